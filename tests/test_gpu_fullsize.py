"""Full-size parity: the 2048 x 2048 two-continuum workload in the launch configuration the
benchmark times (D-scheme, FP64, block IC(0) PCG), checked against stored oracle values on a
seeded sample of cells (tests/golden/c2_oracle.npz, written by tests/golden/make_golden.py
from the CPU oracle alone).  PCG tolerance: 1e-10 as in the workload, and 1e-13 for the
1e-10 parity gate (the stopping test bounds the residual, the error can be up to kappa
times larger)."""
import os

import numpy as np
import pytest

import media

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
from paper_2209_01158_amd import mcdec  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden", "c2_oracle.npz")


def sampled_error(g, z, scheme, step):
    num = den = 0.0
    for a in range(g.n_cont):
        idx = z[f"idx{a}"]
        d = g.get_state(a)[idx] - z[f"{scheme}_s{step}_c{a}"]
        num += float(d @ d)
        den += float(z[f"{scheme}_s{step}_c{a}"] @ z[f"{scheme}_s{step}_c{a}"])
    return np.sqrt(num / den)


@pytest.fixture(scope="module")
def c2():
    return media.config_problem("C2"), np.load(GOLD, allow_pickle=False)


@pytest.mark.parametrize("tol,gate", [(1e-13, 1e-10), (1e-10, 1e-8)])
def test_c2_decoupled_trajectory(c2, tol, gate):
    p, z = c2
    with mcdec.Problem(p, scheme="D", precond="bic0", tol=tol) as g:
        for n in range(1, 101):
            g.step(1)
            if n in (1, 10, 100):
                err = sampled_error(g, z, "D", n)
                print(f"tol {tol}: step {n} sampled rel L2 {err:.2e}", flush=True)
                assert err < gate


def test_c2_coupled_steps(c2):
    p, z = c2
    with mcdec.Problem(p, scheme="coupled", precond="bic0", tol=1e-13) as g:
        for n in range(1, 6):
            g.step(1)
            if n in (1, 5):
                err = sampled_error(g, z, "coupled", n)
                print(f"coupled step {n} sampled rel L2 {err:.2e}", flush=True)
                assert err < 1e-10


def test_c2_mixed_precision(c2):
    p, z = c2
    with mcdec.Problem(p, scheme="D", precision="mixed", precond="bic0", outer_tol=1e-12,
                       inner_tol=1e-4) as g:
        for n in range(1, 11):
            rep = g.step(1)
        err = sampled_error(g, z, "D", 10)
        print(f"mixed step 10 sampled rel L2 {err:.2e}, outer {rep['outer']}", flush=True)
        assert err < 1e-8
