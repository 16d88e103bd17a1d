"""GPU parity of the coarse-grid NLMC path (Section 4) against the oracle (oracle/nlmc.py).

The GPU builds the basis functions by band Cholesky factorizations of the local operators
and the constraint Schur complement; the oracle solves the saddle-point systems of eq.
eq:basis by sparse LU.  Both then form the conservative coarse operator and step the coarse
schemes (eqs. is-nlmc, si-nlmc).  Gates: the coarse operator, storage and right-hand side
to 1e-9 relative (max norm; the local operators at k_f / k_m = 1e6 have condition numbers
near 1e8, so the two factorizations agree to about that), and every scheme's coarse
trajectory to 1e-9 relative L2.
"""
import numpy as np
import pytest

import media
from oracle import nlmc, schemes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2209_01158_amd import mcdec  # noqa: E402


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / (nb if nb > 0 else 1.0)


def _dirichlet3():
    p = media.small_problem(n=48, seed=5, three=True, nseg=6, seg_len=(5, 30))
    return p


CASES = {
    "paper2C_n40_l1": (lambda: media.paper_problem("2C", n=40), 8, 8, 1),
    "paper3C_n40_l2": (lambda: media.paper_problem("3C", n=40), 8, 8, 2),
    "dirichlet3C_n48_l1": (_dirichlet3, 6, 8, 1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_nlmc_system_and_trajectories(name):
    make, bx, by, layers = CASES[name]
    p = make()
    cs = nlmc.coarse_system(nlmc.Basis(p, nlmc.CoarseGrid(p.nx, p.ny, bx, by), layers))
    x0 = nlmc.unit_means(cs.units, p.initial_state())
    with mcdec.Problem(p, scheme="D") as g, mcdec.Nlmc(g, bx, by, layers) as nl:
        inf = nl.info()
        assert inf.n_units == cs.units.n
        assert list(inf.sizes)[:inf.n_cont] == list(cs.units.sizes)
        A, M, F = nl.system()
        ea = np.abs(A - cs.A).max() / np.abs(cs.A).max()
        em = np.abs(M - np.diag(cs.M)).max() / np.abs(np.diag(cs.M)).max()
        ef = np.abs(F - cs.F).max() / max(np.abs(cs.F).max(), 1e-300)
        print(f"{name}: N_H {inf.n_units}, band <= {inf.max_band}, region <= "
              f"{inf.max_region_unknowns}, A {ea:.2e}, M {em:.2e}, F {ef:.2e}, setup ms "
              f"{list(inf.setup_ms)}", flush=True)
        assert ea < 1e-9 and em < 1e-14 and ef < 1e-12
        assert rel(nl.get_state(), x0) < 1e-14
        for scheme in ("coupled", "D", "L", "U"):
            nl.set_state()
            ref = nlmc.run(cs, p.tau, scheme, x0, 10)
            for n in range(1, 11):
                nl.step(scheme, 1)
                e = rel(nl.get_state(), ref[n])
                assert e < 1e-9, (scheme, n, e)
            print(f"  {scheme}: layer 10 rel L2 vs oracle {e:.2e}", flush=True)


def test_nlmc_paper_2c_accuracy():
    """The paper's 2C problem on its 20 x 20 coarse grid with two layers of oversampling: the
    GPU's coarse schemes reach the oracle's e_H against the fine coupled solution (the size
    of Table tab-2c-ms) and agree with the oracle's coarse trajectory."""
    p = media.paper_problem("2C")
    cs = nlmc.coarse_system(nlmc.Basis(p, nlmc.CoarseGrid(200, 200, 10, 10), 2))
    x0 = nlmc.unit_means(cs.units, p.initial_state())
    fine = schemes.run(p, "coupled", 50, keep="last")
    ref_m = nlmc.unit_means(cs.units, fine)
    with mcdec.Problem(p, scheme="D") as g, mcdec.Nlmc(g, 10, 10, 2) as nl:
        for scheme in ("coupled", "D", "L", "U"):
            nl.set_state()
            nl.step(scheme, 50)
            x = nl.get_state()
            xo = nlmc.run(cs, p.tau, scheme, x0, 50, keep="last")
            e_gpu, e_or = nlmc.e_H(x, ref_m), nlmc.e_H(xo, ref_m)
            print(f"2C 20x20 l=2 {scheme}: e_H GPU {100 * e_gpu:.4f} % oracle "
                  f"{100 * e_or:.4f} %, GPU vs oracle {rel(x, xo):.2e}", flush=True)
            assert rel(x, xo) < 1e-9
            assert e_gpu < 5e-3


def test_nlmc_refusals():
    p = media.paper_problem("2C", n=40)
    with mcdec.Problem(p) as g:
        with pytest.raises(mcdec.McError, match="tile"):
            mcdec.Nlmc(g, 7, 8, 1)
    with mcdec.Problem(p, scheme="EX") as g:
        with pytest.raises(mcdec.McError, match="EX"):
            mcdec.Nlmc(g, 8, 8, 1)
