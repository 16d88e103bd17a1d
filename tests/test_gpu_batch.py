"""Batched form: many problems of uneven size advanced by shared launches (mc_batch_step).

Each system keeps its own tiling, partial-sum order and stopping test, so a problem stepped
inside a batch must give bitwise the state it gets when stepped alone with the same options,
whatever else shares the launches.  Against the CPU oracle the bar is the usual one:
relative L2 <= 1e-10 (FP64) and <= 1e-8 (FP32 inner solves in FP64 refinement).  Graph
replay of iteration chunks is checked bitwise against launching the same iterations one by
one.
"""
import os

import numpy as np
import pytest

import media
from oracle import schemes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2209_01158_amd import mcdec  # noqa: E402


def rel(a, b):
    a = np.concatenate([np.ravel(v) for v in a])
    b = np.concatenate([np.ravel(v) for v in b])
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def family(paper=False):
    """Uneven sizes (ragged tiles), two and three continua, lognormal and constant k,
    with and without fractures; with `paper`, also the numerical-results problem with
    wells on a 100 x 100 grid, its fracture permeability lowered from 1e6 to 1e3: at 1e6 the
    FP64 residual floor of the fracture system (eps ||A|| ||x|| / ||b|| ~ 1e-10) lies above
    the 1e-11 outer tolerance of the mixed-precision options."""
    out = [
        media.small_problem(n=70, seed=5, three=True, nseg=6, seg_len=(5, 40)),
        media.small_problem(n=130, seed=8, nseg=10, seg_len=(10, 60)),
        media.small_problem(n=40, seed=2, nseg=4),
        media.small_problem(n=97, seed=9, three=True, nseg=0, lognormal=False),
        media.small_problem(n=200, seed=11, nseg=12, seg_len=(10, 80)),
    ]
    if paper:
        pw = media.paper_problem("3C", n=100)
        pw.k_f = 1e3
        out.append(pw)
    return out


def alone_states(probs, nsteps, **opt):
    out = []
    for p in probs:
        with mcdec.Problem(p, **opt) as g:
            g.step(nsteps)
            out.append(g.get_states())
    return out


def batch_states(probs, nsteps, **opt):
    gs = [mcdec.Problem(p, **opt) for p in probs]
    try:
        with mcdec.Batch(**{k: v for k, v in opt.items()}) as b:
            reps = b.step(gs, nsteps)
        assert all(all(c == 1 for c in r["converged"]) for r in reps), reps
        return [g.get_states() for g in gs], reps
    finally:
        for g in gs:
            g.close()


def assert_bitwise(a_list, b_list):
    for i, (a, b) in enumerate(zip(a_list, b_list)):
        for c, (x, y) in enumerate(zip(a, b)):
            assert np.array_equal(x, y), (i, c, float(np.max(np.abs(x - y))))


OPTS = {
    "fp64_jacobi": dict(scheme="D", precision="fp64", precond="jacobi", tol=1e-12),
    "fp64_bic0": dict(scheme="D", precision="fp64", precond="bic0", tol=1e-12),
    "mixed_bic0": dict(scheme="D", precision="mixed", precond="bic0", outer_tol=1e-11,
                       inner_tol=1e-5),
    "mixed_jacobi": dict(scheme="D", precision="mixed", precond="jacobi", outer_tol=1e-11,
                         inner_tol=1e-5),
    "coupled": dict(scheme="coupled", precision="fp64", precond="bic0", tol=1e-12),
    "fp64_mg": dict(scheme="D", precision="fp64", precond="mg", tol=1e-12),
    "mixed_mg": dict(scheme="D", precision="mixed", precond="mg", outer_tol=1e-11,
                     inner_tol=1e-5),
    "coupled_mg": dict(scheme="coupled", precision="fp64", precond="mg", tol=1e-12),
}


@pytest.mark.parametrize("key", list(OPTS))
def test_batch_equals_alone_bitwise(key):
    print(f"\n[batch {key}]", flush=True)
    probs = family(paper=True)
    opt = OPTS[key]
    alone = alone_states(probs, 3, **opt)
    mixed, reps = batch_states(probs, 3, **opt)
    assert_bitwise(alone, mixed)


@pytest.mark.parametrize("key", ["fp64_bic0", "mixed_bic0", "fp64_mg", "mixed_mg"])
def test_batch_matches_oracle(key):
    print(f"\n[batch oracle {key}]", flush=True)
    probs = family(paper=True)
    nsteps = 3
    opt = dict(OPTS[key])
    if opt["precision"] == "fp64":
        opt["tol"] = 1e-14
    got, reps = batch_states(probs, nsteps, **opt)
    gate = 1e-10 if opt["precision"] == "fp64" else 1e-8
    for p, s in zip(probs, got):
        ref = schemes.run(p, "D", nsteps, keep="last")
        err = rel(s, ref)
        print(p.nx, p.n_cont, err, flush=True)
        assert err < gate


def test_batch_composition_changes():
    """Problems join and leave between steps (the serving pattern): every problem still
    follows its own alone trajectory bitwise."""
    probs = family()
    opt = OPTS["mixed_bic0"]
    alone = alone_states(probs, 3, **opt)
    gs = [mcdec.Problem(p, **opt) for p in probs]
    try:
        with mcdec.Batch(**opt) as b:
            plan = [[0, 1, 2], [0, 2, 3, 4], [1, 3], [0, 1, 2, 4], [2, 3, 4], [1, 3, 4]]
            done = [0] * len(gs)
            for sel in plan:
                sel = [i for i in sel if done[i] < 3]
                if not sel:
                    continue
                b.step([gs[i] for i in sel], 1)
                for i in sel:
                    done[i] += 1
            for i, g in enumerate(gs):
                while done[i] < 3:
                    b.step([g], 1)
                    done[i] += 1
        assert_bitwise(alone, [g.get_states() for g in gs])
    finally:
        for g in gs:
            g.close()


def test_graph_replay_equals_eager(monkeypatch):
    p = media.small_problem(n=130, seed=8, nseg=10, seg_len=(10, 60))
    res = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("MCDEC_GRAPHS", flag)
        with mcdec.Problem(p, precond="bic0", tol=1e-12) as g:
            # the first step captures graphs, later steps replay them; eager work in between
            for _ in range(3):
                g.step(1)
                g.get_states()
            res[flag] = g.get_states()
    assert_bitwise([res["0"]], [res["1"]])


def test_fixed_polling_interval_same_result():
    p = media.small_problem(n=70, seed=5, three=True, nseg=6, seg_len=(5, 40))
    a = alone_states([p], 2, precond="bic0", tol=1e-12)
    b = alone_states([p], 2, precond="bic0", tol=1e-12, check_every=3)
    assert_bitwise(a, b)


def test_batch_failure_is_per_problem():
    """A problem already at its steady state converges at iteration 0; one that needs many
    iterations fails at max_iter = 2.  The first advances, the second keeps its state."""
    steady = media.small_problem(n=33, seed=1, nseg=0, lognormal=False)
    steady.bc_type = np.zeros(4, dtype=steady.bc_type.dtype)      # no-flow everywhere
    steady.p0 = [np.full(s, 0.5) for s in steady.sizes()]
    hard = media.small_problem(n=64, seed=3, nseg=4)
    g1 = mcdec.Problem(steady, tol=1e-12, max_iter=2)
    g2 = mcdec.Problem(hard, tol=1e-12, max_iter=2)
    try:
        before = g2.get_states()
        with mcdec.Batch(tol=1e-12, max_iter=2) as b:
            with pytest.raises(mcdec.McError) as ei:
                b.step([g1, g2], 1)
        assert ei.value.status == mcdec.MC_ENOCONV
        reps = ei.value.report
        assert reps[0]["failed"] == -1 and reps[0]["step"] == 1
        assert reps[1]["failed"] >= 0 and reps[1]["step"] == 0
        for x, y in zip(before, g2.get_states()):
            assert np.array_equal(x, y)
        for x in g1.get_states():
            assert np.allclose(x, 0.5, rtol=0, atol=1e-15)
    finally:
        g1.close()
        g2.close()


def test_batch_rejects_mismatched_options():
    p = media.small_problem(n=16, seed=3, nseg=2)
    with mcdec.Problem(p, precond="jacobi") as g, mcdec.Batch(precond="bic0") as b:
        with pytest.raises(mcdec.McError) as ei:
            b.step([g], 1)
        assert ei.value.status == mcdec.MC_EINVAL
    with mcdec.Problem(p, precond="jacobi") as g, mcdec.Batch(precond="jacobi") as b:
        with pytest.raises(mcdec.McError) as ei:
            b.step([g, g], 1)
        assert ei.value.status == mcdec.MC_EINVAL and "twice" in str(ei.value)


def test_autotune_keeps_state_and_batch_equals_alone():
    mcdec.autotune_clear()
    probs = family()
    opt = OPTS["mixed_bic0"]
    gs = [mcdec.Problem(p, **opt) for p in probs]
    try:
        before = [g.get_states() for g in gs]
        mcdec.autotune(gs, iters=5)
        assert_bitwise(before, [g.get_states() for g in gs])
        til = [mcdec.tilings(g) for g in gs]
        print(til, flush=True)
        alone = alone_states(probs, 2, **opt)      # created after tuning: same tilings
        with mcdec.Batch(**opt) as b:
            b.step(gs, 2)
        assert_bitwise(alone, [g.get_states() for g in gs])
        with mcdec.Problem(probs[1], **opt) as g2:
            assert mcdec.tilings(g2) == til[1]
        ref = schemes.run(probs[4], "D", 2, keep="last")
        assert rel(gs[4].get_states(), ref) < 1e-8
    finally:
        for g in gs:
            g.close()
        mcdec.autotune_clear()


@pytest.mark.parametrize("key", ["fp64_jacobi", "fp64_bic0", "mixed_bic0", "coupled"])
def test_batch_with_3d_problems(key):
    """3-D problems (stacked planes, fracture planes) share launches with 2-D ones: bitwise
    equal to alone, and within the usual gate of the oracle."""
    print(f"\n[batch 3-D {key}]", flush=True)
    probs = [media.box_problem(n=24, nz=12, seed=7, three=True),
             media.small_problem(n=70, seed=5, three=True, nseg=6, seg_len=(5, 40)),
             media.box_problem(n=70, nz=5, seed=3, nplane=6, plane_len=(5, 30))]
    opt = OPTS[key]
    alone = alone_states(probs, 3, **opt)
    mixed, reps = batch_states(probs, 3, **opt)
    assert_bitwise(alone, mixed)
    gate = 1e-8 if opt["precision"] == "mixed" else 1e-9
    for p, s in zip(probs, mixed):
        err = rel(s, schemes.run(p, opt["scheme"], 3, keep="last"))
        print(p.nx, p.nz, err, flush=True)
        assert err < gate
