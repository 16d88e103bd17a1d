"""GPU parity of the HIP path against the CPU oracle (element by element, same seeded inputs).

Tolerances: FP64 operator applications agree to rounding (<= 1e-14 relative, the only
difference is summation order and FMA contraction); FP64 solves and trajectories to a
relative L2 error <= 1e-10; mixed-precision refinement to <= 1e-8.
"""
import ctypes as C

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg  # noqa: F401  (sp.linalg)
import pytest

import media
from oracle import fv, schemes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2209_01158_amd import mcdec  # noqa: E402

DEV = torch.device("cuda:0")


def rel(a, b):
    a = np.concatenate([np.ravel(v) for v in a]) if isinstance(a, (list, tuple)) else np.ravel(a)
    b = np.concatenate([np.ravel(v) for v in b]) if isinstance(b, (list, tuple)) else np.ravel(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def T(v):
    return torch.tensor(np.ascontiguousarray(v, np.float64), device=DEV)


CASES = {
    "c1": lambda: media.config_problem("C1"),
    # ragged: 200 = 3 * 64 + 8 columns, 200 = 12 * 16 + 8 rows; lognormal k, any-angle fractures
    "ragged200": lambda: media.small_problem(n=200, seed=11, nseg=12, seg_len=(10, 80)),
    "three70": lambda: media.small_problem(n=70, seed=5, three=True, nseg=6, seg_len=(5, 40)),
    "tiny1": lambda: media.small_problem(n=1, seed=1, nseg=0, lognormal=False),
}
# a dense fracture network: hundreds of crossing cells on a 48 x 48 grid
DENSE = lambda: media.small_problem(n=48, seed=13, nseg=40, seg_len=(10, 40))  # noqa: E731


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print(f"\n[case {request.param}]", flush=True)
    return request.param, CASES[request.param]()


def test_apply_continuum(case):
    name, p = case
    asm = fv.assemble(p)
    rng = np.random.default_rng(0)
    with mcdec.Problem(p) as g:
        for a in range(p.n_cont):
            K = schemes.continuum_matrix(asm, p.tau, a)
            x = rng.standard_normal(p.sizes()[a])
            y = torch.zeros(p.sizes()[a], dtype=torch.float64, device=DEV)
            g.apply_continuum(a, T(x), y)
            ref = K @ x
            assert rel(y.cpu().numpy(), ref) < 1e-14, (name, a)


def test_apply_coupled(case):
    name, p = case
    asm = fv.assemble(p)
    K = schemes.coupled_matrix(asm, p.tau)
    x = np.random.default_rng(1).standard_normal(p.dof())
    y = torch.zeros(p.dof(), dtype=torch.float64, device=DEV)
    with mcdec.Problem(p) as g:
        g.apply_coupled(T(x), y)
    assert rel(y.cpu().numpy(), K @ x) < 1e-14


def test_assemble_rhs(case):
    name, p = case
    asm = fv.assemble(p)
    rng = np.random.default_rng(2)
    st = [rng.random(s) for s in p.sizes()]
    with mcdec.Problem(p) as g:
        g.set_states(st)
        for a in range(p.n_cont):
            b = torch.zeros(p.sizes()[a], dtype=torch.float64, device=DEV)
            g.assemble_rhs(a, b)
            ref = schemes.decoupled_rhs(asm, p.tau, a, st, "D")
            assert rel(b.cpu().numpy(), ref) < 1e-14, a


def test_solve_continuum(case):
    name, p = case
    asm = fv.assemble(p)
    rng = np.random.default_rng(3)
    with mcdec.Problem(p, tol=1e-14) as g:
        for a in range(p.n_cont):
            K = schemes.continuum_matrix(asm, p.tau, a)
            rhs = rng.random(p.sizes()[a])
            ref = schemes.DirectSolver(K).solve(rhs)
            x = torch.zeros(p.sizes()[a], dtype=torch.float64, device=DEV)
            rep = g.solve_continuum(a, T(rhs), x)
            err = rel(x.cpu().numpy(), ref)
            print(name, a, rep["iters"][a], err)
            assert err < 1e-10


@pytest.mark.parametrize("scheme", ["D", "coupled", "L", "U"])
def test_trajectory(case, scheme):
    name, p = case
    nsteps = 20 if name == "c1" else 4
    ref = schemes.run(p, scheme, nsteps, keep="all")
    with mcdec.Problem(p, scheme=scheme, tol=1e-14) as g:
        for n in range(1, nsteps + 1):
            rep = g.step(1)
            err = rel(g.get_states(), ref[n])
            assert err < 1e-10, (name, scheme, n, err, rep)


@pytest.mark.parametrize("scheme", ["D", "L", "U", "EX"])
@pytest.mark.parametrize("name", ["c1", "three70"])
def test_small_system_path(name, scheme):
    """Small systems (small_max): one workgroup per continuum runs its whole Jacobi PCG in
    one launch; the layers match the oracle's as the general path's do."""
    p = CASES[name]() if scheme != "EX" else media.small_problem(n=40, seed=2, nseg=4,
                                                                   tau=1e-5, nsteps=3)
    nsteps = 4 if scheme != "EX" else 3
    ref = schemes.run(p, scheme, nsteps, keep="all")
    with mcdec.Problem(p, scheme=scheme, precond="jacobi", tol=1e-14, small_max=1 << 20) as g:
        for n in range(1, nsteps + 1):
            rep = g.step(1)
            err = rel(g.get_states(), ref[n])
            assert err < 1e-10, (name, scheme, n, err, rep)
            assert all(rep["converged"]), rep


def test_ex_scheme_small_tau():
    p = media.small_problem(n=40, seed=2, nseg=4, tau=1e-5, nsteps=3)
    ref = schemes.run(p, "EX", 3, keep="last")
    with mcdec.Problem(p, scheme="EX", tol=1e-14) as g:
        g.step(3)
        assert rel(g.get_states(), ref) < 1e-10


@pytest.mark.parametrize("name", ["ragged200", "three70"])
def test_mixed_precision_refinement(name):
    p = CASES[name]()
    ref = schemes.run(p, "D", 3, keep="last")
    with mcdec.Problem(p, precision="mixed", outer_tol=1e-12, inner_tol=1e-5) as g:
        rep = g.step(3)
        err = rel(g.get_states(), ref)
        print(name, rep, err)
        assert err < 1e-8
        assert all(c == 1 for c in rep["converged"])


def test_noconv_is_transactional():
    p = media.small_problem(n=64, seed=3, nseg=4)
    with mcdec.Problem(p, tol=1e-14, max_iter=1) as g:
        before = g.get_states()
        with pytest.raises(mcdec.McError) as ei:
            g.step(1)
        assert ei.value.status == mcdec.MC_ENOCONV
        after = g.get_states()
        for a, b in zip(before, after):
            assert np.array_equal(a, b)


def test_invalid_descriptor_rejected():
    p = media.small_problem(n=16, seed=3, nseg=2)
    p.host = p.host.copy()
    p.host[0] = 16 * 16 + 5
    with pytest.raises(mcdec.McError) as ei:
        mcdec.Problem(p)
    assert ei.value.status == mcdec.MC_EINVAL and "host" in str(ei.value)


# ------------------------------------------------------------------------------------
# block IC(0) preconditioner
# ------------------------------------------------------------------------------------
from oracle import precond  # noqa: E402


@pytest.mark.parametrize("name", ["ragged200", "three70", "c1", "dense48"])
def test_block_ic0_apply(name):
    p = DENSE() if name == "dense48" else CASES[name]()
    asm = fv.assemble(p)
    rng = np.random.default_rng(4)
    with mcdec.Problem(p, precond="bic0") as g:
        for a in range(p.n_cont):
            K = schemes.continuum_matrix(asm, p.tau, a)
            r = rng.standard_normal(p.sizes()[a])
            z = torch.zeros(p.sizes()[a], dtype=torch.float64, device=DEV)
            g.apply_precond(a, T(r), z)
            if a < p.n_omega:
                facs = precond.block_precond(K, precond.grid_tile_blocks(p.nx, p.ny))
                ref = precond.block_precond_apply(facs, r)
                tol = 2e-6   # FP32 copies of the grid factor (about 6e-8 relative rounding)
            else:
                # fracture: chains cut at the crossing cells plus the crossing-cell Schur
                # complement form an exact solve of the fracture system
                ref = schemes.DirectSolver(K).solve(r)
                tol = 1e-10
            err = rel(z.cpu().numpy(), ref)
            print(name, a, err, g.info().n_crossing)
            assert err < tol, (name, a, err)


@pytest.mark.parametrize("scheme", ["D", "coupled", "U"])
def test_trajectory_bic0(case, scheme):
    name, p = case
    nsteps = 5 if name == "c1" else 3
    ref = schemes.run(p, scheme, nsteps, keep="all")
    with mcdec.Problem(p, scheme=scheme, precond="bic0", tol=1e-14) as g:
        for n in range(1, nsteps + 1):
            rep = g.step(1)
            err = rel(g.get_states(), ref[n])
            assert err < 1e-10, (name, scheme, n, err, rep)


def test_chain_ic0_exact_without_crossings():
    # axis-aligned, non-overlapping segments that do not cross: every chain is a segment and
    # block IC(0) on the fracture system is its exact inverse -> one PCG iteration
    p = media.small_problem(n=64, seed=21, nseg=3, axis=True, seg_len=(10, 30))
    cross = (p.edges[:, 1] - p.edges[:, 0]) != 1
    if cross.any():
        pytest.skip("generator produced a crossing")
    with mcdec.Problem(p, precond="bic0", tol=1e-12) as g:
        rep = g.step(1)
    assert rep["iters"][-1] <= 1, rep


@pytest.mark.parametrize("name", ["ragged200", "c1", "dense48"])
def test_fracture_solve_exact_with_crossings(name):
    """With crossing cells the fracture preconditioner is the exact inverse: the fracture
    PCG stops after at most two iterations, in FP64 and inside FP32 refinement; the
    trajectory still matches the oracle."""
    p = DENSE() if name == "dense48" else CASES[name]()
    with mcdec.Problem(p, precond="bic0", tol=1e-12) as g:
        assert g.info().n_crossing > 0
        for _ in range(3):
            rep = g.step(1)
            assert rep["iters"][-1] <= 2, rep
    with mcdec.Problem(p, precond="bic0", precision="mixed", outer_tol=1e-11,
                       inner_tol=1e-6) as g:
        for _ in range(3):
            rep = g.step(1)
        print(rep)
        assert rep["outer"][-1] <= 3 and rep["iters"][-1] <= 2 * rep["outer"][-1] + 2, rep
        ref = schemes.run(p, "D", 3, keep="last")
        assert rel(g.get_states(), ref) < 1e-8


@pytest.mark.parametrize("name", ["ragged200", "three70"])
def test_mixed_precision_bic0(name):
    p = CASES[name]()
    ref = schemes.run(p, "D", 3, keep="last")
    with mcdec.Problem(p, precision="mixed", precond="bic0", outer_tol=1e-12,
                       inner_tol=1e-5) as g:
        rep = g.step(3)
        err = rel(g.get_states(), ref)
        print(name, rep, err)
        assert err < 1e-8


@pytest.mark.parametrize("precond", ["bic0", "jacobi"])
def test_mixed_precision_tiny_magnitudes(precond):
    """Residuals far below FP32's normal range (pressures of order 1e-40) still refine to
    the FP64 answer: the inner FP32 residual is scaled by a power of two."""
    p = media.small_problem(n=64, seed=3, nseg=4)
    p.bc_value = np.asarray(p.bc_value, float) * 1e-40
    ref = schemes.run(p, "D", 3, keep="last")
    with mcdec.Problem(p, precision="mixed", precond=precond, outer_tol=1e-11,
                       inner_tol=1e-6) as g:
        rep = g.step(3)
        err = rel(g.get_states(), ref)
        print(precond, rep, err)
        assert err < 1e-8
        assert all(c == 1 for c in rep["converged"])


# ------------------------------------------------------------------------------------
# multigrid V-cycle preconditioner (option "mg")
# ------------------------------------------------------------------------------------
MG_CASES = {
    # 300 x 270 -> 150 x 135 -> 75 x 68 -> 38 x 34 -> 19 x 17 -> 10 x 9 (dense): ragged
    # tiles and odd sizes on every level
    "rect300x270": lambda: media.rect_problem(300, 270, seed=5),
    # diffusion-dominated (tau = 1e4): the full hierarchy down to the dense coarsest level
    # (the storage-dominated cases above stop after their first coarse level)
    "deep300x270": lambda: media.rect_problem(300, 270, seed=5, tau=1e4),
    "strip1x700": lambda: media.rect_problem(1, 700, seed=6),      # 700 -> 350 -> 175
    # level ratios (row sums over face conductances) 1.0, 4.0, 16 on levels 1-3: FP64
    # solves stop at level 3 (1292 cells, above the tail), mixed precision at level 2
    "mid300x270": lambda: media.rect_problem(300, 270, seed=5, tau=0.046),
    "ragged200": CASES["ragged200"],
    "three70": CASES["three70"],
}


def mg_depth(K, nx, ny, ratio):
    """Coarse levels of the V-cycle for operator K: the hierarchy stops at the first level
    above the 1024-cell tail whose row sums reach `ratio` times its face conductances
    (both summed over the level), else it runs down to the dense coarsest level."""
    full = precond.vcycle_setup(K, nx, ny)
    for l in range(1, len(full)):
        Kl = full[l]["K"]
        if Kl.shape[0] <= 1024:
            break
        rs = float(np.asarray(Kl.sum(axis=1)).sum())
        fs = float(-(Kl - sp.diags(Kl.diagonal())).sum())
        if rs >= ratio * fs:
            return l
    return len(full) - 1


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["mid300x270", "deep300x270", "three70"])
def test_mg_depth(name, precision):
    """Where the hierarchy stops: a row-sum ratio of 8 for FP64 solves, 2 for the inner FP32
    solves of mixed precision."""
    print(f"\n[mg depth {name} {precision}]", flush=True)
    p = MG_CASES[name]()
    asm = fv.assemble(p)
    with mcdec.Problem(p, precond="mg", precision=precision) as g:
        got = list(g.info().mg_levels)
        sw = list(g.info().mg_stop_sweeps)
    want = [mg_depth(schemes.continuum_matrix(asm, p.tau, a), p.nx, p.ny,
                     8.0 if precision == "fp64" else 2.0) for a in range(p.n_omega)]
    print(name, precision, got[:p.n_omega], want, flush=True)
    assert got[:p.n_omega] == want
    if name == "mid300x270":
        assert want == [3 if precision == "fp64" else 2]
        # the FP64 stop level (ratio 16) is smoothed once, the mixed one (ratio 4) twice
        assert sw[0] == (1 if precision == "fp64" else 2), sw


@pytest.mark.parametrize("name", list(MG_CASES))
def test_mg_apply(name):
    """One V-cycle z = V r on every grid continuum against the oracle's cycle (FP32 copies of
    the smoother factors: relative error within 2e-5); the fracture continuum keeps the
    exact solve."""
    print(f"\n[mg apply {name}]", flush=True)
    p = MG_CASES[name]()
    asm = fv.assemble(p)
    rng = np.random.default_rng(4)
    with mcdec.Problem(p, precond="mg") as g:
        inf = g.info()
        for a in range(p.n_cont):
            K = schemes.continuum_matrix(asm, p.tau, a)
            r = rng.standard_normal(p.sizes()[a])
            z = torch.zeros(p.sizes()[a], dtype=torch.float64, device=DEV)
            g.apply_precond(a, T(r), z)
            if a < p.n_omega:
                want = mg_depth(K, p.nx, p.ny, 8.0)
                assert inf.mg_levels[a] == want, (inf.mg_levels[a], want)
                # an FP64 hierarchy stops only where a level's row sums reach 8 times its
                # face conductances: that level is smoothed once
                full = len(precond.vcycle_setup(K, p.nx, p.ny)) - 1
                sweeps = 1 if want < full else 0
                assert inf.mg_stop_sweeps[a] == sweeps, (inf.mg_stop_sweeps[a], sweeps)
                lev = precond.vcycle_setup(K, p.nx, p.ny, max_levels=want, last_sweeps=1)
                ref = precond.vcycle_apply(lev, r)
                tol = 2e-5
            else:
                ref = schemes.DirectSolver(K).solve(r)
                tol = 1e-10
            err = rel(z.cpu().numpy(), ref)
            print(name, a, inf.mg_levels[a], err, flush=True)
            assert err < tol, (name, a, err)


@pytest.mark.parametrize("scheme", ["D", "coupled", "U"])
@pytest.mark.parametrize("name", ["rect300x270", "deep300x270", "ragged200", "three70"])
def test_trajectory_mg(name, scheme):
    print(f"\n[mg trajectory {name} {scheme}]", flush=True)
    p = MG_CASES[name]()
    nsteps = 3
    ref = schemes.run(p, scheme, nsteps, keep="all")
    with mcdec.Problem(p, scheme=scheme, precond="mg", tol=1e-14) as g:
        for n in range(1, nsteps + 1):
            rep = g.step(1)
            err = rel(g.get_states(), ref[n])
            assert err < 1e-10, (name, scheme, n, err, rep)


@pytest.mark.parametrize("name", ["rect300x270", "deep300x270", "three70", "strip1x700"])
def test_mixed_precision_mg(name):
    print(f"\n[mg mixed {name}]", flush=True)
    p = MG_CASES[name]()
    ref = schemes.run(p, "D", 3, keep="last")
    with mcdec.Problem(p, precision="mixed", precond="mg", outer_tol=1e-12,
                       inner_tol=1e-5) as g:
        rep = g.step(3)
        err = rel(g.get_states(), ref)
        print(name, rep, err)
        assert err < 1e-8


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["rect300x270", "deep300x270", "ragged200", "three70"])
def test_fused_restriction_matches_unfused(name, prec, monkeypatch):
    """Inside FP64 PCG the update kernel forms the finest level's in-block share of the
    restriction into level 1 and the level-1 kernel adds the couplings across the block
    edges; the same cycle with the restriction kernel doing it all (MCDEC_MG_FUSE=0) gives the
    same iterations and states up to rounding (mixed precision: the FP32 inner solves keep
    the separate restriction, so both runs agree as well)."""
    print(f"\n[mg fused restriction {name} {prec}]", flush=True)
    p = MG_CASES[name]()
    kw = dict(precond="mg", precision=prec)
    kw.update(dict(tol=1e-12) if prec == "fp64" else dict(outer_tol=1e-12, inner_tol=1e-5))
    out = {}
    for fuse in ("0", "1"):
        monkeypatch.setenv("MCDEC_MG_FUSE", fuse)
        with mcdec.Problem(p, **kw) as g:
            rep = g.step(3)
            out[fuse] = (rep["iters"], np.concatenate(g.get_states()))
    print(out["0"][0], out["1"][0], rel(out["1"][1], out["0"][1]))
    for a, b in zip(out["0"][0], out["1"][0]):
        assert abs(a - b) <= 1, (out["0"][0], out["1"][0])
    assert rel(out["1"][1], out["0"][1]) < 1e-10


def test_mg_fewer_iterations_than_block_ic0():
    """On a 300 x 270 lognormal grid with a long time step (diffusion dominates storage,
    k tau / h^2 of order 100) the V-cycle needs well under half the PCG iterations of
    one-level block IC(0) at the same tolerance."""
    p = media.rect_problem(300, 270, seed=5, tau=10.0)
    its = {}
    for pc in ("bic0", "mg"):
        with mcdec.Problem(p, precond=pc, tol=1e-10) as g:
            its[pc] = g.step(1)["iters"][0]
    print(its)
    assert its["mg"] * 2 < its["bic0"], its


def test_kernel_timing_samples_and_keeps_results():
    """Kernel timing (one iteration in 4 launched with events, the rest replayed from graphs)
    counts every issued launch, samples the grid operator, update and (mg) finest
    post-smoothing kernels, and leaves the trajectory bitwise unchanged."""
    p = MG_CASES["rect300x270"]()
    with mcdec.Problem(p, precond="mg", tol=1e-12) as g:
        g.step(2)
        ref = g.get_states()
    with mcdec.Problem(p, precond="mg", tol=1e-12) as g:
        g.profile(True, every=4)
        rep = g.step(2)
        reads = [g.profile_read(w) for w in range(7)]
        levels = g.info().mg_levels[0]
        sweeps = g.info().mg_stop_sweeps[0]
        g.profile(False)
        got = g.get_states()
    print(rep, reads, levels)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    for sampled, ms, issued in reads[:3]:
        assert sampled >= 1 and ms > 0 and issued >= sum(rep["iters"][:1])
        assert sampled <= issued // 4 + 2
    # the V-cycle's coarse kernels (this storage-dominated problem keeps one coarse level,
    # row sums 45 times its conductances, restricted into with pre-smoothing and smoothed
    # once, no tail): one restriction launch per cycle, a sampled cycle timed whole, and no
    # coarse post-smoothing
    assert levels == 1 and sweeps == 1
    cycles = reads[2][2]
    sampled, ms, issued = reads[3]
    assert issued == cycles and sampled == reads[2][0] and ms > 0
    assert reads[4][2] == 0 and reads[5][2] == 0 and reads[6][2] == 0
    with pytest.raises(mcdec.McError):
        g2 = mcdec.Problem(p, precond="mg")
        try:
            g2.profile_read(7)
        finally:
            g2.close()


def test_reports_are_deterministic():
    """Two identical runs give bitwise the same states and the same per-layer reports
    (iteration and refinement-pass counts), in FP64 and in FP32 refinement, with three
    continua solved by concurrent groups."""
    p = CASES["three70"]()
    for opt in (dict(precond="mg", tol=1e-12),
                dict(precond="mg", precision="mixed", outer_tol=1e-11, inner_tol=1e-4),
                dict(precond="bic0", precision="mixed", outer_tol=1e-11, inner_tol=1e-6)):
        runs = []
        for _ in range(2):
            with mcdec.Problem(p, **opt) as g:
                reps = [g.step(1) for _ in range(4)]
                runs.append(([(r["iters"], r["outer"]) for r in reps], g.get_states()))
        assert runs[0][0] == runs[1][0], (opt, runs[0][0], runs[1][0])
        for a, b in zip(runs[0][1], runs[1][1]):
            assert np.array_equal(a, b)


def test_warm_start_modes_and_history_reset():
    """Every warm start (linear extrapolation, the default; the previous layer; adaptive
    extrapolation) meets the oracle trajectory over 8 layers.  The adaptive mode's order stays
    within the history it has: p^{n-1} at the first layer, linear at the second, then at most
    min(n - 2, 3).  A state change resets the layer history, so stepping after set_states(p0)
    gives bitwise the layers of a fresh problem."""
    p = CASES["ragged200"]()
    ref = schemes.run(p, "D", 8, keep="all")
    for ws in ("extrapolate", "previous", "adaptive"):
        with mcdec.Problem(p, precond="mg", tol=1e-14, warm_start=ws) as g:
            for n in range(1, 9):
                rep = g.step(1)
                assert rel(g.get_states(), ref[n]) < 1e-10, (ws, n)
                for o in rep["warm_order"]:
                    if ws == "previous":
                        assert o == 0
                    elif ws == "extrapolate":
                        assert o == (1 if n >= 2 else 0)
                    else:
                        assert o == (0 if n == 1 else 1) if n <= 2 else 0 <= o <= min(n - 2, 3)
    with mcdec.Problem(p, precond="mg", tol=1e-12) as a, \
            mcdec.Problem(p, precond="mg", tol=1e-12) as b:
        a.step(3)
        a.set_states(p.initial_state())
        a.step(2)
        b.step(2)
        for x, y in zip(a.get_states(), b.get_states()):
            assert np.array_equal(x, y)


def test_adaptive_warm_start_saves_iterations():
    """On a smooth trajectory (300 x 270 lognormal grid, 16 layers) the adaptive warm start
    settles on high extrapolation orders and needs fewer PCG iterations than the linear one
    (the default); both meet the oracle."""
    p = MG_CASES["rect300x270"]()
    ref = schemes.run(p, "D", 16, keep="last")
    its, orders = {}, {}
    for ws in ("extrapolate", "adaptive"):
        with mcdec.Problem(p, precond="mg", tol=1e-12, warm_start=ws) as g:
            its[ws], orders[ws] = 0, []
            for _ in range(16):
                rep = g.step(1)
                its[ws] += rep["iters"][0]
                orders[ws].append(rep["warm_order"][0])
            assert rel(g.get_states(), ref) < 1e-9, ws
    print(its, orders)
    assert its["adaptive"] < its["extrapolate"], its
    assert max(orders["adaptive"][8:]) >= 2, orders


# ------------------------------------------------------------------------------------
# degenerate inputs
# ------------------------------------------------------------------------------------
def _no_transfer():
    p = media.small_problem(n=70, seed=5, three=True, nseg=6, seg_len=(5, 40))
    p.sigma_f = np.zeros_like(p.sigma_f)
    p.sigma_omega = 0.0
    return p


def _zero_k():
    # a quarter of the matrix cells impermeable (their faces carry no flux) and an
    # impermeable natural-fracture continuum
    p = media.small_problem(n=90, seed=6, three=True, nseg=5, seg_len=(5, 40))
    k = p.omega[0].k.copy()
    k[np.random.default_rng(1).random(k.shape) < 0.25] = 0.0
    p.omega[0].k = k
    p.omega[1].k_const = 0.0
    return p


def _isolated_fracture():
    # fracture cells with no fracture-fracture connections at all
    p = media.small_problem(n=64, seed=8, nseg=5, seg_len=(5, 30))
    p.edges = np.zeros((0, 2), np.int32)
    p.edge_d = np.zeros(0)
    return p


DEGENERATE = {"no_transfer": _no_transfer, "zero_k": _zero_k,
              "isolated_fracture": _isolated_fracture}


@pytest.mark.parametrize("precond", ["jacobi", "bic0", "mg"])
@pytest.mark.parametrize("name", list(DEGENERATE))
def test_degenerate_inputs(name, precond):
    print(f"\n[degenerate {name} {precond}]", flush=True)
    p = DEGENERATE[name]()
    p.check()
    for scheme in ("D", "coupled", "U"):
        ref = schemes.run(p, scheme, 3, keep="all")
        with mcdec.Problem(p, scheme=scheme, precond=precond, tol=1e-14) as g:
            for n in range(1, 4):
                rep = g.step(1)
                err = rel(g.get_states(), ref[n])
                assert err < 1e-10, (name, precond, scheme, n, err, rep)
    if name == "no_transfer":
        # with no transfer the continua are independent: every scheme is the coupled one
        d = schemes.run(p, "D", 3, keep="last")
        c = schemes.run(p, "coupled", 3, keep="last")
        assert rel(d, c) < 1e-13


# ------------------------------------------------------------------------------------
# 3-D grids (stacked planes, 7-point stencil) with fracture planes
# ------------------------------------------------------------------------------------
def _box_zdirichlet():
    # Dirichlet bottom and top as well; 70 = 64 + 6 columns and 70 * 5 = 350 = 21 * 16 + 14
    # stacked rows: ragged tiles in both directions, planes meeting inside tiles
    p = media.box_problem(n=70, nz=5, seed=3, nplane=6, plane_len=(5, 30))
    p.bc_type_z = np.array([1, 1], np.int32)
    p.bc_value_z = np.array([0.3, 0.8])
    return p


BOXES = {
    "box24x12_3c": lambda: media.box_problem(n=24, nz=12, seed=7, three=True),
    "box70x5_zdir": _box_zdirichlet,
    "box2x3": lambda: media.box_problem(n=2, nz=3, seed=1, nplane=1, plane_len=(1, 2)),
    # planes of two whole tile rows: the operator kernel takes its tile rows z-fastest
    "box64x5": lambda: media.box_problem(n=64, nz=5, seed=9, nplane=4, plane_len=(4, 24)),
}


@pytest.fixture(scope="module", params=list(BOXES))
def box(request):
    print(f"\n[3-D case {request.param}]", flush=True)
    return request.param, BOXES[request.param]()


def test_3d_operators(box):
    name, p = box
    asm = fv.assemble(p)
    rng = np.random.default_rng(4)
    with mcdec.Problem(p) as g:
        for a in range(p.n_cont):
            K = schemes.continuum_matrix(asm, p.tau, a)
            x = rng.standard_normal(p.sizes()[a])
            y = torch.zeros(p.sizes()[a], dtype=torch.float64, device=DEV)
            g.apply_continuum(a, T(x), y)
            assert rel(y.cpu().numpy(), K @ x) < 1e-14, (name, a)
        K = schemes.coupled_matrix(asm, p.tau)
        x = rng.standard_normal(p.dof())
        y = torch.zeros(p.dof(), dtype=torch.float64, device=DEV)
        g.apply_coupled(T(x), y)
        assert rel(y.cpu().numpy(), K @ x) < 1e-14, name


@pytest.mark.parametrize("precond", ["jacobi", "bic0"])
@pytest.mark.parametrize("scheme", ["D", "coupled", "U"])
def test_3d_trajectory(box, scheme, precond):
    name, p = box
    ref = schemes.run(p, scheme, 3, keep="all")
    with mcdec.Problem(p, scheme=scheme, precond=precond, tol=1e-14) as g:
        for n in range(1, 4):
            rep = g.step(1)
            err = rel(g.get_states(), ref[n])
            assert err < 1e-10, (name, scheme, precond, n, err, rep)


def test_3d_mixed_precision(box):
    name, p = box
    ref = schemes.run(p, "D", 3, keep="last")
    with mcdec.Problem(p, precision="mixed", precond="bic0", outer_tol=1e-12) as g:
        rep = g.step(3)
        err = rel(g.get_states(), ref)
        assert err < 1e-8, (name, err, rep)


# ------------------------------------------------------------------------------------
# two-level block preconditioner of fracture graphs with more crossing cells than the exact
# solve takes (fracture planes, dense networks); MCDEC_FRACTURE_EXACT_MAX = 0 selects it for
# every graph with crossings
# ------------------------------------------------------------------------------------
FRAC_BLOCK_CASES = {
    "dense48": DENSE,
    "box24x12_3c": BOXES["box24x12_3c"],
    "box70x5_zdir": BOXES["box70x5_zdir"],
    "box96x8": lambda: media.box_problem(n=96, nz=8, seed=4, nplane=8, plane_len=(10, 40)),
}


def bfs_blocks(nf, edges, size=64):
    """Blocks of at most `size` connected fracture cells, grown breadth-first from the
    lowest unassigned cell over neighbours in ascending order."""
    nbr = [[] for _ in range(nf)]
    for a, b in np.asarray(edges, np.int64).reshape(-1, 2):
        nbr[a].append(b)
        nbr[b].append(a)
    for v in nbr:
        v.sort()
    blk = -np.ones(nf, np.int64)
    nb = 0
    for s in range(nf):
        if blk[s] >= 0:
            continue
        queue, blk[s] = [s], nb
        h = 0
        while h < len(queue) and len(queue) < size:
            for v in nbr[queue[h]]:
                if blk[v] < 0 and len(queue) < size:
                    blk[v] = nb
                    queue.append(v)
            h += 1
        nb += 1
    return blk, nb


def two_level_apply(K, blk, nb, r):
    """z = B^-1 r + P (P^T K P)^-1 P^T r with B the block diagonal of K."""
    n = K.shape[0]
    Pm = sp.csr_matrix((np.ones(n), (np.arange(n), blk)), shape=(n, nb))
    Kc = sp.coo_matrix(K)
    m = blk[Kc.row] == blk[Kc.col]
    B = sp.csc_matrix((Kc.data[m], (Kc.row[m], Kc.col[m])), shape=(n, n))
    y = sp.linalg.splu(B).solve(r)
    Ac = (Pm.T @ K @ Pm).toarray()
    return y + Pm @ np.linalg.solve(Ac, Pm.T @ r)


@pytest.mark.parametrize("name", list(FRAC_BLOCK_CASES))
def test_fracture_blocks_apply(name, monkeypatch):
    """z = M^-1 r of the two-level block preconditioner against the same formula formed with
    sparse and dense direct solves (FP32 block and coarse inverses: relative error within
    1e-5)."""
    print(f"\n[fracture blocks apply {name}]", flush=True)
    monkeypatch.setenv("MCDEC_FRACTURE_EXACT_MAX", "0")
    p = FRAC_BLOCK_CASES[name]()
    asm = fv.assemble(p)
    a = p.n_omega
    K = schemes.continuum_matrix(asm, p.tau, a)
    blk, nb = bfs_blocks(p.sizes()[a], p.edges)
    rng = np.random.default_rng(8)
    with mcdec.Problem(p, precond="bic0") as g:
        inf = g.info()
        assert inf.n_frac_blocks == nb and inf.n_crossing == 0, (inf.n_frac_blocks, nb)
        r = rng.standard_normal(p.sizes()[a])
        z = torch.zeros(p.sizes()[a], dtype=torch.float64, device=DEV)
        g.apply_precond(a, T(r), z)
    ref = two_level_apply(K, blk, nb, r)
    err = rel(z.cpu().numpy(), ref)
    print(name, nb, err, flush=True)
    assert err < 1e-5, (name, err)


@pytest.mark.parametrize("scheme", ["D", "coupled", "U"])
@pytest.mark.parametrize("name", ["dense48", "box24x12_3c", "box70x5_zdir"])
def test_fracture_blocks_trajectory(name, scheme, monkeypatch):
    print(f"\n[fracture blocks trajectory {name} {scheme}]", flush=True)
    monkeypatch.setenv("MCDEC_FRACTURE_EXACT_MAX", "0")
    p = FRAC_BLOCK_CASES[name]()
    ref = schemes.run(p, scheme, 3, keep="all")
    with mcdec.Problem(p, scheme=scheme, precond="bic0", tol=1e-14) as g:
        assert g.info().n_frac_blocks > 0
        for n in range(1, 4):
            rep = g.step(1)
            err = rel(g.get_states(), ref[n])
            assert err < 1e-10, (name, scheme, n, err, rep)


@pytest.mark.parametrize("name", ["dense48", "box96x8"])
def test_fracture_blocks_mixed(name, monkeypatch):
    """Inside FP32 refinement (the FP32 inner solve reads the same block inverses), and in
    fewer fracture iterations than with the chains alone."""
    print(f"\n[fracture blocks mixed {name}]", flush=True)
    monkeypatch.setenv("MCDEC_FRACTURE_EXACT_MAX", "0")
    p = FRAC_BLOCK_CASES[name]()
    ref = schemes.run(p, "D", 3, keep="last")
    with mcdec.Problem(p, precision="mixed", precond="bic0", outer_tol=1e-12) as g:
        assert g.info().n_frac_blocks > 0
        rep = g.step(3)
        err = rel(g.get_states(), ref)
        print(name, rep, err, flush=True)
        assert err < 1e-8, (name, err, rep)


def test_fracture_preconditioner_switch_on_rebuild(monkeypatch):
    """One problem whose fracture solve changes between the two-level blocks (43 blocks) and
    the exact solve (hundreds of crossing cells) when option changes rebuild its
    coefficients: each layer still matches the oracle (the K-sized arrays, and their FP32
    copies in mixed precision, are made for the preconditioner in use)."""
    p = DENSE()
    ref = schemes.run(p, "D", 4, keep="all")
    mixed = dict(precision="mixed", outer_tol=1e-12, inner_tol=1e-6)
    monkeypatch.setenv("MCDEC_FRACTURE_EXACT_MAX", "0")
    with mcdec.Problem(p, precond="bic0", **mixed) as g:
        assert g.info().n_frac_blocks > 0 and g.info().n_crossing == 0
        g.step(1)
        assert rel(g.get_states(), ref[1]) < 1e-8
        monkeypatch.delenv("MCDEC_FRACTURE_EXACT_MAX")
        g.set_options(precision="fp64", tol=1e-13)          # rebuild: the exact solve
        inf = g.info()
        assert inf.n_frac_blocks == 0 and inf.n_crossing > 43, inf.n_crossing
        g.step(1)
        assert rel(g.get_states(), ref[2]) < 1e-10
        g.set_options(**mixed)                               # rebuild: exact, in FP32 copies
        g.step(1)
        assert rel(g.get_states(), ref[3]) < 1e-8
        monkeypatch.setenv("MCDEC_FRACTURE_EXACT_MAX", "0")
        g.set_options(precision="fp64", tol=1e-13)          # rebuild: the blocks again
        assert g.info().n_frac_blocks > 0
        g.step(1)
        assert rel(g.get_states(), ref[4]) < 1e-10


def test_cu_partition_keeps_results(monkeypatch):
    """A problem whose fracture takes the two-level block preconditioner runs its fracture
    group on its own compute units by default; with every unit shared (MCDEC_FRAC_CUS=0)
    the layers are bitwise the same (the partial sums are reduced in a fixed order)."""
    monkeypatch.setenv("MCDEC_FRACTURE_EXACT_MAX", "0")
    p = BOXES["box64x5"]()
    out = {}
    for cus in (None, "0"):
        if cus is None:
            monkeypatch.delenv("MCDEC_FRAC_CUS", raising=False)
        else:
            monkeypatch.setenv("MCDEC_FRAC_CUS", cus)
        with mcdec.Problem(p, precond="bic0", tol=1e-12) as g:
            assert g.info().n_frac_blocks > 0
            reps = [g.step(1) for _ in range(3)]
            out[cus] = (g.get_states(), [r["iters"] for r in reps])
    (a, ia), (b, ib) = out[None], out["0"]
    assert ia == ib
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_fracture_blocks_fewer_iterations(monkeypatch):
    """On fracture planes the two-level preconditioner needs far fewer PCG iterations than
    the chains alone (MCDEC_FRACTURE_BLOCKS = 0 leaves the chains)."""
    p = FRAC_BLOCK_CASES["box96x8"]()
    monkeypatch.setenv("MCDEC_FRACTURE_EXACT_MAX", "0")
    its = {}
    for on in ("0", "1"):
        monkeypatch.setenv("MCDEC_FRACTURE_BLOCKS", on)
        with mcdec.Problem(p, precond="bic0", tol=1e-10) as g:
            inf = g.info()
            assert (inf.n_frac_blocks > 0) == (on == "1") and inf.n_crossing == 0
            its[on] = sum(g.step(1)["iters"][-1] for _ in range(3))   # fracture continuum
    print(its, flush=True)
    assert its["1"] * 2 < its["0"], its


def test_3d_multigrid_refused():
    p = media.box_problem(n=16, nz=4, seed=2)
    with pytest.raises(mcdec.McError) as ei:
        mcdec.Problem(p, precond="mg")
    assert ei.value.status == mcdec.MC_EINVAL and "2-D" in str(ei.value)
    with mcdec.Problem(p, precond="bic0") as g:
        with pytest.raises(mcdec.McError) as ei:
            g.set_options(precond="mg")
        assert ei.value.status == mcdec.MC_EINVAL


# ------------------------------------------------------------------------------------
# device allocator hooks (mc_options.dev_alloc / dev_free)
# ------------------------------------------------------------------------------------
@pytest.mark.parametrize("precond", ["mg", "bic0"])
def test_torch_allocator_hooks(precond):
    """With torch's caching allocator as the hooks, the problem's device arrays come from
    torch (its allocated bytes grow by at least the problem's device bytes and fall back
    when the problem is destroyed) and the layers are bitwise those of the library's own
    allocation, also when torch hands back blocks that held NaN (no array is read before
    the library writes it)."""
    print(f"\n[allocator hooks {precond}]", flush=True)
    p = CASES["three70"]()
    poison = torch.full((8 << 20,), float("nan"), dtype=torch.float64, device=DEV)
    del poison   # the block stays in torch's cache with this content
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    with mcdec.Problem(p, precond=precond, alloc="torch") as g:
        g.step(3)
        held = torch.cuda.memory_allocated() - base
        dev_bytes = g.info().device_bytes
        a = g.get_states()
    torch.cuda.synchronize()
    left = torch.cuda.memory_allocated() - base
    with mcdec.Problem(p, precond=precond) as g:
        g.step(3)
        b = g.get_states()
    print(precond, held, dev_bytes, left, flush=True)
    assert held >= dev_bytes > 0 and left == 0, (held, dev_bytes, left)
    assert len(a) == len(b) and all(np.array_equal(x, y) for x, y in zip(a, b))


def test_allocator_hooks_both_or_neither():
    p = CASES["three70"]()
    d, keep = mcdec.describe(p)
    o = mcdec.make_options(alloc="torch")
    o.dev_free = None
    h = mcdec._PROBLEM()
    st = mcdec.mc_create_problem(C.byref(d), C.byref(o), C.byref(h))
    assert st == mcdec.MC_EINVAL and not h.value
    assert b"dev_free" in mcdec.mc_last_error(None)
