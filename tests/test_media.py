"""Seeded input generator: reproducibility, sizes and statistics of the workloads (no GPU)."""
import numpy as np
import pytest

import media


def test_reproducible():
    a = media.config_problem("C1")
    b = media.config_problem("C1")
    assert np.array_equal(a.host, b.host) and np.array_equal(a.edges, b.edges)
    assert np.array_equal(a.sigma_f, b.sigma_f)


def test_c1_shape():
    p = media.config_problem("C1")
    assert (p.nx, p.ny, p.n_omega) == (64, 64, 1)
    assert 150 <= p.nf <= 260            # "about 200 fracture cells"
    assert p.tau == 0.01 and p.nsteps == 20
    assert list(p.bc_type) == [1, 1, 0, 0] and list(p.bc_value[:2]) == [1.0, 0.0]
    # axis-aligned, no collinear overlap: no host holds two cells of one orientation
    seg = p.meta["seg_id"]
    hs, cnt = np.unique(p.host, return_counts=True)
    assert cnt.max() <= 2
    np.testing.assert_allclose(p.sigma_f, 1e-4)


def test_c2_shape_and_field():
    p = media.config_problem("C2")
    assert p.nx == 2048 and 55_000 <= p.nf <= 70_000
    lk = np.log(p.omega[0].k)
    assert abs(np.median(lk) - np.log(1e-4)) < 0.5
    assert 1.2 < lk.std() < 1.8
    # chain edges join consecutive cells of one segment; crossings join different segments
    seg = p.meta["seg_id"]
    e = p.edges
    chain = e[:, 1] - e[:, 0] == 1
    assert np.all(seg[e[chain, 0]] == seg[e[chain, 1]])
    assert np.all(p.host[e[~chain, 0]] == p.host[e[~chain, 1]])
    assert np.all(seg[e[~chain, 0]] != seg[e[~chain, 1]])


def test_lognormal_correlation_length():
    rng = np.random.default_rng(0)
    n = 512
    k = media.lognormal_field(n, rng, sigma_log=1.0, corr_len=0.05)
    g = np.log(k / 1e-4)
    assert abs(g.std() - 1.0) < 0.15
    # covariance exp(-r^2/l^2): at r = l the correlation is e^-1
    lag = int(round(0.05 * n))
    c = np.mean(g[:, :-lag] * g[:, lag:]) / g.var()
    assert abs(c - np.exp(-1)) < 0.1


def test_c3_sizes():
    p = media.config_problem("C3")
    assert p.nx == 4096 and p.n_omega == 2 and p.nf >= 150_000
    assert p.sigma_omega == 10.0 and p.omega[1].k_const == 1e-2


def test_c4_c5_families():
    probs = media.c4_problems(count=6, n_range=(128, 160))
    assert len(probs) == 6 and all(128 <= p.nx <= 160 for p in probs)
    tr = media.c5_trace(count=50)
    t = np.array([e[0] for e in tr])
    assert np.all(np.diff(t) > 0)
    assert all(64 <= e[1] <= 2048 and 10 <= e[4] <= 500 for e in tr)


@pytest.mark.parametrize("case,dof", [("2C", 42684), ("3C", 82684)])
def test_paper_problem_shape(case, dof):
    """The numerical-results test problems: 200 x 200 grid, 2684 fracture cells (the DOF
    counts the paper states), wells in both boxes, no-flow sides, p0 = 1, T = 0.002 / 50."""
    p = media.paper_problem(case)
    assert (p.nx, p.ny, p.nf, p.dof()) == (200, 200, 2684, dof)
    assert p.n_omega == (1 if case == "2C" else 2)
    assert len(np.unique(p.meta["seg_id"])) == 25
    assert np.all(p.bc_type == 0)
    assert abs(p.tau * p.nsteps - 0.002) < 1e-15 and p.nsteps == 50
    assert all(np.all(v == 1.0) for v in p.initial_state())
    wells = np.flatnonzero(p.well_q)
    assert np.all(p.well_q[wells] == 1e5) and np.all(p.well_p == 1.2)
    h = p.h
    x = (p.host[wells] % p.nx + 0.5) * h
    y = (p.host[wells] // p.nx + 0.5) * h
    low = (x <= 0.15) & (y <= 0.15)
    high = (x >= 0.6) & (y >= 0.85)
    assert low.any() and high.any() and np.all(low | high)
    assert np.all((x >= 0.1) & (x <= 0.65) & (y >= 0.1) & (y <= 0.9))
