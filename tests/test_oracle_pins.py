"""Pins of the CPU oracle against facts the paper and the mathematics fix (no GPU).

Each test is chosen so that a plausible slip in the oracle (a dropped term, a wrong sign,
a wrong index, a transposed block) fails at least one of them:

* hand-computed fixtures (tests/golden/hand_2x1.json and   -> every assembled entry, F,
  hand_frac.json: aperture, fracture edge, sigma_12 h^2)      coupled and D steps exactly
* textbook eigenvalues of the 5-point operator            -> stencil assembly with BCs
* layered-medium series-resistance solution              -> harmonic mean, Dirichlet faces
* two-cell closed forms (coupled, D, EX)                  -> transfer and the recurrences
* brute-force dense assembly on tiny problems             -> the whole coupled matrix
* constant states, maximum principle, mass identity      -> transfer signs, antisymmetry
* Theorems 2 and 3 (energy decay), symmetry, Q_ab=Q_ba^T  -> operator structure
* first order in tau of decoupled vs coupled              -> the splitting itself
* fast diagonalization vs LU                              -> the large-grid fallback
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import media
from media import OmegaContinuum, Problem
from oracle import dense, fastdiag, fv, schemes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(n=4, ny=None, three=False, nfc=3, seed=0, bc=(1, 1, 0, 0), bcv=(1.0, 0.0, 0, 0),
          tau=0.1, lognormal=True):
    rng = np.random.default_rng(seed)
    ny = n if ny is None else ny
    h = 1.0 / n
    k = np.exp(rng.normal(np.log(1e-1), 1.0, (ny, n))) if lognormal else None
    om = [OmegaContinuum(c=1.0, k=k, k_const=0.3)]
    if three:
        om.append(OmegaContinuum(c=0.05, k_const=2.0))
    host = rng.integers(0, n * ny, nfc).astype(np.int32)
    edges = np.array([[i, i + 1] for i in range(nfc - 1)], np.int32).reshape(-1, 2)
    p = Problem(nx=n, ny=ny, h=h, omega=om, sigma_omega=3.0 if three else 0.0, host=host,
                flen=np.full(nfc, h), edges=edges, edge_d=rng.uniform(0.5, 1.5, len(edges)) * h,
                k_f=5.0, c_f=0.1, aperture=0.2,
                sigma_f=rng.uniform(0.1, 1.0, (len(om), nfc)),
                bc_type=np.array(bc, np.int32), bc_value=np.array(bcv, float), tau=tau)
    p.check()
    return p


# ------------------------------------------------------------------------------------
def test_hand_computed_fixture():
    g = json.load(open(os.path.join(GOLD, "hand_2x1.json")))
    q = g["problem"]
    p = Problem(nx=q["nx"], ny=q["ny"], h=q["h"], omega=[OmegaContinuum(c=q["c"], k_const=q["k"])],
                host=np.array(q["host"], np.int32), flen=np.array(q["flen"]),
                k_f=q["k_f"], c_f=q["c_f"], aperture=q["aperture"],
                sigma_f=np.array(q["sigma_f"]), bc_type=np.array(q["bc_type"], np.int32),
                bc_value=np.array(q["bc_value"]), tau=q["tau"])
    asm = fv.assemble(p)
    K = schemes.coupled_matrix(asm, p.tau).toarray()
    np.testing.assert_array_equal(K, np.array(g["coupled_matrix"]))
    np.testing.assert_array_equal(asm.Ffull(), np.array(g["F"]))
    frac = lambda v: np.array([float(Fraction(a, b)) for a, b in v])
    x = schemes.run(p, "coupled", 1)[-1]
    np.testing.assert_allclose(np.concatenate(x), frac(g["coupled_step1"]), rtol=0, atol=1e-15)
    h = schemes.run(p, "D", 2)
    np.testing.assert_allclose(np.concatenate(h[1]), frac(g["D_step1"]), rtol=0, atol=1e-15)
    assert abs(h[2][1][0] - float(Fraction(*g["D_step2_fracture"]))) < 1e-15


def _exact_solve(A, b):
    """Gaussian elimination in rationals (the fixture's own derivation, no oracle code)."""
    n = len(A)
    m = [list(r) + [bb] for r, bb in zip(A, b)]
    for i in range(n):
        piv = next(r for r in range(i, n) if m[r][i] != 0)
        m[i], m[piv] = m[piv], m[i]
        for r in range(n):
            if r != i and m[r][i] != 0:
                f = m[r][i] / m[i][i]
                m[r] = [x - f * y for x, y in zip(m[r], m[i])]
    return [m[i][n] / m[i][i] for i in range(n)]


def test_hand_computed_fracture_fixture():
    """Three continua, a fracture edge and aperture 1/4 (tests/golden/hand_frac.json): the
    fracture storage c_f a l, the fracture conductance k_f a / d and the per-cell
    sigma_12 h^2 each enter the hand matrix with a value that a dropped factor changes."""
    g = json.load(open(os.path.join(GOLD, "hand_frac.json")))
    q = g["problem"]
    R = lambda v: Fraction(v)
    p = Problem(nx=q["nx"], ny=q["ny"], h=q["h"],
                omega=[OmegaContinuum(c=o["c"], k_const=o["k"]) for o in q["omega"]],
                sigma_omega=q["sigma_omega"], host=np.array(q["host"], np.int32),
                flen=np.array(q["flen"]), edges=np.array(q["edges"], np.int32),
                edge_d=np.array(q["edge_d"]), k_f=q["k_f"], c_f=q["c_f"],
                aperture=q["aperture"], sigma_f=np.array(q["sigma_f"]),
                bc_type=np.array(q["bc_type"], np.int32), bc_value=np.array(q["bc_value"]),
                tau=q["tau"])
    p.check()
    K_hand = [[R(v) for v in row] for row in g["coupled_matrix"]]
    F_hand = [R(v) for v in g["F"]]
    # the stored solutions are the exact solutions of the hand matrix
    assert _exact_solve(K_hand, F_hand) == [R(v) for v in g["coupled_step1"]]
    Dm = [[[R(v) for v in row] for row in blk] for blk in g["D_matrices"]]
    d1 = [R(v) for v in g["D_step1"]]
    assert _exact_solve(Dm[0], F_hand[0:2]) == d1[0:2]
    assert _exact_solve(Dm[1], F_hand[2:4]) == d1[2:4]
    # second D layer of the fracture: m_f/tau p_f^1 + Q_f0 p_0^1 + Q_f1 p_1^1 (p_f^1 = 0)
    sf = q["sigma_f"]
    rf = [R(sf[0][0]) * d1[0] + R(sf[1][0]) * d1[2], R(sf[0][1]) * d1[1] + R(sf[1][1]) * d1[3]]
    assert _exact_solve(Dm[2], rf) == [R(v) for v in g["D_step2_fracture"]]
    # the oracle against the hand values
    asm = fv.assemble(p)
    fl = lambda M: np.array([[float(v) for v in row] for row in M])
    np.testing.assert_array_equal(schemes.coupled_matrix(asm, p.tau).toarray(), fl(K_hand))
    np.testing.assert_array_equal(asm.Ffull(), np.array([float(v) for v in F_hand]))
    for a in range(3):
        np.testing.assert_array_equal(schemes.continuum_matrix(asm, p.tau, a, "D").toarray(),
                                      fl(Dm[a]))
    x = np.concatenate(schemes.run(p, "coupled", 1)[-1])
    np.testing.assert_allclose(x, [float(R(v)) for v in g["coupled_step1"]], rtol=0, atol=1e-15)
    h = schemes.run(p, "D", 2)
    np.testing.assert_allclose(np.concatenate(h[1]), [float(v) for v in d1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(h[2][2], [float(R(v)) for v in g["D_step2_fracture"]], rtol=0,
                               atol=1e-15)


@pytest.mark.parametrize("bc", [(1, 1, 0, 0), (0, 0, 1, 1), (0, 0, 0, 0), (1, 1, 1, 1)])
def test_stencil_eigenvalues_textbook(bc):
    """Constant-k 5-point operator: eigenvalues k (4 sin^2(pi i/2nx) + 4 sin^2(pi j/2ny)) with
    i, j from 1 (Dirichlet half-cell ends) or 0 (no-flow ends)."""
    nx, ny, k = 7, 5, 0.37
    D, _ = fv.omega_diffusion(np.full((ny, nx), k), bc, (0, 0, 0, 0))
    ev = np.sort(np.linalg.eigvalsh(D.toarray()))
    ix = np.arange(1, nx + 1) if bc[0] else np.arange(nx)
    iy = np.arange(1, ny + 1) if bc[2] else np.arange(ny)
    lx = 4 * np.sin(np.pi * ix / (2 * nx)) ** 2
    ly = 4 * np.sin(np.pi * iy / (2 * ny)) ** 2
    ref = np.sort((k * (lx[None, :] + ly[:, None])).ravel())
    np.testing.assert_allclose(ev, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("bc", [(1, 1, 0, 0, 0, 0), (0, 0, 0, 0, 1, 1), (0, 0, 0, 0, 0, 0),
                                (1, 1, 1, 1, 1, 1), (0, 0, 1, 1, 1, 0)])
def test_stencil_eigenvalues_textbook_3d(bc):
    """Constant-k 7-point operator on cubes of side h: eigenvalues k h (4 sin^2(pi i/2nx) +
    4 sin^2(pi j/2ny) + 4 sin^2(pi l/2nz)); a Dirichlet pair of ends shifts an axis's indices
    to 1..n, one Dirichlet end to half-integers (i + 1/2)."""
    nx, ny, nz, k, h = 5, 4, 3, 0.37, 0.25
    D, _ = fv.omega_diffusion_3d(np.full((nz, ny, nx), k), h, bc[:4], (0, 0, 0, 0), bc[4:],
                                 (0, 0))
    ev = np.sort(np.linalg.eigvalsh(D.toarray()))

    def axis(n, lo, hi):
        i = np.arange(n, dtype=float)
        if lo and hi:
            i = i + 1
        elif lo or hi:
            i = i + 0.5
        return 4 * np.sin(np.pi * i / (2 * n)) ** 2

    lx, ly, lz = axis(nx, bc[0], bc[1]), axis(ny, bc[2], bc[3]), axis(nz, bc[4], bc[5])
    ref = np.sort((k * h * (lx[None, None, :] + ly[None, :, None] + lz[:, None, None])).ravel())
    np.testing.assert_allclose(ev, ref, rtol=0, atol=1e-13)


def test_layered_medium_series_resistance_z():
    """Steady flow up a column of layers k_0..k_{n-1} between p = 1 (bottom) and p = 0 (top):
    the profile of 1-D conductances in series, the same in every column."""
    rng = np.random.default_rng(4)
    nz, m = 7, 3
    kl = np.exp(rng.normal(0, 1.5, nz))
    k = np.broadcast_to(kl[:, None, None], (nz, m, m)).copy()
    p = Problem(nx=m, ny=m, nz=nz, h=1.0 / m, omega=[OmegaContinuum(c=1.0, k=k)],
                bc_type=np.zeros(4, np.int32), bc_value=np.zeros(4),
                bc_type_z=np.array([1, 1], np.int32), bc_value_z=np.array([1.0, 0.0]),
                tau=1e18)
    x = schemes.run(p, "coupled", 1)[-1][0].reshape(nz, m * m)
    flux = 1.0 / np.sum(1.0 / kl)
    ref = 1.0 - flux * (np.concatenate([[0], np.cumsum(1.0 / kl)[:-1]]) + 0.5 / kl)
    np.testing.assert_allclose(x, np.repeat(ref[:, None], m * m, axis=1), rtol=0, atol=1e-12)


@pytest.mark.parametrize("scheme", ["coupled", "D", "L", "U"])
def test_3d_constant_state_energy_and_mass(scheme):
    """3-D: a constant state equal to every Dirichlet value stays put; with no-flow sides and
    no sources the A-energy does not grow (Theorems 2 and 3), and the coupled scheme keeps
    the mass."""
    p = _tiny3d(three=True, bc=(1, 1, 1, 1), bcv=(0.7, 0.7, 0.7, 0.7), bcz=(1, 1),
                bcvz=(0.7, 0.7), tau=0.1)
    p.p0 = [np.full(s, 0.7) for s in p.sizes()]
    for st in schemes.run(p, scheme, 3):
        for v in st:
            np.testing.assert_allclose(v, 0.7, rtol=0, atol=1e-13)
    q = _tiny3d(three=True, bc=(0, 0, 0, 0), bcz=(0, 0), tau=0.3)
    rng = np.random.default_rng(6)
    q.p0 = [rng.normal(size=s) for s in q.sizes()]
    asm = fv.assemble(q)
    hist = schemes.run(q, scheme, 5)
    e = [schemes.energy(asm, st) for st in hist]
    assert all(e[i + 1] <= e[i] + 1e-14 * e[0] for i in range(len(e) - 1)), e
    if scheme == "coupled":
        mass = [sum(float(asm.M[a] @ st[a]) for a in range(asm.L)) for st in hist]
        np.testing.assert_allclose(mass, mass[0], rtol=1e-13)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_layered_medium_series_resistance(axis):
    """Steady flow through layers k_0..k_{n-1} between p=1 and p=0 half-cell faces: flux
    1/sum(1/k_i) and p_i = 1 - flux (sum_{j<i} 1/k_j + 1/(2 k_i)) exactly (Darcy's law for
    conductances in series); the transverse direction carries no flow."""
    rng = np.random.default_rng(3)
    n, m = 9, 4
    kl = np.exp(rng.normal(0, 1.5, n))
    if axis == "x":
        k = np.tile(kl, (m, 1)); nx, ny = n, m; bc = (1, 1, 0, 0); bcv = (1, 0, 0, 0)
    else:
        k = np.tile(kl[:, None], (1, m)); nx, ny = m, n; bc = (0, 0, 1, 1); bcv = (0, 0, 1, 0)
    p = Problem(nx=nx, ny=ny, h=1.0 / nx, omega=[OmegaContinuum(c=1.0, k=k)],
                bc_type=np.array(bc, np.int32), bc_value=np.array(bcv, float), tau=1e18)
    x = schemes.run(p, "coupled", 1)[-1][0].reshape(ny, nx)
    flux = 1.0 / np.sum(1.0 / kl)
    ref = 1.0 - flux * (np.concatenate([[0], np.cumsum(1.0 / kl)[:-1]]) + 0.5 / kl)
    got = x[0, :] if axis == "x" else x[:, 0]
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
    assert np.ptp(x, axis=0 if axis == "x" else 1).max() < 1e-12


def _two_cell(mm=0.7, mf=0.2, sig=1.3, tau=0.4, pm=1.0, pf=-0.5):
    p = Problem(nx=1, ny=1, h=1.0, omega=[OmegaContinuum(c=mm, k_const=1.0)],
                host=np.array([0], np.int32), flen=np.array([1.0]), k_f=1.0, c_f=mf,
                aperture=1.0, sigma_f=np.array([[sig]]), tau=tau,
                p0=[np.array([pm]), np.array([pf])])
    return p


def test_two_cell_coupled_closed_form():
    mm, mf, sig, tau = 0.7, 0.2, 1.3, 0.4
    p = _two_cell(mm, mf, sig, tau)
    hist = schemes.run(p, "coupled", 6)
    d0 = 1.5
    mass0 = mm * 1.0 + mf * (-0.5)
    for n, s in enumerate(hist):
        d = s[0][0] - s[1][0]
        assert abs(d - d0 / (1 + tau * sig * (1 / mm + 1 / mf)) ** n) < 1e-14
        assert abs(mm * s[0][0] + mf * s[1][0] - mass0) < 1e-14


def test_two_cell_D_and_EX_closed_form():
    mm, mf, sig, tau = 0.7, 0.2, 1.3, 0.4
    a = sig / (mm / tau + sig)
    b = sig / (mf / tau + sig)
    p = _two_cell(mm, mf, sig, tau)
    hist = schemes.run(p, "D", 8)
    G = np.array([[1 - a, a], [b, 1 - b]])
    v = np.array([1.0, -0.5])
    for s in hist:
        np.testing.assert_allclose([s[0][0], s[1][0]], v, rtol=0, atol=1e-14)
        assert abs(b * s[0][0] + a * s[1][0] - (b * 1.0 + a * -0.5)) < 1e-14
        v = G @ v
    # EX: (m/tau) p^n = (m/tau - sig) p^{n-1} + sig q^{n-1}  (whole transfer lagged)
    e = sig * tau / mm
    f = sig * tau / mf
    G2 = np.array([[1 - e, e], [f, 1 - f]])
    hist = schemes.run(p, "EX", 5)
    v = np.array([1.0, -0.5])
    for s in hist:
        np.testing.assert_allclose([s[0][0], s[1][0]], v, rtol=0, atol=1e-13)
        v = G2 @ v


def test_EX_unstable_where_D_is_not():
    # tau*sigma/m_f = 5 > 2: the EX amplification 1 - tau sigma (1/m_m + 1/m_f) leaves the
    # unit disc, the D-scheme's 1 - a - b stays inside
    p = _two_cell(mm=1.0, mf=0.2, sig=1.0, tau=1.0)
    ex = schemes.run(p, "EX", 20)[-1]
    d = schemes.run(p, "D", 20)[-1]
    assert abs(ex[0][0] - ex[1][0]) > 1e3
    assert abs(d[0][0] - d[1][0]) < 1.5


def _tiny3d(three=False, seed=5, bc=(1, 1, 0, 0), bcv=(1.0, 0.0, 0, 0), bcz=(1, 0),
            bcvz=(0.4, 0.0), tau=0.05):
    """3 x 4 x 2 cubes (h = 0.5) with a lognormal k, and two fracture planes meeting in a
    host cell (a 2 x 2 plane normal to z and a 2 x 1 plane normal to x)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz, h = 3, 4, 2, 0.5
    k = np.exp(rng.normal(np.log(1e-1), 1.0, (nz, ny, nx)))
    om = [OmegaContinuum(c=1.0, k=k)]
    if three:
        om.append(OmegaContinuum(c=0.05, k_const=2.0))
    cell = lambda x, y, z: (z * ny + y) * nx + x  # noqa: E731
    host = np.array([cell(0, 1, 1), cell(1, 1, 1), cell(0, 2, 1), cell(1, 2, 1),
                     cell(1, 1, 0), cell(1, 1, 1)], np.int32)
    edges = np.array([[0, 1], [2, 3], [0, 2], [1, 3], [4, 5], [1, 5]], np.int32)
    p = Problem(nx=nx, ny=ny, nz=nz, h=h, omega=om, sigma_omega=3.0 if three else 0.0,
                host=host, flen=np.full(6, h * h), edges=edges,
                edge_d=rng.uniform(0.5, 1.5, len(edges)), k_f=5.0, c_f=0.1, aperture=0.2,
                sigma_f=rng.uniform(0.1, 1.0, (len(om), 6)),
                bc_type=np.array(bc, np.int32), bc_value=np.array(bcv, float),
                bc_type_z=np.array(bcz, np.int32), bc_value_z=np.array(bcvz, float), tau=tau)
    p.check()
    return p


@pytest.mark.parametrize("wells", [False, True])
@pytest.mark.parametrize("three", [False, True])
@pytest.mark.parametrize("dim", [2, 3])
def test_dense_brute_force(three, wells, dim):
    if dim == 2:
        p = _tiny(n=4, ny=3, three=three, nfc=4, seed=11, tau=0.05)
        wq, wp = [3.0, 0.0, 40.0, 0.5], [1.2, 7.0, -0.3, 2.0]
    else:
        p = _tiny3d(three=three)
        wq, wp = [3.0, 0.0, 40.0, 0.5, 0.0, 2.0], [1.2, 7.0, -0.3, 2.0, 0.0, 0.9]
    if wells:
        p.well_q = np.array(wq)
        p.well_p = np.array(wp)
    K, mdiag, rf, _ = dense.coupled_dense(p, p.tau)
    asm = fv.assemble(p)
    np.testing.assert_allclose(schemes.coupled_matrix(asm, p.tau).toarray(), K, rtol=1e-14,
                               atol=1e-14)
    np.testing.assert_allclose(asm.Ffull(), rf, rtol=1e-14, atol=1e-15)
    rng = np.random.default_rng(5)
    p.p0 = [rng.random(s) for s in p.sizes()]
    x = schemes.run(p, "coupled", 1)[-1]
    np.testing.assert_allclose(np.concatenate(x), dense.coupled_step_dense(p, p.tau, p.p0),
                               rtol=1e-12, atol=1e-13)
    # D-scheme from the dense blocks: block-diagonal implicit part, off-diagonal lagged
    N = K.shape[0]
    off = np.cumsum([0] + p.sizes())
    K0 = np.zeros_like(K)
    for a in range(len(p.sizes())):
        s = slice(off[a], off[a + 1])
        K0[s, s] = K[s, s]
    A1 = K - K0
    xd = np.linalg.solve(K0, mdiag / p.tau * np.concatenate(p.p0) + rf - A1 @ np.concatenate(p.p0))
    np.testing.assert_allclose(np.concatenate(schemes.run(p, "D", 1)[-1]), xd, rtol=1e-12,
                               atol=1e-13)
    # L and U from the dense blocks: triangular implicit parts
    for sch, tri in (("L", np.tril), ("U", np.triu)):
        mask = np.zeros((len(p.sizes()),) * 2)
        mask = tri(np.ones_like(mask))
        KL = np.zeros_like(K)
        for a in range(len(p.sizes())):
            for b in range(len(p.sizes())):
                if mask[a, b]:
                    KL[off[a]:off[a + 1], off[b]:off[b + 1]] = K[off[a]:off[a + 1], off[b]:off[b + 1]]
        xl = np.linalg.solve(KL, mdiag / p.tau * np.concatenate(p.p0) + rf
                             - (K - KL) @ np.concatenate(p.p0))
        np.testing.assert_allclose(np.concatenate(schemes.run(p, sch, 1)[-1]), xl, rtol=1e-12,
                                   atol=1e-13)


@pytest.mark.parametrize("scheme", schemes.SCHEMES)
@pytest.mark.parametrize("three", [False, True])
def test_constant_state_preserved(scheme, three):
    # EX only within its stability bound tau * sigma / m < 1 (rounding grows otherwise)
    tau = 1e-3 if scheme == "EX" else 0.1
    p = _tiny(n=5, three=three, nfc=6, seed=2, bc=(1, 1, 0, 1), bcv=(0.7, 0.7, 0, 0.7), tau=tau)
    p.p0 = [np.full(s, 0.7) for s in p.sizes()]
    for s in schemes.run(p, scheme, 4):
        for v in s:
            np.testing.assert_allclose(v, 0.7, rtol=0, atol=1e-13)


@pytest.mark.parametrize("scheme", ["coupled", "D", "L", "U"])
def test_maximum_principle(scheme):
    p = media.small_problem(n=24, seed=4, nseg=5, tau=1e-2, nsteps=6)
    for s in schemes.run(p, scheme):
        for v in s:
            assert v.min() >= -1e-14 and v.max() <= 1 + 1e-14


@pytest.mark.parametrize("three", [False, True])
def test_symmetry_and_splitting_condition(three):
    p = _tiny(n=5, three=three, nfc=7, seed=9)
    asm = fv.assemble(p)
    A = asm.Afull()
    assert abs(A - A.T).max() < 1e-15
    for (a, b), q in asm.Q.items():
        assert abs(q - asm.Q[(b, a)].T).max() == 0
        assert q.min() >= 0
    # A >= 0 and A0 - A1 >= 0 for the D-split (Section 3.3 condition dc-op)
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > -1e-12
    A0 = sp.block_diag([asm.D[a] + sp.diags(asm.S(a)) for a in range(asm.L)]).toarray()
    A1 = A.toarray() - A0
    assert np.linalg.eigvalsh(A0 - A1).min() > -1e-12


@pytest.mark.parametrize("scheme", ["coupled", "D", "L", "U"])
@pytest.mark.parametrize("tau", [1e-3, 1.0, 1e3])
def test_energy_decay_theorems(scheme, tau):
    """Theorems 2 and 3 with F = 0: ||p^n||_A <= ||p^{n-1}||_A (no-flow sides, no source)."""
    p = _tiny(n=6, three=True, nfc=8, seed=21, bc=(0, 0, 0, 0), tau=tau)
    rng = np.random.default_rng(1)
    p.p0 = [rng.normal(size=s) for s in p.sizes()]
    asm = fv.assemble(p)
    hist = schemes.run(p, scheme, 6)
    e = [schemes.energy(asm, s) for s in hist]
    # rounding floor: ||A|| ||x||^2 * eps relative to the initial energy
    assert all(e[i + 1] <= e[i] + 1e-14 * e[0] for i in range(len(e) - 1)), e
    assert e[-1] < e[0]


def test_mass_identities():
    p = _tiny(n=6, three=True, nfc=8, seed=8, bc=(0, 0, 0, 0), tau=0.3)
    rng = np.random.default_rng(2)
    p.p0 = [rng.random(s) for s in p.sizes()]
    asm = fv.assemble(p)
    mass = lambda s: sum(float(asm.M[a] @ s[a]) for a in range(asm.L))
    hist = schemes.run(p, "coupled", 5)
    for s in hist:
        assert abs(mass(s) - mass(hist[0])) < 1e-13 * abs(mass(hist[0]))
    # D-scheme: each transfer pair (i in a, j in b, sigma) changes the mass by
    # -tau sigma (dp_a,i + dp_b,j) per step
    hist = schemes.run(p, "D", 3)
    for s0, s1 in zip(hist[:-1], hist[1:]):
        dm = mass(s1) - mass(s0)
        pred = 0.0
        for (a, b), q in asm.Q.items():
            if a < b:
                qc = q.tocoo()
                pred -= p.tau * np.sum(qc.data * ((s1[a] - s0[a])[qc.row] + (s1[b] - s0[b])[qc.col]))
        assert abs(dm - pred) < 1e-13


# ------------------------------------------------------------------------------------
# wells of the numerical results (Section 5): source q_w (p_w - p_f) per unit measure on
# fracture cells, implicit
def test_well_isolated_cell_recurrence():
    """A fracture cell with no transfer and no connections, holding a well: the balance
    c_f m (p^n - p^{n-1}) / tau = q_w m (p_w - p^n) gives p^n - p_w = (p^0 - p_w) / (1 + q_w
    tau / c_f)^n in every scheme, and the Omega cell does not move."""
    cf, q, pw, tau = 0.3, 7.0, 1.2, 0.05
    p = Problem(nx=1, ny=1, h=0.5, omega=[OmegaContinuum(c=1.0, k_const=1.0)],
                host=np.array([0], np.int32), flen=np.array([0.37]), k_f=1.0, c_f=cf,
                aperture=0.02, sigma_f=np.array([[0.0]]), tau=tau,
                p0=[np.array([0.4]), np.array([1.0])],
                well_q=np.array([q]), well_p=np.array([pw]))
    for scheme in ("coupled", "D", "L", "U"):
        hist = schemes.run(p, scheme, 6)
        for n, st in enumerate(hist):
            assert abs(st[1][0] - (pw + (1.0 - pw) / (1 + q * tau / cf) ** n)) < 1e-14
            assert st[0][0] == 0.4


@pytest.mark.parametrize("three", [False, True])
def test_well_steady_state_is_well_pressure(three):
    """With no-flow sides the operator annihilates constants, so the steady state of wells
    sharing one p_w is p = p_w in every continuum: one coupled step with a huge tau lands
    there, and short steps from p = 1 move monotonically toward p_w = 1.2 (discrete maximum
    principle)."""
    p = _tiny(n=5, three=three, nfc=6, seed=4, bc=(0, 0, 0, 0), tau=1e12, lognormal=False)
    p.well_q = np.array([0.0, 2.0, 0.0, 0.0, 5.0, 0.0])
    p.well_p = np.full(6, 1.2)
    p.p0 = [np.ones(s) for s in p.sizes()]
    x = schemes.run(p, "coupled", 1)[-1]
    for v in x:
        assert np.max(np.abs(v - 1.2)) < 1e-9
    hist = schemes.run(p, "coupled", 5, tau=0.01)
    for s0, s1 in zip(hist[:-1], hist[1:]):
        for a, b in zip(s0, s1):
            assert np.all(b >= a - 1e-15) and np.all(b <= 1.2 + 1e-15)
    assert hist[1][-1][1] > 1.0 and hist[1][-1][4] > 1.0


def test_well_mass_balance():
    """Coupled scheme, no-flow sides: the stored mass changes by what the wells inject,
    sum_a M_a (p^n - p^{n-1}) = tau sum_l q_l a len_l (p_w,l - p_l^n)."""
    p = _tiny(n=6, three=True, nfc=8, seed=8, bc=(0, 0, 0, 0), tau=0.3)
    rng = np.random.default_rng(3)
    p.p0 = [rng.random(s) for s in p.sizes()]
    p.well_q = np.where(rng.random(8) < 0.5, rng.uniform(1, 50, 8), 0.0)
    p.well_p = rng.uniform(-1, 2, 8)
    asm = fv.assemble(p)
    hist = schemes.run(p, "coupled", 4)
    meas = p.aperture * p.flen
    for s0, s1 in zip(hist[:-1], hist[1:]):
        dm = sum(float(asm.M[a] @ (s1[a] - s0[a])) for a in range(asm.L))
        inj = p.tau * float(np.sum(p.well_q * meas * (p.well_p - s1[-1])))
        assert abs(dm - inj) < 1e-12 * max(1.0, abs(inj))


def test_first_order_in_tau():
    """||p_D(T) - p_C(T)|| / ||p_C(T)|| halves with tau (the lagged coupling is O(tau))."""
    p = media.config_problem("C1")
    errs = []
    for tau in (0.02, 0.01, 0.005, 0.0025):
        ns = int(round(0.2 / tau))
        d = schemes.run(p, "D", ns, tau=tau, keep="last")
        c = schemes.run(p, "coupled", ns, tau=tau, keep="last")
        errs.append(schemes.rel_l2(d, c))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(1.8 <= r <= 2.2 for r in ratios), (errs, ratios)


def test_fast_diagonalization_matches_lu():
    n = 48
    p = Problem(nx=n, ny=n, h=1.0 / n, omega=[OmegaContinuum(c=1.0, k_const=1e-4)],
                bc_type=np.array([1, 1, 0, 0], np.int32), bc_value=np.array([1.0, 0, 0, 0]),
                tau=1e-3)
    rng = np.random.default_rng(0)
    p.p0 = [rng.random(n * n)]
    x = schemes.run(p, "D", 1)[-1][0]
    asm = fv.assemble(p)
    b = asm.M[0] / p.tau * p.p0[0] + asm.F[0]
    y = fastdiag.fd_solve(b, n, n, 1e-4, p.h ** 2 / p.tau, p.bc_type)
    np.testing.assert_allclose(y, x, rtol=1e-12, atol=0)
    # with fracture-host transfer perturbations: CG preconditioned by the exact part
    q = media.small_problem(n=n, seed=3, lognormal=False, axis=True, nseg=6)
    asm = fv.assemble(q)
    K = schemes.continuum_matrix(asm, q.tau, 0)
    b = rng.random(n * n)
    xs = schemes.DirectSolver(K).solve(b)
    xf, it, rr = fastdiag.fd_pcg(K, b, n, n, 1e-4, q.h ** 2 / q.tau, q.bc_type)
    np.testing.assert_allclose(xf, xs, rtol=1e-11, atol=0)


def test_fd_stepper_matches_lu_on_c3_recipe():
    """The stepper that writes the stored 4096 x 4096 three-continuum layers (fast-
    diagonalization CG on the grid continua) against the sparse-LU D-scheme stepper on the
    same recipe at 1024 x 1024 (three continua, about 38k fracture cells): two layers."""
    p = media.config_problem("C3", n=1024, min_cells=37_500)
    fd = fastdiag.FDStepper(p)
    lu = schemes.Stepper(p, None, "D")
    x = y = p.initial_state()
    for _ in range(2):
        x, y = fd.step(x), lu.step(y)
        for a in range(p.n_cont):
            assert np.linalg.norm(x[a] - y[a]) <= 1e-12 * np.linalg.norm(y[a]), a
    assert schemes.rel_l2(x, y) < 1e-13


def test_decoupled_close_to_coupled_c1():
    """The paper reports decoupled-vs-coupled errors well below 1% and the U-scheme as the
    most accurate (qualitative; its geometry cannot be reproduced)."""
    p = media.config_problem("C1")
    c = schemes.run(p, "coupled", keep="last")
    e = {s: schemes.rel_l2(schemes.run(p, s, keep="last"), c) for s in ("D", "L", "U")}
    assert max(e.values()) < 1e-2
    assert e["U"] < e["D"]


def test_dof_counts():
    # the paper's fine-grid sizes: 200^2 + 2684 and 2 * 200^2 + 2684
    assert 200 * 200 + 2684 == 42684 and 2 * 200 * 200 + 2684 == 82684
    p = media.config_problem("C1")
    assert p.dof() == 64 * 64 + p.nf


# ------------------------------------------------------------------------------------
# block incomplete factorization (the preconditioner the GPU path applies)
# ------------------------------------------------------------------------------------
from oracle import precond  # noqa: E402


def test_ilu0_exact_on_tridiagonal_and_dense():
    rng = np.random.default_rng(0)
    n = 30
    off = -rng.uniform(0.1, 1.0, n - 1)
    T = sp.diags([off, np.abs(np.r_[0, off]) + np.abs(np.r_[off, 0]) + rng.uniform(0.01, 1, n),
                  off], [-1, 0, 1]).tocsr()
    r = rng.standard_normal(n)
    z = precond.ilu0_solve(precond.ilu0(T), r)
    np.testing.assert_allclose(z, sp.linalg.spsolve(T.tocsc(), r), rtol=1e-13, atol=0)
    Q = rng.standard_normal((8, 8))
    D = sp.csr_matrix(Q @ Q.T + 8 * np.eye(8))
    z = precond.ilu0_solve(precond.ilu0(D), r[:8])
    np.testing.assert_allclose(z, np.linalg.solve(D.toarray(), r[:8]), rtol=1e-12, atol=0)


def test_ilu0_matches_matrix_on_pattern():
    """ILU(0) property: (L U)_ij = a_ij on the pattern of A; for SPD A, M is SPD."""
    p = media.small_problem(n=12, seed=3, nseg=0)
    K = schemes.continuum_matrix(fv.assemble(p), p.tau, 0)
    rows = precond.ilu0(K)
    n = K.shape[0]
    L = np.eye(n)
    U = np.zeros((n, n))
    for i, row in enumerate(rows):
        for j, v in row.items():
            if j < i:
                L[i, j] = v
            else:
                U[i, j] = v
    M = L @ U
    Kd = K.toarray()
    mask = Kd != 0
    np.testing.assert_allclose(M[mask], Kd[mask], rtol=1e-12, atol=1e-18)
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_block_partitions():
    b = precond.grid_tile_blocks(130, 40)
    assert len(b) == 3 * 3 and sorted(np.concatenate(b).tolist()) == list(range(130 * 40))
    assert b[0][:3].tolist() == [0, 1, 2] and b[0][64] == 130
    ch = precond.chain_blocks(6, np.array([[0, 1], [1, 2], [3, 4], [2, 5]]))
    assert [c.tolist() for c in ch] == [[0, 1, 2], [3, 4], [5]]


# ------------------------------------------------------------------------------------
# multigrid V-cycle (the GPU path's second preconditioner option)
# ------------------------------------------------------------------------------------
def test_aggregation_coarse_operator_by_counting():
    """The coarse operator on a homogeneous 9 x 7 grid, against counts done by hand: a coarse
    face conductance is half the fine conductance times the fine faces it covers (2, or 1
    along the 1-wide last column / row of an odd grid), and a coarse row sum equals the sum
    of the aggregate's fine row sums (P^T K 1 = P^T (K 1)); it is symmetric and positive
    definite."""
    p = media.rect_problem(9, 7, seed=2, lognormal=False)
    K = schemes.continuum_matrix(fv.assemble(p), p.tau, 0).tocsr()
    nx, ny = p.nx, p.ny
    assert K.shape[0] == nx * ny
    t = -K[0, 1]
    assert t > 0 and np.isclose(-K[0, nx], t)
    P, cnx, cny = precond.aggregate_prolongator(nx, ny)
    assert (cnx, cny) == (5, 4)
    Kc = precond.coarse_operator(K, P).toarray()
    for Y in range(cny):
        for X in range(cnx):
            I = Y * cnx + X
            rows = 2 if 2 * Y + 1 < ny else 1
            cols = 2 if 2 * X + 1 < nx else 1
            if X + 1 < cnx:
                assert np.isclose(-Kc[I, I + 1], 0.5 * rows * t)
            if Y + 1 < cny:
                assert np.isclose(-Kc[I, I + cnx], 0.5 * cols * t)
            nb = [J for J in range(cnx * cny) if J != I and Kc[I, J] != 0]
            assert len(nb) == (X > 0) + (X + 1 < cnx) + (Y > 0) + (Y + 1 < cny)
    fine_rowsum = np.asarray(K.sum(axis=1)).ravel()
    np.testing.assert_allclose(Kc.sum(axis=1), P.T @ fine_rowsum, rtol=1e-12)
    assert np.abs(Kc - Kc.T).max() == 0 and np.linalg.eigvalsh(Kc).min() > 0


def _dense_inverse_of(apply, n):
    return np.column_stack([apply(e) for e in np.eye(n)])


def test_two_grid_cycle_error_propagation():
    """Two levels (20 x 18 cells, coarse 10 x 9 solved exactly): the cycle equals
    (I - E) K^-1 with E = (I - M^-1 K)(I - P Kc^-1 P^T K)(I - M^-1 K), the product of the
    smoothing and coarse-correction error propagators; V is symmetric and V K has its
    spectrum in (0, 2) (the halved coarse faces over-correct, by at most a factor 2, since
    Kc >= P^T K P / 2)."""
    p = media.rect_problem(20, 18, seed=9)
    asm = fv.assemble(p)
    K = schemes.continuum_matrix(asm, p.tau, 0).toarray()
    n = K.shape[0]
    assert n == 360
    lev = precond.vcycle_setup(K, p.nx, p.ny)
    assert len(lev) == 2 and "inv" in lev[1]
    Minv = _dense_inverse_of(lambda e: precond.block_precond_apply(lev[0]["facs"], e), n)
    P = lev[0]["P"].toarray()
    Kc = precond.coarse_operator(sp.csr_matrix(K), sp.csr_matrix(P)).toarray()
    I = np.eye(n)
    S = I - Minv @ K
    Cc = I - P @ np.linalg.solve(Kc, P.T @ K)
    E = S @ Cc @ S
    Vref = (I - E) @ np.linalg.inv(K)
    V = _dense_inverse_of(lambda e: precond.vcycle_apply(lev, e), n)
    assert np.abs(V - Vref).max() < 1e-10 * np.abs(Vref).max()
    assert np.abs(V - V.T).max() < 1e-12 * np.abs(V).max()
    ev = np.linalg.eigvals(V @ K).real
    assert ev.min() > 0 and ev.max() < 2


@pytest.mark.parametrize("sweeps", [1, 2])
def test_truncated_cycle_error_propagation(sweeps):
    """A cycle truncated after its first coarse level (36 x 32 -> 18 x 16, whose own coarser
    levels are dropped): the coarse solve Kc^-1 of the two-grid cycle becomes s sweeps of
    the coarse smoother, (I - (I - Mc^-1 Kc)^s) Kc^-1 (for s = 1 just Mc^-1), so
    V = (I - E) K^-1 with E = S (I - P (I - Sc^s) Kc^-1 P^T K) S; V stays symmetric positive
    definite."""
    p = media.rect_problem(36, 32, seed=4)
    K = schemes.continuum_matrix(fv.assemble(p), p.tau, 0).toarray()
    n = K.shape[0]
    lev = precond.vcycle_setup(K, p.nx, p.ny, max_levels=1, last_sweeps=sweeps)
    assert len(lev) == 2 and lev[1].get("sweeps") == sweeps and "inv" not in lev[1]
    Minv = _dense_inverse_of(lambda e: precond.block_precond_apply(lev[0]["facs"], e), n)
    P = lev[0]["P"].toarray()
    Kc = precond.coarse_operator(sp.csr_matrix(K), sp.csr_matrix(P)).toarray()
    nc = Kc.shape[0]
    Mc = _dense_inverse_of(lambda e: precond.block_precond_apply(lev[1]["facs"], e), nc)
    Sc = np.eye(nc) - Mc @ Kc
    coarse = (np.eye(nc) - np.linalg.matrix_power(Sc, sweeps)) @ np.linalg.inv(Kc)
    I = np.eye(n)
    S = I - Minv @ K
    E = S @ (I - P @ coarse @ P.T @ K) @ S
    Vref = (I - E) @ np.linalg.inv(K)
    V = _dense_inverse_of(lambda e: precond.vcycle_apply(lev, e), n)
    assert np.abs(V - Vref).max() < 1e-10 * np.abs(Vref).max()
    assert np.abs(V - V.T).max() < 1e-12 * np.abs(V).max()
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0


def test_three_level_cycle_symmetric_positive():
    """Three levels (36 x 32 -> 18 x 16 -> 9 x 8): (r1, V r2) = (r2, V r1), (r, V r) > 0."""
    p = media.rect_problem(36, 32, seed=4)
    K = schemes.continuum_matrix(fv.assemble(p), p.tau, 0)
    lev = precond.vcycle_setup(K, p.nx, p.ny)
    assert [(l["nx"], l["ny"]) for l in lev] == [(36, 32), (18, 16), (9, 8)]
    rng = np.random.default_rng(1)
    for _ in range(3):
        a, b = rng.standard_normal((2, 36 * 32))
        va, vb = precond.vcycle_apply(lev, a), precond.vcycle_apply(lev, b)
        assert abs(a @ vb - b @ va) < 1e-12 * np.linalg.norm(a) * np.linalg.norm(vb)
        assert a @ va > 0
    p2 = media.rect_problem(16, 16, seed=4)
    K2 = schemes.continuum_matrix(fv.assemble(p2), p2.tau, 0)
    lev2 = precond.vcycle_setup(K2, 16, 16)   # 256 cells: plain block IC(0)
    assert len(lev2) == 1
    r = rng.standard_normal(256)
    np.testing.assert_array_equal(precond.vcycle_apply(lev2, r),
                                  precond.block_precond_apply(lev2[0]["facs"], r))
