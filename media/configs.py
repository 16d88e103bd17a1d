"""Seeded recipes for the five benchmark workloads and for small parity cases.

All randomness comes from ``numpy.random.default_rng`` with fixed seeds, so every
array is reproducible.  The recipes are stand-ins for the paper's fracture network,
whose geometry exists only in a figure: a unit square, a matrix continuum, an optional
natural-fracture continuum on the same grid, and straight fracture segments cut into
cells of length h.

Matrix-fracture transfer input: the discrete transfer coefficient of fracture cell l with
its host cell in Omega continuum a is supplied as ``sigma_f[a, l] = k_a(host) * len_l / h``
(the workload's "sigma = k_m / h between each fracture cell and its host" stated per unit
fracture length).  Fracture cells of different segments that share a host cell are joined
by an edge with centre distance h; consecutive cells of one segment by an edge of centre
distance equal to the cell length.
"""
from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np
from scipy.signal import fftconvolve

from .problem import BC_DIRICHLET, BC_NOFLOW, OmegaContinuum, Problem

CONFIG_NAMES = ("C1", "C2", "C3", "C4", "C5")

# fracture physics shared by every workload
K_F, C_F, APERTURE = 1.0, 0.1, 1e-3
# natural-fracture continuum of the three-continuum workloads
K_NAT, C_NAT, SIGMA_NAT = 1e-2, 0.05, 10.0


# --------------------------------------------------------------------------------------
# permeability fields
# --------------------------------------------------------------------------------------
def lognormal_field(n: int, rng: np.random.Generator, median: float = 1e-4,
                    sigma_log: float = 1.5, corr_len: float = 0.05,
                    ny: Optional[int] = None) -> np.ndarray:
    """ln k = ln(median) + sigma_log * g with g a unit-variance Gaussian field whose
    covariance is exp(-r^2 / corr_len^2) on the unit square (h = 1/n).

    g is white noise convolved with exp(-2 r^2 / corr_len^2) (zero-padded, so the field is
    not periodic) and divided by the kernel's L2 norm, which gives unit variance.
    """
    ny = n if ny is None else ny
    h = 1.0 / n
    pad = int(np.ceil(2.0 * corr_len / h))
    off = np.arange(-pad, pad + 1) * h
    kern = np.exp(-2.0 * (off[:, None] ** 2 + off[None, :] ** 2) / corr_len ** 2)
    kern /= np.sqrt(np.sum(kern ** 2))
    noise = rng.standard_normal((ny + 2 * pad, n + 2 * pad))
    g = fftconvolve(noise, kern, mode="valid")
    assert g.shape == (ny, n)
    return np.exp(np.log(median) + sigma_log * g)


# --------------------------------------------------------------------------------------
# fracture geometry
# --------------------------------------------------------------------------------------
def _axis_segments(n: int, nseg: int, lmin: int, lmax: int, rng: np.random.Generator,
                   min_cells: int = 0) -> List[np.ndarray]:
    """Axis-aligned segments on an n x n grid, each a list of host cells (in order).

    Orientation ~ Bernoulli(1/2); length ~ U{lmin..lmax} cells; row (or column) ~ U{0..n-1};
    start ~ U{0..n-L}.  A segment that overlaps a collinear one is redrawn.  With
    ``min_cells`` > 0, segments are added past ``nseg`` until that many cells exist.
    """
    used_h = {}   # row -> list of (start, end) occupied by horizontal segments
    used_v = {}
    segs: List[np.ndarray] = []
    total = 0
    while len(segs) < nseg or total < min_cells:
        horiz = bool(rng.integers(0, 2))
        L = int(rng.integers(lmin, lmax + 1))
        L = min(L, n)
        line = int(rng.integers(0, n))
        start = int(rng.integers(0, n - L + 1))
        book = used_h if horiz else used_v
        if any(not (start + L <= s or e <= start) for (s, e) in book.get(line, [])):
            continue                                   # collinear overlap: redraw
        book.setdefault(line, []).append((start, start + L))
        j = np.arange(start, start + L)
        cells = line * n + j if horiz else j * n + line
        segs.append(cells.astype(np.int64))
        total += L
    return segs


def _angle_segments(n: int, nseg: int, lmin: int, lmax: int,
                    rng: np.random.Generator) -> List[np.ndarray]:
    """Any-angle segments: midpoint ~ U[0,1]^2, angle ~ U[0, pi), L ~ U{lmin..lmax} cells of
    length h centred at x0 + (j - (L-1)/2) h (cos t, sin t); the host is the grid cell that
    contains the centre, and cells whose centre falls outside (0,1)^2 are dropped."""
    h = 1.0 / n
    segs: List[np.ndarray] = []
    for _ in range(nseg):
        x0, y0 = rng.random(2)
        th = rng.random() * np.pi
        L = int(rng.integers(lmin, lmax + 1))
        j = np.arange(L) - (L - 1) / 2.0
        cx = x0 + j * h * np.cos(th)
        cy = y0 + j * h * np.sin(th)
        keep = (cx > 0) & (cx < 1) & (cy > 0) & (cy < 1)
        ix = np.minimum(np.floor(cx[keep] / h).astype(np.int64), n - 1)
        iy = np.minimum(np.floor(cy[keep] / h).astype(np.int64), n - 1)
        if len(ix):
            segs.append(iy * n + ix)
    return segs


def _fracture_arrays(segs: List[np.ndarray], h: float):
    """Concatenate segments (segment-major cell order) and build the connection list:
    chain edges between consecutive cells of a segment (distance h) and, for every host
    cell holding cells of different segments, an edge between each such pair (distance h).
    """
    if not segs:
        return (np.zeros(0, np.int32), np.zeros(0), np.zeros((0, 2), np.int32), np.zeros(0),
                np.zeros(0, np.int32))
    host = np.concatenate(segs).astype(np.int64)
    seg_id = np.concatenate([np.full(len(s), i) for i, s in enumerate(segs)])
    nf = len(host)
    flen = np.full(nf, h)
    chain = []
    off = 0
    for s in segs:
        L = len(s)
        if L > 1:
            a = np.arange(off, off + L - 1)
            chain.append(np.stack([a, a + 1], axis=1))
        off += L
    chain = np.concatenate(chain) if chain else np.zeros((0, 2), np.int64)
    # crossings: cells of different segments sharing a host
    order = np.lexsort((np.arange(nf), host))
    hs = host[order]
    cross = []
    starts = np.flatnonzero(np.r_[True, hs[1:] != hs[:-1]])
    ends = np.r_[starts[1:], nf]
    for s0, e0 in zip(starts, ends):
        if e0 - s0 < 2:
            continue
        grp = order[s0:e0]
        for i in range(len(grp)):
            for j in range(i + 1, len(grp)):
                a, b = int(grp[i]), int(grp[j])
                if seg_id[a] != seg_id[b]:
                    cross.append((min(a, b), max(a, b)))
    cross = np.array(sorted(cross), np.int64).reshape(-1, 2)
    edges = np.concatenate([chain, cross]).astype(np.int32)
    edge_d = np.full(len(edges), h)
    return host.astype(np.int32), flen, edges, edge_d, seg_id.astype(np.int32)


def _sigma_f(omega: List[OmegaContinuum], host: np.ndarray, flen: np.ndarray, n: int,
             h: float) -> np.ndarray:
    """Transfer input sigma_f[a, l] = k_a(host(l)) * len_l / h."""
    out = np.zeros((len(omega), len(host)))
    for a, o in enumerate(omega):
        k = o.k_field(n, n).reshape(-1)
        out[a] = k[host] * flen / h
    return out


def _bc_c1() -> Tuple[np.ndarray, np.ndarray]:
    # Dirichlet p = 1 on the west side, p = 0 on the east side, no-flow south and north
    return (np.array([BC_DIRICHLET, BC_DIRICHLET, BC_NOFLOW, BC_NOFLOW], np.int32),
            np.array([1.0, 0.0, 0.0, 0.0]))


def build_problem(n: int, omega: List[OmegaContinuum], segs: List[np.ndarray], tau: float,
                  nsteps: int, sigma_omega: float = 0.0, meta: Optional[dict] = None,
                  k_f: float = K_F, c_f: float = C_F, aperture: float = APERTURE) -> Problem:
    h = 1.0 / n
    host, flen, edges, edge_d, seg_id = _fracture_arrays(segs, h)
    bct, bcv = _bc_c1()
    m = dict(meta or {})
    m["seg_id"] = seg_id
    p = Problem(nx=n, ny=n, h=h, omega=omega, sigma_omega=sigma_omega, host=host, flen=flen,
                edges=edges, edge_d=edge_d, k_f=k_f, c_f=c_f, aperture=aperture,
                sigma_f=_sigma_f(omega, host, flen, n, h), bc_type=bct, bc_value=bcv,
                src=None, p0=None, tau=tau, nsteps=nsteps, meta=m)
    p.check()
    return p


# --------------------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------------------
def _c1(seed: int = 1, n: int = 64) -> Problem:
    rng = np.random.default_rng(seed)
    segs = _axis_segments(n, 8, 10, 40, rng)
    return build_problem(n, [OmegaContinuum(c=1.0, k_const=1e-4)], segs, tau=0.01, nsteps=20,
                         meta=dict(name="C1", precond="jacobi", tol=1e-12, precision="fp64"))


def _c2(seed: int = 2, n: int = 2048, nseg: int = 400) -> Problem:
    rng = np.random.default_rng(seed)
    k = lognormal_field(n, rng, median=1e-4, sigma_log=1.5, corr_len=0.05)
    segs = _angle_segments(n, nseg, 20, 300, rng)
    return build_problem(n, [OmegaContinuum(c=1.0, k=k)], segs, tau=1e-3, nsteps=100,
                         meta=dict(name="C2", precond="ic0", tol=1e-10, precision="fp64"))


def _c3(seed: int = 3, n: int = 4096, min_cells: int = 150_000) -> Problem:
    rng = np.random.default_rng(seed)
    scale = n // 64
    segs = _axis_segments(n, 8, 10 * scale, 40 * scale, rng, min_cells=min_cells)
    omega = [OmegaContinuum(c=1.0, k_const=1e-4), OmegaContinuum(c=C_NAT, k_const=K_NAT)]
    return build_problem(n, omega, segs, tau=1e-3, nsteps=50, sigma_omega=SIGMA_NAT,
                         meta=dict(name="C3", precond="jacobi", tol=1e-10, precision="mixed"))


def _3d(seed: int = 8, n: int = 256, nz: int = 256) -> Problem:
    # plane sides scale with the grid (16..96 cells at n = 256)
    lo, hi = max(2, 16 * n // 256), max(4, 96 * n // 256)
    p = box_problem(n=n, nz=nz, seed=seed, nplane=40, plane_len=(lo, hi), nsteps=20)
    p.meta.update(name="3D", precond="bic0", tol=1e-10, precision="fp64")
    return p


def config_problem(name: str, **kw) -> Problem:
    """Problem of workload C1, C2, C3 or the 3-D extension (C4 and C5 are families: see
    c4_problems, c5_trace)."""
    return {"C1": _c1, "C2": _c2, "C3": _c3, "3D": _3d}[name](**kw)


def _family_member(rng: np.random.Generator, n: int, three: bool, sigma_log: Optional[float],
                   k_m_const: Optional[float], nseg: int, nsteps: int, name: str) -> Problem:
    if k_m_const is None:
        k = lognormal_field(n, rng, median=1e-4, sigma_log=sigma_log, corr_len=0.05)
        omega = [OmegaContinuum(c=1.0, k=k)]
    else:
        omega = [OmegaContinuum(c=1.0, k_const=k_m_const)]
    if three:
        omega.append(OmegaContinuum(c=C_NAT, k_const=K_NAT))
    segs = _angle_segments(n, nseg, 20, 300, rng)
    return build_problem(n, omega, segs, tau=1e-3, nsteps=nsteps,
                         sigma_omega=SIGMA_NAT if three else 0.0,
                         meta=dict(name=name, precond="jacobi", tol=1e-10, precision="mixed"))


def _c4_draw(ss, n_range):
    rng = np.random.default_rng(ss)
    three = bool(rng.integers(0, 2))
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    sl = float(rng.uniform(0.5, 2.5))
    nseg = int(rng.integers(20, 201))
    return rng, three, n, sl, nseg


def c4_problems(count: int = 256, seed: int = 4, n_range=(128, 1024),
                only: Optional[List[int]] = None) -> List[Problem]:
    """Batched realizations: two- or three-continuum (1/2 each), side n ~ U{n_range},
    lognormal matrix permeability with sigma_log ~ U[0.5, 2.5], 20..200 segments.
    Realization i depends only on its own spawned seed; `only` builds a subset."""
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(count)):
        if only is not None and i not in only:
            continue
        rng, three, n, sl, nseg = _c4_draw(ss, n_range)
        out.append(_family_member(rng, n, three, sl, None, nseg, 50, f"C4[{i}]"))
    return out


def c4_shapes(count: int = 256, seed: int = 4, n_range=(128, 1024)):
    """(n, three_continuum) of every realization, without building the fields."""
    out = []
    for ss in np.random.SeedSequence(seed).spawn(count):
        _, three, n, _, _ = _c4_draw(ss, n_range)
        out.append((n, three))
    return out


def c5_trace(count: int = 400, seed: int = 5, rate: float = 40.0, n_range=(64, 2048),
             steps_range=(10, 500)):
    """Serving trace: list of (arrival_time_s, n, three, contrast, nsteps, seed_seq).  The
    problems are built on demand with ``c5_problem`` so the trace itself stays small."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    kids = np.random.SeedSequence(seed + 1000).spawn(count)
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(round(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        three = bool(rng.integers(0, 2))
        contrast = float(np.exp(rng.uniform(np.log(1e2), np.log(1e6))))
        ns = int(rng.integers(steps_range[0], steps_range[1] + 1))
        out.append((t, n, three, contrast, ns, kids[i]))
    return out


def c5_problem(entry) -> Problem:
    t, n, three, contrast, ns, ss = entry
    rng = np.random.default_rng(ss)
    nseg = int(rng.integers(20, 201))
    return _family_member(rng, n, three, None, K_F / contrast, nseg, ns, "C5")


def rect_problem(nx: int, ny: int, seed: int = 7, lognormal: bool = True,
                 sigma_log: float = 1.5, tau: float = 1e-3, nsteps: int = 3) -> Problem:
    """A grid-only (no fracture) two-continuum problem on an nx x ny grid with h = 1/nx:
    lognormal or constant matrix permeability, the C1 boundary conditions."""
    rng = np.random.default_rng(seed)
    if lognormal:
        om = OmegaContinuum(c=1.0, k=lognormal_field(nx, rng, sigma_log=sigma_log, ny=ny))
    else:
        om = OmegaContinuum(c=1.0, k_const=1e-4)
    bct, bcv = _bc_c1()
    h = 1.0 / nx
    p = Problem(nx=nx, ny=ny, h=h, omega=[om], sigma_omega=0.0,
                sigma_f=np.zeros((1, 0)), bc_type=bct, bc_value=bcv, src=None, p0=None,
                tau=tau, nsteps=nsteps,
                meta=dict(name=f"rect{nx}x{ny}", precond="jacobi", tol=1e-12, precision="fp64",
                          seg_id=np.zeros(0, np.int32)))
    p.check()
    return p


def small_problem(n: int = 40, seed: int = 7, three: bool = False, nseg: int = 6,
                  lognormal: bool = True, axis: bool = False, tau: float = 1e-3,
                  nsteps: int = 5, sigma_log: float = 1.5, seg_len=(5, 30)) -> Problem:
    """Small problems with the workloads' structure, for parity tests the oracle finishes
    in seconds (lognormal or constant matrix k, any-angle or axis-aligned segments)."""
    rng = np.random.default_rng(seed)
    if lognormal:
        omega = [OmegaContinuum(c=1.0, k=lognormal_field(n, rng, sigma_log=sigma_log))]
    else:
        omega = [OmegaContinuum(c=1.0, k_const=1e-4)]
    if three:
        omega.append(OmegaContinuum(c=C_NAT, k_const=K_NAT))
    if axis:
        segs = _axis_segments(n, nseg, seg_len[0], min(seg_len[1], n), rng)
    else:
        segs = _angle_segments(n, nseg, seg_len[0], seg_len[1], rng)
    return build_problem(n, omega, segs, tau=tau, nsteps=nsteps,
                         sigma_omega=SIGMA_NAT if three else 0.0,
                         meta=dict(name=f"small{n}", precond="jacobi", tol=1e-12,
                                   precision="fp64"))


# --------------------------------------------------------------------------------------
# the paper's own test problems (Section 5): 2C and 3C with wells
# --------------------------------------------------------------------------------------
WELL_BOXES = ((0.10, 0.15, 0.10, 0.15), (0.60, 0.65, 0.85, 0.90))   # x0, x1, y0, y1
WELL_Q, WELL_P, PAPER_T, PAPER_STEPS = 1e5, 1.2, 0.002, 50
PAPER_FRACTURE_CELLS = 2684


def _rays(n: int, mids: np.ndarray, dirs: np.ndarray, lens: np.ndarray) -> List[np.ndarray]:
    """Segments of lens[s] cells of length h centred on mids[s] along dirs[s] (cells whose
    centre leaves the open unit square are dropped), as host-cell lists."""
    h = 1.0 / n
    out = []
    for m, d, L in zip(mids, dirs, lens):
        j = np.arange(int(L)) - (int(L) - 1) / 2.0
        cx, cy = m[0] + j * h * d[0], m[1] + j * h * d[1]
        keep = (cx > 0) & (cx < 1) & (cy > 0) & (cy < 1)
        ix = np.minimum(np.floor(cx[keep] / h).astype(np.int64), n - 1)
        iy = np.minimum(np.floor(cy[keep] / h).astype(np.int64), n - 1)
        if len(ix):
            out.append(iy * n + ix)
    return out


def _paper_network(n: int, nseg: int, total: int, rng: np.random.Generator) -> List[np.ndarray]:
    """A stand-in for the paper's 25-line network (its geometry is only drawn): nseg
    any-angle segments, the first two centred inside the two well boxes so that both boxes
    hold fracture cells, the others centred uniformly; relative lengths U[0.3, 1] scaled by
    one common factor (bisection) so that the network has `total` cells after clipping, the
    last segment's length then adjusted by whole cells towards that count."""
    mids = rng.random((nseg, 2))
    for b, (x0, x1, y0, y1) in enumerate(WELL_BOXES[:min(2, nseg)]):
        mids[b] = (x0 + (x1 - x0) * rng.random(), y0 + (y1 - y0) * rng.random())
    th = rng.random(nseg) * np.pi
    dirs = np.stack([np.cos(th), np.sin(th)], axis=1)
    w = rng.uniform(0.3, 1.0, nseg)
    count = lambda lens: sum(len(s) for s in _rays(n, mids, dirs, lens))  # noqa: E731
    lo, hi = 0.0, 4.0 * total / w.sum()
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if count(np.maximum(1, np.round(w * mid))) < total:
            lo = mid
        else:
            hi = mid
    lens = np.maximum(1, np.round(w * hi)).astype(np.int64)
    best = (abs(count(lens) - total), lens[-1])
    for L in range(max(1, int(lens[-1]) - 40), int(lens[-1]) + 41):
        lens[-1] = L
        best = min(best, (abs(count(lens) - total), L))
    lens[-1] = best[1]
    return _rays(n, mids, dirs, lens)


def paper_problem(case: str = "2C", n: int = 200, seed: int = 11,
                  nsteps: int = PAPER_STEPS) -> Problem:
    """The test problems of the paper's numerical results on an n x n grid (200 there).

    2C: matrix c = 0.1, k = 1; explicit fractures c = 1, k = 1e6.  3C: matrix c = 0.05,
    k = 1e-3; natural fractures c = 0.1, k = 1; explicit fractures c = 1, k = 1e6.  No-flow
    sides, p0 = 1 everywhere, T = 0.002 in 50 layers, wells q_w = 1e5, p_w = 1.2 on the
    fracture cells whose host cell centre lies in one of the two boxes.  The paper leaves
    the network geometry to a figure and sigma and the aperture unstated; here: a synthetic
    25-segment network of about 2684 cells, aperture 1 (the fracture measure is the cell
    length, as in the paper's 1-D fracture balance), matrix-fracture sigma_il = k_a len_l /
    h, and in 3C a matrix-natural-fracture coefficient sigma_12 = k_1 / h^2 per unit area
    (sigma_12 |cell| = k_1: the two-point conductance of co-located cells at distance h).
    """
    if case not in ("2C", "3C"):
        raise ValueError(case)
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    total = int(round(PAPER_FRACTURE_CELLS * (n / 200.0)))
    segs = _paper_network(n, 25, total, rng)
    if case == "2C":
        omega = [OmegaContinuum(c=0.1, k_const=1.0)]
        sig12 = 0.0
    else:
        omega = [OmegaContinuum(c=0.05, k_const=1e-3), OmegaContinuum(c=0.1, k_const=1.0)]
        sig12 = 1e-3 / h ** 2
    host, flen, edges, edge_d, seg_id = _fracture_arrays(segs, h)
    nf = len(host)
    hx = (host % n + 0.5) * h
    hy = (host // n + 0.5) * h
    inbox = np.zeros(nf, bool)
    for (x0, x1, y0, y1) in WELL_BOXES:
        inbox |= (hx >= x0) & (hx <= x1) & (hy >= y0) & (hy <= y1)
    p = Problem(nx=n, ny=n, h=h, omega=omega, sigma_omega=sig12, host=host, flen=flen,
                edges=edges, edge_d=edge_d, k_f=1e6, c_f=1.0, aperture=1.0,
                sigma_f=_sigma_f(omega, host, flen, n, h),
                bc_type=np.zeros(4, np.int32), bc_value=np.zeros(4),
                src=None, p0=[np.ones(n * n)] * len(omega) + [np.ones(nf)],
                well_q=np.where(inbox, WELL_Q, 0.0), well_p=np.full(nf, WELL_P),
                tau=PAPER_T / PAPER_STEPS, nsteps=nsteps,
                meta=dict(name=case, precond="mg", tol=1e-10, precision="fp64",
                          seg_id=seg_id, wells=int(inbox.sum())))
    p.check()
    return p


# --------------------------------------------------------------------------------------
# 3-D problems (the paper's stated extension): stacked planes, fracture planes
# --------------------------------------------------------------------------------------
def _fracture_planes(n: int, nz: int, nplane: int, lmin: int, lmax: int,
                     rng: np.random.Generator) -> List[np.ndarray]:
    """Axis-aligned fracture rectangles through cell centres of an n x n x nz grid, each a
    list of host cells (in-plane row-major order) with its in-plane shape: normal ~ U{x, y,
    z}; position ~ U over the cells along the normal; side lengths ~ U{lmin..lmax} cells
    (clipped to the grid); corner ~ U."""
    dims = (n, n, nz)   # cells along x, y, z
    out = []
    for _ in range(nplane):
        normal = int(rng.integers(0, 3))
        ax = [a for a in range(3) if a != normal]
        pos = int(rng.integers(0, dims[normal]))
        L = [min(int(rng.integers(lmin, lmax + 1)), dims[a]) for a in ax]
        c0 = [int(rng.integers(0, dims[a] - L[k] + 1)) for k, a in enumerate(ax)]
        u, v = np.meshgrid(np.arange(c0[0], c0[0] + L[0]), np.arange(c0[1], c0[1] + L[1]))
        xyz = [None, None, None]
        xyz[normal] = np.full(u.size, pos)
        xyz[ax[0]] = u.ravel()
        xyz[ax[1]] = v.ravel()
        host = (xyz[2] * n + xyz[1]) * n + xyz[0]
        out.append((host.astype(np.int64), (L[1], L[0])))   # rows along ax[1], columns ax[0]
    return out


def box_problem(n: int = 24, nz: int = 12, seed: int = 7, three: bool = False,
                nplane: int = 4, lognormal: bool = True, tau: float = 1e-3, nsteps: int = 5,
                plane_len=(4, 16)) -> Problem:
    """A 3-D problem on an n x n x nz grid of cubes (h = 1/n): lognormal matrix permeability
    (independent 2-D fields per plane, correlated in x and y) or constant 1e-4, the optional
    natural-fracture continuum, and axis-aligned fracture planes cut into h x h cells
    (measure aperture * h^2).  Fracture cells connect to their in-plane neighbours and,
    where planes meet in a host cell, to each other; a connection's `edge_d` is the centre
    distance over the interface measure, h / h = 1 here.  sigma_f = k_a(host) * area / h.
    Dirichlet p = 1 on the west side, p = 0 on the east side, no-flow elsewhere."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    if lognormal:
        k = np.stack([lognormal_field(n, rng, sigma_log=1.0) for _ in range(nz)])
        omega = [OmegaContinuum(c=1.0, k=k)]
    else:
        omega = [OmegaContinuum(c=1.0, k_const=1e-4)]
    if three:
        omega.append(OmegaContinuum(c=C_NAT, k_const=K_NAT))
    planes = _fracture_planes(n, nz, nplane, plane_len[0], plane_len[1], rng)
    host = np.concatenate([p[0] for p in planes]) if planes else np.zeros(0, np.int64)
    nf = len(host)
    edges = []
    off = 0
    seg_id = []
    for s, (hp, (rows, cols)) in enumerate(planes):
        idx = off + np.arange(rows * cols).reshape(rows, cols)
        edges.append(np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], axis=1))
        edges.append(np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], axis=1))
        seg_id.append(np.full(rows * cols, s))
        off += rows * cols
    seg_id = np.concatenate(seg_id) if seg_id else np.zeros(0, np.int64)
    order = np.lexsort((np.arange(nf), host))
    hs = host[order]
    starts = np.flatnonzero(np.r_[True, hs[1:] != hs[:-1]]) if nf else np.zeros(0, int)
    ends = np.r_[starts[1:], nf]
    cross = []
    for s0, e0 in zip(starts, ends):
        grp = order[s0:e0]
        for i in range(len(grp)):
            for j in range(i + 1, len(grp)):
                a, b = int(grp[i]), int(grp[j])
                if seg_id[a] != seg_id[b]:
                    cross.append((min(a, b), max(a, b)))
    edges.append(np.array(sorted(cross), np.int64).reshape(-1, 2))
    edges = np.concatenate(edges).astype(np.int32) if nf else np.zeros((0, 2), np.int32)
    flen = np.full(nf, h * h)
    sig = np.zeros((len(omega), nf))
    for a, o in enumerate(omega):
        sig[a] = o.k_field(n, n, nz).reshape(-1)[host] * flen / h
    bct, bcv = _bc_c1()
    p = Problem(nx=n, ny=n, nz=nz, h=h, omega=omega, sigma_omega=SIGMA_NAT if three else 0.0,
                host=host.astype(np.int32), flen=flen, edges=edges,
                edge_d=np.ones(len(edges)), k_f=K_F, c_f=C_F, aperture=APERTURE,
                sigma_f=sig, bc_type=bct, bc_value=bcv, src=None, p0=None, tau=tau,
                nsteps=nsteps, meta=dict(name=f"box{n}x{n}x{nz}", precond="jacobi",
                                         tol=1e-12, precision="fp64", seg_id=seg_id))
    p.check()
    return p
