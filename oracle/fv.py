"""Finite-volume assembly of the multicontinuum system (oracle; test infrastructure only).

Follows Section 3.1 of the paper:

* storage  m_{a,i} = c_a |cell_i|                                (matrix M, eq. app-mc)
* diffusion: two-point flux T_ij = k |E_ij| / d_ij between neighbouring cells; the
  operator D_a has a_ii = sum_j T_ij and a_ij = -T_ij          (eqs. app-md, app-mc)
* transfer: q_{ab,ij} = sigma_{ab,ij} where cell i of continuum a meets cell j of b;
  Q_ab = Q_ba^T, and the diagonal block of Q for continuum a is the row-sum diagonal of
  sum_{b != a} Q_ab                                              (eqs. app, app-mc)
* right-hand side F_a = f_a |cell| plus boundary contributions.

Readings where the paper is silent (each is also listed in the design notes):
* square cells of side h, so |E|/d = 1 for interior faces; with a cellwise permeability the
  face value is the harmonic mean 2 k_i k_j / (k_i + k_j) (the two half-cell conductances
  in series), which is k for a constant k;
* a Dirichlet side (the workloads replace the paper's no-flow condition on the west and east
  sides) is a half-cell conductance T_b = 2 k_i added to a_ii, with T_b p_D added to F;
* fracture cell measure |iota_l| = aperture * len_l; fracture connection
  T_e = k_f * aperture / d_e; the discrete matrix-fracture coefficients sigma_il are inputs;
* the Omega-Omega transfer of the three-continuum model is sigma_12 |cell| per cell;
* 3-D (the paper's stated extension, nz > 1 stacked planes): cubic cells of side h, so
  |cell| = h^3 and |E| / d = h for interior faces (T = k h, harmonic mean for a cellwise k),
  a Dirichlet side face T_b = 2 k_i h, and fracture planes whose cells have measure
  aperture * area;
* the wells of the numerical results (Section 5) are a fracture source q_w (p_w - p_f) per
  unit measure: the paper prints q_w (p - p_w), which with q_w = 1e5 on the right-hand side
  would be an anti-diffusive term that makes the system indefinite, so the physical sign is
  taken.  The term is implicit: q_w |iota_l| joins the diagonal of the fracture operator D_f
  and q_w p_w |iota_l| joins F_f.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp

BC_DIRICHLET = 1   # input code for a Dirichlet side (0 = no-flow)


def omega_transmissibilities(k: np.ndarray):
    """Face transmissibilities of an ny x nx cell grid with square cells.

    Returns (tx, ty): tx[y, x] couples cells (x, y) and (x+1, y), shape (ny, nx-1);
    ty[y, x] couples (x, y) and (x, y+1), shape (ny-1, nx).  T = k|E|/d with |E| = d = h
    for constant k; harmonic mean for a cellwise k.
    """
    k = np.asarray(k, np.float64)
    def harm(a, b):
        s = a + b
        out = np.zeros_like(s)
        nz = s > 0
        out[nz] = 2.0 * a[nz] * b[nz] / s[nz]
        return out
    tx = harm(k[:, :-1], k[:, 1:])
    ty = harm(k[:-1, :], k[1:, :])
    return tx, ty


def _harm(a, b):
    s = a + b
    out = np.zeros_like(s)
    nz = s > 0
    out[nz] = 2.0 * a[nz] * b[nz] / s[nz]
    return out


def omega_diffusion_3d(k: np.ndarray, h: float, bc_type, bc_value, bc_type_z,
                       bc_value_z) -> Tuple[sp.csr_matrix, np.ndarray]:
    """D_a of an nz x ny x nx grid of cubes of side h (cells (z*ny + y)*nx + x): every interior
    face T = h * harmonic mean of k, each Dirichlet side face T_b = 2 k_i h.  Sides W, E, S, N
    from bc_type / bc_value, bottom and top from bc_type_z / bc_value_z."""
    nz_, ny, nx = k.shape
    n = nx * ny * nz_
    idx = np.arange(n).reshape(nz_, ny, nx)
    faces = ((h * _harm(k[:, :, :-1], k[:, :, 1:]), idx[:, :, :-1], idx[:, :, 1:]),
             (h * _harm(k[:, :-1, :], k[:, 1:, :]), idx[:, :-1, :], idx[:, 1:, :]),
             (h * _harm(k[:-1], k[1:]), idx[:-1], idx[1:]))
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for t, a, b in faces:
        t, a, b = t.ravel(), a.ravel(), b.ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-t, -t]
        np.add.at(diag, a, t)
        np.add.at(diag, b, t)
    fb = np.zeros(n)
    kf = k.ravel()
    sides = [(idx[:, :, 0], bc_type[0], bc_value[0]), (idx[:, :, -1], bc_type[1], bc_value[1]),
             (idx[:, 0, :], bc_type[2], bc_value[2]), (idx[:, -1, :], bc_type[3], bc_value[3]),
             (idx[0], bc_type_z[0], bc_value_z[0]), (idx[-1], bc_type_z[1], bc_value_z[1])]
    for cells, bt, bv in sides:
        if int(bt) == BC_DIRICHLET:
            cells = cells.ravel()
            tb = 2.0 * kf[cells] * h
            np.add.at(diag, cells, tb)
            np.add.at(fb, cells, tb * float(bv))
    rows.append(np.arange(n)); cols.append(np.arange(n)); vals.append(diag)
    D = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    D.sum_duplicates()
    return D, fb


def omega_diffusion(k: np.ndarray, bc_type, bc_value) -> Tuple[sp.csr_matrix, np.ndarray]:
    """D_a (sparse, n x n with n = nx*ny, row-major cells) and its boundary right-hand side.

    Each interior face contributes T to both diagonals and -T to both off-diagonals; each
    Dirichlet side face contributes T_b = 2 k_i to a_ii and T_b p_D to F_i.
    """
    ny, nx = k.shape
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    tx, ty = omega_transmissibilities(k)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for t, a, b in ((tx, idx[:, :-1], idx[:, 1:]), (ty, idx[:-1, :], idx[1:, :])):
        t, a, b = t.ravel(), a.ravel(), b.ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-t, -t]
        np.add.at(diag, a, t)
        np.add.at(diag, b, t)
    fb = np.zeros(n)
    sides = {0: idx[:, 0], 1: idx[:, -1], 2: idx[0, :], 3: idx[-1, :]}   # W, E, S, N
    kf = k.ravel()
    for s in range(4):
        if int(bc_type[s]) == BC_DIRICHLET:
            cells = sides[s]
            tb = 2.0 * kf[cells]
            np.add.at(diag, cells, tb)
            np.add.at(fb, cells, tb * float(bc_value[s]))
    rows.append(np.arange(n)); cols.append(np.arange(n)); vals.append(diag)
    D = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    D.sum_duplicates()
    return D, fb


def fracture_diffusion(nf: int, edges: np.ndarray, edge_d: np.ndarray, k_f: float,
                       aperture: float) -> sp.csr_matrix:
    """D_f on the fracture-cell graph: T_e = k_f * aperture / d_e per connection."""
    if nf == 0:
        return sp.csr_matrix((0, 0))
    e = np.asarray(edges, np.int64).reshape(-1, 2)
    t = k_f * aperture / np.asarray(edge_d, np.float64)
    diag = np.zeros(nf)
    np.add.at(diag, e[:, 0], t)
    np.add.at(diag, e[:, 1], t)
    rows = np.concatenate([e[:, 0], e[:, 1], np.arange(nf)])
    cols = np.concatenate([e[:, 1], e[:, 0], np.arange(nf)])
    vals = np.concatenate([-t, -t, diag])
    D = sp.csr_matrix((vals, (rows, cols)), shape=(nf, nf))
    D.sum_duplicates()
    return D


@dataclass
class Assembled:
    """All blocks of M dp/dt + (D + Q) p = F for one problem (continuum order: Omega
    continua, then the fracture).  D_f carries the implicit well term besides the fracture
    diffusion."""
    sizes: List[int]
    M: List[np.ndarray]                         # diagonal of M_a
    D: List[sp.csr_matrix]                      # D_a
    Q: Dict[Tuple[int, int], sp.csr_matrix]     # Q_ab for a != b (N_a x N_b), nonnegative
    F: List[np.ndarray]                         # F_a (sources and boundary terms)

    @property
    def L(self) -> int:
        return len(self.sizes)

    def S(self, a: int) -> np.ndarray:
        """Row-sum diagonal of sum_{b != a} Q_ab (the diagonal block of Q)."""
        s = np.zeros(self.sizes[a])
        for b in range(self.L):
            if b != a and (a, b) in self.Q:
                s += np.asarray(self.Q[(a, b)].sum(axis=1)).ravel()
        return s

    def Qfull(self) -> sp.csr_matrix:
        """The block matrix Q with row-sum diagonal blocks and -Q_ab off-diagonal blocks."""
        blocks = [[None] * self.L for _ in range(self.L)]
        for a in range(self.L):
            blocks[a][a] = sp.diags(self.S(a))
            for b in range(self.L):
                if b != a and (a, b) in self.Q:
                    blocks[a][b] = -self.Q[(a, b)]
        return sp.bmat(blocks, format="csr")

    def Afull(self) -> sp.csr_matrix:
        return (sp.block_diag(self.D, format="csr") + self.Qfull()).tocsr()

    def Mfull(self) -> np.ndarray:
        return np.concatenate(self.M)

    def Ffull(self) -> np.ndarray:
        return np.concatenate(self.F)


def assemble(prob) -> Assembled:
    """Assemble M, D, Q, F for a ``media.Problem``."""
    nx, ny, h = prob.nx, prob.ny, prob.h
    nz = getattr(prob, "nz", 1)
    nc = nx * ny * nz
    vol = h ** (3 if nz > 1 else 2)      # cell measure
    no = prob.n_omega
    nf = prob.nf
    sizes = [nc] * no + ([nf] if nf > 0 else [])
    M, D, F = [], [], []
    for a, o in enumerate(prob.omega):
        if nz > 1:
            Da, fb = omega_diffusion_3d(o.k_field(nx, ny, nz), h, prob.bc_type, prob.bc_value,
                                        prob.bc_type_z, prob.bc_value_z)
        else:
            Da, fb = omega_diffusion(o.k_field(nx, ny), prob.bc_type, prob.bc_value)
        D.append(Da)
        M.append(np.full(nc, o.c * vol))
        src = prob.source(a)
        F.append(fb + (0.0 if src is None else src * vol))
    if nf > 0:
        meas = prob.aperture * np.asarray(prob.flen, np.float64)
        M.append(prob.c_f * meas)
        Df = fracture_diffusion(nf, prob.edges, prob.edge_d, prob.k_f, prob.aperture)
        src = prob.source(no)
        Ff = np.zeros(nf) if src is None else src * meas
        wq = getattr(prob, "well_q", None)
        if wq is not None:
            wq = np.asarray(wq, np.float64)
            wp = getattr(prob, "well_p", None)
            wp = np.zeros(nf) if wp is None else np.asarray(wp, np.float64)
            Df = (Df + sp.diags(wq * meas)).tocsr()
            Ff = Ff + wq * wp * meas
        D.append(Df)
        F.append(Ff)
    Q: Dict[Tuple[int, int], sp.csr_matrix] = {}
    if no == 2 and prob.sigma_omega != 0.0:
        q = sp.diags(np.full(nc, prob.sigma_omega * vol)).tocsr()
        Q[(0, 1)] = q
        Q[(1, 0)] = q.T.tocsr()
    if nf > 0:
        fi = no
        host = np.asarray(prob.host, np.int64)
        for a in range(no):
            sig = np.asarray(prob.sigma_f[a], np.float64)
            qaf = sp.csr_matrix((sig, (host, np.arange(nf))), shape=(nc, nf))
            qaf.sum_duplicates()
            Q[(a, fi)] = qaf
            Q[(fi, a)] = qaf.T.tocsr()
    return Assembled(sizes=sizes, M=M, D=D, Q=Q, F=F)
