"""Brute-force dense assembly for tiny problems (oracle cross-check; test infrastructure only).

Builds the coupled matrix M/tau + A row by row from the semi-discrete balance of each cell
(Section 3.1, eqs. app-md / app-tc / app): storage c|cell|/tau on the diagonal, one
two-point flux term T (p_i - p_j) per face or fracture connection, one transfer term
sigma (p_i - p_j) per matrix-fracture or matrix-natural-fracture pair, one exchange
q_w |cell| (p_l - p_w) per fracture well (Section 5, physical sign).  In 3-D (nz > 1) the
cells are cubes: faces of measure h^2, storage and sources over h^3.  Written as plain
Python loops over cells and faces, independently of the vectorized sparse assembly.
"""
from __future__ import annotations

import numpy as np


def coupled_dense(prob, tau: float):
    nx, ny, h = prob.nx, prob.ny, prob.h
    nz = getattr(prob, "nz", 1)
    dim = 3 if nz > 1 else 2
    nc = nx * ny * nz
    vol = h ** dim                 # cell measure; a face has measure h^(dim-1)
    no = prob.n_omega
    nf = prob.nf
    off = [a * nc for a in range(no)] + [no * nc]
    N = no * nc + nf
    K = np.zeros((N, N))
    rhs_f = np.zeros(N)

    def flux(i, j, t):
        K[i, i] += t
        K[i, j] -= t

    face = h ** (dim - 1)
    bct = list(prob.bc_type) + (list(prob.bc_type_z) if dim == 3 else [])
    bcv = list(prob.bc_value) + (list(prob.bc_value_z) if dim == 3 else [])
    for a, o in enumerate(prob.omega):
        k = o.k_field(nx, ny, nz).reshape(nz, ny, nx)
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    c = (z * ny + y) * nx + x
                    i = off[a] + c
                    K[i, i] += o.c * vol / tau
                    nbrs = [(x - 1, y, z, 0), (x + 1, y, z, 1), (x, y - 1, z, 2), (x, y + 1, z, 3)]
                    if dim == 3:
                        nbrs += [(x, y, z - 1, 4), (x, y, z + 1, 5)]
                    for (xx, yy, zz, side) in nbrs:
                        if 0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz:
                            k1, k2 = k[z, y, x], k[zz, yy, xx]
                            # two half-cell resistances (d/2) / (k |E|) in series, d = h
                            t = face / (0.5 * h / k1 + 0.5 * h / k2) if k1 > 0 and k2 > 0 else 0.0
                            flux(i, off[a] + (zz * ny + yy) * nx + xx, t)
                        elif int(bct[side]) == 1:
                            t = k[z, y, x] / (0.5 * h) * face      # d = h/2 to the side
                            K[i, i] += t
                            rhs_f[i] += t * bcv[side]
                    src = prob.source(a)
                    if src is not None:
                        rhs_f[i] += src[c] * vol
        if no == 2:
            b = 1 - a
            for c in range(nc):
                flux(off[a] + c, off[b] + c, prob.sigma_omega * vol)
    if nf:
        fo = off[no]
        for l in range(nf):
            meas = prob.aperture * prob.flen[l]
            K[fo + l, fo + l] += prob.c_f * meas / tau
            src = prob.source(no)
            if src is not None:
                rhs_f[fo + l] += src[l] * meas
            wq = getattr(prob, "well_q", None)
            if wq is not None:
                # a well exchanges with a reservoir held at p_w, like a Dirichlet face
                t = float(wq[l]) * meas
                K[fo + l, fo + l] += t
                rhs_f[fo + l] += t * (0.0 if prob.well_p is None else float(prob.well_p[l]))
        for e in range(len(prob.edges)):
            l, m = int(prob.edges[e, 0]), int(prob.edges[e, 1])
            t = prob.k_f * prob.aperture / prob.edge_d[e]
            flux(fo + l, fo + m, t)
            flux(fo + m, fo + l, t)
        for a in range(no):
            for l in range(nf):
                s = prob.sigma_f[a, l]
                i = off[a] + int(prob.host[l])
                flux(i, fo + l, s)
                flux(fo + l, i, s)
    mdiag = np.zeros(N)
    for a, o in enumerate(prob.omega):
        mdiag[off[a]:off[a] + nc] = o.c * vol
    if nf:
        mdiag[off[no]:] = prob.c_f * prob.aperture * np.asarray(prob.flen)
    return K, mdiag, rhs_f, off


def coupled_step_dense(prob, tau: float, p_prev):
    """One backward-Euler step of the coupled system by a dense solve."""
    K, mdiag, rf, off = coupled_dense(prob, tau)
    x = np.linalg.solve(K, mdiag / tau * np.concatenate(p_prev) + rf)
    return x
