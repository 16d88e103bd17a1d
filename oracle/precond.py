"""Block incomplete factorization with zero fill (oracle; test infrastructure only).

The paper solves every SPD system with CG and an incomplete factorization preconditioner;
the GPU path uses a block form of it.  This module states that preconditioner by its plain
definition so the GPU sweep can be compared with it:

* blocks: the Omega grid cut into 64-column x 16-row blocks; the fracture cells cut into
  chains (maximal runs of consecutive cells l, l+1 joined by a connection); inside a chain
  only the couplings between consecutive cells are kept;
* inside a block, ILU(0) in natural order (Saad, Iterative Methods for Sparse Linear
  Systems, ILU(0) in IKJ form): for each row i and each k < i in the pattern,
  a_ik <- a_ik / a_kk, then a_ij <- a_ij - a_ik a_kj for j > k in the pattern of row i.
  For a symmetric matrix this is IC(0) written as L U; M = L U;
* couplings between blocks are dropped; z = M^-1 r block by block.

Written with plain Python loops over sparse rows: meant for small test problems.
"""
from __future__ import annotations

from typing import Dict, List

import numpy as np
import scipy.sparse as sp


def ilu0(B: sp.spmatrix):
    """ILU(0) of a square sparse matrix in natural order.  Returns (rows, diag) where rows[i]
    is a dict col -> value holding L (strictly lower, unit diagonal implied) and U (upper,
    diagonal included) in the pattern of B."""
    B = sp.csr_matrix(B)
    n = B.shape[0]
    rows: List[Dict[int, float]] = []
    for i in range(n):
        rows.append({int(j): float(v) for j, v in zip(B.indices[B.indptr[i]:B.indptr[i + 1]],
                                                     B.data[B.indptr[i]:B.indptr[i + 1]])})
    for i in range(1, n):
        ri = rows[i]
        for k in sorted(c for c in ri if c < i):
            ri[k] = ri[k] / rows[k][k]
            for j, ukj in rows[k].items():
                if j > k and j in ri:
                    ri[j] -= ri[k] * ukj
    return rows


def ilu0_solve(rows, r: np.ndarray) -> np.ndarray:
    n = len(rows)
    y = np.array(r, np.float64)
    for i in range(n):
        for k, v in rows[i].items():
            if k < i:
                y[i] -= v * y[k]
    z = y
    for i in range(n - 1, -1, -1):
        s = z[i]
        for j, v in rows[i].items():
            if j > i:
                s -= v * z[j]
        z[i] = s / rows[i][i]
    return z


def grid_tile_blocks(nx: int, ny: int, tx: int = 64, ty: int = 16) -> List[np.ndarray]:
    """Row-major cell indices of each tile, in natural (row-major) order inside the tile."""
    out = []
    for y0 in range(0, ny, ty):
        for x0 in range(0, nx, tx):
            ys = np.arange(y0, min(y0 + ty, ny))
            xs = np.arange(x0, min(x0 + tx, nx))
            out.append((ys[:, None] * nx + xs[None, :]).ravel())
    return out


def chain_blocks(nf: int, edges: np.ndarray) -> List[np.ndarray]:
    linked = set()
    for a, b in np.asarray(edges).reshape(-1, 2):
        if abs(int(a) - int(b)) == 1:
            linked.add(min(int(a), int(b)))
    out, start = [], 0
    for l in range(nf - 1):
        if l not in linked:
            out.append(np.arange(start, l + 1))
            start = l + 1
    if nf:
        out.append(np.arange(start, nf))
    return out


def block_precond(K: sp.spmatrix, blocks: List[np.ndarray], tridiagonal: bool = False):
    """Factors of the block preconditioner of K; with tridiagonal=True each block keeps
    only its diagonal and the couplings between consecutive cells."""
    K = sp.csr_matrix(K)
    facs = []
    for idx in blocks:
        B = K[idx][:, idx].tocsr()
        if tridiagonal:
            B = sp.triu(sp.tril(B, 1), -1).tocsr()
        facs.append((idx, ilu0(B)))
    return facs


def block_precond_apply(facs, r: np.ndarray) -> np.ndarray:
    z = np.zeros_like(np.asarray(r, np.float64))
    for idx, rows in facs:
        z[idx] = ilu0_solve(rows, r[idx])
    return z


# ------------------------------------------------------------------------------------
# Multigrid V-cycle (the GPU path's MC_MG option).  Not from the paper: a second
# preconditioner for the same SPD continuum systems, stated here by its textbook definition
# (aggregation two-grid / V-cycle with a symmetric pre- and post-smoothing, e.g. Saad,
# Iterative Methods for Sparse Linear Systems, multigrid chapter; Vanek, Mandel and Brezina
# on aggregation) so that the GPU cycle can be compared with it.
# ------------------------------------------------------------------------------------
def aggregate_prolongator(nx: int, ny: int):
    """Piecewise-constant prolongation over 2 x 2 cell aggregates (1-wide at an odd last
    column or row): column J of P is the indicator of aggregate J, numbered row-major on the
    coarse (ceil(nx/2) x ceil(ny/2)) grid.  Returns (P, cnx, cny)."""
    cnx, cny = (nx + 1) // 2, (ny + 1) // 2
    ys, xs = np.divmod(np.arange(nx * ny), nx)
    J = (ys // 2) * cnx + xs // 2
    P = sp.csr_matrix((np.ones(nx * ny), (np.arange(nx * ny), J)), shape=(nx * ny, cnx * cny))
    return P, cnx, cny


def coarse_operator(K: sp.spmatrix, P: sp.spmatrix) -> sp.csr_matrix:
    """The coarse operator of one aggregation level: the Galerkin product P^T K P with its
    off-diagonal (face) conductances halved and the diagonal lowered by the same amount, so
    that row sums are kept.  With piecewise-constant 2 x 2 aggregates the Galerkin product
    carries twice the conductance a coarse cell of side 2h has (two fine faces of
    conductance T in parallel, against T for the rediscretized face), while its storage and
    transfer terms (the row sums) are exact; halving the faces restores the balance."""
    Kc = sp.csr_matrix(P.T @ K @ P)
    d = Kc.diagonal()
    off = Kc - sp.diags(d)
    rs = np.asarray(off.sum(axis=1)).ravel()          # minus the cell's face conductances
    return sp.csr_matrix(0.5 * off + sp.diags(d + 0.5 * rs))


def vcycle_setup(K: sp.spmatrix, nx: int, ny: int, coarse: int = 256, coarse_rows: int = 4,
                 max_levels=None, last_sweeps: int = 2):
    """Levels of the V-cycle of the grid operator K (nx x ny cells, row-major): coarse
    operators from `coarse_operator` until at most `coarse` cells remain; block IC(0) factors on
    64 x 16 blocks on the finest level and 64 x `coarse_rows` blocks on the coarse levels
    above the coarsest; the coarsest level's dense inverse.  A grid of at most `coarse`
    cells has one level and the cycle is plain block IC(0).  With `max_levels`, the cycle
    is truncated after that many coarse levels: its last level (if above `coarse` cells) has
    no coarser correction and is smoothed `last_sweeps` times (1: z = M^-1 r; 2: then
    z += M^-1 (r - K z)), a truncated V-cycle, symmetric either way."""
    K = sp.csr_matrix(K)
    levels = [dict(K=K, nx=nx, ny=ny, facs=block_precond(K, grid_tile_blocks(nx, ny)))]
    while nx * ny > coarse:
        if max_levels is not None and len(levels) - 1 >= max_levels:
            levels[-1]["sweeps"] = last_sweeps
            break
        P, nx, ny = aggregate_prolongator(nx, ny)
        levels[-1]["P"] = P
        K = coarse_operator(K, P)
        lev = dict(K=K, nx=nx, ny=ny)
        if nx * ny > coarse:
            lev["facs"] = block_precond(K, grid_tile_blocks(nx, ny, ty=coarse_rows))
        else:
            lev["inv"] = np.linalg.inv(K.toarray())
        levels.append(lev)
    return levels


def vcycle_apply(levels, r: np.ndarray, l: int = 0) -> np.ndarray:
    """z = V r: pre-smoothing z_p = M^-1 r, coarse correction with the restricted residual
    P^T (r - K z_p), post-smoothing with the same M (so V is symmetric)."""
    L = levels[l]
    r = np.asarray(r, np.float64)
    if "inv" in L:
        return L["inv"] @ r
    if "sweeps" in L:            # last level of a truncated cycle: one or two sweeps
        zp = block_precond_apply(L["facs"], r)
        if L["sweeps"] == 1:
            return zp
        return zp + block_precond_apply(L["facs"], r - L["K"] @ zp)
    if "P" not in L:
        return block_precond_apply(L["facs"], r)
    K, P = L["K"], L["P"]
    zp = block_precond_apply(L["facs"], r)
    e = vcycle_apply(levels, P.T @ (r - K @ zp), l + 1)
    z1 = zp + P @ e
    return z1 + block_precond_apply(L["facs"], r - K @ z1)
