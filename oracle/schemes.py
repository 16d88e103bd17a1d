"""Time stepping for the multicontinuum system (oracle; test infrastructure only).

Schemes (Section 3.2 and 3.3 of the paper), with A = D + Q, A = A0 + A1:

* ``coupled``  backward Euler on the whole system:  (M/tau + A) p^n = M/tau p^{n-1} + F
  (eq. ct-mc), one system of size sum_a N_a.
* ``D``        block-diagonal A0 (eq. si-mc, D-scheme): every continuum solves
  (M_a/tau + D_a + S_a) p_a^n = M_a/tau p_a^{n-1} + sum_{b != a} Q_ab p_b^{n-1} + F_a
  where S_a is the row-sum diagonal of sum_{b != a} Q_ab.
* ``L``        block lower-triangular A0: continua in ascending-permeability order, each
  using the new values of the continua solved before it.
* ``U``        block upper-triangular A0: highest permeability first, each continuum
  using the new values of the continua of higher index.
* ``EX``       A0 = D, A1 = Q (the whole transfer lagged):
  (M_a/tau + D_a) p_a^n = (M_a/tau - S_a) p_a^{n-1} + sum_b Q_ab p_b^{n-1} + F_a.
  A0 - A1 = D - Q is not nonnegative, so this split is only conditionally stable.

Every system matrix is time invariant, so each is factored once with SuperLU; every
solve is certified by an independent residual check.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fv import Assembled, assemble

SCHEMES = ("coupled", "D", "L", "U", "EX")
CERT_TOL = 1e-13


class CertificationError(RuntimeError):
    pass


class DirectSolver:
    """Sparse LU of an SPD matrix, with a residual certificate on every solve.

    Every system matrix of the schemes is symmetric positive definite (storage over tau
    plus a symmetric nonnegative-definite flux and transfer part, Sections 3.1-3.3), so
    the factorization keeps the symmetric fill-reducing order and takes its pivots from
    the diagonal (no row interchanges).  The certificate is the normwise backward error:
    ||b - K x|| <= CERT_TOL (||b|| + ||K|| ||x||) with ||K|| bounded by the largest
    absolute row sum (K is symmetric)."""

    def __init__(self, K: sp.spmatrix):
        self.K = K.tocsr()
        self.knorm = float(abs(self.K).sum(axis=1).max()) if self.K.shape[0] else 0.0
        t = time.perf_counter()
        self.lu = spla.splu(self.K.tocsc(), permc_spec="MMD_AT_PLUS_A",
                            diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
        self.factor_seconds = time.perf_counter() - t

    def solve(self, b: np.ndarray) -> np.ndarray:
        x = self.lu.solve(b)
        nb = np.linalg.norm(b)
        for _ in range(4):
            r = b - self.K @ x
            nr = np.linalg.norm(r)
            bound = CERT_TOL * (nb + self.knorm * np.linalg.norm(x))
            if nr <= bound:
                return x
            x = x + self.lu.solve(r)      # a step of FP64 iterative refinement
        raise CertificationError(f"backward error {nr / max(bound / CERT_TOL, 1e-300):.3e}")


def continuum_matrix(asm: Assembled, tau: float, a: int, scheme: str = "D") -> sp.csr_matrix:
    """System matrix of continuum a in a decoupled scheme: M_a/tau + D_a + S_a (D, L, U),
    or M_a/tau + D_a (EX)."""
    K = asm.D[a] + sp.diags(asm.M[a] / tau)
    if scheme != "EX":
        K = K + sp.diags(asm.S(a))
    return K.tocsr()


def coupled_matrix(asm: Assembled, tau: float) -> sp.csr_matrix:
    return (sp.diags(asm.Mfull() / tau) + asm.Afull()).tocsr()


def transfer_sum(asm: Assembled, a: int, states: Sequence[np.ndarray],
                 which: Optional[Sequence[int]] = None) -> np.ndarray:
    """sum_{b != a} Q_ab p_b over the continua b listed in ``which`` (default: all)."""
    out = np.zeros(asm.sizes[a])
    for b in range(asm.L):
        if b == a or (a, b) not in asm.Q:
            continue
        if which is not None and b not in which:
            continue
        out += asm.Q[(a, b)] @ states[b]
    return out


def decoupled_rhs(asm: Assembled, tau: float, a: int, p_prev: Sequence[np.ndarray],
                  scheme: str = "D", p_new: Optional[Sequence[np.ndarray]] = None) -> np.ndarray:
    """Right-hand side of continuum a in a decoupled scheme.

    D/EX use only the previous layer; L uses new values for b < a; U uses new values for
    b > a (``p_new`` holds them)."""
    L = asm.L
    if scheme in ("D", "EX"):
        rhs = asm.M[a] / tau * p_prev[a] + transfer_sum(asm, a, p_prev) + asm.F[a]
        if scheme == "EX":
            rhs = rhs - asm.S(a) * p_prev[a]
        return rhs
    if scheme == "L":
        new_set = [b for b in range(L) if b < a]
    elif scheme == "U":
        new_set = [b for b in range(L) if b > a]
    else:
        raise ValueError(scheme)
    old_set = [b for b in range(L) if b != a and b not in new_set]
    rhs = asm.M[a] / tau * p_prev[a] + asm.F[a]
    rhs = rhs + transfer_sum(asm, a, p_prev, old_set)
    if new_set:
        rhs = rhs + transfer_sum(asm, a, p_new, new_set)
    return rhs


class Stepper:
    """Advances the state p = (p_1, ..., p_L) one time layer with a given scheme."""

    def __init__(self, prob_or_asm, tau: Optional[float] = None, scheme: str = "D"):
        if scheme not in SCHEMES:
            raise ValueError(scheme)
        self.asm = prob_or_asm if isinstance(prob_or_asm, Assembled) else assemble(prob_or_asm)
        self.tau = float(prob_or_asm.tau if tau is None else tau)
        self.scheme = scheme
        self.factor_seconds = 0.0
        if scheme == "coupled":
            self.solver = DirectSolver(coupled_matrix(self.asm, self.tau))
            self.factor_seconds = self.solver.factor_seconds
        else:
            self.solvers = [DirectSolver(continuum_matrix(self.asm, self.tau, a, scheme))
                            for a in range(self.asm.L)]
            self.factor_seconds = sum(s.factor_seconds for s in self.solvers)

    def step(self, p_prev: Sequence[np.ndarray]) -> List[np.ndarray]:
        asm, tau = self.asm, self.tau
        if self.scheme == "coupled":
            b = asm.Mfull() / tau * np.concatenate(p_prev) + asm.Ffull()
            x = self.solver.solve(b)
            return list(np.split(x, np.cumsum(asm.sizes)[:-1]))
        L = asm.L
        new: List[Optional[np.ndarray]] = [None] * L
        order = range(L - 1, -1, -1) if self.scheme == "U" else range(L)
        for a in order:
            rhs = decoupled_rhs(asm, tau, a, p_prev, self.scheme, new)
            new[a] = self.solvers[a].solve(rhs)
        return new  # type: ignore[return-value]


def run(prob, scheme: str = "D", nsteps: Optional[int] = None, tau: Optional[float] = None,
        p0: Optional[Sequence[np.ndarray]] = None, keep: str = "all"):
    """Run ``nsteps`` layers; returns the list of states (index 0 = initial) when
    keep='all', else only the final state."""
    st = Stepper(prob, tau, scheme)
    p = [np.array(v, np.float64) for v in (prob.initial_state() if p0 is None else p0)]
    nsteps = prob.nsteps if nsteps is None else nsteps
    hist = [p] if keep == "all" else None
    for _ in range(nsteps):
        p = st.step(p)
        if hist is not None:
            hist.append(p)
    return hist if keep == "all" else p


def rel_l2(p: Sequence[np.ndarray], p_ref: Sequence[np.ndarray]) -> float:
    """Relative L2 error over the concatenation of all continua (absolute if the reference
    is zero); the paper's e_h without the percent factor."""
    a = np.concatenate([np.ravel(v) for v in p])
    b = np.concatenate([np.ravel(v) for v in p_ref])
    nb = np.linalg.norm(b)
    d = np.linalg.norm(a - b)
    return d / nb if nb > 1e-300 else d


def energy(asm: Assembled, p: Sequence[np.ndarray]) -> float:
    """||p||_A^2 = (A p, p)."""
    x = np.concatenate(p)
    return float(x @ (asm.Afull() @ x))
