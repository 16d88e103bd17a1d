"""Fast diagonalization of constant-coefficient grid systems (oracle; test infrastructure).

For a constant permeability k, unit-ratio square cells and a uniform shift s, the Omega
system s I + D on an ny x nx grid separates into 1-D three-point operators:

* a direction with no-flow at both ends has the Neumann matrix (diagonal 1 at the ends),
  diagonalized by the type-II cosine transform with eigenvalues 4 sin^2(pi j / 2n),
  j = 0..n-1;
* a direction with Dirichlet half-cell faces at both ends (the end diagonal gains
  T_b / k = 2) is diagonalized by the type-II sine transform with eigenvalues
  4 sin^2(pi j / 2n), j = 1..n.

``fd_solve`` is exact for such systems.  ``fd_pcg`` solves a grid system whose matrix
is that constant part plus a nonnegative diagonal perturbation (transfer to fracture
host cells) by conjugate gradients preconditioned with ``fd_solve``; it is used where a
sparse LU of the grid system is too large.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def _axis_eigs(n: int, dirichlet: bool) -> np.ndarray:
    j = np.arange(1, n + 1) if dirichlet else np.arange(n)
    return 4.0 * np.sin(np.pi * j / (2.0 * n)) ** 2


def _fwd(v, axis, dirichlet):
    return (sfft.dst if dirichlet else sfft.dct)(v, type=2, norm="ortho", axis=axis,
                                                  workers=-1)


def _inv(v, axis, dirichlet):
    return (sfft.idst if dirichlet else sfft.idct)(v, type=2, norm="ortho", axis=axis,
                                                    workers=-1)


def fd_solve(b: np.ndarray, nx: int, ny: int, k: float, shift: float, bc_type) -> np.ndarray:
    """Solve (shift I + D) x = b for constant k; bc_type = (W, E, S, N), 1 = Dirichlet.
    Both ends of a direction must share the same kind."""
    dx = int(bc_type[0]) == 1
    dy = int(bc_type[2]) == 1
    if dx != (int(bc_type[1]) == 1) or dy != (int(bc_type[3]) == 1):
        raise ValueError("fast diagonalization needs matching side types per direction")
    lam = shift + k * (_axis_eigs(nx, dx)[None, :] + _axis_eigs(ny, dy)[:, None])
    B = b.reshape(ny, nx)
    c = _fwd(_fwd(B, 1, dx), 0, dy)
    c = c / lam
    x = _inv(_inv(c, 0, dy), 1, dx)
    return x.reshape(-1)


def fd_pcg(K, b: np.ndarray, nx: int, ny: int, k: float, shift: float, bc_type,
           x0=None, rtol: float = 1e-14, maxit: int = 500):
    """CG on K x = b preconditioned by the exact constant-coefficient solve.
    Returns (x, iterations, final relative residual); raises if not converged."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    r = b - K @ x
    nb = np.linalg.norm(b)
    if nb == 0:
        return x, 0, 0.0
    z = fd_solve(r, nx, ny, k, shift, bc_type)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = K @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= rtol * nb:
            rt = np.linalg.norm(b - K @ x) / nb        # certify with the true residual
            if rt <= 10 * rtol:
                return x, it, rt
            r = b - K @ x
        z = fd_solve(r, nx, ny, k, shift, bc_type)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise RuntimeError("fd_pcg did not converge")


class FDStepper:
    """D-scheme layers (Section 3.3, eq. si-mc with block-diagonal A0) for problems whose
    Omega continua have constant permeability on a 2-D grid with matching side types per
    direction, at sizes where a sparse LU of the grid systems is out of reach.

    Each continuum's system matrix and right-hand side are the ones the sparse-direct
    stepper uses (``schemes.continuum_matrix``, ``schemes.decoupled_rhs``).  A grid continuum
    is solved by ``fd_pcg``, preconditioned by the exact solve of its constant part
    (storage c h^2 / tau, the Omega-Omega transfer sigma_omega h^2 and the diffusion) and
    started from the previous layer; the fracture continuum by the certified sparse LU.
    Only the transfer to the fracture host cells is left to the CG iterations."""

    def __init__(self, prob, rtol: float = 1e-14):
        from . import fv, schemes
        if getattr(prob, "nz", 1) > 1 or any(o.k is not None for o in prob.omega):
            raise ValueError("FDStepper needs constant-permeability 2-D grid continua")
        self.prob, self.rtol = prob, rtol
        self.asm = fv.assemble(prob)
        self.tau = float(prob.tau)
        self.K = [schemes.continuum_matrix(self.asm, self.tau, a, "D")
                  for a in range(self.asm.L)]
        vol = prob.h ** 2
        self.shift = [o.c * vol / self.tau + (prob.sigma_omega * vol if prob.n_omega == 2
                                              else 0.0) for o in prob.omega]
        self.frac = (schemes.DirectSolver(self.K[-1]) if prob.nf > 0 else None)
        self.iterations: list = []

    def step(self, p_prev):
        from . import schemes
        prob, asm = self.prob, self.asm
        new, its = [], []
        for a in range(asm.L):
            rhs = schemes.decoupled_rhs(asm, self.tau, a, p_prev, "D")
            if a < prob.n_omega:
                x, it, _ = fd_pcg(self.K[a], rhs, prob.nx, prob.ny, prob.omega[a].k_const,
                                  self.shift[a], prob.bc_type, x0=p_prev[a], rtol=self.rtol)
                its.append(it)
            else:
                x = self.frac.solve(rhs)
            new.append(x)
        self.iterations.append(its)
        return new
