"""Problem descriptor: the discrete data a multicontinuum finite-volume problem is built from.

The fields follow the paper's problem statement (Section 2, the general L-continuum model
with its boundary and initial conditions) and the quantities its finite-volume
discretization names (Section 3.1): an h x h cell grid on Omega, per-continuum storage c
and permeability k, a 1-D fracture mesh embedded in the grid with cell lengths, the
fracture-fracture connections, the matrix-fracture transfer coefficients sigma_il,
the time step tau and the initial pressures.

Index conventions
-----------------
* Omega cells are row-major: cell (x, y) with column x in [0, nx) (west -> east) and row
  y in [0, ny) (south -> north) has index y * nx + x.  A 3-D problem (nz > 1) stacks nz such
  planes bottom to top: cell (x, y, z) has index (z * ny + y) * nx + x.  Cells are squares
  (cubes in 3-D) of side h; a fracture cell's `flen` is its measure per unit aperture (its
  length for the 1-D fractures of a 2-D problem, its area for fracture planes in 3-D).
* Continua are ordered Omega continua first (ascending permeability: matrix, then the
  natural-fracture continuum in three-continuum media), then the explicit fracture.
* Boundary sides are ordered W, E, S, N, and in 3-D the bottom and top sides follow
  (bc_type_z / bc_value_z).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

BC_NOFLOW = 0
BC_DIRICHLET = 1


@dataclass
class OmegaContinuum:
    """One continuum living on the 2-D grid: storage c and permeability k."""
    c: float
    k_const: float = 0.0
    k: Optional[np.ndarray] = None          # (ny, nx) float64 cell permeability, or None = k_const

    def k_field(self, nx: int, ny: int, nz: int = 1) -> np.ndarray:
        shape = (ny, nx) if nz == 1 else (nz, ny, nx)
        if self.k is not None:
            return np.asarray(self.k, dtype=np.float64).reshape(shape)
        return np.full(shape, float(self.k_const))


@dataclass
class Problem:
    nx: int
    ny: int
    h: float                                 # cell side (square cells)
    omega: List[OmegaContinuum]              # 1 (two-continuum) or 2 (three-continuum)
    sigma_omega: float = 0.0                 # Omega-Omega transfer coefficient per unit area
    # explicit fracture continuum (may be empty)
    host: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))   # [nf] host cell
    flen: np.ndarray = field(default_factory=lambda: np.zeros(0))             # [nf] cell length
    edges: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))  # [ne, 2]
    edge_d: np.ndarray = field(default_factory=lambda: np.zeros(0))           # [ne] centre distance
    k_f: float = 1.0
    c_f: float = 1.0
    aperture: float = 1.0
    sigma_f: np.ndarray = field(default_factory=lambda: np.zeros((1, 0)))     # [n_omega, nf]
    bc_type: np.ndarray = field(default_factory=lambda: np.zeros(4, np.int32))
    bc_value: np.ndarray = field(default_factory=lambda: np.zeros(4))
    src: Optional[List[Optional[np.ndarray]]] = None    # per continuum, per unit measure
    p0: Optional[List[Optional[np.ndarray]]] = None     # per continuum initial pressure
    # wells on fracture cells (Section 5): a source q_w (p_w - p_f) per unit measure, taken
    # implicitly; q_w = 0 where there is no well
    well_q: Optional[np.ndarray] = None                 # [nf] q_w >= 0, or None
    well_p: Optional[np.ndarray] = None                 # [nf] p_w, or None (= 0)
    tau: float = 1e-3
    nsteps: int = 1
    meta: dict = field(default_factory=dict)
    # 3-D: planes stacked in z (1 = the 2-D model), bottom and top boundary sides
    nz: int = 1
    bc_type_z: np.ndarray = field(default_factory=lambda: np.zeros(2, np.int32))
    bc_value_z: np.ndarray = field(default_factory=lambda: np.zeros(2))

    # ---- sizes -----------------------------------------------------------------------
    @property
    def n_omega(self) -> int:
        return len(self.omega)

    @property
    def nf(self) -> int:
        return int(len(self.host))

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dim(self) -> int:
        return 3 if self.nz > 1 else 2

    @property
    def n_cont(self) -> int:
        """Number of continua: Omega continua plus the fracture continuum when nf > 0."""
        return self.n_omega + (1 if self.nf > 0 else 0)

    def sizes(self) -> List[int]:
        s = [self.ncell] * self.n_omega
        if self.nf > 0:
            s.append(self.nf)
        return s

    def dof(self) -> int:
        return int(sum(self.sizes()))

    def initial_state(self) -> List[np.ndarray]:
        out = []
        for a, n in enumerate(self.sizes()):
            v = None if self.p0 is None else self.p0[a]
            out.append(np.zeros(n) if v is None else np.asarray(v, np.float64).reshape(n).copy())
        return out

    def source(self, a: int) -> Optional[np.ndarray]:
        if self.src is None:
            return None
        v = self.src[a]
        return None if v is None else np.asarray(v, np.float64).reshape(-1)

    def check(self) -> None:
        """Shape and range checks on the raw input arrays (no physics)."""
        assert self.nx >= 1 and self.ny >= 1 and self.nz >= 1 and self.h > 0 and self.tau > 0
        assert len(self.bc_type_z) == 2 and len(self.bc_value_z) == 2
        assert self.n_omega in (1, 2)
        nf = self.nf
        assert self.flen.shape == (nf,)
        assert self.sigma_f.shape == (self.n_omega, nf)
        assert self.edges.ndim == 2 and self.edges.shape[1] == 2
        assert self.edge_d.shape == (len(self.edges),)
        if nf:
            assert self.host.min() >= 0 and self.host.max() < self.ncell
        if len(self.edges):
            assert self.edges.min() >= 0 and self.edges.max() < nf
            assert np.all(self.edges[:, 0] != self.edges[:, 1])
            assert np.all(self.edge_d > 0)
        if self.well_q is not None:
            q = np.asarray(self.well_q, np.float64)
            assert q.shape == (nf,) and np.all(np.isfinite(q)) and np.all(q >= 0)
        if self.well_p is not None:
            w = np.asarray(self.well_p, np.float64)
            assert w.shape == (nf,) and np.all(np.isfinite(w))
        for o in self.omega:
            assert o.c > 0
            k = o.k_field(self.nx, self.ny, self.nz)
            assert np.all(np.isfinite(k)) and np.all(k >= 0)
