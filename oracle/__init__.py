"""CPU FP64 oracle for the decoupled multicontinuum scheme -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The GPU library never calls it and shares no code with it; both read the same
seeded input arrays (``media``) and nothing else.

Contents
--------
fv        explicit sparse assembly of M, D, Q, F (Section 3.1: the two-point-flux
          semi-discrete forms for the two- and three-continuum and general models,
          and the block matrix form M dp/dt + A p = F with A = D + Q), with the implicit
          fracture wells of Section 5
schemes   time stepping: coupled backward Euler (Section 3.2) and the decoupled
          D-, L-, U-schemes (Section 3.3), plus the fully-lagged "EX" split, each system
          solved by sparse LU (SuperLU) with a certified residual
fastdiag  exact solver for constant-coefficient grid systems by sine/cosine transforms,
          and a CG solver preconditioned by it for the largest grids
dense     a loop-by-loop dense assembler for tiny problems (brute-force cross-check)

Every function is pinned by ``tests/test_oracle_pins.py`` against closed forms,
invariants stated in the paper (Theorems 2 and 3, symmetry of A, Q_ab = Q_ba^T),
textbook special cases and brute force.  The paper's own table values are not pinned:
its fracture geometry exists only in a figure and sigma and the aperture are not given,
so its 2C / 3C errors can be compared for size and order only.
"""
