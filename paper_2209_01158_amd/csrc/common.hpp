// Device-visible descriptors shared by the kernels and the host runtime.
//
// A "system" is one SPD linear system solved by PCG (one continuum in the decoupled
// schemes, or all continua together in the coupled scheme).  A system is made of "parts":
// one part per continuum block, either a structured grid (Omega continuum, 5-point operator)
// or a graph (fracture cells, CSR operator).  Every launch walks a table of tiles; each
// workgroup takes one tile of one part.  Scalars of a system (alpha, beta, dot products,
// convergence flags) live in device memory and are finalized by the last workgroup of that
// system to finish a launch, so no host round trip is needed between iterations.
#pragma once
#include <stdint.h>

#define MC_BLOCK 256           // threads per workgroup (4 waves of 64)
#define MC_TX 64               // grid tile width: one wavefront across 64 consecutive cells
#define MC_GRAPH_ROWS 256      // fracture rows per workgroup
#define MC_SLOT 4              // doubles per partial-sum slot

enum { PART_GRID = 0, PART_GRAPH = 1 };
enum { PREC_JACOBI = 0, PREC_BIC0 = 1 };
enum { ST_RUN = 0, ST_CONV = 1, ST_NOCONV = 2, ST_BREAK = 3 };

// kernel ids for arrival counters (one counter per kernel family, so consecutive launches of
// different kernels never share a counter)
enum { KC_INIT = 0, KC_A = 1, KC_B = 2, KC_RES = 3, KC_N = 4 };

struct SysState {
  double rz, pq, rr, bb, alpha, beta, tol2, rr0;   // PCG scalars (FP64 always); tol2 = tol^2
  double orr, obb, otol2;                          // outer refinement scalars (MC_MIXED)
  int iter, done, status, first, max_iter, total_iter;
  int outer, outer_done, outer_status, max_outer;
  unsigned int cnt[KC_N];                          // arrival counters per kernel family
  int nslots;                                      // tiles of this system per launch
  int pad;
  double* partials;                                // [nslots * MC_SLOT]
  int* active;                                     // shared counter of unfinished systems
  int* oactive;                                    // shared counter of unfinished outer loops
};

// One continuum block of a system.  Pointers are device memory.  Coefficient arrays exist in
// FP64 and (for MC_MIXED inner solves) FP32; vectors are typed by the launch precision.
struct PartD {
  int kind;          // PART_GRID / PART_GRAPH
  int sys;           // owning system
  int cont;          // continuum index inside the problem
  int n;             // unknowns
  int nx, ny;        // grid shape
  int tiles_x;       // grid tiles per row of tiles
  int trows;         // grid tile height in rows
  int slot0;         // first partial slot of this part inside its system
  int coupled;       // operator includes the off-diagonal transfer blocks (coupled scheme)
  int ex;            // EX split: diagonal excludes S, RHS subtracts S p^{n-1}
  int has_t;         // grid: per-face conductance arrays (0 = constant tconst)
  int n_omega;
  int other;         // (grid, 3C) part index of the other Omega continuum in this table or -1
  int frac;          // (grid) part index of the fracture part in this table or -1
  int omg[2];        // (graph) part indices of the Omega parts in this table or -1
  double tconst, tconst32pad;
  double mtau;       // grid storage over tau: c h^2 / tau
  double s12;        // Omega-Omega discrete transfer sigma_omega h^2
  // FP64 coefficients
  const double* diag;      // [n] full system diagonal (storage/tau + conductances + S unless ex)
  const double* tx;        // [n] conductance to the east neighbour (0 on the last column)
  const double* ty;        // [n] conductance to the north neighbour (0 on the last row)
  const double* F;         // [n] sources and Dirichlet terms (may be null)
  const int* rowptr;       // graph CSR of off-diagonal conductances (positive values)
  const int* col;
  const double* val;
  const double* mt;        // (graph) [n] storage / tau per fracture cell
  // FP32 copies
  const float* diag32;
  const float* tx32;
  const float* ty32;
  const float* val32;
  // IC(0) block factors (inverse pivots)
  const double* fdinv;
  const float* fdinv32;
  const int* chain_ptr;    // (graph) chain boundaries [nchains+1]
  int nchains;
  int pad2;
  // transfer structure
  const int* hptr;         // (grid) [n+1] fracture cells hosted per cell (CSR)
  const int* hidx;         // (grid) [nf]   their fracture indices
  const double* hsig;      // (grid) sigma_{a f, l} indexed by fracture cell l (row a of sigma_f)
  const int* host;         // (graph) [n] host cell per fracture cell
  const double* fsig0;     // (graph) sigma_{0 f, l}
  const double* fsig1;     // (graph) sigma_{1 f, l} (3C) or null
  // state used for transfer terms in the right-hand side: tsrc[c] = array of continuum c
  const double* tsrc[3];
  const double* pold;      // own previous layer
  // PCG vectors (typed by the launch precision)
  void* x;
  void* r;
  void* p;           // search direction, double-buffered: iteration k reads p[k&1 ? p2 : p]
  void* p2;          // and writes the other buffer (neighbouring tiles still read the old one)
  void* q;
  void* z;
  double* b;               // FP64 right-hand side
  double* r64;             // FP64 residual scratch (refinement)
  double* x64;             // FP64 iterate (refinement)
};

struct Tile {
  int part;
  int tile;
};
