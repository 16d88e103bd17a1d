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
#define MC_SLOT 8              // doubles per partial-sum slot
#define MC_TY 32               // grid tile height (rows) of the LDS-staged operator
#define MC_ICY 16              // rows of a grid block of the block IC(0) preconditioner
#define MC_ICB (MC_TY / MC_ICY)  // IC(0) blocks per grid tile
#define MC_ICYC 4              // rows of an IC(0) block on the coarse levels of a V-cycle
#define MC_SCHUR_ROWS 4        // rows of the crossing-cell inverse per workgroup (one per wave)
#define MC_SCHUR_KMAX 6144     // most crossing cells solved exactly (FP64 right-hand side in LDS)
#define MC_MG_COARSE 256       // multigrid levels stop at this many cells (dense inverse there)
#define MC_MG_TAIL 1024        // levels of at most this many cells run in one workgroup
#define MC_MG_DOMINANCE 8.0    // a V-cycle stops at a level whose row sums reach this many
                               // times its face conductances (summed over the level)
#define MC_TAIL_THREADS 1024   // threads of that workgroup

enum { PART_GRID = 0, PART_GRAPH = 1 };
enum { PREC_JACOBI = 0, PREC_BIC0 = 1 };
enum { ST_RUN = 0, ST_CONV = 1, ST_NOCONV = 2, ST_BREAK = 3 };
// warm start of a layer's PCG: 2 p^{n-1} - p^{n-2}; p^{n-1}; the order (0-3) of the polynomial
// extrapolation of the layer history that best predicted the previous layer
enum { WS_LINEAR = 0, WS_PREVIOUS = 1, WS_ADAPTIVE = 2 };

// Per-system state.  Reductions never cross workgroups inside a kernel: every kernel writes
// one partial-sum slot per workgroup, and the next kernel in stream order has each of its
// workgroups sum all slots of its system in slot order (the same order in every workgroup,
// so every workgroup obtains the bitwise-identical scalar).  Workgroup 0 of a kernel records
// the scalars later kernels and the host need; a kernel never reads a field that a
// workgroup of the same kernel writes.
struct SysState {
  double rzh[2];        // (r,z) of iterations with even / odd index
  double bb;            // ||b||^2 (inner solves: ||r_start||^2)
  double rr;            // last ||r||^2
  double rr0;           // ||r||^2 at the start of the (inner) solve
  double obb, orr;      // refinement: ||b||^2 and the last FP64 ||r||^2
  double tol2, otol2;   // squared relative tolerances (inner / outer)
  int iter;             // iterations done by the last (inner) solve
  int done;             // the (inner) solve has ended
  int status;           // ST_* of the (inner) solve
  int total_iter;       // inner iterations summed over refinement passes
  int outer, outer_done, outer_status;
  int max_iter, max_outer;
  // PCG iteration index, kept on the device so that launches carry no per-iteration
  // argument: the operator kernel reads ka and records it in kb; the update kernel reads kb
  // and sets ka = kb + 1 for the next operator kernel
  int ka, kb;
  int mixed;            // inner solve of FP64 refinement: iteration 0 first tests the outer residual
  int hist;             // layers computed in a row before the current one (warm start)
  double rscale;        // refinement: power-of-two scale of the FP32 residual of the inner solve
  int nslotsA;          // workgroups (partial slots) of this system in an operator launch
  int nslotsB;          // ... in an update / init / residual launch (its own tiling)
  int wsorder;          // extrapolation order of the current layer's warm start
  int pad1;
  double* partA;        // [nslotsA * MC_SLOT] written by operator kernels
  double* partB;        // [nslotsB * MC_SLOT] written by update / init / residual kernels
};

// One continuum block of a system.  Pointers are device memory.  Coefficient arrays exist in
// FP64 and (for MC_MIXED inner solves) FP32; vectors are typed by the launch precision.
struct PartD {
  int kind;          // PART_GRID / PART_GRAPH
  int sys;           // owning system
  int cont;          // continuum index inside the problem
  int n;             // unknowns
  int nx, ny;        // grid shape (3-D: ny counts the rows of all planes, stacked in z)
  int tiles_x;       // grid tiles per row of tiles
  int slot0A, slot0B; // first partial slot of this part inside its system (per tiling)
  int coupled;       // operator includes the off-diagonal transfer blocks (coupled scheme)
  int ex;            // EX split: diagonal excludes S, RHS subtracts S p^{n-1}
  int extrap;        // warm start (WS_*): the PCG initial guess of a layer (k_rhs)
  int has_t;         // grid: per-face conductance arrays (0 = constant tconst)
  int fp32;          // the PCG vectors are FP32 (inner solve of FP64 refinement)
  int n_omega;
  int other;         // (grid, 3C) part index of the other Omega continuum in this table or -1
  int frac;          // (grid) part index of the fracture part in this table or -1
  int omg[2];        // (graph) part indices of the Omega parts in this table or -1
  double tconst, tconst32pad;
  long plane;        // (3-D grid) cells per plane, the index step in z; 0 for a 2-D grid
  double mtau;       // grid storage over tau: c h^2 / tau
  double s12;        // Omega-Omega discrete transfer sigma_omega h^2
  // FP64 coefficients
  const double* diag;      // [n] full system diagonal (storage/tau + conductances + S unless ex)
  const double* tx;        // [n] conductance to the east neighbour (0 on the last column)
  const double* ty;        // [n] conductance to the north neighbour (0 on the last row)
  const double* tz;        // (3-D) [n] conductance to the cell above (0 on the top plane)
  const double* F;         // [n] sources and Dirichlet terms (may be null)
  const int* rowptr;       // graph CSR of off-diagonal conductances (positive values)
  const int* col;
  const double* val;
  const double* mt;        // (graph) [n] storage / tau per fracture cell
  // FP32 copies
  const float* diag32;
  const float* tx32;
  const float* ty32;
  const float* tz32;
  const float* val32;
  // IC(0) block factors (inverse pivots)
  const double* fdinv;
  const float* fdinv32;
  const int* chain_ptr;    // (graph) chain boundaries [nchains+1]
  const int* gtile;        // (graph) work tiles as chain ranges [ntiles+1]
  const double* cT;        // (graph) coupling of cell l to l-1 inside its block (0 at block starts)
  const float* cT32;
  int nchains;
  // (graph) exact solve through the crossing cells: blocks are the runs of chains between
  // crossing cells, the crossing cells are solved by the inverse of their Schur complement
  int K;                   // crossing cells (0: none, or too many: crossings left out)
  int slotS;               // first partial slot of the Schur product (after the update slots)
  int blocks;              // 1: two-level block preconditioner instead (K = blocks, below)
  const int* xcells;       // [K] crossing cells, ascending
  const int* xtile;        // [ntiles + 1] crossing cells of each work tile
  const int* xlr;          // [2n] crossing neighbours (left, right) of each cell's block or -1
  const double* cl;        // [n] responses of the block to its left / right crossing neighbour
  const double* cr;
  const float* cl32;
  const float* cr32;
  const double* cxl;       // [K] conductance of crossing cell k to its chain neighbours
  const double* cxr;
  const double* sinv;      // [K*K] inverse of the Schur complement (symmetric)
  const float* sinv32;
  // two-level block preconditioner: connected blocks of at most 64 cells solved by their
  // dense inverses, the coarse system over the blocks by sinv (the inverse of P^T A P); xtile
  // then holds the first block of each work tile, xlr / cl the block of each cell and 1
  const int* bnode;        // [K*64] cells of each block, -1 padding
  const float* binv;       // [K*64*64] block inverses, entry (i, j) at j*64 + i
  void* gX;                // [K] crossing right-hand side g = r_X - A_XI y (launch precision)
  void* zX;                // [K] crossing solution S^-1 g (launch precision)
  // (grid) multigrid V-cycle: this part is level mg_level of a continuum; coarser and finer
  // levels are other parts of the same table
  int mg_level;            // 0: the continuum itself
  int mg_next;             // part of the next coarser level, -1 at the coarsest (or no V-cycle)
  int mg_prev;             // part of the next finer level (levels >= 1)
  int mg_slot;             // (level 0) first partial slot of the final smoothing
  const double* mg_inv;    // (coarsest) dense inverse of the level operator [n*n]
  const float* mg_inv32;
  void* mg_r;              // right-hand side of the level (level 0: the PCG residual r)
  void* mg_zp;             // level solution after pre-smoothing
  void* mg_z;              // level solution after the coarse correction and post-smoothing
  // copies of the neighbouring levels' fields the V-cycle kernels read, filled when the
  // launch table is built, so that a kernel needs this one descriptor: the coarser level's
  // solution and width (post-smoothing), the finer level's vectors, FP32 operator and shape
  // (restriction)
  const void* mg_e;        // coarser level's z
  int mg_cnx;              // coarser level's nx
  int mg_fnx, mg_fny, mg_ftiles_x, mg_fhas_t;
  int mg_fuse;             // (level 0) the update kernel forms this level's share of the
                           // restriction into level 1 (level 1 is not in the small-level tail)
  int mg_once;             // (last level above the tail) smoothed once: the finer level takes
                           // its pre-smoothed z_p as the correction, no post-smoothing here
  int mg_pad0;
  double mg_ftc;           // finer level's constant conductance (no conductance field)
  const void* mg_fr;       // finer level's right-hand side (level 0: the PCG residual)
  const void* mg_fzp;      // finer level's z_p
  const float* mg_fd32;    // finer level's FP32 diagonal and face conductances
  const float* mg_ftx32;
  const float* mg_fty32;
  // block edges of a fused restriction (level 0 writes them, level 1 reads the copies): per
  // IC(0) block column k (64 grid columns) and grid row y, z_p of the block's first and last
  // column at [(k * ny + y) * 2 + 0 / 1] (launch precision) and the east face conductance of
  // its last column at [k * ny + y] (FP32)
  void* mg_edz;
  float* mg_edt;
  const void* mg_fedz;
  const float* mg_fedt;
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
  double* hx[3];           // (WS_ADAPTIVE) states p^{n-3}, p^{n-4}, p^{n-5} of the layer history
  double* b;               // FP64 right-hand side
  double* r64;             // FP64 residual scratch (refinement)
  double* x64;             // FP64 iterate (refinement)
};

// One workgroup's work: tiles [t0, t1) of a part, reporting into partial slot `slot`.  The
// owning system is copied here so that a kernel's end test loads the system's done flag
// straight from the tile, without waiting for the part's descriptor.
struct Tile {
  int part;   // -1: padding workgroup (does nothing)
  int slot;
  int t0, t1;
  int sys;    // parts[part].sys
};
