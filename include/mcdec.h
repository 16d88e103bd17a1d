/*
 * mcdec.h -- C ABI of the MI355X (gfx950) decoupled multicontinuum flow library.
 *
 * What it computes (Vasilyeva, "Efficient decoupling schemes for multiscale multicontinuum
 * problems in fractured porous media"):
 *   the L-continuum model  c_a dp_a/dt - div(k_a grad p_a) + sum_b sigma_ab (p_a - p_b) = f_a
 *   (Section 2, eq. mm) discretized by two-point-flux finite volumes on an h x h grid with an
 *   embedded 1-D fracture mesh (Section 3.1, eqs. app-md, app-tc, app, app-mc):
 *       M dp/dt + (D + Q) p = F,
 *   and advanced in time by
 *     - the coupled backward-Euler scheme  (M/tau + A) p^n = M/tau p^{n-1} + F  (Section 3.2,
 *       eq. ct-mc), or
 *     - the decoupled D-scheme (Section 3.3, eq. si-mc with block-diagonal A0): each
 *       continuum solves its own SPD system
 *         (M_a/tau + D_a + S_a) p_a^n = M_a/tau p_a^{n-1} + sum_{b!=a} Q_ab p_b^{n-1} + F_a,
 *       S_a = row-sum diagonal of sum_{b!=a} Q_ab; or the L-/U-schemes (block lower/upper
 *       triangular A0, Section 3.3); or the fully lagged split "EX" (A0 = D, A1 = Q, only
 *       conditionally stable).
 *   Every linear system is solved on the GPU by preconditioned conjugate gradients.
 *
 * Conventions
 *   - All functions return mc_status; no C++ exception crosses this boundary.
 *   - Omega cells are row-major: cell (x, y), x in [0,nx) west->east, y in [0,ny)
 *     south->north, has index y*nx + x.  Sides are ordered W, E, S, N.
 *   - Continuum index a: 0 = matrix (lowest permeability), 1 = natural-fracture continuum
 *     (three-continuum media only), then the explicit fracture continuum (if nf > 0).
 *     This is the ascending-permeability order the L-/U-schemes use.
 *   - Descriptor arrays are HOST memory owned by the caller, read only during
 *     mc_create_problem / mc_server_submit; the library copies what it needs to the device.
 *   - Pointers named *_dev are DEVICE memory owned by the caller, accessed in stream order on
 *     the problem's stream.
 *   - One handle is used by one host thread at a time.  All device work of a handle is
 *     ordered on its stream (mc_options.stream, or a stream the library creates).
 *   - After MC_EDEVICE a handle may only be destroyed.
 */
#ifndef MCDEC_H
#define MCDEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MC_OK = 0,
  MC_EINVAL = -1,      /* invalid argument or descriptor (message in mc_last_error)        */
  MC_ENOMEM = -2,      /* device allocation failed / request can never fit the budget        */
  MC_ENOCONV = -3,     /* PCG reached max_iter (or refinement max_outer) before tolerance     */
  MC_EBREAKDOWN = -4,  /* PCG breakdown: p.Ap <= 0 or a non-finite value                      */
  MC_EDEVICE = -5,     /* HIP runtime error                                                   */
  MC_ENOTFOUND = -6,   /* unknown request id (server)                                         */
  MC_ETIMEOUT = -7     /* server wait ended before the requests did                           */
} mc_status;

typedef enum {
  MC_SCHEME_D = 0,        /* decoupled, block-diagonal A0 (Section 3.3)                       */
  MC_SCHEME_COUPLED = 1,  /* coupled backward Euler (Section 3.2)                             */
  MC_SCHEME_L = 2,        /* block lower-triangular A0 (ascending permeability first)          */
  MC_SCHEME_U = 3,        /* block upper-triangular A0 (highest permeability first)            */
  MC_SCHEME_EX = 4        /* A0 = D, A1 = Q: whole transfer lagged; stable only if
                             tau * max(S_a / m_a) < 1 per cell (not unconditionally stable)     */
} mc_scheme;

typedef enum {
  MC_FP64 = 0,   /* FP64 storage and arithmetic throughout                                     */
  MC_MIXED = 1   /* FP32 operator copies and inner PCG (FP64 dot products) inside FP64
                    iterative refinement; residual, right-hand side and transfer stay FP64     */
} mc_precision;

typedef enum {
  MC_JACOBI = 0, /* z = r / diag                                                               */
  MC_BIC0 = 1,   /* grid: block incomplete Cholesky, zero fill, on 64-column x 16-row blocks
                    (IC(0) in natural order inside a block, couplings between blocks dropped);
                    fracture graph: an exact solve -- its chains cut at the crossing cells
                    (cells joined to cells other than their chain neighbours) are tridiagonal
                    blocks solved exactly, and the crossing cells are solved through the
                    inverse of their Schur complement (formed once at setup, up to 6144
                    crossing cells; beyond that the crossing couplings are dropped)            */
  MC_MG = 2      /* grid: one symmetric multigrid V-cycle -- 2 x 2 cell aggregates, coarse
                    operators P^T A P with their face conductances halved (again 5-point
                    conductance stencils; row sums kept), block IC(0) as the
                    pre- and post-smoother on every level, the coarsest level (at most 256
                    cells) solved by its dense inverse; fracture graph: as MC_BIC0.  Grids of
                    at most 256 cells use plain block IC(0).  2-D grids only (nz <= 1)    */
} mc_precond;

/* One continuum on the Omega grid. */
typedef struct {
  double c;              /* storage coefficient c_a > 0                                       */
  double k_const;        /* permeability when k == NULL (>= 0)                                */
  const double *k;       /* [ny*nx] cell permeability (>= 0, finite) or NULL                  */
  const double *src;     /* [ny*nx] source f_a per unit area (volume in 3-D), or NULL (= 0)    */
  const double *p0;      /* [ny*nx] initial pressure, or NULL (= 0)                           */
} mc_omega_desc;

/* A problem: grid, continua, fracture mesh, boundary data, time step. */
typedef struct {
  int32_t nx, ny;        /* grid cells (>= 1)                                                 */
  double h;              /* cell side (> 0); cell area h^2, interior |E|/d = 1                */
  int32_t n_omega;       /* 1 (matrix only) or 2 (matrix + natural fractures)                  */
  mc_omega_desc omega[2];
  double sigma_omega;    /* Omega-Omega transfer coefficient per unit area (>= 0); the discrete
                            coefficient of each cell pair is sigma_omega * h^2                  */
  int32_t nf;            /* fracture cells (0 = no explicit fracture continuum)                */
  const int32_t *host;   /* [nf] row-major index of the Omega cell containing fracture cell l  */
  const double *flen;    /* [nf] fracture cell length (> 0); measure = aperture * flen         */
  int32_t ne;            /* fracture-fracture connections                                      */
  const int32_t *edges;  /* [2*ne] endpoint pairs (distinct, in [0,nf))                        */
  const double *edge_d;  /* [ne] centre distance (> 0); conductance k_f * aperture / d         */
  double k_f, c_f, aperture;   /* fracture permeability (>= 0), storage (> 0), aperture (> 0)  */
  const double *sigma_f; /* [n_omega*nf] (continuum-major) discrete matrix-fracture transfer
                            coefficient sigma_il of fracture cell l with its host in continuum a */
  const double *src_f;   /* [nf] fracture source per unit measure, or NULL                     */
  const double *p0_f;    /* [nf] initial fracture pressure, or NULL                            */
  int32_t bc_type[4];    /* W,E,S,N for every Omega continuum: 0 no-flow, 1 Dirichlet given by a
                            half-cell conductance 2 k_i; fracture tips are always no-flow      */
  double bc_value[4];    /* Dirichlet pressures                                                */
  double tau;            /* time step (> 0)                                                    */
  const double *well_q;  /* [nf] well coefficient q_w >= 0 per unit measure, or NULL (no wells).
                            Each fracture cell l gets the source q_w,l (p_w,l - p_f,l) per unit
                            measure (the wells of Section 5, with the sign that injects when
                            p_f < p_w), treated implicitly in every scheme                      */
  const double *well_p;  /* [nf] well pressure p_w, or NULL (= 0); read only with well_q         */
  int32_t nz;            /* 3-D grid (the extension the paper names as future work): nz > 1
                            planes of nx*ny cubes of side h stacked bottom to top, cell (x,y,z)
                            at (z*ny + y)*nx + x; every per-cell array then holds nz*ny*nx
                            values and host indexes them.  Faces have |E|/d = h (conductance
                            k h, Dirichlet side 2 k h), cells |cell| = h^3 (storage, sources,
                            sigma_omega h^3).  Fracture cells are then cells of fracture planes:
                            flen is their area, edge_d the centre distance over the interface
                            length.  0 or 1: the 2-D model.  MC_MG needs a 2-D grid           */
  int32_t bc_type_z[2];  /* (nz > 1) bottom (z = 0) and top (z = nz-1) sides: as bc_type       */
  double bc_value_z[2];
} mc_problem_desc;

typedef struct {
  int32_t scheme;        /* mc_scheme                                                          */
  int32_t precision;     /* mc_precision                                                       */
  int32_t precond;       /* mc_precond                                                         */
  double tol;            /* PCG stop: ||b - A x||_2 <= tol ||b||_2 (recursive residual), 0<tol<1 */
  int32_t max_iter;      /* per solve (per inner solve in MC_MIXED), >= 1                      */
  double outer_tol;      /* MC_MIXED: FP64 residual target relative to ||b||                   */
  int32_t max_outer;     /* MC_MIXED: maximum refinement passes                                */
  double inner_tol;      /* MC_MIXED: inner FP32 PCG tolerance relative to the outer residual  */
  int32_t check_every;   /* PCG iterations launched between host convergence polls (0 = auto:
                            estimated from the observed residual decrease); the device stops
                            each system at its own tolerance either way                        */
  int32_t tile_rows;     /* grid tile height in rows: 0 (default) or 32                         */
  int32_t warm_start;    /* PCG initial guess of a layer: 0 (default) the linear extrapolation
                            2 p^{n-1} - p^{n-2}; 1 always p^{n-1}; 2 adaptive: the order (0-3)
                            of the polynomial extrapolation of the last layers that best
                            predicted the previous layer (the problem keeps three more states
                            per continuum).  Extrapolation uses only layers this problem
                            computed in a row (after creation, mc_set_state or a failed layer
                            it starts from p^{n-1}).  Changes iteration counts only, never the
                            tolerance the solution meets                                    */
  int32_t small_max;     /* 0 (default) or N >= 1: when every continuum has at most N unknowns,
                            the decoupled schemes (D, L, U, EX) in FP64 with MC_JACOBI solve
                            each continuum by one workgroup running its whole PCG in a single
                            launch (mc_step only; batches and the server keep the general
                            path).  Same stopping test; the solution meets the same tolerance
                            but differs from the general path's in rounding                 */
  void *stream;          /* hipStream_t to order all work on, or NULL (library-owned stream)   */
  /* Device allocator hooks (both or neither; NULL: hipMalloc / hipFree).  A problem, batch or
     server takes its device arrays (coefficients, states, PCG and level vectors, launch
     tables) from dev_alloc(bytes, alloc_ctx), which must return memory of the current device
     aligned to at least 256 bytes, or NULL (the call then fails with MC_ENOMEM), and gives
     each back once through dev_free(ptr, alloc_ctx) when it is destroyed, after its streams
     are idle.  The hooks in force at creation stay with the object (mc_set_options does not
     move memory).  They are called on the creating thread, except that a server creates its
     admitted problems on its own setup thread.  The per-system records (a few hundred bytes),
     pinned host mirrors and one-off setup scratch stay with hipMalloc.  This is how a caller
     hands the library torch's caching allocator (the Python binding does with alloc="torch"). */
  void *(*dev_alloc)(size_t bytes, void *ctx);
  void (*dev_free)(void *ptr, void *ctx);
  void *alloc_ctx;
} mc_options;

typedef struct {
  int32_t n_cont;        /* continua in the problem                                            */
  int32_t iters[3];      /* PCG iterations of the last step per continuum (coupled: all equal;
                            mixed: total inner iterations)                                     */
  int32_t outer[3];      /* refinement passes of the last step (MC_MIXED), else 0             */
  int32_t converged[3];  /* 1 if that continuum's last solve met its tolerance                 */
  double relres[3];      /* final ||r||/||b|| (FP64 true residual for MC_MIXED)                */
  double seconds;        /* host wall time of the call                                         */
  int64_t step;          /* time layers completed since creation or the last mc_set_time       */
  int32_t failed;        /* -1, or the continuum whose solve failed                            */
  int32_t warm_order[3]; /* order of the warm start's extrapolation in the last step per
                            continuum (0 = the previous layer; see mc_options.warm_start)    */
} mc_report;

typedef struct {
  int32_t n_cont;
  int32_t sizes[3];      /* unknowns per continuum                                             */
  int64_t device_bytes;  /* device memory held by the problem                                  */
  int32_t grid_tiles;    /* grid tiles per Omega continuum                                     */
  int32_t n_chains;      /* fracture chains (blocks of the fracture preconditioner)            */
  int32_t tiles[3];      /* work tiles per continuum (grid: 64 x 32 cells; fracture: whole
                            chains of about 256 cells)                                          */
  int32_t blocks[3][2];  /* workgroups per launch per continuum: [0] operator kernel,
                            [1] update / residual kernels (equal to its partial-sum slots)      */
  int32_t n_crossing;    /* fracture cells solved through the crossing-cell Schur complement
                            (MC_BIC0 / MC_MG; 0 with Jacobi, without crossings, or beyond 6144) */
  int32_t mg_levels[3];  /* (MC_MG) coarse levels of each grid continuum's V-cycle, else 0;
                            the last one holds at most 256 cells                               */
  int32_t n_frac_blocks; /* (MC_BIC0 / MC_MG) blocks of the two-level fracture preconditioner
                            that replaces the exact solve beyond 6144 crossing cells (connected
                            blocks of at most 64 cells, dense block inverses, and the Galerkin
                            coarse system over the blocks); 0 when the solve is exact or with
                            more than 6144 blocks (the chains alone then)                       */
  int32_t mg_stop_sweeps[3]; /* (MC_MG) 0 if the continuum's V-cycle runs down to its dense
                            coarsest level; else its last level, above the one-workgroup tail,
                            is smoothed by 1 block IC(0) sweep (its row sums reach 8 times its
                            face conductances) or 2 (z_p, then z = z_p + M^-1 (r - A z_p))      */
} mc_info;

typedef struct mc_problem mc_problem;

/* Fill *opt with defaults: D-scheme, FP64, Jacobi, tol 1e-10, max_iter 20000, outer_tol
   1e-10, max_outer 30, inner_tol 1e-6, automatic polling and tiles, NULL stream. */
mc_status mc_options_default(mc_options *opt);

/* Validate *desc (MC_EINVAL with a message on any violation of the ranges stated above),
   allocate device memory for the problem, copy the inputs and build every coefficient on the
   device (storage, face conductances, Dirichlet terms, transfer row sums, fracture graph,
   preconditioner factors).  The state is set to the initial pressures.  *out is NULL on
   failure. */
mc_status mc_create_problem(const mc_problem_desc *desc, const mc_options *opt,
                            mc_problem **out);

/* Release everything; NULL-safe. */
mc_status mc_destroy(mc_problem *p);

/* Advance n_steps (>= 1) time layers with the problem's scheme.  Transactional per layer: if a
   solve fails (MC_ENOCONV, MC_EBREAKDOWN) the state stays at the last completed layer and
   last->failed names the continuum.  last may be NULL. */
mc_status mc_step(mc_problem *p, int32_t n_steps, mc_report *last);

/* Solve (M_a/tau + D_a + S_a) x = rhs for one continuum a (the D-scheme system of Section 3.3;
   without S_a under MC_SCHEME_EX).  rhs_dev and x_dev are device arrays of that continuum's
   size; x_dev holds the initial guess on entry and the solution on return.  The problem's
   state is not touched. */
mc_status mc_solve_continuum(mc_problem *p, int32_t alpha, const double *rhs_dev,
                             double *x_dev, mc_report *rep);

/* Size of the static device workspace of mc_solve_continuum_noalloc, per device. */
#define MC_NOALLOC_BYTES (64L << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): the solve of mc_solve_continuum (same
   system, FP64, same kernels, the problem's tiling and options) with every buffer beyond
   rhs_dev, x_dev and the problem's own coefficients (launch descriptor, tile lists, system
   record, partial sums, the PCG vectors and the crossing-cell vectors) taken from one static
   device array of MC_NOALLOC_BYTES per device, held until the process ends.  No device
   memory is allocated or freed by this call.
   - Preconditioner: Jacobi or block IC(0) (MC_EINVAL under MC_MG or MC_MIXED).
   - Size: MC_EINVAL if the continuum needs more than MC_NOALLOC_BYTES (about 40 bytes per
     unknown: roughly 1.6 million unknowns).
   - The problem's device must be current (MC_EINVAL otherwise); the work runs on the
     problem's stream and the call returns after it has finished.
   - Every call on one device shares that device's workspace, which keeps the last call's
     contents (each call initialises what it reads): calls that overlap on one device, from
     any thread or problem, race and must not be made.
   rhs_dev, x_dev and rep as for mc_solve_continuum. */
mc_status mc_solve_continuum_noalloc(mc_problem *p, int32_t alpha, const double *rhs_dev,
                                     double *x_dev, mc_report *rep);

/* y = (M_a/tau + D_a + S_a) x for continuum a (the operator mc_solve_continuum inverts).
   Device arrays of that continuum's size.  Runs the same operator kernel the solver uses. */
mc_status mc_apply_continuum(mc_problem *p, int32_t alpha, const double *x_dev, double *y_dev);

/* y = (M/tau + D + Q) x on the concatenated vector [p_0; p_1; (p_2)] (the coupled operator of
   Section 3.2).  Device arrays of the total size. */
mc_status mc_apply_coupled(mc_problem *p, const double *x_dev, double *y_dev);

/* z = M_a^-1 r for continuum a with the problem's preconditioner: Jacobi (z = r / diag) or
   block IC(0) (MC_BIC0).  M approximates the D-scheme matrix of mc_solve_continuum; PCG
   converges to the same solution with either (the preconditioner changes only iteration
   counts; no preconditioner appears in the paper's scheme itself).  Device arrays of that
   continuum's size; r and z must not overlap. */
mc_status mc_apply_precond(mc_problem *p, int32_t alpha, const double *r_dev, double *z_dev);

/* b_dev = right-hand side of continuum a in the D-scheme from the current state p^{n-1}:
   M_a/tau p_a^{n-1} + sum_{b!=a} Q_ab p_b^{n-1} + F_a (Section 3.3).  Always FP64. */
mc_status mc_assemble_rhs(mc_problem *p, int32_t alpha, double *b_dev);

/* Copy continuum a of the current state to / from host memory (synchronous). */
mc_status mc_get_state(mc_problem *p, int32_t alpha, double *host_out);
mc_status mc_set_state(mc_problem *p, int32_t alpha, const double *host_in);

/* Replace the solver options (scheme, precision, preconditioner, tolerances); coefficients
   that depend on the scheme are rebuilt on the device.  The stream cannot change. */
mc_status mc_set_options(mc_problem *p, const mc_options *opt);

mc_status mc_get_info(const mc_problem *p, mc_info *info);

/* Message of the last failure on this handle, or (p == NULL) of the calling thread's last
   failed mc_create_problem / server call.  Never NULL. */
const char *mc_last_error(const mc_problem *p);

/* Kernel timing on the problem's streams: HIP events bound to the dispatch of sampled
   launches of the grid PCG kernels time the kernel execution itself.  which: 0 = grid
   operator kernel (p = z + beta p, q = A p), 1 = grid update kernel (x, r, z = M^-1 r;
   under MC_MG its sweep is the finest pre-smoothing), 2 = (MC_MG) the finest level's
   correction and post-smoothing, which writes z; the V-cycle's coarse kernels over all its
   levels (MC_MG): 3 = restriction into a coarse level with its pre-smoothing, 4 = coarse
   correction with post-smoothing, 5 = the small-level tail (one workgroup), 6 = restriction
   into the tail's first level (a sampled V-cycle is timed whole).  enable >= 1 starts recording and clears
   the totals, sampling the kernels of one PCG iteration in `enable` (1 = every iteration;
   each sampled launch costs the stream a few microseconds); 0 stops.  Sampled iterations
   are launched one by one, the others still replayed from captured graphs.
   mc_profile_read returns the number of sampled launches and their summed duration, and
   the number of launches issued while timing was on (sampled or not); which outside 0..6
   gives MC_EINVAL. */
mc_status mc_profile(mc_problem *p, int32_t enable);
mc_status mc_profile_read(mc_problem *p, int32_t which, int64_t *sampled, double *sampled_ms,
                          int64_t *issued);

/* As mc_profile_read, restricted to the sampled launches that lasted at least min_ms (for
   instance to leave out launches that returned at once because their systems had already
   converged): their number and summed duration. */
mc_status mc_profile_read_above(mc_problem *p, int32_t which, double min_ms, int64_t *sampled,
                                double *sampled_ms);

/* Device bytes mc_create_problem allocates for *desc under *opt (NULL = defaults): an upper
   bound computed from the sizes alone, used for admission by the server. */
mc_status mc_footprint(const mc_problem_desc *desc, const mc_options *opt, int64_t *bytes);

/* Autotuner of the launch shapes.  For every size class (work tiles rounded down to a power
   of two, per continuum kind, precision and preconditioner) present among probs[0..n), time
   candidate workgroup counts of the PCG operator and update launches (1, 2 or 4 tiles per
   workgroup; 2, 4 or 8 for the grid block IC(0) update, whose wavefronts each sweep 64 x 16
   blocks) over `iters` (<= 0: 20) iterations of a real PCG run on one continuum of that class,
   and keep the fastest (classes already tuned in this process are kept).  The choices apply
   to these problems and to every problem created later in the process; a problem's result then depends on its own size class only, so it is
   still the same alone and in any batch.  Only scratch vectors are written (the state is
   kept).  Problems must not be in use by another thread. */
mc_status mc_autotune(mc_problem *const *probs, int32_t n, int32_t iters);

/* Forget every tuned choice (problems created afterwards use the built-in shapes). */
mc_status mc_autotune_clear(void);

/* ---- batches: many problems advanced by shared launches ---------------------------------
 *
 * A batch executor advances a list of problems by one time layer per step with every
 * continuum of every problem in the same kernel launches: one launch per PCG kernel covers
 * the tiles of all grid continua of all problems, another those of all fracture continua
 * (each system keeps its own scalars and stopping test, Section 3.3 D-scheme per problem).
 * Iterations are replayed from captured HIP graphs.  Each problem keeps its own tiling and
 * partial-sum order, so its result is bitwise the one mc_step gives it alone with the same
 * options.  Problems may differ in size, continua and fracture network.
 */
typedef struct mc_batch mc_batch;

/* Create a batch executor.  opt gives the solver options of every batch step (tolerances,
   max_iter, refinement) and the stream (NULL = library-owned).  scheme must be D, EX or
   COUPLED.  *out is NULL on failure (message from mc_batch_last_error(NULL)). */
mc_status mc_batch_create(const mc_options *opt, mc_batch **out);

/* Release the executor (not the problems); NULL-safe. */
mc_status mc_batch_destroy(mc_batch *b);

/* Advance the n (>= 1) distinct problems probs[0..n) by n_steps layers together.  Every
   problem must have been created with the batch's scheme class (D/EX, or COUPLED),
   precision and preconditioner (MC_EINVAL otherwise).  Per problem and per layer the step is
   transactional: a problem whose solve fails keeps its state (reps[i].failed names the
   continuum) while the others advance; the call then returns the first failure after that
   layer.  reps (nullable) receives one report per problem.  The problems must not be used by
   another thread during the call; their device memory is accessed on the batch's stream. */
mc_status mc_batch_step(mc_batch *b, mc_problem *const *probs, int32_t n, int32_t n_steps,
                        mc_report *reps);

const char *mc_batch_last_error(const mc_batch *b);

/* Kernel timing of the batch's grid PCG kernels, as mc_profile / mc_profile_read /
   mc_profile_read_above. */
mc_status mc_batch_profile(mc_batch *b, int32_t enable);
mc_status mc_batch_profile_read(mc_batch *b, int32_t which, int64_t *sampled,
                                double *sampled_ms, int64_t *issued);
mc_status mc_batch_profile_read_above(mc_batch *b, int32_t which, double min_ms,
                                      int64_t *sampled, double *sampled_ms);

/* ---- serving: continuous batching of simulation requests ------------------------------
 *
 * A server owns a worker thread and a batch executor.  Requests (a problem descriptor and a
 * number of time layers) are queued by mc_server_submit and admitted in arrival order while
 * their device footprint (mc_footprint) fits the memory budget and a resident slot is free;
 * a later request may bypass a waiting head that does not fit, at most max_bypass times per
 * head.  Admitted requests are created on the device and stay resident; every server step
 * advances all resident requests by one layer in shared launches (mc_batch_step).  A request
 * that finishes copies its final state to host memory and frees its device memory, which
 * admits the next ones.  Each request's result is the one mc_step gives the same problem
 * alone with the server's options (per-problem tilings and reductions, see mc_batch_step).
 * All server calls may be made from one client thread while the worker runs.
 */
typedef struct mc_server mc_server;

typedef struct {
  int64_t hbm_budget;    /* device bytes the resident requests may hold (> 0)                 */
  int32_t max_resident;  /* resident requests at most (0 = 256)                               */
  int32_t max_bypass;    /* times a waiting head request may be bypassed (>= 0)                */
  int32_t autotune;      /* 1: run mc_autotune on each admitted request (new size classes only) */
} mc_server_config;

typedef struct {
  int32_t state;         /* 0 queued, 1 running (or finishing), 2 done, 3 failed               */
  int32_t status;        /* mc_status of a failed request                                      */
  int32_t steps_done, n_steps;
  int64_t bytes;         /* device bytes charged against the budget                            */
  double t_submit, t_admit, t_finish;   /* seconds since the server started (-1: not yet)     */
} mc_request_info;

typedef struct {
  int64_t submitted, finished, failed, queued, resident;
  int64_t bytes_in_use, budget;
  int64_t steps;         /* server steps (one layer of every resident request)                 */
  double cell_updates;   /* unknowns advanced, summed over server steps                        */
  double busy_seconds;   /* time inside server steps                                           */
  double elapsed_seconds;/* since mc_server_create                                             */
} mc_server_stats;

/* opt: solver options of every request (scheme D or EX; NULL = defaults). */
mc_status mc_server_create(const mc_server_config *cfg, const mc_options *opt, mc_server **out);

/* Stops the worker after the current step and releases everything; NULL-safe. */
mc_status mc_server_destroy(mc_server *s);

/* Queue a request; *desc's arrays are copied before return.  MC_ENOMEM if its footprint
   exceeds the whole budget (it could never be admitted). */
mc_status mc_server_submit(mc_server *s, const mc_problem_desc *desc, int32_t n_steps,
                           uint64_t *id);

mc_status mc_server_poll(mc_server *s, uint64_t id, mc_request_info *info);

/* Final state of continuum alpha of a done request (host array of that continuum's size). */
mc_status mc_server_fetch(mc_server *s, uint64_t id, int32_t alpha, double *host_out);

/* Forget a done or failed request and its host copy of the state. */
mc_status mc_server_release(mc_server *s, uint64_t id);

/* Block until no request is queued, running or finishing (timeout_s < 0: no limit);
   MC_ETIMEOUT if the time ran out first. */
mc_status mc_server_wait(mc_server *s, double timeout_s);

mc_status mc_server_get_stats(mc_server *s, mc_server_stats *st);

/* Durations of the server steps so far (seconds): *n receives the count, out (nullable)
   the first min(cap, count) of them. */
mc_status mc_server_step_seconds(mc_server *s, double *out, int64_t cap, int64_t *n);

const char *mc_server_last_error(const mc_server *s);

/* ---- coarse-grid schemes: nonlocal multicontinuum (NLMC) upscaling (Section 4) ---------
   A coarse grid of bx x by fine cells per coarse cell (nx % bx == ny % by == 0).  A coarse
   unit is one continuum inside one coarse cell (K_j^a; a fracture unit only where the
   coarse cell hosts fracture cells); units are ordered continuum by continuum, coarse cells
   row-major.  For every unit a basis function minimizes the energy of the fine operator
   A = D + Q (wells included) over vectors that vanish outside the oversampled region K_i^+
   (K_i grown by `layers` coarse cells) and have mean one on their own unit and zero on
   every other unit of K_i^+ (eq. eq:basis; the means weigh cells by their measure).  The
   coarse operator A_bar takes its off-diagonal entries (nonlocal transmissibilities) from
   R A R^T, R the matrix of basis functions, and its diagonal from conservation: each row
   sums to the unit's summed fine row sums (zero away from Dirichlet sides and wells).
   M_bar (diagonal) and F_bar sum the fine storage c|K| and right-hand side over each unit
   (eq. app-nlmc and the direct coarse formulas after it).  Layers advance eq. is-nlmc
   (coupled) or eq. si-nlmc (D, L, U: block-diagonal, block-lower or block-upper A_bar_0)
   with direct solves (dense inverses of the coarse systems, formed at creation). */
typedef struct mc_nlmc mc_nlmc;

typedef struct {
  int32_t n_units;               /* N_H, coarse unknowns                                       */
  int32_t n_cont;                /* continua (grid continua, then the fracture if any)         */
  int32_t sizes[3];              /* units per continuum                                        */
  int32_t n_regions;             /* oversampled regions (one per coarse cell)                  */
  int32_t max_region_unknowns;   /* largest local problem                                      */
  int32_t max_band;              /* largest lower band width of a local operator               */
  int32_t max_constraints;       /* most units inside one region                               */
  int32_t pad;
  int64_t n_pairs;               /* unit pairs whose basis functions interact                  */
  int64_t device_bytes;          /* device memory held after creation                          */
  double setup_ms[4];            /* GPU time of creation: [0] unit sums and local factors,     */
                                 /* [1] basis functions, [2] coarse operator, [3] inverses     */
  int64_t steps;                 /* layers advanced since the last mc_nlmc_set_state           */
} mc_nlmc_info;

/* Build the coarse system of fine problem `fine` (2-D grid; any scheme but MC_SCHEME_EX),
   on its device (which must be current) and stream.  The coarse state starts as the unit
   means of the fine problem's current state.  The fine problem is only read here.
   MC_EINVAL: coarse cells that do not tile the grid, layers < 0, fracture connections
   between hosts more than one cell apart, local bands too wide for the forward solve.
   MC_EBREAKDOWN: a local operator or constraint system not positive definite (for example
   a region covering a whole domain without Dirichlet sides or wells). */
mc_status mc_nlmc_create(mc_problem *fine, int32_t bx, int32_t by, int32_t layers,
                         mc_nlmc **out);
mc_status mc_nlmc_destroy(mc_nlmc *nl);   /* NULL-safe */
mc_status mc_nlmc_get_info(const mc_nlmc *nl, mc_nlmc_info *info);

/* Copies of A_bar (row-major n_units x n_units), the diagonal of M_bar and F_bar to host
   arrays (each may be NULL). */
mc_status mc_nlmc_get_system(mc_nlmc *nl, double *A_host, double *M_host, double *F_host);

/* Coarse state to / from host arrays of n_units values; host_in NULL restores the unit
   means of the fine state at creation.  Synchronous. */
mc_status mc_nlmc_set_state(mc_nlmc *nl, const double *host_in);
mc_status mc_nlmc_get_state(mc_nlmc *nl, double *host_out);

/* Advance n_steps layers of `scheme` (MC_SCHEME_COUPLED, _D, _L or _U) with the fine
   problem's tau; synchronous. */
mc_status mc_nlmc_step(mc_nlmc *nl, int32_t scheme, int32_t n_steps);

/* Message of the last failure on this handle, or (NULL) of the calling thread's last failed
   mc_nlmc_create.  Never NULL. */
const char *mc_nlmc_last_error(const mc_nlmc *nl);

#ifdef __cplusplus
}
#endif
#endif /* MCDEC_H */
