// Runtime of the MI355X multicontinuum library: device memory of a problem, coefficient
// setup, launch tables, PCG orchestration for every scheme and precision, and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mcdec.h"
#include "common.hpp"
#include "host_setup.hpp"
#include "kernels.hpp"

namespace mc {

struct Error {
  mc_status st;
  std::string msg;
};

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw Error{MC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)};      \
  } while (0)

static thread_local std::string g_thread_error = "";

static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

static bool env_flag(const char* name, bool dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v) != 0;
}

// ------------------------------------------------------------------------------------
// device buffers
// ------------------------------------------------------------------------------------
struct DevArena {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  template <class T>
  T* alloc(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{MC_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed"};
    }
    ptrs.push_back(p);
    bytes += n * sizeof(T);
    return (T*)p;
  }
  template <class T>
  T* upload(const T* h, size_t n, hipStream_t s) {
    T* d = alloc<T>(n);
    if (n) HIPCHK(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
};

// A launch table: parts + tiles in device memory, plus per-system slot counts.
struct Table {
  PartD* parts = nullptr;
  Tile* tiles = nullptr;
  int nblocks = 0;
  int nparts = 0;
  std::vector<PartD> hparts;
};

struct Cont {  // one continuum
  int kind;    // PART_GRID / PART_GRAPH
  long n;
  int tiles;   // tiles of its part
  // FP64 coefficients
  double *diag = nullptr, *tx = nullptr, *ty = nullptr, *F = nullptr, *val = nullptr,
         *mt = nullptr;
  float *diag32 = nullptr, *tx32 = nullptr, *ty32 = nullptr, *val32 = nullptr;
  double* fdinv = nullptr;
  float* fdinv32 = nullptr;
  // state and PCG vectors
  double* ps[2] = {nullptr, nullptr};
  double *b = nullptr, *r = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr, *z = nullptr;
  float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *p232 = nullptr, *q32 = nullptr,
        *z32 = nullptr;
  double mtau = 0, tconst = 0;
  int has_t = 1;
};

}  // namespace mc

using namespace mc;

struct mc_problem {
  mc_problem_desc d{};   // scalars only (array pointers are not kept)
  mc_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int ncont = 0, n_omega = 0, nf = 0, ne = 0;
  long ncell = 0;
  int ty = 16;
  DevArena mem;
  std::vector<Cont> cont;
  // inputs kept on the device (for re-setup)
  double* k[2] = {nullptr, nullptr};
  double* src[3] = {nullptr, nullptr, nullptr};
  int *host = nullptr, *rowptr = nullptr, *col = nullptr, *eidx = nullptr, *hptr = nullptr,
      *hidx = nullptr, *chain_ptr = nullptr;
  double *flen = nullptr, *edge_d = nullptr, *sigma_f = nullptr;
  int nchains = 0;
  // systems: 0..ncont-1 decoupled per continuum, ncont = coupled
  SysState* sys = nullptr;
  std::vector<double*> partials;
  int* counters = nullptr;       // [0] active, [1] outer active
  int* h_counters = nullptr;     // pinned
  SysState* h_sys = nullptr;     // pinned
  int cur = 0;                   // state ping-pong index
  long step_count = 0;
  std::map<std::string, Table> tables;
  std::string err;
  // profiling
  bool prof = false;
  struct Ev { hipEvent_t a, b; int which; };
  std::vector<Ev> ev_free, ev_pending;
  long prof_launch[2] = {0, 0};
  double prof_ms[2] = {0, 0};
};

namespace mc {

static void fail(mc_problem* p, const std::string& m) { throw Error{MC_EINVAL, m}; }

// ------------------------------------------------------------------------------------
// tables
// ------------------------------------------------------------------------------------
static PartD base_part(mc_problem* P, int c, int sys, int slot0, bool fp32) {
  Cont& C = P->cont[c];
  PartD q;
  std::memset(&q, 0, sizeof(q));
  q.kind = C.kind;
  q.sys = sys;
  q.cont = c;
  q.n = (int)C.n;
  q.nx = P->d.nx;
  q.ny = P->d.ny;
  q.trows = P->ty;
  q.tiles_x = (int)cdiv(P->d.nx, MC_TX);
  q.slot0 = slot0;
  q.ex = P->opt.scheme == MC_SCHEME_EX;
  q.has_t = C.has_t;
  q.n_omega = P->n_omega;
  q.other = -1;
  q.frac = -1;
  q.omg[0] = q.omg[1] = -1;
  q.tconst = C.tconst;
  q.mtau = C.mtau;
  q.s12 = P->n_omega == 2 ? P->d.sigma_omega * P->d.h * P->d.h : 0.0;
  q.diag = C.diag;
  q.tx = C.tx;
  q.ty = C.ty;
  q.F = C.F;
  q.rowptr = P->rowptr;
  q.col = P->col;
  q.val = C.val;
  q.mt = C.mt;
  q.diag32 = C.diag32;
  q.tx32 = C.tx32;
  q.ty32 = C.ty32;
  q.val32 = C.val32;
  q.fdinv = C.fdinv;
  q.fdinv32 = C.fdinv32;
  q.chain_ptr = P->chain_ptr;
  q.nchains = P->nchains;
  if (C.kind == PART_GRID) {
    q.hptr = P->nf ? P->hptr : nullptr;
    q.hidx = P->hidx;
    q.hsig = P->nf ? P->sigma_f + (long)c * P->nf : nullptr;
  } else {
    q.host = P->host;
    q.fsig0 = P->sigma_f;
    q.fsig1 = P->n_omega > 1 ? P->sigma_f + P->nf : nullptr;
  }
  q.pold = C.ps[P->cur];
  for (int b = 0; b < P->ncont; ++b) q.tsrc[b] = P->cont[b].ps[P->cur];
  q.b = C.b;
  if (fp32) {
    q.x = C.x32;
    q.r = C.r32;
    q.p = C.p32;
    q.p2 = C.p232;
    q.q = C.q32;
    q.z = C.z32;
    q.x64 = C.ps[1 - P->cur];
  } else {
    q.x = C.ps[1 - P->cur];
    q.x64 = C.ps[1 - P->cur];
    q.r = C.r;
    q.p = C.p;
    q.p2 = C.p2;
    q.q = C.q;
    q.z = C.z;
  }
  return q;
}

static Table& upload_table(mc_problem* P, const std::string& key, std::vector<PartD> parts) {
  auto it = P->tables.find(key);
  if (it != P->tables.end() && it->second.hparts.size() == parts.size() &&
      std::memcmp(it->second.hparts.data(), parts.data(), parts.size() * sizeof(PartD)) == 0)
    return it->second;
  Table T;
  if (it != P->tables.end()) T = it->second;
  // tile list: parts in order, tiles in natural order, then the XCD-aware launch order
  std::vector<Tile> nat;
  for (int pi = 0; pi < (int)parts.size(); ++pi) {
    int nt = parts[pi].kind == PART_GRID
                 ? (int)(cdiv(parts[pi].nx, MC_TX) * cdiv(parts[pi].ny, parts[pi].trows))
                 : (int)cdiv(parts[pi].n, MC_GRAPH_ROWS);
    for (int t = 0; t < nt; ++t) nat.push_back(Tile{pi, t});
  }
  std::vector<int> ord = xcd_order((int)nat.size(), env_flag("MCDEC_XCD", true) ? 8 : 1);
  std::vector<Tile> tiles(ord.size());
  for (size_t b = 0; b < ord.size(); ++b) tiles[b] = ord[b] >= 0 ? nat[ord[b]] : Tile{-1, 0};
  if (!T.parts || T.nparts < (int)parts.size()) T.parts = P->mem.alloc<PartD>(parts.size() + 2);
  if (!T.tiles || T.nblocks < (int)tiles.size()) T.tiles = P->mem.alloc<Tile>(tiles.size() + 8);
  HIPCHK(hipMemcpyAsync(T.parts, parts.data(), parts.size() * sizeof(PartD),
                        hipMemcpyHostToDevice, P->stream));
  HIPCHK(hipMemcpyAsync(T.tiles, tiles.data(), tiles.size() * sizeof(Tile),
                        hipMemcpyHostToDevice, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));   // host vectors die at return
  T.nblocks = (int)tiles.size();
  T.nparts = (int)parts.size();
  T.hparts = std::move(parts);
  P->tables[key] = T;
  return P->tables[key];
}

static int part_tiles(mc_problem* P, int c) { return P->cont[c].tiles; }

// ------------------------------------------------------------------------------------
// setup
// ------------------------------------------------------------------------------------
static void build_coefficients(mc_problem* P) {
  const bool ex = P->opt.scheme == MC_SCHEME_EX;
  const double h = P->d.h, tau = P->d.tau;
  for (int a = 0; a < P->n_omega; ++a) {
    Cont& C = P->cont[a];
    GridSetup g;
    std::memset(&g, 0, sizeof(g));
    g.nx = P->d.nx;
    g.ny = P->d.ny;
    g.k = P->k[a];
    g.kc = P->d.omega[a].k_const;
    g.c = P->d.omega[a].c;
    g.h = h;
    g.tau = tau;
    g.s12 = P->n_omega == 2 ? P->d.sigma_omega * h * h : 0.0;
    for (int s = 0; s < 4; ++s) {
      g.bc_type[s] = P->d.bc_type[s];
      g.bc_value[s] = P->d.bc_value[s];
    }
    g.src = P->src[a];
    g.hptr = P->nf ? P->hptr : nullptr;
    g.hidx = P->hidx;
    g.hsig = P->nf ? P->sigma_f + (long)a * P->nf : nullptr;
    g.ex = ex;
    g.diag = C.diag;
    g.tx = C.tx;
    g.ty = C.ty;
    g.F = C.F;
    hipLaunchKernelGGL(k_setup_grid, dim3(cdiv(C.n, 256)), dim3(256), 0, P->stream, g);
    C.mtau = P->d.omega[a].c * h * h / tau;
    C.has_t = P->k[a] != nullptr;
    C.tconst = P->d.omega[a].k_const;
  }
  if (P->nf) {
    Cont& C = P->cont[P->n_omega];
    GraphSetup g;
    std::memset(&g, 0, sizeof(g));
    g.nf = P->nf;
    g.n_omega = P->n_omega;
    g.rowptr = P->rowptr;
    g.eidx = P->eidx;
    g.edge_d = P->edge_d;
    g.flen = P->flen;
    g.sig0 = P->sigma_f;
    g.sig1 = P->n_omega > 1 ? P->sigma_f + P->nf : nullptr;
    g.src = P->src[P->n_omega];
    g.k_f = P->d.k_f;
    g.c_f = P->d.c_f;
    g.aperture = P->d.aperture;
    g.tau = tau;
    g.ex = ex;
    g.val = C.val;
    g.diag = C.diag;
    g.mt = C.mt;
    g.F = C.F;
    hipLaunchKernelGGL(k_setup_graph, dim3(cdiv(P->nf, 256)), dim3(256), 0, P->stream, g);
  }
  HIPCHK(hipGetLastError());
  if (P->opt.precision == MC_MIXED) {
    for (auto& C : P->cont) {
      auto cv = [&](double* a, float*& b, long n) {
        if (!a || n == 0) return;
        if (!b) b = P->mem.alloc<float>(n);
        hipLaunchKernelGGL(k_to_f32, dim3(cdiv(n, 256)), dim3(256), 0, P->stream, a, b, n);
      };
      cv(C.diag, C.diag32, C.n);
      if (C.kind == PART_GRID) {
        cv(C.tx, C.tx32, C.n);
        cv(C.ty, C.ty32, C.n);
      } else {
        cv(C.val, C.val32, 2L * P->ne);
      }
      if (!C.x32) {
        C.x32 = P->mem.alloc<float>(C.n);
        C.r32 = P->mem.alloc<float>(C.n);
        C.p32 = P->mem.alloc<float>(C.n);
        C.p232 = P->mem.alloc<float>(C.n);
        C.q32 = P->mem.alloc<float>(C.n);
      }
    }
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(P->stream));
  P->tables.clear();
}

static void create(mc_problem* P, const mc_problem_desc& d, const mc_options& o) {
  std::string m = validate_desc(d);
  if (!m.empty()) fail(P, m);
  m = validate_options(o);
  if (!m.empty()) fail(P, m);
  if (o.precond == MC_BIC0) fail(P, "block IC(0) is not available in this build");
  P->d = d;
  P->opt = o;
  P->ty = o.tile_rows > 0 ? o.tile_rows : 16;
  P->n_omega = d.n_omega;
  P->nf = d.nf;
  P->ne = d.ne;
  P->ncell = (long)d.nx * d.ny;
  P->ncont = d.n_omega + (d.nf > 0 ? 1 : 0);
  if (o.stream) {
    P->stream = (hipStream_t)o.stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking));
    P->own_stream = true;
  }
  hipStream_t s = P->stream;
  DevArena& M = P->mem;
  // inputs
  for (int a = 0; a < d.n_omega; ++a) {
    if (d.omega[a].k) P->k[a] = M.upload(d.omega[a].k, P->ncell, s);
    if (d.omega[a].src) P->src[a] = M.upload(d.omega[a].src, P->ncell, s);
  }
  GraphCSR g;
  HostMap hm;
  std::vector<int> chains;
  if (d.nf) {
    g = build_graph(d.nf, d.ne, d.edges);
    hm = build_host_map((int)P->ncell, d.nf, d.host);
    chains = build_chains(d.nf, g);
    P->host = M.upload(d.host, d.nf, s);
    P->flen = M.upload(d.flen, d.nf, s);
    P->sigma_f = M.upload(d.sigma_f, (size_t)d.n_omega * d.nf, s);
    P->rowptr = M.upload(g.rowptr.data(), g.rowptr.size(), s);
    P->col = M.upload(g.col.data(), g.col.size(), s);
    P->eidx = M.upload(g.eidx.data(), g.eidx.size(), s);
    P->edge_d = d.ne ? M.upload(d.edge_d, d.ne, s) : M.alloc<double>(1);
    P->hptr = M.upload(hm.hptr.data(), hm.hptr.size(), s);
    P->hidx = M.upload(hm.hidx.data(), hm.hidx.size(), s);
    P->chain_ptr = M.upload(chains.data(), chains.size(), s);
    P->nchains = (int)chains.size() - 1;
    if (d.src_f) P->src[d.n_omega] = M.upload(d.src_f, d.nf, s);
  }
  // continua
  P->cont.resize(P->ncont);
  for (int c = 0; c < P->ncont; ++c) {
    Cont& C = P->cont[c];
    const bool grid = c < d.n_omega;
    C.kind = grid ? PART_GRID : PART_GRAPH;
    C.n = grid ? P->ncell : d.nf;
    C.tiles = grid ? (int)(cdiv(d.nx, MC_TX) * cdiv(d.ny, P->ty)) : (int)cdiv(d.nf, MC_GRAPH_ROWS);
    C.diag = M.alloc<double>(C.n);
    C.F = M.alloc<double>(C.n);
    if (grid) {
      C.tx = M.alloc<double>(C.n);
      C.ty = M.alloc<double>(C.n);
    } else {
      C.val = M.alloc<double>(std::max<long>(1, 2L * d.ne));
      C.mt = M.alloc<double>(C.n);
    }
    for (int k = 0; k < 2; ++k) C.ps[k] = M.alloc<double>(C.n);
    C.b = M.alloc<double>(C.n);
    C.r = M.alloc<double>(C.n);
    C.p = M.alloc<double>(C.n);
    C.p2 = M.alloc<double>(C.n);
    C.q = M.alloc<double>(C.n);
    const double* p0 = grid ? d.omega[c].p0 : d.p0_f;
    if (p0) HIPCHK(hipMemcpyAsync(C.ps[0], p0, C.n * sizeof(double), hipMemcpyHostToDevice, s));
    else HIPCHK(hipMemsetAsync(C.ps[0], 0, C.n * sizeof(double), s));
  }
  // systems: one per continuum + the coupled one
  const int nsys = P->ncont + 1;
  P->sys = M.alloc<SysState>(nsys);
  P->counters = M.alloc<int>(4);
  HIPCHK(hipHostMalloc((void**)&P->h_counters, 4 * sizeof(int), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void**)&P->h_sys, nsys * sizeof(SysState), hipHostMallocDefault));
  std::vector<SysState> hs(nsys);
  std::memset(hs.data(), 0, nsys * sizeof(SysState));
  int coupled_slots = 0;
  for (int c = 0; c < P->ncont; ++c) coupled_slots += P->cont[c].tiles;
  for (int sI = 0; sI < nsys; ++sI) {
    int ns = sI < P->ncont ? P->cont[sI].tiles : coupled_slots;
    hs[sI].nslots = ns;
    hs[sI].partials = M.alloc<double>((size_t)ns * MC_SLOT);
    hs[sI].active = P->counters;
    hs[sI].oactive = P->counters + 1;
  }
  HIPCHK(hipMemcpyAsync(P->sys, hs.data(), nsys * sizeof(SysState), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  build_coefficients(P);
}

// ------------------------------------------------------------------------------------
// profiling helpers
// ------------------------------------------------------------------------------------
static void prof_begin(mc_problem* P, int which, mc_problem::Ev& e) {
  if (P->ev_free.empty()) {
    mc_problem::Ev n;
    HIPCHK(hipEventCreate(&n.a));
    HIPCHK(hipEventCreate(&n.b));
    P->ev_free.push_back(n);
  }
  e = P->ev_free.back();
  P->ev_free.pop_back();
  e.which = which;
  HIPCHK(hipEventRecord(e.a, P->stream));
}
static void prof_end(mc_problem* P, mc_problem::Ev& e) {
  HIPCHK(hipEventRecord(e.b, P->stream));
  P->ev_pending.push_back(e);
}
static void prof_harvest(mc_problem* P) {
  for (auto& e : P->ev_pending) {
    float ms = 0;
    HIPCHK(hipEventSynchronize(e.b));
    HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
    P->prof_ms[e.which] += ms;
    P->prof_launch[e.which] += 1;
    P->ev_free.push_back(e);
  }
  P->ev_pending.clear();
}

// ------------------------------------------------------------------------------------
// solve orchestration
// ------------------------------------------------------------------------------------
template <class T, int PREC>
static void launch_iter(mc_problem* P, const Table& Tb) {
  mc_problem::Ev e;
  if (P->prof) prof_begin(P, 0, e);
  hipLaunchKernelGGL((k_pcg_A<T, PREC>), dim3(Tb.nblocks), dim3(MC_BLOCK), 0, P->stream,
                     Tb.parts, Tb.tiles, P->sys);
  if (P->prof) prof_end(P, e);
  if (P->prof) prof_begin(P, 1, e);
  hipLaunchKernelGGL((k_pcg_B<T, PREC>), dim3(Tb.nblocks), dim3(MC_BLOCK), 0, P->stream,
                     Tb.parts, Tb.tiles, P->sys);
  if (P->prof) prof_end(P, e);
}

static void poll(mc_problem* P) {
  HIPCHK(hipMemcpyAsync(P->h_counters, P->counters, 2 * sizeof(int), hipMemcpyDeviceToHost,
                        P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  if (P->prof) prof_harvest(P);
}

static void set_sys_params(mc_problem* P, const std::vector<int>& systems, double tol,
                           int max_iter, bool mixed) {
  // small per-solve parameters written into the device system records
  for (int sI : systems) {
    SysState* S = P->sys + sI;
    double t2 = tol * tol;
    HIPCHK(hipMemcpyAsync(&S->tol2, &t2, sizeof(double), hipMemcpyHostToDevice, P->stream));
    HIPCHK(hipMemcpyAsync(&S->max_iter, &max_iter, sizeof(int), hipMemcpyHostToDevice,
                          P->stream));
    if (mixed) {
      double o2 = P->opt.outer_tol * P->opt.outer_tol;
      HIPCHK(hipMemcpyAsync(&S->otol2, &o2, sizeof(double), hipMemcpyHostToDevice, P->stream));
      HIPCHK(hipMemcpyAsync(&S->max_outer, &P->opt.max_outer, sizeof(int),
                            hipMemcpyHostToDevice, P->stream));
    }
  }
  HIPCHK(hipStreamSynchronize(P->stream));   // sources are stack values
}

// Runs PCG to completion for the systems of table Tb (FP64).  Returns after every system is
// done; statuses are in the device system records.
template <int PREC>
static void run_pcg64(mc_problem* P, const Table& Tb, int nsys_active, int max_iter) {
  int K = P->opt.check_every > 0 ? P->opt.check_every : 8;
  long launched = 0;
  for (;;) {
    for (int k = 0; k < K; ++k) launch_iter<double, PREC>(P, Tb);
    HIPCHK(hipGetLastError());
    launched += K;
    poll(P);
    if (P->h_counters[0] <= 0) break;
    if (launched > (long)max_iter + 2L * K + 4)
      throw Error{MC_EDEVICE, "PCG did not report completion within max_iter launches"};
    if (K < 64) K *= 2;   // long solves poll less often
  }
}

static void solve_systems64(mc_problem* P, const Table& Tb, const std::vector<int>& systems,
                            bool assemble) {
  const int ns = (int)systems.size();
  set_sys_params(P, systems, P->opt.tol, P->opt.max_iter, false);
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, P->stream, P->sys, P->ncont + 1,
                     P->counters, ns, 0, 0);
  if (assemble)
    hipLaunchKernelGGL(k_rhs, dim3(Tb.nblocks), dim3(MC_BLOCK), 0, P->stream, Tb.parts,
                       Tb.tiles);
  hipLaunchKernelGGL((k_init<PREC_JACOBI>), dim3(Tb.nblocks), dim3(MC_BLOCK), 0, P->stream,
                     Tb.parts, Tb.tiles, P->sys);
  HIPCHK(hipGetLastError());
  run_pcg64<PREC_JACOBI>(P, Tb, ns, P->opt.max_iter);
}

static void solve_systems_mixed(mc_problem* P, const Table& Tb, const std::vector<int>& systems,
                                bool assemble) {
  const int ns = (int)systems.size();
  set_sys_params(P, systems, P->opt.inner_tol, P->opt.max_iter, true);
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, P->stream, P->sys, P->ncont + 1,
                     P->counters, 0, ns, 1);
  if (assemble)
    hipLaunchKernelGGL(k_rhs, dim3(Tb.nblocks), dim3(MC_BLOCK), 0, P->stream, Tb.parts,
                       Tb.tiles);
  const double it2 = P->opt.inner_tol * P->opt.inner_tol;
  for (int outer = 0; outer <= P->opt.max_outer + 1; ++outer) {
    hipLaunchKernelGGL(k_residual, dim3(Tb.nblocks), dim3(MC_BLOCK), 0, P->stream, Tb.parts,
                       Tb.tiles, P->sys, it2);
    HIPCHK(hipGetLastError());
    poll(P);
    if (P->h_counters[1] <= 0) return;
    int K = P->opt.check_every > 0 ? P->opt.check_every : 8;
    long launched = 0;
    while (P->h_counters[0] > 0) {
      for (int k = 0; k < K; ++k) launch_iter<float, PREC_JACOBI>(P, Tb);
      HIPCHK(hipGetLastError());
      launched += K;
      poll(P);
      if (launched > (long)P->opt.max_iter + 2L * K + 4)
        throw Error{MC_EDEVICE, "inner PCG did not report completion"};
      if (K < 64) K *= 2;
    }
    hipLaunchKernelGGL(k_correct, dim3(Tb.nblocks), dim3(MC_BLOCK), 0, P->stream, Tb.parts,
                       Tb.tiles, P->sys);
    hipLaunchKernelGGL(k_outer_count, dim3(1), dim3(64), 0, P->stream, P->sys, P->ncont + 1);
  }
  throw Error{MC_EDEVICE, "refinement loop did not terminate"};
}

// Reads back the system records; fills the report; returns the first failing status.
static mc_status collect(mc_problem* P, const std::vector<int>& systems,
                         const std::vector<int>& conts_of_sys, mc_report* rep, bool mixed) {
  const int nsys = P->ncont + 1;
  HIPCHK(hipMemcpyAsync(P->h_sys, P->sys, nsys * sizeof(SysState), hipMemcpyDeviceToHost,
                        P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  mc_status st = MC_OK;
  int failed = -1;
  for (size_t k = 0; k < systems.size(); ++k) {
    const SysState& S = P->h_sys[systems[k]];
    const int status = mixed ? S.outer_status : S.status;
    const int c = conts_of_sys[k];
    if (rep && c >= 0 && c < 3) {
      rep->iters[c] = mixed ? S.total_iter : S.iter;
      rep->outer[c] = mixed ? S.outer : 0;
      rep->converged[c] = status == ST_CONV;
      rep->relres[c] = mixed ? (S.obb > 0 ? std::sqrt(S.orr / S.obb) : std::sqrt(S.orr))
                             : (S.bb > 0 ? std::sqrt(S.rr / S.bb) : std::sqrt(S.rr));
    }
    if (status != ST_CONV && st == MC_OK) {
      st = status == ST_NOCONV ? MC_ENOCONV : MC_EBREAKDOWN;
      failed = c;
    }
  }
  if (rep) rep->failed = failed;
  return st;
}

static void fill_coupled_report(mc_problem* P, mc_report* rep) {
  if (!rep) return;
  for (int c = 1; c < P->ncont; ++c) {
    rep->iters[c] = rep->iters[0];
    rep->outer[c] = rep->outer[0];
    rep->converged[c] = rep->converged[0];
    rep->relres[c] = rep->relres[0];
  }
}

static std::vector<PartD> decoupled_parts(mc_problem* P, const std::vector<int>& conts,
                                          bool fp32) {
  std::vector<PartD> parts;
  for (int c : conts) parts.push_back(base_part(P, c, c, 0, fp32));
  return parts;
}

static std::vector<PartD> coupled_parts(mc_problem* P) {
  std::vector<PartD> parts;
  int slot = 0;
  const int sysI = P->ncont;
  for (int c = 0; c < P->ncont; ++c) {
    PartD q = base_part(P, c, sysI, slot, false);
    slot += P->cont[c].tiles;
    q.coupled = 1;
    parts.push_back(q);
  }
  for (int c = 0; c < P->ncont; ++c) {
    if (c < P->n_omega) {
      parts[c].other = P->n_omega == 2 ? 1 - c : -1;
      parts[c].frac = P->nf ? P->n_omega : -1;
    } else {
      parts[c].omg[0] = 0;
      parts[c].omg[1] = P->n_omega > 1 ? 1 : -1;
    }
  }
  return parts;
}

static mc_status step_once(mc_problem* P, mc_report* rep) {
  const bool mixed = P->opt.precision == MC_MIXED;
  const int sch = P->opt.scheme;
  std::vector<int> all;
  for (int c = 0; c < P->ncont; ++c) all.push_back(c);
  mc_status st;
  if (sch == MC_SCHEME_COUPLED) {
    Table& T = upload_table(P, "coupled" + std::to_string(P->cur), coupled_parts(P));
    solve_systems64(P, T, {P->ncont}, true);
    st = collect(P, {P->ncont}, {0}, rep, false);
    fill_coupled_report(P, rep);
  } else if (sch == MC_SCHEME_D || sch == MC_SCHEME_EX) {
    Table& T = upload_table(P, std::string(mixed ? "dm" : "d") + std::to_string(P->cur),
                            decoupled_parts(P, all, mixed));
    if (mixed) solve_systems_mixed(P, T, all, true);
    else solve_systems64(P, T, all, true);
    st = collect(P, all, all, rep, mixed);
  } else {
    // L: ascending index order, each continuum sees the new values of those before it;
    // U: descending order, new values of those after it.
    st = MC_OK;
    std::vector<int> order = all;
    if (sch == MC_SCHEME_U) std::reverse(order.begin(), order.end());
    for (size_t k = 0; k < order.size(); ++k) {
      const int c = order[k];
      std::vector<PartD> parts = decoupled_parts(P, {c}, mixed);
      for (size_t j = 0; j < k; ++j) parts[0].tsrc[order[j]] = P->cont[order[j]].ps[1 - P->cur];
      Table& T = upload_table(P, std::string(mixed ? "sm" : "s") + std::to_string(c) + "_" +
                                     std::to_string(P->cur), parts);
      if (mixed) solve_systems_mixed(P, T, {c}, true);
      else solve_systems64(P, T, {c}, true);
      mc_status s1 = collect(P, {c}, {c}, rep, mixed);
      if (s1 != MC_OK) {
        st = s1;
        break;
      }
    }
  }
  if (st == MC_OK) {
    P->cur ^= 1;
    P->step_count += 1;
  }
  return st;
}

}  // namespace mc

// ======================================================================================
// C ABI
// ======================================================================================
#define ABI_BEGIN try {
#define ABI_END(P)                                                                       \
  }                                                                                      \
  catch (const mc::Error& e) {                                                           \
    if (P) (P)->err = e.msg; else mc::g_thread_error = e.msg;                            \
    return e.st;                                                                         \
  }                                                                                      \
  catch (const std::exception& e) {                                                      \
    if (P) (P)->err = e.what(); else mc::g_thread_error = e.what();                      \
    return MC_EDEVICE;                                                                   \
  }

extern "C" {

mc_status mc_options_default(mc_options* o) {
  if (!o) return MC_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->scheme = MC_SCHEME_D;
  o->precision = MC_FP64;
  o->precond = MC_JACOBI;
  o->tol = 1e-10;
  o->max_iter = 20000;
  o->outer_tol = 1e-10;
  o->max_outer = 30;
  o->inner_tol = 1e-6;
  return MC_OK;
}

mc_status mc_create_problem(const mc_problem_desc* d, const mc_options* o, mc_problem** out) {
  if (!out) {
    mc::g_thread_error = "out is NULL";
    return MC_EINVAL;
  }
  *out = nullptr;
  if (!d) {
    mc::g_thread_error = "desc is NULL";
    return MC_EINVAL;
  }
  mc_options od;
  mc_options_default(&od);
  if (o) od = *o;
  mc_problem* P = new mc_problem();
  try {
    mc::create(P, *d, od);
  } catch (const mc::Error& e) {
    mc::g_thread_error = e.msg;
    mc_destroy(P);
    return e.st;
  } catch (const std::exception& e) {
    mc::g_thread_error = e.what();
    mc_destroy(P);
    return MC_EDEVICE;
  }
  *out = P;
  return MC_OK;
}

mc_status mc_destroy(mc_problem* P) {
  if (!P) return MC_OK;
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  for (auto& e : P->ev_free) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto& e : P->ev_pending) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  P->mem.release();
  if (P->h_counters) (void)hipHostFree(P->h_counters);
  if (P->h_sys) (void)hipHostFree(P->h_sys);
  if (P->own_stream && P->stream) (void)hipStreamDestroy(P->stream);
  delete P;
  return MC_OK;
}

mc_status mc_step(mc_problem* P, int32_t n_steps, mc_report* last) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (n_steps < 1) throw mc::Error{MC_EINVAL, "n_steps must be >= 1"};
  auto t0 = std::chrono::steady_clock::now();
  mc_report rep;
  std::memset(&rep, 0, sizeof(rep));
  rep.n_cont = P->ncont;
  rep.failed = -1;
  mc_status st = MC_OK;
  for (int k = 0; k < n_steps && st == MC_OK; ++k) st = mc::step_once(P, &rep);
  rep.step = P->step_count;
  rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (last) *last = rep;
  if (st != MC_OK) P->err = "solve failed in continuum " + std::to_string(rep.failed);
  return st;
  ABI_END(P)
}

mc_status mc_solve_continuum(mc_problem* P, int32_t alpha, const double* rhs, double* x,
                             mc_report* rep) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (alpha < 0 || alpha >= P->ncont) throw mc::Error{MC_EINVAL, "alpha out of range"};
  if (!rhs || !x) throw mc::Error{MC_EINVAL, "rhs and x must be device pointers"};
  if (P->opt.precision == MC_MIXED)
    throw mc::Error{MC_EINVAL, "mc_solve_continuum solves in FP64; set precision MC_FP64"};
  auto t0 = std::chrono::steady_clock::now();
  std::vector<PartD> parts = mc::decoupled_parts(P, {alpha}, false);
  parts[0].x = x;
  parts[0].x64 = x;
  parts[0].b = const_cast<double*>(rhs);
  mc::Table& T = mc::upload_table(P, "solve" + std::to_string(alpha), parts);
  mc::solve_systems64(P, T, {alpha}, false);
  mc_report r;
  std::memset(&r, 0, sizeof(r));
  r.n_cont = P->ncont;
  mc_status st = mc::collect(P, {alpha}, {alpha}, &r, false);
  r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  r.step = P->step_count;
  if (rep) *rep = r;
  return st;
  ABI_END(P)
}

mc_status mc_apply_continuum(mc_problem* P, int32_t alpha, const double* x, double* y) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (alpha < 0 || alpha >= P->ncont) throw mc::Error{MC_EINVAL, "alpha out of range"};
  if (!x || !y) throw mc::Error{MC_EINVAL, "x and y must be device pointers"};
  std::vector<PartD> parts = mc::decoupled_parts(P, {alpha}, false);
  parts[0].x = const_cast<double*>(x);
  parts[0].q = y;
  mc::Table& T = mc::upload_table(P, "apply" + std::to_string(alpha), parts);
  hipLaunchKernelGGL(mc::k_apply, dim3(T.nblocks), dim3(MC_BLOCK), 0, P->stream, T.parts,
                     T.tiles);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(P->stream));
  return MC_OK;
  ABI_END(P)
}

mc_status mc_apply_coupled(mc_problem* P, const double* x, double* y) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (!x || !y) throw mc::Error{MC_EINVAL, "x and y must be device pointers"};
  std::vector<PartD> parts = mc::coupled_parts(P);
  long off = 0;
  for (int c = 0; c < P->ncont; ++c) {
    parts[c].x = const_cast<double*>(x) + off;
    parts[c].q = y + off;
    off += P->cont[c].n;
  }
  mc::Table& T = mc::upload_table(P, "applyc", parts);
  hipLaunchKernelGGL(mc::k_apply, dim3(T.nblocks), dim3(MC_BLOCK), 0, P->stream, T.parts,
                     T.tiles);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(P->stream));
  return MC_OK;
  ABI_END(P)
}

mc_status mc_assemble_rhs(mc_problem* P, int32_t alpha, double* b) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (alpha < 0 || alpha >= P->ncont) throw mc::Error{MC_EINVAL, "alpha out of range"};
  if (!b) throw mc::Error{MC_EINVAL, "b must be a device pointer"};
  std::vector<PartD> parts = mc::decoupled_parts(P, {alpha}, false);
  parts[0].b = b;
  parts[0].x64 = P->cont[alpha].r;    // warm-start copy goes to scratch
  parts[0].coupled = 0;
  mc::Table& T = mc::upload_table(P, "rhs" + std::to_string(alpha), parts);
  hipLaunchKernelGGL(mc::k_rhs, dim3(T.nblocks), dim3(MC_BLOCK), 0, P->stream, T.parts,
                     T.tiles);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(P->stream));
  return MC_OK;
  ABI_END(P)
}

mc_status mc_get_state(mc_problem* P, int32_t alpha, double* out) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (alpha < 0 || alpha >= P->ncont || !out) throw mc::Error{MC_EINVAL, "bad argument"};
  HIPCHK(hipMemcpyAsync(out, P->cont[alpha].ps[P->cur], P->cont[alpha].n * sizeof(double),
                        hipMemcpyDeviceToHost, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  return MC_OK;
  ABI_END(P)
}

mc_status mc_set_state(mc_problem* P, int32_t alpha, const double* in) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (alpha < 0 || alpha >= P->ncont || !in) throw mc::Error{MC_EINVAL, "bad argument"};
  HIPCHK(hipMemcpyAsync(P->cont[alpha].ps[P->cur], in, P->cont[alpha].n * sizeof(double),
                        hipMemcpyHostToDevice, P->stream));
  HIPCHK(hipStreamSynchronize(P->stream));
  return MC_OK;
  ABI_END(P)
}

mc_status mc_set_options(mc_problem* P, const mc_options* o) {
  if (!P || !o) return MC_EINVAL;
  ABI_BEGIN
  std::string m = mc::validate_options(*o);
  if (!m.empty()) throw mc::Error{MC_EINVAL, m};
  const int ty = o->tile_rows > 0 ? o->tile_rows : 16;
  if (ty != P->ty) throw mc::Error{MC_EINVAL, "tile_rows cannot change after creation"};
  if (o->stream && o->stream != (void*)P->stream)
    throw mc::Error{MC_EINVAL, "the stream cannot change after creation"};
  const bool rebuild = (o->scheme == MC_SCHEME_EX) != (P->opt.scheme == MC_SCHEME_EX) ||
                       (o->precision != P->opt.precision) || (o->precond != P->opt.precond);
  P->opt = *o;
  P->opt.stream = P->stream;
  if (rebuild) mc::build_coefficients(P);
  P->tables.clear();
  return MC_OK;
  ABI_END(P)
}

mc_status mc_get_info(const mc_problem* P, mc_info* info) {
  if (!P || !info) return MC_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->n_cont = P->ncont;
  for (int c = 0; c < P->ncont && c < 3; ++c) info->sizes[c] = (int32_t)P->cont[c].n;
  info->device_bytes = (int64_t)P->mem.bytes;
  info->grid_tiles = P->ncont ? P->cont[0].tiles : 0;
  info->n_chains = P->nchains;
  return MC_OK;
}

const char* mc_last_error(const mc_problem* P) {
  if (P) return P->err.c_str();
  return mc::g_thread_error.c_str();
}

mc_status mc_profile(mc_problem* P, int32_t enable) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  HIPCHK(hipStreamSynchronize(P->stream));
  mc::prof_harvest(P);
  P->prof = enable != 0;
  if (enable) {
    P->prof_launch[0] = P->prof_launch[1] = 0;
    P->prof_ms[0] = P->prof_ms[1] = 0;
  }
  return MC_OK;
  ABI_END(P)
}

mc_status mc_profile_read(mc_problem* P, int32_t which, int64_t* launches, double* total_ms) {
  if (!P || which < 0 || which > 1) return MC_EINVAL;
  ABI_BEGIN
  HIPCHK(hipStreamSynchronize(P->stream));
  mc::prof_harvest(P);
  if (launches) *launches = P->prof_launch[which];
  if (total_ms) *total_ms = P->prof_ms[which];
  return MC_OK;
  ABI_END(P)
}

}  // extern "C"
