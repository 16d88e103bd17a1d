// Runtime of the MI355X multicontinuum library: device memory of a problem, coefficient
// setup, launch tables, PCG orchestration for every scheme and precision, batches of
// problems advanced by shared launches, and the C ABI.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <condition_variable>
#include <functional>
#include <thread>
#include <vector>

#include "../../include/mcdec.h"
#include "common.hpp"
#include "fine_view.hpp"
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

// Block IC(0) factors (grid) and the exact fracture solve are used by MC_BIC0 and MC_MG.
static inline bool ic_precond(int p) { return p == MC_BIC0 || p == MC_MG; }

static bool env_flag(const char* name, bool dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v) != 0;
}

static int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atoi(v);
}

// Coarse levels of at most this many cells form the small-level tail of a V-cycle
// (MCDEC_MG_TAIL overrides the size; the coarsest level is always in the tail).
// Most crossing cells a fracture graph's exact solve takes (MC_SCHUR_KMAX; the environment
// variable MCDEC_FRACTURE_EXACT_MAX lowers it, 0 = the two-level block preconditioner for
// every graph with crossings).  Beyond it the two-level block preconditioner takes over
// (MCDEC_FRACTURE_BLOCKS = 0 leaves the chains alone instead).
static bool fracture_blocks_on() { return env_int("MCDEC_FRACTURE_BLOCKS", 1) != 0; }

static int exact_crossing_max() {
  const int v = env_int("MCDEC_FRACTURE_EXACT_MAX", MC_SCHUR_KMAX);
  return std::min(MC_SCHUR_KMAX, std::max(0, v));
}

static long mg_tail_cells();

// The last level of a truncated V-cycle, above the small-level tail, smoothed once (its
// dominance reached MC_MG_DOMINANCE; MCDEC_MG_STOP_ONCE = 0 / 1 forces twice / once).
static bool stop_smoothed_once(const PartD& c) {
  if (c.mg_level == 0 || c.mg_next >= 0 || c.mg_inv != nullptr || (long)c.n <= mg_tail_cells())
    return false;
  const int f = env_int("MCDEC_MG_STOP_ONCE", -1);
  return f < 0 ? c.mg_once != 0 : f != 0;
}

static long mg_tail_cells() {
  static const long n = std::max(env_int("MCDEC_MG_TAIL", MC_MG_TAIL), MC_MG_COARSE);
  return n;
}

// Workgroups per launch over a continuum, for the operator tiling (fam 0) and for the
// update / init / residual tiling (fam 1).  A tuned choice (tiles per workgroup, recorded
// per size class by mc_autotune) wins; otherwise one workgroup per tile up to a cap, beyond
// which each workgroup takes a contiguous run of tiles, and with block IC(0) the grid update
// workgroups take four tiles (eight 64 x 16 blocks) so that all four wavefronts sweep.
// Depends only on the continuum's size, kind and solver configuration, so the reduction order
// of a system never depends on what else shares the launch.
static std::mutex g_tune_mu;
static std::map<std::vector<int>, int> g_tune;   // key -> tiles per workgroup

static int size_class(int ntiles) {
  int b = 0;
  while ((2L << b) <= ntiles) ++b;
  return b;   // floor(log2(ntiles))
}

static std::vector<int> tune_key(int ntiles, int kind, int fam, bool bic0, bool fp32) {
  return {kind, fam, bic0 ? 1 : 0, fp32 ? 1 : 0, size_class(ntiles)};
}

static int blocks_for(int ntiles, int kind, int fam, bool bic0, bool fp32) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(ntiles, kind, fam, bic0, fp32));
    if (it != g_tune.end()) return std::max(1, (ntiles + it->second - 1) / it->second);
  }
  // untuned defaults: a fracture graph gets one workgroup per tile (its chain solves are
  // latency-bound), the grid operator up to 2048 workgroups, the update with block IC(0)
  // four tiles per workgroup
  int cap;
  if (kind == PART_GRAPH) cap = env_int("MCDEC_GRAPH_BLOCKS", std::max(256, ntiles));
  else if (fam == 0) cap = env_int("MCDEC_GRID_BLOCKS_A", 2048);
  else cap = bic0 ? std::max(1, env_int("MCDEC_GRID_BLOCKS_B", (ntiles + 3) / 4))
                  : env_int("MCDEC_GRID_BLOCKS_A", 2048);
  return std::max(1, std::min(ntiles, std::max(cap, 1)));
}

// ------------------------------------------------------------------------------------
// device buffers
// ------------------------------------------------------------------------------------
struct DevArena {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  // the caller's allocator (mc_options.dev_alloc / dev_free), fixed when the owner is created
  void* (*hook_alloc)(size_t, void*) = nullptr;
  void (*hook_free)(void*, void*) = nullptr;
  void* hook_ctx = nullptr;
  void use_hooks(const mc_options& o) {
    hook_alloc = o.dev_alloc;
    hook_free = o.dev_free;
    hook_ctx = o.alloc_ctx;
  }
  template <class T>
  T* alloc(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    if (hook_alloc) {
      p = hook_alloc(n * sizeof(T), hook_ctx);
      if (!p)
        throw Error{MC_ENOMEM, "dev_alloc of " + std::to_string(n * sizeof(T)) + " bytes failed"};
      if ((uintptr_t)p % 256 != 0) {
        hook_free(p, hook_ctx);
        throw Error{MC_EINVAL, "dev_alloc returned memory not aligned to 256 bytes"};
      }
    } else {
      hipError_t e = hipMalloc(&p, n * sizeof(T));
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{MC_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed"};
      }
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
    for (void* p : ptrs) {
      if (hook_free) hook_free(p, hook_ctx);
      else (void)hipFree(p);
    }
    ptrs.clear();
    bytes = 0;
  }
};

// ------------------------------------------------------------------------------------
// launch tables
// ------------------------------------------------------------------------------------
// Parts in device memory and, per tiling and part kind (grid / graph), the list of tiles in
// launch order.  Kernels are instantiated per kind, so a launch covers the tiles of one
// kind only.  Graphs of captured PCG iteration chunks over this table are cached with it.
struct Table {
  PartD* parts = nullptr;
  int pcap = 0;
  // [tiling][kind]; tiling 0: operator, 1: update / init / residual, 2: crossing-cell rows
  Tile* tiles[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  int nblk[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  int cap[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  int nparts = 0;
  bool has_blocks = false;   // a fracture part with the two-level block preconditioner
  std::vector<PartD> hparts;
  std::vector<int> htil;                      // tiles and the three workgroup counts per part
  // multigrid tile lists per level: [0] restriction into the level when it starts the tail,
  // [1] restriction into the level with its pre-smoothing (the other coarse levels), [2] the
  // small levels from this one down in one workgroup, [3] post-smoothing (level 0: the final
  // one, writing partial slots)
  struct List {
    Tile* t = nullptr;
    int n = 0, cap = 0;
  };
  std::vector<std::array<List, 4>> mg;
  bool mg_fused = false;   // the finest parts' update kernels restrict into level 1
  std::map<long, hipGraphExec_t> graphs;
};

static void drop_graphs(Table& T) {
  for (auto& g : T.graphs) (void)hipGraphExecDestroy(g.second);
  T.graphs.clear();
}

// Tiling of one part: its tiles and the workgroups of its operator / update launches and of
// its crossing-cell product (one workgroup per MC_SCHUR_ROWS rows).
struct PartTiling {
  int tiles;
  int blocks[3];
};

static bool table_matches(const Table& T, const std::vector<PartD>& parts,
                          const std::vector<PartTiling>& til) {
  if (T.hparts.size() != parts.size() || T.htil.size() != 4 * til.size()) return false;
  if (std::memcmp(T.hparts.data(), parts.data(), parts.size() * sizeof(PartD)) != 0) return false;
  for (size_t i = 0; i < til.size(); ++i)
    if (T.htil[4 * i] != til[i].tiles || T.htil[4 * i + 1] != til[i].blocks[0] ||
        T.htil[4 * i + 2] != til[i].blocks[1] || T.htil[4 * i + 3] != til[i].blocks[2])
      return false;
  return true;
}

// Appends the workgroup tiles of part `pi` for tiling `fam` (0 operator, 1 update, 2
// crossing-cell rows) to `tiles`: workgroup b of the part takes tiles [b*nt/nb,
// (b+1)*nt/nb); in launch order, die j of the 8 XCDs (round-robin dispatch) receives a
// contiguous band of workgroups.
static void part_tiles(const PartD& q, int pi, const PartTiling& til, int fam, bool xcd,
                       std::vector<Tile>& tiles) {
  const int nb = til.blocks[fam];
  if (nb == 0 || q.mg_level > 0 || (fam == 2 && q.kind == PART_GRID)) return;
  const int nt = fam == 2 ? nb : til.tiles;
  const int slot0 = fam == 0 ? q.slot0A : (fam == 1 ? q.slot0B : q.slotS);
  std::vector<int> ord = xcd_order(nb, xcd ? 8 : 1);
  for (int b : ord) {
    if (b < 0) {
      tiles.push_back(Tile{-1, 0, 0, 0, 0});
      continue;
    }
    const int t0 = (int)((long)b * nt / nb), t1 = (int)((long)(b + 1) * nt / nb);
    tiles.push_back(Tile{pi, slot0 + b, t0, t1, q.sys});
  }
  while (xcd && tiles.size() % 8) tiles.push_back(Tile{-1, 0, 0, 0, 0});
}

// Writes parts and their tile lists into T (reusing its device buffers when large enough).
static void fill_table(Table& T, DevArena& M, hipStream_t s, std::vector<PartD> parts,
                       const std::vector<PartTiling>& til) {
  drop_graphs(T);
  if (!T.parts || T.pcap < (int)parts.size()) {
    T.pcap = (int)parts.size() + 2;
    T.parts = M.alloc<PartD>(T.pcap);
  }
  HIPCHK(hipMemcpyAsync(T.parts, parts.data(), parts.size() * sizeof(PartD),
                        hipMemcpyHostToDevice, s));
  const bool xcd = env_flag("MCDEC_XCD", true);
  std::vector<Tile> kept[3][2];
  for (int fam = 0; fam < 3; ++fam)
    for (int kind = 0; kind < 2; ++kind) {
      std::vector<Tile>& tiles = kept[fam][kind];
      for (int pi = 0; pi < (int)parts.size(); ++pi)
        if (parts[pi].kind == kind) part_tiles(parts[pi], pi, til[pi], fam, xcd, tiles);
      if (!tiles.empty() && (!T.tiles[fam][kind] || T.cap[fam][kind] < (int)tiles.size())) {
        T.cap[fam][kind] = (int)tiles.size() + 8;
        T.tiles[fam][kind] = M.alloc<Tile>(T.cap[fam][kind]);
      }
      if (!tiles.empty())
        HIPCHK(hipMemcpyAsync(T.tiles[fam][kind], tiles.data(), tiles.size() * sizeof(Tile),
                              hipMemcpyHostToDevice, s));
      T.nblk[fam][kind] = (int)tiles.size();
    }
  // multigrid lists
  T.mg_fused = false;
  for (auto& q : parts) T.mg_fused = T.mg_fused || (q.kind == PART_GRID && q.mg_fuse);
  int L = 0;
  for (auto& q : parts)
    if (q.kind == PART_GRID && (q.mg_next >= 0 || q.mg_level > 0)) L = std::max(L, q.mg_level + 1);
  if ((int)T.mg.size() < L) T.mg.resize(L);
  std::vector<std::vector<Tile>> mgv(4 * std::max(L, 1));
  // a coarse level of at most MC_MG_TAIL cells belongs to its chain's tail (a suffix of the
  // levels), which one workgroup runs from the tail's first level down and back up
  // (MCDEC_MG_TAIL overrides the size; the coarsest level is always in the tail)
  const long tail_n = mg_tail_cells();
  auto in_tail = [&](const PartD& q) { return q.mg_level > 0 && (long)q.n <= tail_n; };
  for (int pi = 0; pi < (int)parts.size(); ++pi) {
    const PartD& q = parts[pi];
    if (q.kind != PART_GRID || (q.mg_next < 0 && q.mg_level == 0)) continue;
    const int l = q.mg_level;
    const int nt = (int)(cdiv(q.nx, MC_TX) * cdiv(q.ny, MC_TY));
    auto add = [&](int op, int nb, int ntile, int slot0) {
      std::vector<Tile>& v = mgv[4 * l + op];
      for (int b = 0; b < nb; ++b)
        v.push_back(Tile{pi, slot0 + b, (int)((long)b * ntile / nb),
                         (int)((long)(b + 1) * ntile / nb), q.sys});
    };
    bool tail_start = false;
    if (l > 0) {
      if (q.mg_prev < 0 || q.mg_prev >= (int)parts.size())
        throw Error{MC_EDEVICE, "multigrid level without a finer level"};
      const PartD& f = parts[q.mg_prev];
      if (in_tail(q) && in_tail(f)) continue;          // run inside its tail's workgroup
      // the last level is either the coarsest (dense inverse, solved in the tail) or a
      // truncated level above the tail (smoothed twice, no coarser correction)
      if (q.mg_next < 0 && in_tail(q) != (q.mg_inv != nullptr))
        throw Error{MC_EDEVICE, "last multigrid level does not match the small-level tail"};
      tail_start = in_tail(q);
      if (tail_start) {                                // restriction into l: finer tiles
        const int ntf = (int)(cdiv(f.nx, MC_TX) * cdiv(f.ny, MC_TY));
        add(0, ntf, ntf, 0);
      }
    }
    if (tail_start) {
      add(2, 1, 1, 0);
      continue;
    }
    // coarse levels: ranges of IC(0) blocks (MC_ICYC rows), one per wavefront
    const int units = nt * (MC_TY / MC_ICYC);
    if (l > 0) add(1, (int)cdiv(units, 4), units, 0);  // restriction + pre-smoothing
    if (l == 0) add(3, til[pi].blocks[1], nt, q.mg_slot);
    else if (!stop_smoothed_once(q))
      add(3, (int)cdiv(units, 4), units, 0);           // post-smoothing
  }
  for (int l = 0; l < L; ++l)
    for (int op = 0; op < 4; ++op) {
      Table::List& li = T.mg[l][op];
      const std::vector<Tile>& v = mgv[4 * l + op];
      if (!v.empty() && (!li.t || li.cap < (int)v.size())) {
        li.cap = (int)v.size() + 8;
        li.t = M.alloc<Tile>(li.cap);
      }
      if (!v.empty())
        HIPCHK(hipMemcpyAsync(li.t, v.data(), v.size() * sizeof(Tile), hipMemcpyHostToDevice, s));
      li.n = (int)v.size();
    }
  for (int l = L; l < (int)T.mg.size(); ++l)
    for (auto& li : T.mg[l]) li.n = 0;
  HIPCHK(hipStreamSynchronize(s));   // host vectors die at return
  T.nparts = (int)parts.size();
  T.has_blocks = std::any_of(parts.begin(), parts.end(), [](const PartD& q) { return q.blocks; });
  T.hparts = std::move(parts);
  T.htil.clear();
  for (auto& t : til) {
    T.htil.push_back(t.tiles);
    T.htil.push_back(t.blocks[0]);
    T.htil.push_back(t.blocks[1]);
    T.htil.push_back(t.blocks[2]);
  }
}

// A coarse level of a grid continuum's V-cycle (level 0 is the continuum itself).
struct MgLevel {
  int nx = 0, ny = 0, tiles = 0;
  long n = 0;
  bool coarsest = false;
  bool smooth_once = false;   // last level, truncated where its row sums reach MC_MG_DOMINANCE
                              // times its face conductances: one block IC(0) sweep
  double *diag = nullptr, *tx = nullptr, *ty = nullptr, *fdinv = nullptr;
  float *diag32 = nullptr, *tx32 = nullptr, *ty32 = nullptr, *fdinv32 = nullptr;
  double *r = nullptr, *zp = nullptr, *z = nullptr;
  float *r32 = nullptr, *zp32 = nullptr, *z32 = nullptr;
  double* inv = nullptr;   // coarsest: dense inverse of the level operator
  float* inv32 = nullptr;
};

struct Cont {  // one continuum
  int kind;    // PART_GRID / PART_GRAPH
  long n;
  int tiles;      // tiles of its part
  int blocks[3];  // workgroups (and partial slots) per launch: operator / update tiling /
                  // crossing-cell product (graph with crossing cells only)
  // FP64 coefficients
  double *diag = nullptr, *tx = nullptr, *ty = nullptr, *F = nullptr, *val = nullptr,
         *mt = nullptr;
  float *diag32 = nullptr, *tx32 = nullptr, *ty32 = nullptr, *val32 = nullptr;
  double* tz = nullptr;      // (3-D grid) conductance to the cell above
  float* tz32 = nullptr;
  double* fdinv = nullptr;   // block IC(0) inverse pivots
  float* fdinv32 = nullptr;
  double* cT = nullptr;      // (graph) block couplings to the previous cell
  float* cT32 = nullptr;
  // (graph) exact solve through the crossing cells
  int K = 0;
  int *xcells = nullptr, *xtile = nullptr, *xlr = nullptr;
  double *cl = nullptr, *cr = nullptr, *cxl = nullptr, *cxr = nullptr, *sinv = nullptr;
  float *cl32 = nullptr, *cr32 = nullptr, *sinv32 = nullptr;
  double *gX = nullptr, *zX = nullptr;
  float *gX32 = nullptr, *zX32 = nullptr;
  // (graph) two-level block preconditioner in place of the exact solve (K = blocks)
  bool fblocks = false;
  int fmode = 0;   // preconditioner the K-sized arrays above were made for: 1 exact, 2 blocks
  int* bnode = nullptr;
  float* binv = nullptr;
  // (grid) multigrid levels 1.. and the finest level's pre-smoothed solution
  std::vector<MgLevel> mg;
  bool mg_on = false;
  double* zpre = nullptr;
  float* zpre32 = nullptr;
  double* mg_edz = nullptr;   // block edges of the fused restriction into level 1
  float* mg_edt = nullptr;
  // state and PCG vectors
  double* ps[2] = {nullptr, nullptr};
  double* hx[3] = {nullptr, nullptr, nullptr};   // (adaptive warm start) p^{n-3}, p^{n-4}, p^{n-5}
  double *b = nullptr, *r = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr, *z = nullptr;
  float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *p232 = nullptr, *q32 = nullptr,
        *z32 = nullptr;
  double mtau = 0, tconst = 0;
  int has_t = 1;
};

// ------------------------------------------------------------------------------------
// execution context: streams, system records, polling, graphs, kernel timing
// ------------------------------------------------------------------------------------
struct Exec {
  mc_options opt{};
  hipStream_t stream = nullptr;    // main stream (grid group, coupled systems, setup)
  hipStream_t stream2 = nullptr;   // fracture group of a decoupled solve (created on first use)
  // CU-partitioned streams of a decoupled solve (see create_cu_streams): the fracture group
  // gets its own compute units
  hipStream_t stream_grid = nullptr, stream_frac = nullptr;
  bool own_stream = false, side = false;
  bool auto_cus = false;           // a single problem's executor (batches share all units)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_poll[2] = {nullptr, nullptr};
  SysState* sys = nullptr;         // device system records
  SysState* h_sys = nullptr;       // pinned mirror
  int nsys = 0, sys_cap = 0;
  bool graphs = true;              // replay captured iteration chunks
  std::mutex graph_mu;
  // kernel timing
  bool prof = false;
  struct Ev { hipEvent_t a, b; int which; };
  std::vector<Ev> ev_free, ev_pending;
  // [0] grid operator, [1] grid update, [2] finest V-cycle post-smoothing kernel, and the
  // V-cycle's coarse kernels over all levels: [3] restriction with pre-smoothing, [4]
  // coarse correction with post-smoothing, [5] small-level tail, [6] restriction into the
  // tail.  A V-cycle is timed whole when its finest post-smoothing is due for a sample.
  static constexpr int NPROF = 7;
  long prof_launch[NPROF] = {0, 0, 0, 0, 0, 0, 0};
  double prof_ms[NPROF] = {0, 0, 0, 0, 0, 0, 0};
  long prof_count[NPROF] = {0, 0, 0, 0, 0, 0, 0};
  std::vector<float> prof_samples[NPROF];   // every sampled duration (ms)
  int prof_every = 8;
  // host threads that drive the extra groups of a solve (kept for the problem's lifetime)
  struct Worker {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    std::function<void()> job;
    bool quit = false;
  };
  std::vector<std::unique_ptr<Worker>> workers;
};

static void worker_loop(Exec::Worker* w) {
  std::unique_lock<std::mutex> lk(w->mu);
  for (;;) {
    w->cv.wait(lk, [&] { return w->quit || (bool)w->job; });
    if (w->quit) return;
    std::function<void()> job = std::move(w->job);
    w->job = nullptr;
    lk.unlock();
    job();
    lk.lock();
    w->cv.notify_all();
  }
}

// Runs job(k) for k = 1..n-1 on the Exec's worker threads and job(0) on the caller, and
// returns once all have finished.
static void run_on_workers(Exec& X, int n, const std::function<void(int)>& job) {
  while ((int)X.workers.size() < n - 1) {
    X.workers.emplace_back(new Exec::Worker());
    Exec::Worker* w = X.workers.back().get();
    w->th = std::thread(worker_loop, w);
  }
  std::vector<bool> done(n, false);
  std::mutex dm;
  std::condition_variable dcv;
  for (int k = 1; k < n; ++k) {
    Exec::Worker* w = X.workers[k - 1].get();
    std::lock_guard<std::mutex> lk(w->mu);
    w->job = [&, k] {
      job(k);
      std::lock_guard<std::mutex> g(dm);
      done[k] = true;
      dcv.notify_all();
    };
    w->cv.notify_all();
  }
  job(0);
  std::unique_lock<std::mutex> lk(dm);
  dcv.wait(lk, [&] {
    for (int k = 1; k < n; ++k)
      if (!done[k]) return false;
    return true;
  });
}

static void exec_init(Exec& X, void* user_stream) {
  if (user_stream) {
    X.stream = (hipStream_t)user_stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&X.stream, hipStreamNonBlocking));
    X.own_stream = true;
  }
  HIPCHK(hipEventCreateWithFlags(&X.ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&X.ev_join, hipEventDisableTiming));
  for (auto& e : X.ev_poll) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  X.graphs = env_flag("MCDEC_GRAPHS", true);
}

// CU partition of a split solve (grid and fracture groups on their own streams): the
// fracture group gets groups of 8 consecutive compute units spread evenly over the chip, the
// grid group the rest (the runtime refused masks of single scattered units here).  By
// default a problem whose fracture takes the two-level block preconditioner (a
// latency-bound solve of many more iterations than the grid's, slowed severalfold by the
// grid kernels' traffic when they share every unit) gets a quarter of the units, one group
// per 32, i.e. one per die of the chip; other solves and batches share all units.
// MCDEC_FRAC_CUS sets the fracture's units (rounded up to a multiple of 8; 0 = no
// partition).  Left out if the masked streams cannot be created.
static void create_cu_streams(Exec& X, bool frac_blocks) {
  int dev = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  constexpr int G = 8;
  const int ngroups = ncu / G;
  const int dflt = X.auto_cus && frac_blocks ? ncu / 4 : 0;
  const int fg = (env_int("MCDEC_FRAC_CUS", dflt) + G - 1) / G;   // groups for the fracture
  if (fg <= 0 || fg >= ngroups) return;
  const int words = (ncu + 31) / 32;
  std::vector<uint32_t> fm(words, 0u), gm(words, 0u);
  int taken = 0;
  for (int gi = 0; gi < ngroups; ++gi) {
    // group gi goes to the fracture when it starts a new 1/fg share of the groups
    const bool frac = taken < fg && (long)gi * fg >= (long)taken * ngroups;
    if (frac) ++taken;
    for (int c = gi * G; c < gi * G + G; ++c) (frac ? fm : gm)[c / 32] |= 1u << (c % 32);
  }
  for (int c = ngroups * G; c < ncu; ++c) gm[c / 32] |= 1u << (c % 32);
  hipStream_t a = nullptr, b = nullptr;
  if (hipExtStreamCreateWithCUMask(&a, words, gm.data()) != hipSuccess ||
      hipExtStreamCreateWithCUMask(&b, words, fm.data()) != hipSuccess) {
    (void)hipGetLastError();
    if (a) (void)hipStreamDestroy(a);
    if (b) (void)hipStreamDestroy(b);
    return;
  }
  X.stream_grid = a;
  X.stream_frac = b;
}

static void exec_side_streams(Exec& X, bool frac_blocks) {
  if (X.side) return;
  HIPCHK(hipStreamCreateWithFlags(&X.stream2, hipStreamNonBlocking));
  create_cu_streams(X, frac_blocks);
  X.side = true;
}

// Device and pinned records for n systems; returns true if they moved (graphs that captured
// the old address must then be dropped).
static bool exec_sys_capacity(Exec& X, int n) {
  X.nsys = n;
  if (n <= X.sys_cap) return false;
  if (X.sys) {
    HIPCHK(hipStreamSynchronize(X.stream));
    (void)hipFree(X.sys);
    X.sys = nullptr;
  }
  if (X.h_sys) {
    (void)hipHostFree(X.h_sys);
    X.h_sys = nullptr;
  }
  const int cap = std::max(n, 2 * X.sys_cap);
  X.sys_cap = 0;
  if (hipMalloc((void**)&X.sys, cap * sizeof(SysState)) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{MC_ENOMEM, "hipMalloc of the system records failed"};
  }
  HIPCHK(hipHostMalloc((void**)&X.h_sys, cap * sizeof(SysState), hipHostMallocDefault));
  std::memset(X.h_sys, 0, cap * sizeof(SysState));
  X.sys_cap = cap;
  return true;
}

static void exec_release(Exec& X) {
  for (auto& w : X.workers) {
    {
      std::lock_guard<std::mutex> lk(w->mu);
      w->quit = true;
    }
    w->cv.notify_all();
    if (w->th.joinable()) w->th.join();
  }
  X.workers.clear();
  if (X.stream) (void)hipStreamSynchronize(X.stream);
  for (hipStream_t st : {X.stream2, X.stream_grid, X.stream_frac})
    if (st) (void)hipStreamSynchronize(st);
  for (auto& e : X.ev_free) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto& e : X.ev_pending) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  X.ev_free.clear();
  X.ev_pending.clear();
  if (X.sys) (void)hipFree(X.sys);
  if (X.h_sys) (void)hipHostFree(X.h_sys);
  X.sys = nullptr;
  X.h_sys = nullptr;
  if (X.ev_fork) (void)hipEventDestroy(X.ev_fork);
  if (X.ev_join) (void)hipEventDestroy(X.ev_join);
  for (auto e : X.ev_poll)
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t st : {X.stream2, X.stream_grid, X.stream_frac})
    if (st) (void)hipStreamDestroy(st);
  if (X.own_stream && X.stream) (void)hipStreamDestroy(X.stream);
  X.stream = X.stream2 = X.stream_grid = X.stream_frac = nullptr;
}

}  // namespace mc

using namespace mc;

struct mc_problem {
  mc_problem_desc d{};   // scalars only (array pointers are not kept)
  Exec X;                // X.opt: the problem's options
  int ncont = 0, n_omega = 0, nf = 0, ne = 0;
  long ncell = 0;
  int nz = 1;            // planes of a 3-D grid (1: 2-D)
  int device = 0;        // HIP device current at creation
  DevArena mem;
  std::vector<Cont> cont;
  // inputs kept on the device (for re-setup)
  double* k[2] = {nullptr, nullptr};
  double* src[3] = {nullptr, nullptr, nullptr};
  double* well_q = nullptr;   // [nf] or null
  double* well_p = nullptr;   // [nf] or null (only with well_q)
  int *host = nullptr, *rowptr = nullptr, *col = nullptr, *eidx = nullptr, *hptr = nullptr,
      *hidx = nullptr, *chain_ptr = nullptr, *gtile = nullptr;
  GraphCSR gh;                       // host copies of the fracture graph structure
  std::vector<int> host_h;           // host copy of the fracture cells' host cells
  std::vector<int> chains_h, gtile_h;
  int K_all = 0;                     // crossing cells of the fracture graph
  int nb_frac = 0;                   // blocks of its two-level preconditioner (if K_all > 0)
  double *flen = nullptr, *edge_d = nullptr, *sigma_f = nullptr;
  int nchains = 0, ngtiles = 0;
  // systems: 0..ncont-1 decoupled per continuum, ncont = coupled; their partial-sum slots
  std::vector<double*> partA, partB;
  int cur = 0;                   // state ping-pong index
  long step_count = 0;
  int hist = 0;   // consecutive layers computed since creation / the last state change: with
                  // hist >= 1 the other state buffer holds the layer before the current one
  std::map<std::string, Table> tables;
  std::string err;
};

// Many problems advanced together: every launch covers the tiles of all of them.
struct mc_batch {
  Exec X;          // X.opt: the batch's solver options
  DevArena mem;    // launch tables
  Table tab[2];    // the two most recent compositions (consecutive steps alternate state buffers)
  int lru = 0;
  std::string err;
};

namespace mc {

static void fail(const std::string& m) { throw Error{MC_EINVAL, m}; }

static void clear_tables(mc_problem* P) {
  for (auto& t : P->tables) drop_graphs(t.second);
  P->tables.clear();
}

// Omega-Omega transfer coefficient of one cell pair: sigma_omega |cell| (h^2, or h^3 in 3-D).
static double omega_transfer(const mc_problem* P) {
  const double h = P->d.h;
  return P->nz > 1 ? P->d.sigma_omega * h * h * h : P->d.sigma_omega * h * h;
}

// ------------------------------------------------------------------------------------
// parts of a problem
// ------------------------------------------------------------------------------------
static PartD base_part(mc_problem* P, int c, int sys, int slot0A, int slot0B, bool fp32) {
  Cont& C = P->cont[c];
  PartD q;
  std::memset(&q, 0, sizeof(q));
  q.kind = C.kind;
  q.sys = sys;
  q.cont = c;
  q.n = (int)C.n;
  q.nx = P->d.nx;
  q.ny = P->d.ny * P->nz;   // 3-D: the planes' rows stacked
  q.tiles_x = (int)cdiv(P->d.nx, MC_TX);
  q.plane = P->nz > 1 && C.kind == PART_GRID ? (long)P->d.nx * P->d.ny : 0;
  q.slot0A = slot0A;
  q.slot0B = slot0B;
  q.ex = P->X.opt.scheme == MC_SCHEME_EX;
  q.extrap = P->X.opt.warm_start;   // WS_* (the history depth comes from the system record)
  for (int k = 0; k < 3; ++k) q.hx[k] = C.hx[k];
  q.has_t = C.has_t;
  q.n_omega = P->n_omega;
  q.other = -1;
  q.frac = -1;
  q.omg[0] = q.omg[1] = -1;
  q.tconst = C.tconst;
  q.mtau = C.mtau;
  q.s12 = P->n_omega == 2 ? omega_transfer(P) : 0.0;
  q.diag = C.diag;
  q.tx = C.tx;
  q.ty = C.ty;
  q.tz = C.tz;
  q.tz32 = C.tz32;
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
  q.gtile = P->gtile;
  q.cT = C.cT;
  q.cT32 = C.cT32;
  q.K = C.K;
  q.slotS = slot0B + C.blocks[1];
  q.xcells = C.xcells;
  q.xtile = C.xtile;
  q.xlr = C.xlr;
  q.cl = C.cl;
  q.cr = C.cr;
  q.cl32 = C.cl32;
  q.cr32 = C.cr32;
  q.cxl = C.cxl;
  q.cxr = C.cxr;
  q.sinv = C.sinv;
  q.sinv32 = C.sinv32;
  q.blocks = C.fblocks ? 1 : 0;
  q.bnode = C.bnode;
  q.binv = C.binv;
  q.gX = fp32 ? (void*)C.gX32 : (void*)C.gX;
  q.zX = fp32 ? (void*)C.zX32 : (void*)C.zX;
  q.mg_level = 0;
  q.mg_next = -1;   // set by add_mg_levels when the continuum has a V-cycle
  q.mg_prev = -1;
  q.mg_slot = slot0B + C.blocks[1];
  q.mg_zp = fp32 ? (void*)C.zpre32 : (void*)C.zpre;
  q.fp32 = fp32 ? 1 : 0;
  q.mg_edz = C.mg_edz;
  q.mg_edt = C.mg_edt;
  if (C.kind == PART_GRID) {
    q.hptr = P->nf ? P->hptr : nullptr;
    q.hidx = P->hidx;
    q.hsig = P->nf ? P->sigma_f + (long)c * P->nf : nullptr;
  } else {
    q.host = P->host;
    q.fsig0 = P->sigma_f;
    q.fsig1 = P->n_omega > 1 ? P->sigma_f + P->nf : nullptr;
  }
  q.r64 = C.r;   // FP64 residual of the refinement (the FP64 PCG vector r is idle then)
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

// Fills the copies of neighbouring V-cycle levels' fields in every level part (after the
// parts' own pointers are final: a caller may have redirected r or z of a finest part).
static void link_mg(std::vector<PartD>& parts) {
  // the update kernel forms the finest level's share of the restriction into level 1 when
  // that level is smoothed by its own kernel, in FP64 solves (an FP32 update kernel moves half
  // the bytes, and its added latency outweighs the bytes it saves); MCDEC_MG_FUSE=0: the
  // restriction kernel does it all
  const bool fuse = env_flag("MCDEC_MG_FUSE", true);
  for (auto& q : parts) {
    if (q.kind != PART_GRID) continue;
    const int n = (int)parts.size();
    if ((q.mg_next >= n) || (q.mg_level > 0 && (q.mg_prev < 0 || q.mg_prev >= n)))
      throw Error{MC_EDEVICE, "multigrid level link outside the launch table"};
    q.mg_fuse = 0;
    if (q.mg_next >= 0) {
      const PartD& c = parts[q.mg_next];
      q.mg_e = stop_smoothed_once(c) ? c.mg_zp : c.mg_z;   // once: its pre-smoothed z_p
      q.mg_cnx = c.nx;
      q.mg_fuse = fuse && !q.fp32 && q.mg_level == 0 && q.plane == 0 && q.mg_edz &&
                  (long)c.n > mg_tail_cells();
    }
    if (q.mg_level > 0) {
      const PartD& f = parts[q.mg_prev];
      q.mg_fnx = f.nx;
      q.mg_fny = f.ny;
      q.mg_ftiles_x = f.tiles_x;
      q.mg_fhas_t = f.has_t;
      q.mg_ftc = f.tconst;
      q.mg_fr = f.mg_level == 0 ? f.r : f.mg_r;
      q.mg_fzp = f.mg_zp;
      q.mg_fd32 = f.diag32;
      q.mg_ftx32 = f.tx32;
      q.mg_fty32 = f.ty32;
      q.mg_fedz = f.mg_edz;
      q.mg_fedt = f.mg_edt;
    }
  }
}

static PartTiling tiling_of(const mc_problem* P, int c) {
  const Cont& C = P->cont[c];
  return PartTiling{C.tiles, {C.blocks[0], C.blocks[1], C.blocks[2]}};
}

static Table& upload_table(mc_problem* P, const std::string& key, std::vector<PartD> parts) {
  link_mg(parts);
  std::vector<PartTiling> til;
  for (auto& q : parts) til.push_back(tiling_of(P, q.cont));
  Table& T = P->tables[key];
  if (table_matches(T, parts, til)) return T;
  fill_table(T, P->mem, P->X.stream, std::move(parts), til);
  return T;
}

// Appends the coarse levels of the V-cycle of grid part parts[i] (a continuum of P) and
// links them to it (links are launch-table indices: vector index + base); nothing when the
// option is off or the grid has no coarse level.
static void add_mg_levels(mc_problem* P, std::vector<PartD>& parts, int i, bool fp32,
                          int base = 0) {
  const Cont& C = P->cont[parts[i].cont];
  if (P->X.opt.precond != MC_MG || C.kind != PART_GRID || !C.mg_on) return;
  int prev = i;
  for (size_t l = 0; l < C.mg.size(); ++l) {
    const MgLevel& L = C.mg[l];
    PartD q;
    std::memset(&q, 0, sizeof(q));
    q.kind = PART_GRID;
    q.sys = parts[i].sys;
    q.cont = parts[i].cont;
    q.n = (int)L.n;
    q.nx = L.nx;
    q.ny = L.ny;
    q.tiles_x = (int)cdiv(L.nx, MC_TX);
    q.has_t = 1;
    q.other = -1;
    q.frac = -1;
    q.omg[0] = q.omg[1] = -1;
    q.diag = L.diag;
    q.tx = L.tx;
    q.ty = L.ty;
    q.diag32 = L.diag32;
    q.tx32 = L.tx32;
    q.ty32 = L.ty32;
    q.fdinv = L.fdinv;
    q.fdinv32 = L.fdinv32;
    q.mg_level = (int)l + 1;
    q.mg_once = L.smooth_once && l + 1 == C.mg.size() ? 1 : 0;
    q.mg_prev = base + prev;
    q.mg_next = -1;
    q.mg_inv = L.coarsest ? L.inv : nullptr;
    q.mg_inv32 = L.coarsest ? L.inv32 : nullptr;
    q.mg_r = fp32 ? (void*)L.r32 : (void*)L.r;
    q.mg_zp = fp32 ? (void*)L.zp32 : (void*)L.zp;
    q.mg_z = fp32 ? (void*)L.z32 : (void*)L.z;
    const int idx = (int)parts.size();
    parts[prev].mg_next = base + idx;
    parts.push_back(q);
    prev = idx;
  }
}

// Parts of the decoupled systems of continua `conts` (system index = continuum index), with
// the V-cycle levels appended after them unless `with_mg` is false.
static std::vector<PartD> decoupled_parts(mc_problem* P, const std::vector<int>& conts,
                                          bool fp32, bool with_mg = true) {
  std::vector<PartD> parts;
  for (int c : conts) parts.push_back(base_part(P, c, c, 0, 0, fp32));
  if (with_mg)
    for (int i = 0, n = (int)parts.size(); i < n; ++i) add_mg_levels(P, parts, i, fp32);
  return parts;
}

// Parts of the coupled system `sysI` of a problem (the continua, then any V-cycle levels);
// cross-part references are indices into the returned vector plus `base` (the position of
// its first part in the launch table).
static std::vector<PartD> coupled_parts(mc_problem* P, int sysI, int base) {
  std::vector<PartD> parts;
  int slotA = 0, slotB = 0;
  for (int c = 0; c < P->ncont; ++c) {
    PartD q = base_part(P, c, sysI, slotA, slotB, false);
    slotA += P->cont[c].blocks[0];
    slotB += P->cont[c].blocks[1] + P->cont[c].blocks[2];
    q.coupled = 1;
    if (q.blocks) {   // the coupled system keeps the chain solves of the fracture block (the
      q.blocks = 0;   // two-level one did not lower its iterations); its crossing-cell
      q.K = 0;        // workgroups then add nothing
    }
    parts.push_back(q);
  }
  for (int c = 0; c < P->ncont; ++c) {
    if (c < P->n_omega) {
      parts[c].other = P->n_omega == 2 ? base + 1 - c : -1;
      parts[c].frac = P->nf ? base + P->n_omega : -1;
    } else {
      parts[c].omg[0] = base;
      parts[c].omg[1] = P->n_omega > 1 ? base + 1 : -1;
    }
  }
  for (int c = 0; c < P->ncont; ++c) add_mg_levels(P, parts, c, false, base);
  return parts;
}

// ------------------------------------------------------------------------------------
// setup
// ------------------------------------------------------------------------------------
static std::mutex g_blas_mu;
static rocblas_handle g_blas = nullptr;

// In place: the K x K SPD matrix S (column-major, device) -> S^-1 (full, symmetric), by a
// Cholesky factorization and its inverse (rocSOLVER potrf, potri) and a copy of the lower
// triangle to the upper one.  Runs once per problem at setup.
static void invert_spd(double* S, int K, hipStream_t s, int lda = 0) {
  if (lda < K) lda = K;
  std::lock_guard<std::mutex> lk(g_blas_mu);
  if (!g_blas && rocblas_create_handle(&g_blas) != rocblas_status_success) {
    g_blas = nullptr;
    throw Error{MC_EDEVICE, "rocblas_create_handle failed"};
  }
  if (rocblas_set_stream(g_blas, s) != rocblas_status_success)
    throw Error{MC_EDEVICE, "rocblas_set_stream failed"};
  rocblas_int* info = nullptr;
  HIPCHK(hipMalloc((void**)&info, 2 * sizeof(rocblas_int)));
  rocblas_status a = rocsolver_dpotrf(g_blas, rocblas_fill_lower, K, S, lda, info);
  rocblas_status b = rocsolver_dpotri(g_blas, rocblas_fill_lower, K, S, lda, info + 1);
  rocblas_int h[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(h, info, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(info);
  HIPCHK(e);
  if (a != rocblas_status_success || b != rocblas_status_success || h[0] != 0 || h[1] != 0)
    throw Error{MC_EDEVICE, "inverse of the crossing-cell Schur complement failed (status " +
                                std::to_string((int)a) + "/" + std::to_string((int)b) +
                                ", info " + std::to_string(h[0]) + "/" + std::to_string(h[1]) + ")"};
  hipLaunchKernelGGL(k_symmetrize, dim3(cdiv((long)K * K, 256)), dim3(256), 0, s, S, K, lda);
  HIPCHK(hipGetLastError());
}

// Two-level block preconditioner of a fracture graph whose crossing cells are too many for the
// exact solve: dense inverses of connected blocks of at most 64 cells and the inverse of the
// Galerkin coarse operator over the blocks, which the crossing-cell kernels apply (K = blocks,
// every cell's response is the coarse value of its own block).  False (nothing changed) if
// the graph needs more blocks than the coarse inverse takes.
static bool setup_block_solve(mc_problem* P, Cont& C, const std::vector<double>& diag,
                              const std::vector<double>& val) {
  hipStream_t s = P->X.stream;
  const long nf = C.n;
  BlockHost H = build_block_solve((int)nf, P->gh, (int)P->gtile_h.size() - 1, diag.data(),
                                  val.data(), MC_SCHUR_KMAX);
  if (!H.ok) throw Error{MC_EDEVICE, "a fracture block matrix is not positive definite"};
  if (H.nb == 0) return false;
  const int K = H.nb;
  DevArena& M = P->mem;
  // device arrays are made on the first setup of this preconditioner (the graph does not
  // change afterwards, so neither does K); the FP32 copies sized by K are made again
  if (C.fmode != 2) {
    C.fmode = 2;
    C.sinv32 = nullptr;
    C.gX32 = C.zX32 = nullptr;
    C.bnode = M.alloc<int>((size_t)K * kBlockCells);
    C.binv = M.alloc<float>((size_t)K * kBlockCells * kBlockCells);
    C.xtile = M.alloc<int>(H.xtile.size());
    C.xlr = M.alloc<int>(2 * nf);
    C.cl = M.alloc<double>(nf);
    C.cr = M.alloc<double>(nf);
    C.sinv = M.alloc<double>((size_t)K * K);
    C.gX = M.alloc<double>(K);
    C.zX = M.alloc<double>(K);
  }
  std::vector<int> xlr(2 * nf);
  std::vector<double> one(nf, 1.0), zero(nf, 0.0);
  for (long l = 0; l < nf; ++l) {
    xlr[2 * l] = H.blk[l];
    xlr[2 * l + 1] = -1;
  }
  HIPCHK(hipMemcpyAsync(C.bnode, H.node.data(), H.node.size() * sizeof(int),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(C.binv, H.binv.data(), H.binv.size() * sizeof(float),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(C.xtile, H.xtile.data(), H.xtile.size() * sizeof(int),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(C.xlr, xlr.data(), 2 * nf * sizeof(int), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(C.cl, one.data(), nf * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(C.cr, zero.data(), nf * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(C.sinv, H.Ac.data(), (size_t)K * K * sizeof(double),
                        hipMemcpyHostToDevice, s));
  invert_spd(C.sinv, K, s);
  if (!C.sinv32) C.sinv32 = M.alloc<float>((size_t)K * K);   // the coarse solve reads FP32
  hipLaunchKernelGGL(k_to_f32, dim3(cdiv((long)K * K, 256)), dim3(256), 0, s, C.sinv, C.sinv32,
                     (long)K * K);
  HIPCHK(hipGetLastError());
  C.K = K;
  C.fblocks = true;
  HIPCHK(hipStreamSynchronize(s));   // host vectors die at return
  return true;
}

// Fracture block preconditioner of the block IC(0) option: factors of the chain blocks cut at
// the crossing cells and the inverse Schur complement of the crossing cells (an exact solve
// of the fracture system), built on the host in FP64 from the device coefficients.
static void setup_fracture_solve(mc_problem* P, Cont& C) {
  hipStream_t s = P->X.stream;
  const long nf = C.n, ne2 = 2L * P->ne;
  std::vector<double> diag(nf), val(std::max<long>(ne2, 1));
  HIPCHK(hipMemcpyAsync(diag.data(), C.diag, nf * sizeof(double), hipMemcpyDeviceToHost, s));
  if (ne2) HIPCHK(hipMemcpyAsync(val.data(), C.val, ne2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int kmax = exact_crossing_max();
  SchurHost H = build_schur((int)nf, P->gh, P->chains_h, P->gtile_h, diag.data(), val.data(),
                            kmax);
  DevArena& M = P->mem;
  C.fblocks = false;
  if (!C.cT) C.cT = M.alloc<double>(nf);
  HIPCHK(hipMemcpyAsync(C.fdinv, H.dinv.data(), nf * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(C.cT, H.cT.data(), nf * sizeof(double), hipMemcpyHostToDevice, s));
  // beyond the exact solve's limit the decoupled fracture solve takes the two-level block
  // preconditioner; the chain factors stay for the coupled system
  if (H.K == 0 && H.K_all > kmax && fracture_blocks_on() && setup_block_solve(P, C, diag, val))
    return;
  C.K = H.K;
  std::vector<int> xlr;
  if (H.K > 0) {
    const int K = H.K;
    if (C.fmode != 1) {   // first setup of the exact solve (K fixed by the graph)
      C.fmode = 1;
      C.sinv32 = nullptr;   // FP32 copies sized by K are made again for this solve's K
      C.gX32 = C.zX32 = nullptr;
      C.xcells = M.alloc<int>(K);
      C.xtile = M.alloc<int>(H.xtile.size());
      C.xlr = M.alloc<int>(2 * nf);
      C.cl = M.alloc<double>(nf);
      C.cr = M.alloc<double>(nf);
      C.cxl = M.alloc<double>(K);
      C.cxr = M.alloc<double>(K);
      C.sinv = M.alloc<double>((size_t)K * K);
      C.gX = M.alloc<double>(K);
      C.zX = M.alloc<double>(K);
    }
    xlr.resize(2 * nf);
    for (long l = 0; l < nf; ++l) {
      xlr[2 * l] = H.xl[l];
      xlr[2 * l + 1] = H.xr[l];
    }
    HIPCHK(hipMemcpyAsync(C.xcells, H.xcells.data(), K * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(C.xtile, H.xtile.data(), H.xtile.size() * sizeof(int),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(C.xlr, xlr.data(), 2 * nf * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(C.cl, H.cl.data(), nf * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(C.cr, H.cr.data(), nf * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(C.cxl, H.cxl.data(), K * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(C.cxr, H.cxr.data(), K * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(C.sinv, H.S.data(), (size_t)K * K * sizeof(double),
                          hipMemcpyHostToDevice, s));
    invert_spd(C.sinv, K, s);
  }
  HIPCHK(hipStreamSynchronize(s));   // host vectors die at return
}

// Levels of the V-cycle of grid continuum C (option MC_MG): 2 x 2 aggregation until at most
// MC_MG_COARSE cells remain; Galerkin coarse operators, their block IC(0) factors (with the
// FP32 copies the sweeps read) and the dense inverse of the coarsest operator.  Arrays are
// allocated on the first call and refilled on later ones.
static void setup_multigrid(mc_problem* P, Cont& C) {
  hipStream_t s = P->X.stream;
  DevArena& M = P->mem;
  const bool mixed = P->X.opt.precision == MC_MIXED;
  auto cv = [&](const double* a, float*& b, long n) {
    if (!b) b = M.alloc<float>(n);
    hipLaunchKernelGGL(k_to_f32, dim3(cdiv(n, 256)), dim3(256), 0, s, a, b, n);
  };
  int nx = P->d.nx, ny = P->d.ny;
  const double *fd = C.diag, *ftx = C.tx, *fty = C.ty;
  size_t l = 0;
  // The hierarchy stops early at a level above the small-level tail whose operator is
  // strongly diagonally dominant: summed over its cells, the row sums (storage over tau,
  // transfer) at least MC_MG_DOMINANCE times the face conductances.  Block IC(0) nearly
  // solves such a level, so it is smoothed twice instead of corrected from coarser levels
  // (MCDEC_MG_DOMINANCE overrides the ratio, 0 = never stop early; MCDEC_MG_LEVELS caps the
  // number of coarse levels).  The inner FP32 solves of mixed precision stop at a ratio of
  // 2: they reduce the residual by 1e-3 at a time, which the deeper levels do not speed
  // up, while a FP64 solve to 1e-10 over many layers needs them for the smooth part of the
  // increments.
  constexpr double dominance_mixed = 2.0;
  const long tail_n = mg_tail_cells();
  const int max_levels = std::max(1, env_int("MCDEC_MG_LEVELS", 1 << 20));
  const char* dom_env = std::getenv("MCDEC_MG_DOMINANCE");
  const double dominance = dom_env ? std::atof(dom_env)
                                  : mixed ? dominance_mixed : MC_MG_DOMINANCE;
  constexpr int dom_blocks = 128;
  double* dom_part = nullptr;
  bool stop = false;
  while ((long)nx * ny > MC_MG_COARSE) {
    if (((int)l >= max_levels || stop) && (long)nx * ny > tail_n) break;
    const int cnx = (nx + 1) / 2, cny = (ny + 1) / 2;
    if (C.mg.size() <= l) C.mg.emplace_back();
    MgLevel& L = C.mg[l];
    L.nx = cnx;
    L.ny = cny;
    L.n = (long)cnx * cny;
    L.tiles = (int)(cdiv(cnx, MC_TX) * cdiv(cny, MC_TY));
    L.smooth_once = false;
    L.coarsest = L.n <= MC_MG_COARSE;   // a level the hierarchy stops at above the tail is
                                         // not: it gets IC(0) factors for its smoothing
    if (!L.diag) {
      L.diag = M.alloc<double>(L.n);
      L.tx = M.alloc<double>(L.n);
      L.ty = M.alloc<double>(L.n);
      L.fdinv = M.alloc<double>(L.n);
      L.r = M.alloc<double>(L.n);
      L.zp = M.alloc<double>(L.n);
      L.z = M.alloc<double>(L.n);
    }
    if (mixed && !L.r32) {
      L.r32 = M.alloc<float>(L.n);
      L.zp32 = M.alloc<float>(L.n);
      L.z32 = M.alloc<float>(L.n);
    }
    CoarsenSetup g{nx, ny, cnx, cny, fd, ftx, fty, L.diag, L.tx, L.ty};
    hipLaunchKernelGGL(k_mg_coarsen, dim3(cdiv(L.n, 256)), dim3(256), 0, s, g);
    if (!L.coarsest) {
      GridIC0Setup gi;
      gi.nx = cnx;
      gi.ny = cny;
      gi.tiles_x = (int)cdiv(cnx, MC_TX);
      gi.ntiles = L.tiles;
      gi.diag = L.diag;
      gi.tx = L.tx;
      gi.ty = L.ty;
      gi.dinv = L.fdinv;
      gi.rows = MC_ICYC;
      hipLaunchKernelGGL(k_setup_grid_ic0, dim3(cdiv((long)L.tiles * (MC_TY / MC_ICYC), 64)),
                         dim3(64), 0, s, gi);
      cv(L.fdinv, L.fdinv32, L.n);
    } else {
      // even leading dimension, zero padding: the product reads rows in pairs
      const int ld = (int)(L.n + (L.n & 1));
      const long nn = (long)ld * ld;
      if (!L.inv) L.inv = M.alloc<double>(nn);
      hipLaunchKernelGGL(k_fill0, dim3(cdiv(nn, 256)), dim3(256), 0, s, L.inv, nn);
      hipLaunchKernelGGL(k_mg_dense_fill, dim3(cdiv(L.n, 256)), dim3(256), 0, s, L.diag, L.tx,
                         L.ty, cnx, cny, ld, L.inv);
      HIPCHK(hipGetLastError());
      invert_spd(L.inv, (int)L.n, s, ld);
      cv(L.inv, L.inv32, nn);   // the cycle reads the FP32 copy
    }
    cv(L.diag, L.diag32, L.n);
    cv(L.tx, L.tx32, L.n);
    cv(L.ty, L.ty32, L.n);
    HIPCHK(hipGetLastError());
    if (dominance > 0 && L.n > tail_n) {
      if (!dom_part) dom_part = M.alloc<double>(2 * dom_blocks);
      hipLaunchKernelGGL(k_mg_dominance, dim3(dom_blocks), dim3(256), 0, s, cnx, cny, L.diag,
                         L.tx, L.ty, dom_part);
      HIPCHK(hipGetLastError());
      std::vector<double> h(2 * dom_blocks);
      HIPCHK(hipMemcpyAsync(h.data(), dom_part, h.size() * sizeof(double),
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double rs = 0.0, fs = 0.0;
      for (int b = 0; b < dom_blocks; ++b) {
        rs += h[2 * b];
        fs += h[2 * b + 1];
      }
      stop = rs >= dominance * fs;
      // a level that strongly dominant is nearly solved by one sweep of its block IC(0)
      L.smooth_once = stop && rs >= MC_MG_DOMINANCE * fs;
    }
    fd = L.diag;
    ftx = L.tx;
    fty = L.ty;
    nx = cnx;
    ny = cny;
    ++l;
  }
  C.mg.resize(l);
  C.mg_on = l > 0;
  if (C.mg_on && !C.zpre) C.zpre = M.alloc<double>(C.n);
  if (C.mg_on && mixed && !C.zpre32) C.zpre32 = M.alloc<float>(C.n);
  if (C.mg_on && !C.mg_edz) {   // (sized for FP64; an FP32 solve uses the same indices)
    const long ne = cdiv(P->d.nx, MC_TX) * (long)P->d.ny;
    C.mg_edz = M.alloc<double>(2 * ne);
    C.mg_edt = M.alloc<float>(ne);
  }
}

static void build_coefficients(mc_problem* P) {
  const bool ex = P->X.opt.scheme == MC_SCHEME_EX;
  const double h = P->d.h, tau = P->d.tau;
  hipStream_t s = P->X.stream;
  for (int a = 0; a < P->n_omega; ++a) {
    Cont& C = P->cont[a];
    GridSetup g;
    std::memset(&g, 0, sizeof(g));
    g.nx = P->d.nx;
    g.ny = P->d.ny;
    g.nz = P->nz;
    g.k = P->k[a];
    g.kc = P->d.omega[a].k_const;
    g.c = P->d.omega[a].c;
    g.h = h;
    g.tau = tau;
    g.s12 = P->n_omega == 2 ? omega_transfer(P) : 0.0;
    for (int k = 0; k < 4; ++k) {
      g.bc_type[k] = P->d.bc_type[k];
      g.bc_value[k] = P->d.bc_value[k];
    }
    for (int k = 0; k < 2; ++k) {
      g.bc_type_z[k] = P->d.bc_type_z[k];
      g.bc_value_z[k] = P->d.bc_value_z[k];
    }
    g.src = P->src[a];
    g.hptr = P->nf ? P->hptr : nullptr;
    g.hidx = P->hidx;
    g.hsig = P->nf ? P->sigma_f + (long)a * P->nf : nullptr;
    g.ex = ex;
    g.diag = C.diag;
    g.tx = C.tx;
    g.ty = C.ty;
    g.tz = C.tz;
    g.F = C.F;
    hipLaunchKernelGGL(k_setup_grid, dim3(cdiv(C.n, 256)), dim3(256), 0, s, g);
    C.mtau = (P->nz > 1 ? P->d.omega[a].c * h * h * h : P->d.omega[a].c * h * h) / tau;
    // a 3-D grid always uses the conductance arrays (ty is 0 across plane boundaries)
    C.has_t = P->k[a] != nullptr || P->nz > 1;
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
    g.wq = P->well_q;
    g.wp = P->well_q ? P->well_p : nullptr;
    g.k_f = P->d.k_f;
    g.c_f = P->d.c_f;
    g.aperture = P->d.aperture;
    g.tau = tau;
    g.ex = ex;
    g.val = C.val;
    g.diag = C.diag;
    g.mt = C.mt;
    g.F = C.F;
    hipLaunchKernelGGL(k_setup_graph, dim3(cdiv(P->nf, 256)), dim3(256), 0, s, g);
  }
  HIPCHK(hipGetLastError());
  for (auto& C : P->cont) {   // set again below for block IC(0)
    C.K = 0;
    C.fblocks = false;
  }
  if (ic_precond(P->X.opt.precond)) {
    for (auto& C : P->cont) {
      if (!C.fdinv) C.fdinv = P->mem.alloc<double>(C.n);
      if (!C.z) C.z = P->mem.alloc<double>(C.n);
      if (C.kind == PART_GRID) {
        GridIC0Setup g;
        g.nx = P->d.nx;
        g.ny = P->d.ny * P->nz;
        g.tiles_x = (int)cdiv(P->d.nx, MC_TX);
        g.ntiles = C.tiles;
        g.diag = C.diag;
        g.tx = C.tx;
        g.ty = C.ty;
        g.dinv = C.fdinv;
        g.rows = MC_ICY;
        hipLaunchKernelGGL(k_setup_grid_ic0, dim3(cdiv((long)C.tiles * MC_ICB, 64)), dim3(64),
                           0, s, g);
      } else {
        setup_fracture_solve(P, C);
      }
    }
    HIPCHK(hipGetLastError());
    // FP32 copies of the grid factor and conductances read by the tile sweeps
    for (auto& C : P->cont) {
      if (C.kind != PART_GRID) continue;
      auto cv = [&](double* a, float*& b, long n) {
        if (!b) b = P->mem.alloc<float>(n);
        hipLaunchKernelGGL(k_to_f32, dim3(cdiv(n, 256)), dim3(256), 0, s, a, b, n);
      };
      cv(C.fdinv, C.fdinv32, C.n);
      cv(C.tx, C.tx32, C.n);
      cv(C.ty, C.ty32, C.n);
    }
    HIPCHK(hipGetLastError());
  }
  for (auto& C : P->cont) C.mg_on = false;
  if (P->X.opt.precond == MC_MG) {
    for (auto& C : P->cont)   // the V-cycle's residuals use the operator's FP32 copies
      if (C.kind == PART_GRID) {
        if (!C.diag32) C.diag32 = P->mem.alloc<float>(C.n);
        hipLaunchKernelGGL(k_to_f32, dim3(cdiv(C.n, 256)), dim3(256), 0, s, C.diag, C.diag32,
                           C.n);
      }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    for (auto& C : P->cont)
      if (C.kind == PART_GRID) setup_multigrid(P, C);
  }
  if (P->X.opt.precision == MC_MIXED) {
    for (auto& C : P->cont) {
      auto cv = [&](double* a, float*& b, long n) {
        if (!a || n == 0) return;
        if (!b) b = P->mem.alloc<float>(n);
        hipLaunchKernelGGL(k_to_f32, dim3(cdiv(n, 256)), dim3(256), 0, s, a, b, n);
      };
      cv(C.diag, C.diag32, C.n);
      if (ic_precond(P->X.opt.precond)) {
        cv(C.fdinv, C.fdinv32, C.n);
        if (C.kind == PART_GRAPH) cv(C.cT, C.cT32, C.n);
        if (!C.z32) C.z32 = P->mem.alloc<float>(C.n);
        if (C.kind == PART_GRAPH && C.K > 0) {
          cv(C.cl, C.cl32, C.n);
          cv(C.cr, C.cr32, C.n);
          cv(C.sinv, C.sinv32, (long)C.K * C.K);
          if (!C.gX32) {
            C.gX32 = P->mem.alloc<float>(C.K);
            C.zX32 = P->mem.alloc<float>(C.K);
          }
        }
      }
      if (C.kind == PART_GRID) {
        cv(C.tx, C.tx32, C.n);
        cv(C.ty, C.ty32, C.n);
        if (C.tz) cv(C.tz, C.tz32, C.n);
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
  HIPCHK(hipStreamSynchronize(s));
  clear_tables(P);
}

// Workgroup counts of every continuum for the current preconditioner, and the slot counts
// of the system records (in host memory `hs`).
static void set_slot_counts(mc_problem* P, SysState* hs) {
  const bool bic0 = ic_precond(P->X.opt.precond);
  const bool fp32 = P->X.opt.precision == MC_MIXED;
  int ca = 0, cb = 0;
  for (int c = 0; c < P->ncont; ++c) {
    Cont& C = P->cont[c];
    C.blocks[0] = blocks_for(C.tiles, C.kind, 0, bic0, fp32);
    C.blocks[1] = blocks_for(C.tiles, C.kind, 1, bic0, fp32);
    // fracture: crossing-cell product; grid with a V-cycle: its final smoothing
    C.blocks[2] = C.K > 0 ? (int)cdiv(C.K, MC_SCHUR_ROWS) : (C.mg_on ? C.blocks[1] : 0);
    hs[c].nslotsA = C.blocks[0];
    hs[c].nslotsB = C.blocks[1] + C.blocks[2];
    ca += C.blocks[0];
    cb += C.blocks[1] + C.blocks[2];
  }
  hs[P->ncont].nslotsA = ca;
  hs[P->ncont].nslotsB = cb;
}

// The layer history the adaptive warm start keeps (three more states per continuum).
static void ensure_history(mc_problem* P) {
  if (P->X.opt.warm_start != WS_ADAPTIVE) return;
  for (auto& C : P->cont)
    for (int k = 0; k < 3; ++k)
      if (!C.hx[k]) C.hx[k] = P->mem.alloc<double>(C.n);
}

static void create(mc_problem* P, const mc_problem_desc& d, const mc_options& o) {
  std::string m = validate_desc(d);
  if (!m.empty()) fail(m);
  m = validate_options(o);
  if (!m.empty()) fail(m);
  P->d = d;
  P->X.opt = o;
  P->X.auto_cus = true;
  P->mem.use_hooks(o);
  P->n_omega = d.n_omega;
  P->nf = d.nf;
  P->ne = d.ne;
  P->nz = d.nz > 1 ? d.nz : 1;
  P->ncell = (long)d.nx * d.ny * P->nz;
  if (P->nz > 1 && o.precond == MC_MG)
    fail("the multigrid preconditioner needs a 2-D grid (nz <= 1); use MC_JACOBI or MC_BIC0");
  P->ncont = d.n_omega + (d.nf > 0 ? 1 : 0);
  HIPCHK(hipGetDevice(&P->device));
  exec_init(P->X, o.stream);
  P->X.opt.stream = P->X.stream;
  hipStream_t s = P->X.stream;
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
    std::vector<int> gt = build_graph_tiles(chains, MC_GRAPH_ROWS);
    P->gtile = M.upload(gt.data(), gt.size(), s);
    P->ngtiles = (int)gt.size() - 1;
    P->K_all = count_crossing_cells(d.nf, d.ne, d.edges);
    if (P->K_all > 0) {
      std::vector<int> bn, bb;
      P->nb_frac = build_blocks(d.nf, g, bn, bb);
    }
    P->gh = g;
    P->host_h.assign(d.host, d.host + d.nf);
    P->chains_h = chains;
    P->gtile_h = gt;
    if (d.src_f) P->src[d.n_omega] = M.upload(d.src_f, d.nf, s);
    if (d.well_q) P->well_q = M.upload(d.well_q, d.nf, s);
    if (d.well_q && d.well_p) P->well_p = M.upload(d.well_p, d.nf, s);
  }
  // continua
  P->cont.resize(P->ncont);
  for (int c = 0; c < P->ncont; ++c) {
    Cont& C = P->cont[c];
    const bool grid = c < d.n_omega;
    C.kind = grid ? PART_GRID : PART_GRAPH;
    C.n = grid ? P->ncell : d.nf;
    C.tiles = grid ? (int)(cdiv(d.nx, MC_TX) * cdiv((long)d.ny * P->nz, MC_TY)) : P->ngtiles;
    C.blocks[0] = blocks_for(C.tiles, C.kind, 0, ic_precond(o.precond), o.precision == MC_MIXED);
    C.blocks[1] = blocks_for(C.tiles, C.kind, 1, ic_precond(o.precond), o.precision == MC_MIXED);
    C.blocks[2] = 0;
    C.diag = M.alloc<double>(C.n);
    C.F = M.alloc<double>(C.n);
    if (grid) {
      C.tx = M.alloc<double>(C.n);
      C.ty = M.alloc<double>(C.n);
      if (P->nz > 1) C.tz = M.alloc<double>(C.n);
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
  ensure_history(P);
  // systems: one per continuum + the coupled one
  const int nsys = P->ncont + 1;
  exec_sys_capacity(P->X, nsys);
  std::vector<SysState> hs(nsys);
  std::memset(hs.data(), 0, nsys * sizeof(SysState));
  // partial-slot arrays sized for one workgroup per tile (the most any tiling uses), so the
  // tilings can follow option changes
  // (a fracture continuum adds the workgroups of its crossing-cell product)
  // (its rows are the crossing cells of the exact solve or the blocks of the two-level one)
  const int krows = std::max(P->K_all <= MC_SCHUR_KMAX ? P->K_all : 0,
                             P->nb_frac <= MC_SCHUR_KMAX ? P->nb_frac : 0);
  const int kslots = (int)cdiv(krows, MC_SCHUR_ROWS);
  // (a grid continuum with a V-cycle adds the workgroups of its final smoothing)
  auto slots_of = [&](int c) {
    return P->cont[c].tiles + (P->cont[c].kind == PART_GRAPH ? kslots : P->cont[c].tiles);
  };
  int coupled_tiles = 0;
  for (int c = 0; c < P->ncont; ++c) coupled_tiles += slots_of(c);
  for (int sI = 0; sI < nsys; ++sI) {
    const int ns = sI < P->ncont ? slots_of(sI) : coupled_tiles;
    hs[sI].partA = M.alloc<double>((size_t)ns * MC_SLOT);
    hs[sI].partB = M.alloc<double>((size_t)ns * MC_SLOT);
    hs[sI].done = 1;
    P->partA.push_back(hs[sI].partA);
    P->partB.push_back(hs[sI].partB);
  }
  set_slot_counts(P, hs.data());
  HIPCHK(hipMemcpyAsync(P->X.sys, hs.data(), nsys * sizeof(SysState), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  build_coefficients(P);
  set_slot_counts(P, hs.data());   // the crossing-cell workgroups are known now
  HIPCHK(hipMemcpyAsync(P->X.sys, hs.data(), nsys * sizeof(SysState), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------------------------
// kernel timing
// ------------------------------------------------------------------------------------
static Exec::Ev prof_take(Exec& X, int which) {
  if (X.ev_free.empty()) {
    Exec::Ev n;
    HIPCHK(hipEventCreate(&n.a));
    HIPCHK(hipEventCreate(&n.b));
    X.ev_free.push_back(n);
  }
  Exec::Ev e = X.ev_free.back();
  X.ev_free.pop_back();
  e.which = which;
  return e;
}
static void prof_harvest(Exec& X) {
  for (auto& e : X.ev_pending) {
    float ms = 0;
    HIPCHK(hipEventSynchronize(e.b));
    HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
    X.prof_ms[e.which] += ms;
    X.prof_launch[e.which] += 1;
    X.prof_samples[e.which].push_back(ms);
    X.ev_free.push_back(e);
  }
  X.ev_pending.clear();
}

// ------------------------------------------------------------------------------------
// solve orchestration
// ------------------------------------------------------------------------------------
// A group is a set of systems (a contiguous range of system records) whose tiles are
// launched together on one stream.  Decoupled continua of different kinds form separate
// groups on separate streams, so the small, latency-bound fracture solves overlap the
// bandwidth-bound grid solves.  The host advances each group as a small state machine and
// only ever waits on an event recorded after a copy of that group's system records.
struct Group {
  hipStream_t s = nullptr;
  Table* T = nullptr;
  int kinds = 0;      // bit k set: launch the kind-k tiles of the table
  int s0 = 0, s1 = 0; // system records [s0, s1)
  bool mixed = false, assemble = true;
  int phase = 0;      // 0 start, 1 iterating, 3 finished
  int K = 8;
  long k = 0;         // PCG iterations launched in the current (inner) solve
  int outer = 0;
  SysState* hbuf = nullptr;
  hipEvent_t ev = nullptr;
  bool inflight = false;
};

// z_X = S^-1 g for the fracture parts with crossing cells (after their update, init or
// residual kernel), completing (r, z) in the update slots.
template <class T>
static void launch_schur(Exec& X, const Table& Tb, hipStream_t s) {
  if (Tb.nblk[2][PART_GRAPH])
    hipLaunchKernelGGL(k_schur<T>, dim3(Tb.nblk[2][PART_GRAPH]), dim3(MC_BLOCK), 0, s, Tb.parts,
                       Tb.tiles[2][PART_GRAPH], X.sys);
}

// V-cycle of the grid parts that have coarse levels, after the kernel that wrote their
// finest pre-smoothed z_p: restriction and smoothing going down (the small levels, the
// coarsest solve among them, in one workgroup per chain), the corrections with
// post-smoothing going up.  The finest post-smoothing writes z and, when
// `final`, (r, z) to the update slots.  `sys` null: no test of the solve's end.
// after_update: the cycle follows the PCG update kernel, which has summed the finest
// level's in-block share of the restriction into level 1 (fused tables)
template <class T>
static void launch_vcycle(const Table& Tb, hipStream_t s, SysState* sys, bool final,
                          Exec* X = nullptr, bool after_update = false) {
  const int L = (int)Tb.mg.size();
  if (L == 0 || Tb.mg[0][3].n == 0) return;
  // X: count the launches for kernel timing, and time them all when the finest
  // post-smoothing of this cycle is due for a sample
  const bool timed = X && X->prof && final && (X->prof_count[2] % X->prof_every) == 0;
  auto go = [&](auto kern, const Table::List& li, int slot, int threads) {
    if (!li.n) return;
    if (X && X->prof) X->prof_count[slot] += 1;
    if (timed) {
      Exec::Ev e = prof_take(*X, slot);
      hipExtLaunchKernelGGL(kern, dim3(li.n), dim3(threads), 0, s, e.a, e.b, 0, Tb.parts, li.t,
                            sys);
      X->ev_pending.push_back(e);
    } else {
      hipLaunchKernelGGL(kern, dim3(li.n), dim3(threads), 0, s, Tb.parts, li.t, sys);
    }
  };
  for (int l = 1; l < L; ++l) {
    if (l == 1 && after_update && Tb.mg_fused) go(k_mg_fix_smooth<T>, Tb.mg[l][1], 3, MC_BLOCK);
    else go(k_mg_restrict_smooth<T>, Tb.mg[l][1], 3, MC_BLOCK);
    go(k_mg_restrict<T>, Tb.mg[l][0], 6, MC_BLOCK);
    go(k_mg_tail<T>, Tb.mg[l][2], 5, MC_TAIL_THREADS);
  }
  for (int l = L - 1; l >= 1; --l) go(k_mg_post_c<T>, Tb.mg[l][3], 4, MC_BLOCK);
  if (!final) {
    hipLaunchKernelGGL((k_mg_post<T, false>), dim3(Tb.mg[0][3].n), dim3(MC_BLOCK), 0, s,
                       Tb.parts, Tb.mg[0][3].t, sys);
  } else {
    if (X && X->prof) X->prof_count[2] += 1;
    if (timed) {
      Exec::Ev e = prof_take(*X, 2);   // timed like the PCG kernels
      hipExtLaunchKernelGGL((k_mg_post<T, true>), dim3(Tb.mg[0][3].n), dim3(MC_BLOCK), 0, s,
                            e.a, e.b, 0, Tb.parts, Tb.mg[0][3].t, sys);
      X->ev_pending.push_back(e);
    } else {
      hipLaunchKernelGGL((k_mg_post<T, true>), dim3(Tb.mg[0][3].n), dim3(MC_BLOCK), 0, s,
                         Tb.parts, Tb.mg[0][3].t, sys);
    }
  }
}

// Launches of V-cycle kernel timing slot `slot` (3..6) in one cycle over table Tb.
static int vcycle_launches(const Table& Tb, int slot) {
  const int L = (int)Tb.mg.size();
  int n = 0;
  for (int l = 1; l < L; ++l) {
    if (slot == 3 && Tb.mg[l][1].n) ++n;
    if (slot == 6 && Tb.mg[l][0].n) ++n;
    if (slot == 5 && Tb.mg[l][2].n) ++n;
    if (slot == 4 && Tb.mg[l][3].n) ++n;
  }
  return n;
}

// One PCG iteration over the group's tiles: operator kernels, then update kernels.
template <class T, int PREC>
static void launch_iter(Exec& X, Group& G, bool timed) {
  const Table& Tb = *G.T;
  auto L = [&](auto kern, int kind, int which) {
    const int fam = which;   // operator kernels: tiling 0, update kernels: tiling 1
    if (!(G.kinds >> kind & 1) || Tb.nblk[fam][kind] == 0) return;
    if (timed && X.prof && kind == PART_GRID &&
        (X.prof_count[which]++ % X.prof_every) == 0) {
      // events bound to this dispatch time the kernel itself; they cost the stream a few
      // microseconds per dispatch, so only every prof_every-th launch is sampled
      Exec::Ev e = prof_take(X, which);
      hipExtLaunchKernelGGL(kern, dim3(Tb.nblk[fam][kind]), dim3(MC_BLOCK), 0, G.s, e.a, e.b,
                            0, Tb.parts, Tb.tiles[fam][kind], X.sys);
      X.ev_pending.push_back(e);
    } else {
      hipLaunchKernelGGL(kern, dim3(Tb.nblk[fam][kind]), dim3(MC_BLOCK), 0, G.s, Tb.parts,
                         Tb.tiles[fam][kind], X.sys);
    }
  };
  L(k_pcg_A<T, PREC, PART_GRID>, PART_GRID, 0);
  L(k_pcg_A<T, PREC, PART_GRAPH>, PART_GRAPH, 0);
  L(k_pcg_B<T, PREC, PART_GRID>, PART_GRID, 1);
  if (G.kinds & 1) launch_vcycle<T>(Tb, G.s, X.sys, true, timed ? &X : nullptr, true);
  L(k_pcg_B<T, PREC, PART_GRAPH>, PART_GRAPH, 1);
  if (G.kinds & 2) launch_schur<T>(X, Tb, G.s);
}

// Executable graph of K iterations over the group's tiles (captured on first use).  The
// launches carry no per-iteration argument, so one graph serves every chunk of that length.
template <class T, int PREC>
static hipGraphExec_t chunk_graph(Exec& X, Group& G, int K) {
  const long key = ((long)G.kinds << 40) | ((long)sizeof(T) << 32) | ((long)PREC << 24) | K;
  std::lock_guard<std::mutex> lk(X.graph_mu);
  auto it = G.T->graphs.find(key);
  if (it != G.T->graphs.end()) return it->second;
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(G.s, hipStreamCaptureModeThreadLocal));
  for (int j = 0; j < K; ++j) launch_iter<T, PREC>(X, G, false);
  hipError_t le = hipGetLastError();
  hipError_t ce = hipStreamEndCapture(G.s, &g);
  if (le != hipSuccess || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    throw Error{MC_EDEVICE, std::string("graph capture failed: ") +
                                hipGetErrorString(le != hipSuccess ? le : ce)};
  }
  hipGraphExec_t e = nullptr;
  hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) throw Error{MC_EDEVICE, std::string("graph instantiate failed: ") +
                                                    hipGetErrorString(ie)};
  G.T->graphs[key] = e;
  return e;
}

// K iterations: replayed from captured graphs of power-of-two lengths (or launched one by one
// when graphs are switched off).  While kernel timing is on, the iterations whose grid
// kernels are due for a sample (one in prof_every) are launched one by one with timing
// events, the others still replayed; the issue counters count both.
template <class T, int PREC>
static void launch_chunk(Exec& X, Group& G, int K) {
  if (!X.graphs) {
    for (int j = 0; j < K; ++j) launch_iter<T, PREC>(X, G, true);
    return;
  }
  auto replay = [&](int m) {
    for (int b = 0; (1 << b) <= m; ++b)
      if (m >> b & 1) HIPCHK(hipGraphLaunch(chunk_graph<T, PREC>(X, G, 1 << b), G.s));
  };
  const bool grid = (G.kinds & 1) && G.T->nblk[0][PART_GRID] > 0;
  if (!X.prof || !grid) {
    replay(K);
    return;
  }
  const bool post = G.T->mg.size() > 0 && G.T->mg[0][3].n > 0;
  while (K > 0) {
    const long c = X.prof_count[1];
    if (c % X.prof_every == 0) {
      launch_iter<T, PREC>(X, G, true);
      --K;
      continue;
    }
    const int m = (int)std::min<long>(K, X.prof_every - c % X.prof_every);
    replay(m);
    for (int w = 0; w < 3; ++w)
      if (w < 2 || post) X.prof_count[w] += m;
    if (post)
      for (int w = 3; w < Exec::NPROF; ++w) X.prof_count[w] += (long)m * vcycle_launches(*G.T, w);
    K -= m;
  }
}

// launch the grid-kind kernel over the grid tiles and the graph-kind kernel over the graph
// tiles of the group's table (each only if the group has tiles of that kind)
template <class KG, class KF, class... A>
static void launch2(const Group& G, int fam, KG kg, KF kf, A... args) {
  if ((G.kinds & 1) && G.T->nblk[fam][PART_GRID])
    hipLaunchKernelGGL(kg, dim3(G.T->nblk[fam][PART_GRID]), dim3(MC_BLOCK), 0, G.s,
                       G.T->parts, G.T->tiles[fam][PART_GRID], args...);
  if ((G.kinds & 2) && G.T->nblk[fam][PART_GRAPH])
    hipLaunchKernelGGL(kf, dim3(G.T->nblk[fam][PART_GRAPH]), dim3(MC_BLOCK), 0, G.s,
                       G.T->parts, G.T->tiles[fam][PART_GRAPH], args...);
}

template <class KG, class KF, class... A>
static void launch_all(hipStream_t s, Table& T, int fam, KG kg, KF kf, A... args) {
  Group g;
  g.s = s;
  g.T = &T;
  g.kinds = 3;
  launch2(g, fam, kg, kf, args...);
}

static void submit_poll(Exec& X, Group& G) {
  HIPCHK(hipMemcpyAsync(G.hbuf, X.sys + G.s0, (G.s1 - G.s0) * sizeof(SysState),
                        hipMemcpyDeviceToHost, G.s));
  HIPCHK(hipEventRecord(G.ev, G.s));
  G.inflight = true;
}

// Chunk size from the observed convergence: the number of further iterations the slowest
// unfinished system needs if its residual keeps shrinking at its average rate so far.
static int next_chunk(const Group& G) {
  double need = 0;
  bool any = false;
  for (int k = 0; k < G.s1 - G.s0; ++k) {
    const SysState& S = G.hbuf[k];
    if (S.done) continue;
    any = true;
    const double target = S.tol2 * S.bb;
    if (S.iter < 2 || !(S.rr < S.rr0) || !(S.rr > 0) || !(target > 0)) {
      need = std::max(need, 16.0);
      continue;
    }
    const double rate = std::log(S.rr / S.rr0) / S.iter;   // per-iteration log decrease
    double rem = std::log(target / S.rr) / rate;
    if (!(rem > 0)) rem = 1;
    need = std::max(need, rem);
  }
  if (!any) return 1;
  int K = (int)std::ceil(0.85 * need) + 1;
  return std::max(2, std::min(K, 256));
}

// First chunk of a solve: nine tenths of the iterations the group's slowest system took in
// its previous solve (consecutive time layers need nearly the same number), at least 8, so
// that most solves need one or two host polls; a chunk that overshoots convergence costs
// only launches whose workgroups return at once.
static int first_chunk(const Exec& X, const Group& G) {
  int prev = 0;
  for (int k = 0; k < G.s1 - G.s0; ++k) {
    const int it = G.hbuf[k].iter;   // last values polled for these records (any before use)
    if (it > 0 && it <= X.opt.max_iter) prev = std::max(prev, it);
  }
  return std::max(8, std::min(256, (int)(0.9 * prev)));
}

static bool all_done(const Group& G, bool outer) {
  for (int k = 0; k < G.s1 - G.s0; ++k)
    if (!(outer ? G.hbuf[k].outer_done : G.hbuf[k].done)) return false;
  return true;
}

// Runs a fixed launch sequence of the group (solve start, refinement restart) from a
// captured graph cached with the table, or eagerly while graphs are off.  `tag` names the
// sequence; the key also holds the group's kinds and record range.
template <class F>
static void launch_seq(Exec& X, Group& G, long tag, const F& seq) {
  if (!X.graphs) {
    seq();
    return;
  }
  const long key = (1L << 62) | (tag << 48) | ((long)G.kinds << 44) | ((long)G.s0 << 22) |
                   (long)G.s1;
  hipGraphExec_t e = nullptr;
  {
    std::lock_guard<std::mutex> lk(X.graph_mu);
    auto it = G.T->graphs.find(key);
    if (it != G.T->graphs.end()) {
      e = it->second;
    } else {
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(G.s, hipStreamCaptureModeThreadLocal));
      seq();
      hipError_t le = hipGetLastError();
      hipError_t ce = hipStreamEndCapture(G.s, &g);
      if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        throw Error{MC_EDEVICE, std::string("graph capture failed: ") +
                                    hipGetErrorString(le != hipSuccess ? le : ce)};
      }
      hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess)
        throw Error{MC_EDEVICE, std::string("graph instantiate failed: ") + hipGetErrorString(ie)};
      G.T->graphs[key] = e;
    }
  }
  HIPCHK(hipGraphLaunch(e, G.s));
}

template <int PREC>
static void advance_t(Exec& X, Group& G) {
  const int max_iter = X.opt.max_iter;
  auto chunk = [&](auto tag) {
    using T = decltype(tag);
    const long room = (long)max_iter + 2 - G.k;
    const int K = (int)std::max<long>(1, std::min<long>(G.K, room));
    launch_chunk<T, PREC>(X, G, K);
    G.k += K;
    HIPCHK(hipGetLastError());
    submit_poll(X, G);
  };
  auto pick_K = [&]() {
    G.K = X.opt.check_every > 0 ? X.opt.check_every : next_chunk(G);
  };
  if (!G.mixed) {
    if (G.phase == 0) {
      launch_seq(X, G, (long)PREC << 3 | (long)G.assemble << 2 | 0, [&] {
        hipLaunchKernelGGL(k_reset, dim3(cdiv(G.s1 - G.s0, 64)), dim3(64), 0, G.s, X.sys,
                           G.s0, G.s1);
        if (G.assemble) {
          launch2(G, 0, k_extrap_err<PART_GRID>, k_extrap_err<PART_GRAPH>, X.sys);
          launch2(G, 0, k_rhs<PART_GRID>, k_rhs<PART_GRAPH>, X.sys);
        }
        launch2(G, 1, k_init<PREC, PART_GRID>, k_init<PREC, PART_GRAPH>, X.sys);
        if (G.kinds & 1) launch_vcycle<double>(*G.T, G.s, X.sys, true);
        if (G.kinds & 2) launch_schur<double>(X, *G.T, G.s);
      });
      G.k = 0;
      G.K = X.opt.check_every > 0 ? X.opt.check_every : first_chunk(X, G);
      G.phase = 1;
    } else {
      if (all_done(G, false)) {
        G.phase = 3;
        return;
      }
      if (G.k > (long)max_iter + 1)
        throw Error{MC_EDEVICE, "PCG did not report completion within max_iter iterations"};
      pick_K();
    }
    chunk(double(0));
    return;
  }
  // mixed precision: FP64 residual -> FP32 inner PCG -> FP64 correction, repeated
  if (G.phase == 0) {
    launch_seq(X, G, (long)PREC << 3 | (long)G.assemble << 2 | 1, [&] {
      hipLaunchKernelGGL(k_reset, dim3(cdiv(G.s1 - G.s0, 64)), dim3(64), 0, G.s, X.sys, G.s0,
                         G.s1);
      if (G.assemble) {
        launch2(G, 0, k_extrap_err<PART_GRID>, k_extrap_err<PART_GRAPH>, X.sys);
        launch2(G, 0, k_rhs<PART_GRID>, k_rhs<PART_GRAPH>, X.sys);
      }
      launch2(G, 0, k_residual64<PART_GRID>, k_residual64<PART_GRAPH>, X.sys);
      launch2(G, 1, k_residual<PREC, PART_GRID>, k_residual<PREC, PART_GRAPH>, X.sys);
      if (G.kinds & 1) launch_vcycle<float>(*G.T, G.s, X.sys, true);
      if (G.kinds & 2) launch_schur<float>(X, *G.T, G.s);
    });
    G.outer = 0;
    G.k = 0;
    G.K = X.opt.check_every > 0 ? X.opt.check_every : 8;
    G.phase = 1;
    chunk(float(0));
    return;
  }
  if (all_done(G, true)) {
    G.phase = 3;
    return;
  }
  if (all_done(G, false)) {
    // every unfinished system ended its inner solve: correct, new residual, restart
    if (G.outer > X.opt.max_outer + 1) throw Error{MC_EDEVICE, "refinement did not terminate"};
    launch_seq(X, G, (long)PREC << 3 | 2, [&] {
      launch2(G, 0, k_correct<PART_GRID>, k_correct<PART_GRAPH>, X.sys);
      launch2(G, 0, k_residual64<PART_GRID>, k_residual64<PART_GRAPH>, X.sys);
      launch2(G, 1, k_residual<PREC, PART_GRID>, k_residual<PREC, PART_GRAPH>, X.sys);
      if (G.kinds & 1) launch_vcycle<float>(*G.T, G.s, X.sys, true);
      if (G.kinds & 2) launch_schur<float>(X, *G.T, G.s);
    });
    G.outer += 1;
    G.k = 0;
    G.K = X.opt.check_every > 0 ? X.opt.check_every : 8;
    chunk(float(0));
    return;
  }
  if (G.k > (long)max_iter + 1) throw Error{MC_EDEVICE, "inner PCG did not finish"};
  pick_K();
  chunk(float(0));
}

static void advance(Exec& X, Group& G) {
  if (ic_precond(X.opt.precond)) advance_t<PREC_BIC0>(X, G);
  else advance_t<PREC_JACOBI>(X, G);
}

// Runs one group's state machine to completion on the calling host thread.
static void drive_group(Exec& X, Group& g) {
  advance(X, g);
  while (g.phase != 3) {
    if (!g.inflight) {
      advance(X, g);
      continue;
    }
    hipError_t q = hipEventQuery(g.ev);
    if (q == hipSuccess) {
      g.inflight = false;
      advance(X, g);
    } else if (q != hipErrorNotReady) {
      HIPCHK(q);
    }
  }
}

// Runs every group to completion.  With more than one group, each group is driven by its
// own host thread, so that enqueueing a long chunk of one group never delays the next
// chunk of another.
static void run_groups(Exec& X, std::vector<Group>& G) {
  // streams of the groups start after all work already ordered on the main stream
  HIPCHK(hipEventRecord(X.ev_fork, X.stream));
  for (size_t k = 0; k < G.size(); ++k) {
    Group& g = G[k];
    if (g.s != X.stream) HIPCHK(hipStreamWaitEvent(g.s, X.ev_fork, 0));
    g.phase = 0;
    g.inflight = false;
    g.hbuf = X.h_sys + g.s0;   // disjoint ranges of the pinned mirror
    g.ev = X.ev_poll[k];
  }
  if (G.size() == 1) {
    drive_group(X, G[0]);
  } else {
    std::vector<Error> errs(G.size(), Error{MC_OK, ""});
    run_on_workers(X, (int)G.size(), [&](int k) {
      try {
        drive_group(X, G[k]);
      } catch (const Error& e) {
        errs[k] = e;
      } catch (const std::exception& e) {
        errs[k] = Error{MC_EDEVICE, e.what()};
      }
    });
    for (auto& e : errs)
      if (e.st != MC_OK) throw e;
  }
  for (auto& g : G)
    if (g.s != X.stream) {
      HIPCHK(hipEventRecord(X.ev_join, g.s));
      HIPCHK(hipStreamWaitEvent(X.stream, X.ev_join, 0));
    }
}

static void sys_params(const Exec& X, SysState& S, double tol, bool mixed) {
  S.tol2 = tol * tol;
  S.max_iter = X.opt.max_iter;
  S.otol2 = X.opt.outer_tol * X.opt.outer_tol;
  S.max_outer = X.opt.max_outer;
  S.mixed = mixed ? 1 : 0;
}

// Solve parameters of the records [s0, s1), set by a kernel in stream order (no host wait).
// hist: layers the problem computed in a row before this one (the warm start's history)
static void set_sys_params(Exec& X, int s0, int s1, double tol, bool mixed, int hist = 0) {
  SysState S;
  std::memset(&S, 0, sizeof(S));
  sys_params(X, S, tol, mixed);
  hipLaunchKernelGGL(k_set_params, dim3(cdiv(s1 - s0, 64)), dim3(64), 0, X.stream, X.sys, s0,
                     s1, S.tol2, S.otol2, S.max_iter, S.max_outer, S.mixed, hist);
  HIPCHK(hipGetLastError());
}

// Solve the systems [s0, s1) of table Tb (system parameters already set).  On return the
// pinned mirror X.h_sys holds the final records of [s0, s1) (the groups' last polls).  Decoupled
// tables (split_kinds) number their grid systems first: they form one group on the main
// stream and the fracture systems a second group on the side stream.
static void solve_table(Exec& X, Table& Tb, int s0, int s1, bool assemble, bool mixed,
                        bool split_kinds) {
  std::vector<Group> G;
  auto mk = [&](int kinds, int a, int b, hipStream_t st) {
    Group g;
    g.s = st;
    g.T = &Tb;
    g.kinds = kinds;
    g.s0 = a;
    g.s1 = b;
    g.mixed = mixed;
    g.assemble = assemble;
    G.push_back(g);
  };
  if (split_kinds && Tb.nblk[0][PART_GRID] && Tb.nblk[0][PART_GRAPH]) {
    int ngrid = 0;
    for (auto& q : Tb.hparts) ngrid += q.kind == PART_GRID && q.mg_level == 0;
    const bool one = env_flag("MCDEC_ONE_STREAM", false);
    if (!one) exec_side_streams(X, Tb.has_blocks);
    const bool part = X.stream_grid && !one;
    mk(1, s0, s0 + ngrid, part ? X.stream_grid : X.stream);
    mk(2, s0 + ngrid, s1, one ? X.stream : (part ? X.stream_frac : X.stream2));
  } else {
    mk(3, s0, s1, X.stream);
  }
  run_groups(X, G);
}

// Fills the report from the (already read) system records; returns the first failing
// status.
static mc_status fill_report(const Exec& X, const std::vector<int>& systems,
                             const std::vector<int>& conts_of_sys, mc_report* rep, bool mixed) {
  mc_status st = MC_OK;
  int failed = -1;
  for (size_t k = 0; k < systems.size(); ++k) {
    const SysState& S = X.h_sys[systems[k]];
    const int status = mixed ? S.outer_status : S.status;
    const int c = conts_of_sys[k];
    if (rep && c >= 0 && c < 3) {
      rep->iters[c] = mixed ? S.total_iter : S.iter;
      rep->outer[c] = mixed ? S.outer : 0;
      rep->converged[c] = status == ST_CONV;
      rep->relres[c] = mixed ? (S.obb > 0 ? std::sqrt(S.orr / S.obb) : std::sqrt(S.orr))
                             : (S.bb > 0 ? std::sqrt(S.rr / S.bb) : std::sqrt(S.rr));
      rep->warm_order[c] = S.wsorder;
    }
    if (status != ST_CONV && st == MC_OK) {
      st = status == ST_NOCONV ? MC_ENOCONV : MC_EBREAKDOWN;
      failed = c;
    }
  }
  if (rep) rep->failed = failed;
  return st;
}

static void fill_coupled_report(int ncont, mc_report* rep) {
  if (!rep) return;
  for (int c = 1; c < ncont; ++c) {
    rep->iters[c] = rep->iters[0];
    rep->outer[c] = rep->outer[0];
    rep->converged[c] = rep->converged[0];
    rep->relres[c] = rep->relres[0];
    rep->warm_order[c] = rep->warm_order[0];
  }
}

// The small-system path applies: FP64 Jacobi decoupled schemes with every continuum at
// most opt.small_max unknowns.
static bool small_path(const mc_problem* P) {
  const mc_options& o = P->X.opt;
  if (o.small_max <= 0 || o.precision != MC_FP64 || o.precond != MC_JACOBI ||
      o.scheme == MC_SCHEME_COUPLED)
    return false;
  for (const Cont& C : P->cont)
    if (C.n > o.small_max) return false;
  return true;
}

// Right-hand sides and warm starts of table T (k_rhs), then one workgroup per system of
// parts [0, nsys) runs its whole PCG, all systems in one launch; the records of systems
// [s0, s0 + nsys) are read back.
static void small_solve(mc_problem* P, Table& T, int s0, int nsys) {
  Exec& X = P->X;
  set_sys_params(X, s0, s0 + nsys, X.opt.tol, false, P->hist);
  launch_all(X.stream, T, 0, k_extrap_err<PART_GRID>, k_extrap_err<PART_GRAPH>, X.sys);
  launch_all(X.stream, T, 0, k_rhs<PART_GRID>, k_rhs<PART_GRAPH>, X.sys);
  // LDS-resident form when every system fits: 2-D grids of at most 4096 cells, fracture
  // systems whose p and CSR take at most 64 KiB
  size_t lds = 0;
  bool fits = true;
  for (int k = 0; k < nsys; ++k) {
    const PartD& q = T.hparts[k];
    size_t b = (size_t)q.n * sizeof(double);
    if (q.kind == PART_GRID) {
      fits = fits && q.n <= 1024 * 4 && q.plane == 0;
    } else {
      const size_t nnz = P->gh.col.size();
      b += nnz * (sizeof(double) + sizeof(int)) + (size_t)(q.n + 1) * sizeof(int);
      fits = fits && q.n <= 1024 * 4;
    }
    lds = std::max(lds, b);
  }
  if (fits && lds <= 64 * 1024)
    hipLaunchKernelGGL((k_small_pcg_lds<1024, 4>), dim3(nsys), dim3(1024), lds, X.stream,
                       T.parts, X.sys);
  else
    hipLaunchKernelGGL(k_small_pcg<1024>, dim3(nsys), dim3(1024), 0, X.stream, T.parts, 0,
                       X.sys);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(X.h_sys + s0, X.sys + s0, nsys * sizeof(SysState),
                        hipMemcpyDeviceToHost, X.stream));
  HIPCHK(hipStreamSynchronize(X.stream));
}

static mc_status step_once(mc_problem* P, mc_report* rep) {
  Exec& X = P->X;
  const bool mixed = X.opt.precision == MC_MIXED;
  const int sch = X.opt.scheme;
  std::vector<int> all;
  for (int c = 0; c < P->ncont; ++c) all.push_back(c);
  mc_status st;
  const bool small = small_path(P);
  if (small && (sch == MC_SCHEME_D || sch == MC_SCHEME_EX)) {
    Table& T = upload_table(P, "d" + std::to_string(P->cur), decoupled_parts(P, all, false));
    small_solve(P, T, 0, P->ncont);
    st = fill_report(X, all, all, rep, false);
  } else if (small) {
    st = MC_OK;
    std::vector<int> order = all;
    if (sch == MC_SCHEME_U) std::reverse(order.begin(), order.end());
    for (size_t k = 0; k < order.size(); ++k) {
      const int c = order[k];
      std::vector<PartD> parts = decoupled_parts(P, {c}, false);
      for (size_t j = 0; j < k; ++j) parts[0].tsrc[order[j]] = P->cont[order[j]].ps[1 - P->cur];
      Table& T = upload_table(P, "s" + std::to_string(c) + "_" + std::to_string(P->cur), parts);
      small_solve(P, T, c, 1);
      mc_status s1 = fill_report(X, {c}, {c}, rep, false);
      if (s1 != MC_OK) {
        st = s1;
        break;
      }
    }
  } else if (sch == MC_SCHEME_COUPLED) {
    Table& T = upload_table(P, "coupled" + std::to_string(P->cur), coupled_parts(P, P->ncont, 0));
    set_sys_params(X, P->ncont, P->ncont + 1, X.opt.tol, false, P->hist);
    solve_table(X, T, P->ncont, P->ncont + 1, true, false, false);
    st = fill_report(X, {P->ncont}, {0}, rep, false);
    fill_coupled_report(P->ncont, rep);
  } else if (sch == MC_SCHEME_D || sch == MC_SCHEME_EX) {
    Table& T = upload_table(P, std::string(mixed ? "dm" : "d") + std::to_string(P->cur),
                            decoupled_parts(P, all, mixed));
    set_sys_params(X, 0, P->ncont, mixed ? X.opt.inner_tol : X.opt.tol, mixed, P->hist);
    solve_table(X, T, 0, P->ncont, true, mixed, true);
    st = fill_report(X, all, all, rep, mixed);
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
      set_sys_params(X, c, c + 1, mixed ? X.opt.inner_tol : X.opt.tol, mixed, P->hist);
      solve_table(X, T, c, c + 1, true, mixed, false);
      mc_status s1 = fill_report(X, {c}, {c}, rep, mixed);
      if (s1 != MC_OK) {
        st = s1;
        break;
      }
    }
  }
  if (st == MC_OK) {
    P->cur ^= 1;
    P->step_count += 1;
    P->hist += 1;
  } else {
    P->hist = 0;   // a failed layer may have overwritten the other state buffer
  }
  return st;
}

// ------------------------------------------------------------------------------------
// batches
// ------------------------------------------------------------------------------------
static bool coupled_class(int scheme) { return scheme == MC_SCHEME_COUPLED; }

static void batch_check(const mc_batch* B, mc_problem* const* probs, int n) {
  if (n < 1 || !probs) fail("a batch step needs at least one problem");
  const mc_options& o = B->X.opt;
  for (int i = 0; i < n; ++i) {
    const mc_problem* P = probs[i];
    if (!P) fail("problem " + std::to_string(i) + " is NULL");
    for (int j = 0; j < i; ++j)
      if (probs[j] == P) fail("problem " + std::to_string(i) + " appears twice");
    const mc_options& q = P->X.opt;
    if (q.scheme == MC_SCHEME_L || q.scheme == MC_SCHEME_U)
      fail("problem " + std::to_string(i) + ": the L- and U-schemes are not batched");
    if (coupled_class(q.scheme) != coupled_class(o.scheme) || q.precision != o.precision ||
        q.precond != o.precond)
      fail("problem " + std::to_string(i) +
           ": scheme class, precision and preconditioner must match the batch options");
  }
}

// One time layer of every problem.  Decoupled: system records and parts list the grid
// continua of all problems first, then their fracture continua; coupled: one system per
// problem.  Each problem keeps its own tilings and partial-sum slots, so its arithmetic is
// the same as when it is stepped alone.
static mc_status batch_step_once(mc_batch* B, mc_problem* const* probs, int n, mc_report* reps) {
  Exec& X = B->X;
  const bool coupled = coupled_class(X.opt.scheme);
  const bool mixed = X.opt.precision == MC_MIXED;
  std::vector<PartD> parts;
  std::vector<PartTiling> til;
  std::vector<SysState> hs;
  std::vector<std::vector<int>> sys_of(n), cont_of(n);
  std::vector<mc_problem*> owner;
  auto rec = [&](mc_problem* P, int sI, int nA, int nB) {
    SysState S;
    std::memset(&S, 0, sizeof(S));
    S.partA = P->partA[sI];
    S.partB = P->partB[sI];
    S.nslotsA = nA;
    S.nslotsB = nB;
    S.hist = P->hist;
    S.done = 1;
    sys_params(X, S, mixed ? X.opt.inner_tol : X.opt.tol, mixed);
    hs.push_back(S);
  };
  if (!coupled) {
    for (int pass = 0; pass < 2; ++pass)          // grid continua, then fracture continua
      for (int i = 0; i < n; ++i) {
        mc_problem* P = probs[i];
        for (int c = 0; c < P->ncont; ++c) {
          if ((P->cont[c].kind == PART_GRID) != (pass == 0)) continue;
          const int sI = (int)hs.size();
          rec(P, c, P->cont[c].blocks[0], P->cont[c].blocks[1] + P->cont[c].blocks[2]);
          parts.push_back(base_part(P, c, sI, 0, 0, mixed));
          til.push_back(tiling_of(P, c));
          owner.push_back(P);
          sys_of[i].push_back(sI);
          cont_of[i].push_back(c);
        }
      }
    for (int j = 0, np = (int)parts.size(); j < np; ++j) {   // V-cycle levels after all parts
      const size_t before = parts.size();
      add_mg_levels(owner[j], parts, j, mixed);
      for (size_t k = before; k < parts.size(); ++k) til.push_back(tiling_of(owner[j], parts[k].cont));
    }
  } else {
    for (int i = 0; i < n; ++i) {
      mc_problem* P = probs[i];
      const int sI = (int)hs.size();
      int nA = 0, nB = 0;
      for (auto& C : P->cont) {
        nA += C.blocks[0];
        nB += C.blocks[1] + C.blocks[2];
      }
      rec(P, P->ncont, nA, nB);
      std::vector<PartD> cp = coupled_parts(P, sI, (int)parts.size());
      for (auto& q : cp) {
        parts.push_back(q);
        til.push_back(tiling_of(P, q.cont));
      }
      sys_of[i].push_back(sI);
      cont_of[i].push_back(0);
    }
  }
  const int nsys = (int)hs.size();
  if (exec_sys_capacity(X, nsys)) {
    drop_graphs(B->tab[0]);
    drop_graphs(B->tab[1]);
  }
  HIPCHK(hipMemcpyAsync(X.sys, hs.data(), nsys * sizeof(SysState), hipMemcpyHostToDevice,
                        X.stream));
  link_mg(parts);
  Table* T = nullptr;
  for (auto& t : B->tab)
    if (table_matches(t, parts, til)) T = &t;
  if (!T) {
    T = &B->tab[B->lru];
    B->lru ^= 1;
    fill_table(*T, B->mem, X.stream, std::move(parts), til);
  }
  HIPCHK(hipStreamSynchronize(X.stream));
  solve_table(X, *T, 0, nsys, true, mixed, !coupled);
  mc_status st = MC_OK;
  for (int i = 0; i < n; ++i) {
    mc_problem* P = probs[i];
    mc_report* r = reps ? &reps[i] : nullptr;
    if (r) {
      std::memset(r, 0, sizeof(*r));
      r->n_cont = P->ncont;
    }
    mc_status si = fill_report(X, sys_of[i], cont_of[i], r, mixed && !coupled);
    if (coupled) fill_coupled_report(P->ncont, r);
    if (si == MC_OK) {
      P->cur ^= 1;
      P->step_count += 1;
      P->hist += 1;
    } else {
      P->hist = 0;
    }
    if (si != MC_OK && st == MC_OK) {
      st = si;
      B->err = "problem " + std::to_string(i) + " failed in continuum " +
               std::to_string(r ? r->failed : -1);
    }
    if (r) r->step = P->step_count;
  }
  return st;
}

// ------------------------------------------------------------------------------------
// autotuner: workgroups per launch, chosen by timing
// ------------------------------------------------------------------------------------
// Median time (microseconds) of the operator (fam 0) or update (fam 1) kernel of continuum c
// of P in its current tilings, over `iters` iterations of a real PCG run on the device (the
// record's tolerance is 0, so the system never stops).  Only scratch vectors and the next
// state buffer are written; the current state is untouched.
template <class T, int PREC>
static double time_tiling(mc_problem* P, int c, int fam, int iters) {
  Exec& X = P->X;
  Cont& C = P->cont[c];
  const bool fp32 = sizeof(T) == 4;
  hipStream_t s = X.stream;
  Table& Tb = upload_table(P, "tune", decoupled_parts(P, {c}, fp32, false));
  SysState S;
  std::memset(&S, 0, sizeof(S));
  S.partA = P->partA[c];
  S.partB = P->partB[c];
  S.nslotsA = C.blocks[0];
  S.nslotsB = C.blocks[1] + (C.kind == PART_GRAPH ? C.blocks[2] : 0);   // no V-cycle here
  S.max_iter = 1 << 30;
  S.max_outer = 1;
  S.done = 1;
  HIPCHK(hipMemcpyAsync(X.sys + c, &S, sizeof(S), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, X.sys, c, c + 1);
  launch_all(s, Tb, 0, k_rhs<PART_GRID>, k_rhs<PART_GRAPH>, X.sys);
  if (fp32) {
    launch_all(s, Tb, 0, k_residual64<PART_GRID>, k_residual64<PART_GRAPH>, X.sys);
    launch_all(s, Tb, 1, k_residual<PREC, PART_GRID>, k_residual<PREC, PART_GRAPH>, X.sys);
    launch_schur<float>(X, Tb, s);
  }
  else {
    launch_all(s, Tb, 1, k_init<PREC, PART_GRID>, k_init<PREC, PART_GRAPH>, X.sys);
    launch_schur<double>(X, Tb, s);
  }
  const int warm = 3, tot = warm + iters;
  std::vector<hipEvent_t> ev(3 * tot, nullptr);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  Group g;
  g.s = s;
  g.T = &Tb;
  g.kinds = 3;
  for (int j = 0; j < tot; ++j) {
    HIPCHK(hipEventRecord(ev[3 * j], s));
    launch2(g, 0, k_pcg_A<T, PREC, PART_GRID>, k_pcg_A<T, PREC, PART_GRAPH>, X.sys);
    HIPCHK(hipEventRecord(ev[3 * j + 1], s));
    launch2(g, 1, k_pcg_B<T, PREC, PART_GRID>, k_pcg_B<T, PREC, PART_GRAPH>, X.sys);
    HIPCHK(hipEventRecord(ev[3 * j + 2], s));
    launch_schur<T>(X, Tb, s);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  std::vector<float> t;
  for (int j = warm; j < tot; ++j) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ev[3 * j + fam], ev[3 * j + fam + 1]));
    t.push_back(ms);
  }
  for (auto e : ev) (void)hipEventDestroy(e);
  std::sort(t.begin(), t.end());
  return 1e3 * t[t.size() / 2];
}

static double time_tiling_any(mc_problem* P, int c, int fam, int iters) {
  const bool fp32 = P->X.opt.precision == MC_MIXED, bic0 = ic_precond(P->X.opt.precond);
  if (fp32) return bic0 ? time_tiling<float, PREC_BIC0>(P, c, fam, iters)
                        : time_tiling<float, PREC_JACOBI>(P, c, fam, iters);
  return bic0 ? time_tiling<double, PREC_BIC0>(P, c, fam, iters)
              : time_tiling<double, PREC_JACOBI>(P, c, fam, iters);
}

// Re-derive every continuum's tilings (tuned choices included) and the records' slot counts.
static void refresh_tilings(mc_problem* P) {
  const size_t nb = (P->ncont + 1) * sizeof(SysState);
  HIPCHK(hipMemcpy(P->X.h_sys, P->X.sys, nb, hipMemcpyDeviceToHost));
  set_slot_counts(P, P->X.h_sys);
  HIPCHK(hipMemcpy(P->X.sys, P->X.h_sys, nb, hipMemcpyHostToDevice));
  clear_tables(P);
}

// For every size class present among the problems' continua, time candidate workgroup
// counts of the operator tiling, then of the update tiling, on the first continuum of that
// class, and record the fastest as tiles per workgroup for the class.
static void autotune(mc_problem* const* probs, int n, int iters) {
  std::vector<std::vector<int>> seen;
  for (int i = 0; i < n; ++i) {
    mc_problem* P = probs[i];
    const bool bic0 = ic_precond(P->X.opt.precond), fp32 = P->X.opt.precision == MC_MIXED;
    for (int c = 0; c < P->ncont; ++c) {
      Cont& C = P->cont[c];
      for (int fam = 0; fam < 2; ++fam) {
        std::vector<int> key = tune_key(C.tiles, C.kind, fam, bic0, fp32);
        if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
        seen.push_back(key);
        {
          std::lock_guard<std::mutex> lk(g_tune_mu);
          if (g_tune.count(key)) continue;   // tuned earlier in this process
        }
        std::vector<int> tpw = (fam == 1 && bic0 && C.kind == PART_GRID)
                                   ? std::vector<int>{2, 4, 8}
                                   : std::vector<int>{1, 2, 4};
        const int keep = C.blocks[fam];
        double best = 1e300;
        int best_b = keep;
        std::vector<int> tried;
        for (int t : tpw) {
          const int b = std::max(1, (C.tiles + t - 1) / t);
          if (std::find(tried.begin(), tried.end(), b) != tried.end()) continue;
          tried.push_back(b);
          C.blocks[fam] = b;
          const double us = time_tiling_any(P, c, fam, iters);
          if (us < best) {
            best = us;
            best_b = b;
          }
        }
        C.blocks[fam] = best_b;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = (C.tiles + best_b - 1) / best_b;
      }
    }
    clear_tables(P);
  }
  // the timing runs wrote PCG iterates into the next-state buffers, which a following layer
  // would otherwise take for the layer before the current one (its extrapolated warm start)
  for (int i = 0; i < n; ++i) {
    probs[i]->hist = 0;
    refresh_tilings(probs[i]);
  }
}

// Device bytes mc_create_problem allocates for a descriptor under options o (the sizes of
// every array create() and build_coefficients() request; chains and fracture tiles are
// bounded by nf + 1), plus launch tables and a rounding allowance per allocation.
static int64_t footprint(const mc_problem_desc& d, const mc_options& o) {
  const int64_t nzp = d.nz > 1 ? d.nz : 1;
  const int64_t nc = (int64_t)d.nx * d.ny * nzp, nf = d.nf, ne = d.ne;
  const int64_t gt = (int64_t)cdiv(d.nx, MC_TX) * cdiv((int64_t)d.ny * nzp, MC_TY);
  const bool bic0 = ic_precond(o.precond), mixed = o.precision == MC_MIXED;
  int64_t b = 0, nalloc = 0;
  auto A = [&](int64_t bytes) {
    b += std::max<int64_t>(bytes, 8);
    nalloc += 1;
  };
  for (int a = 0; a < d.n_omega; ++a) {
    if (d.omega[a].k) A(8 * nc);
    if (d.omega[a].src) A(8 * nc);
  }
  if (nf) {
    A(4 * nf);                    // host
    A(8 * nf);                    // flen
    A(8 * d.n_omega * nf);        // sigma_f
    A(4 * (nf + 1));              // rowptr
    A(4 * 2 * ne);                // col
    A(4 * 2 * ne);                // eidx
    A(8 * std::max<int64_t>(ne, 1));
    A(4 * (nc + 1));              // hptr
    A(4 * nf);                    // hidx
    A(4 * (nf + 1));              // chain_ptr
    A(4 * (nf + 1));              // gtile
    if (d.src_f) A(8 * nf);
    if (d.well_q) A(8 * nf);
    if (d.well_q && d.well_p) A(8 * nf);
  }
  const int ncont = d.n_omega + (nf ? 1 : 0);
  int64_t ctiles = 0;
  for (int c = 0; c < ncont; ++c) {
    const bool grid = c < d.n_omega;
    const int64_t n = grid ? nc : nf;
    const int64_t tiles = grid ? gt : nf + 1;
    const int64_t slots = grid ? 2 * tiles : tiles;   // grid: room for a V-cycle's slots
    ctiles += slots;
    A(8 * n);                     // diag
    A(8 * n);                     // F
    if (grid) {
      A(8 * n);                   // tx
      A(8 * n);                   // ty
      if (nzp > 1) {
        A(8 * n);                 // tz
        if (mixed) A(4 * n);      // tz32
      }
    } else {
      A(8 * std::max<int64_t>(1, 2 * ne));
      A(8 * n);                   // mt
    }
    for (int k = 0; k < 7; ++k) A(8 * n);   // two states, b, r, p, p2, q
    if (o.warm_start == WS_ADAPTIVE)
      for (int k = 0; k < 3; ++k) A(8 * n);   // the adaptive warm start's layer history
    A(8 * MC_SLOT * slots);       // partials of its decoupled system
    A(8 * MC_SLOT * slots);
    if (grid && o.precond == MC_MG) {   // V-cycle levels
      if (!mixed) A(4 * n);               // FP32 diagonal of the V-cycle's residuals
      int64_t lx = d.nx, ly = d.ny;
      if (lx * ly > MC_MG_COARSE) {
        A(8 * n);                 // pre-smoothed z of the finest level
        if (mixed) A(4 * n);
        A(8 * 2 * 128);           // partial sums of the levels' dominance test
        const int64_t ne = (lx + MC_TX - 1) / MC_TX * ly;
        A(8 * 2 * ne);            // block edges of the fused restriction
        A(4 * ne);
      }
      while (lx * ly > MC_MG_COARSE) {   // (a hierarchy that stops early holds less)
        lx = (lx + 1) / 2;
        ly = (ly + 1) / 2;
        const int64_t m = lx * ly;
        for (int k = 0; k < 7; ++k) A(8 * m);   // operator, factor, r, z_p, z
        for (int k = 0; k < 3; ++k) A(4 * m);   // FP32 operator copies
        if (m > MC_MG_COARSE) A(4 * m);          // FP32 factor
        else {
          const int64_t ld = m + (m & 1);
          A(8 * ld * ld);                        // dense inverse (even leading dimension)
          A(4 * ld * ld);                        // its FP32 copy
        }
        if (mixed) for (int k = 0; k < 3; ++k) A(4 * m);
      }
    }
    if (bic0) {
      A(8 * n);                   // fdinv
      A(8 * n);                   // z
      if (grid) {
        A(4 * n);                 // FP32 factor and conductances of the tile sweeps
        A(4 * n);
        A(4 * n);
      } else {
        A(8 * n);                 // cT
      }
    }
    if (mixed) {
      A(4 * n);                   // diag32
      if (bic0) {
        if (!grid) A(4 * n);      // fdinv32 (grid: above)
        if (!grid) A(4 * n);      // cT32
        A(4 * n);                 // z32
      }
      if (grid && !bic0) {
        A(4 * n);                 // tx32
        A(4 * n);                 // ty32
      }
      if (!grid) A(4 * std::max<int64_t>(1, 2 * ne));
      for (int k = 0; k < 5; ++k) A(4 * n);   // x32, r32, p32, p232, q32
    }
  }
  // exact fracture solve (block IC(0)): inverse Schur complement of the crossing cells,
  // responses and indices
  if (nf && bic0) {
    const int64_t Kall = count_crossing_cells(d.nf, d.ne, d.edges);
    const int64_t kmax = exact_crossing_max();
    int64_t K = Kall <= kmax ? Kall : 0;
    if (Kall > kmax && fracture_blocks_on()) {   // the two-level block preconditioner
      std::vector<int> node, blk;
      const int64_t nb = build_blocks(d.nf, build_graph(d.nf, d.ne, d.edges), node, blk);
      if (nb <= MC_SCHUR_KMAX) {
        K = nb;
        A(4 * K * kBlockCells);                 // block cells
        A(4 * K * kBlockCells * kBlockCells);   // block inverses
      }
    }
    if (K > 0) {
      A(4 * K);                   // xcells
      A(4 * (nf + 2));            // xtile
      A(8 * nf);                  // xlr
      A(8 * nf);                  // cl
      A(8 * nf);                  // cr
      A(8 * K);                   // cxl
      A(8 * K);                   // cxr
      A(8 * K * K);               // S^-1
      A(8 * K);                   // g
      A(8 * K);                   // z_X
      if (mixed) {
        A(4 * nf);
        A(4 * nf);
        A(4 * K * K);
        A(4 * K);
        A(4 * K);
      }
      const int64_t ks = (K + MC_SCHUR_ROWS - 1) / MC_SCHUR_ROWS;
      A(8 * MC_SLOT * ks);        // partial slots of the crossing product (decoupled and coupled)
      A(8 * MC_SLOT * ks);
      ctiles += ks;
    }
  }
  A(8 * MC_SLOT * ctiles);        // partials of the coupled system
  A(8 * MC_SLOT * ctiles);
  // launch tables: parts and tile lists of a few keys
  b += 8 * (int64_t)(sizeof(PartD) * 8 + sizeof(Tile) * 4 * (ctiles + 64));
  return b + nalloc * 4096 + (1 << 20);
}

// ------------------------------------------------------------------------------------
// solve without allocation
// ------------------------------------------------------------------------------------
// A variant of the continuum solve for callers that cannot allocate device memory: every
// buffer the solve needs beyond the caller's right-hand side and solution and the
// problem's own coefficients (the launch descriptor and tile lists, the system record, the
// partial-sum slots, the PCG vectors r, p, p', q, z and the crossing-cell vectors) is
// carved out of one static device array.  Each device holds its own copy of the array
// for the life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device.  Every call on a device shares that copy:
// calls that overlap on one device race.
static __device__ __align__(256) unsigned char scratch[MC_NOALLOC_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, unsigned char*> g_scratch_addr;   // device -> its copy of `scratch`

// Address of the calling thread's current device's copy of `scratch` (looked up once per
// device, with that device current).
static unsigned char* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    throw Error{MC_EDEVICE, std::string("hipGetSymbolAddress of the static workspace failed: ") +
                                hipGetErrorString(e)};
  }
  g_scratch_addr[dev] = (unsigned char*)ptr;
  return (unsigned char*)ptr;
}

// Consecutive 256-byte aligned pieces of a workspace; with base == nullptr it only counts.
struct Carve {
  unsigned char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

// Bytes of the static workspace a solve of continuum `c` needs in the current tiling.
static size_t noalloc_bytes(const mc_problem* P, int c, const std::vector<Tile>* tl) {
  const Cont& C = P->cont[c];
  Carve cv{nullptr};
  cv.take<SysState>(1);
  cv.take<PartD>(1);
  for (int f = 0; f < 3; ++f) cv.take<Tile>(tl[f].size());
  cv.take<double>((size_t)C.blocks[0] * MC_SLOT);
  cv.take<double>((size_t)(C.blocks[1] + C.blocks[2]) * MC_SLOT);
  for (int v = 0; v < 5; ++v) cv.take<double>(C.n);
  if (C.K > 0) {
    cv.take<double>(C.K);
    cv.take<double>(C.K);
  }
  return cv.off;
}

template <int PREC, int KIND>
static void noalloc_iterate(hipStream_t s, const PartD* dp, Tile* const* dt, const int* nb,
                            SysState* dsys, SysState& hs, int max_iter) {
  const bool schur = PREC == PREC_BIC0 && KIND == PART_GRAPH && nb[2] > 0;
  hipLaunchKernelGGL((k_init<PREC, KIND>), dim3(nb[1]), dim3(MC_BLOCK), 0, s, dp, dt[1], dsys);
  if (schur)
    hipLaunchKernelGGL(k_schur<double>, dim3(nb[2]), dim3(MC_BLOCK), 0, s, dp, dt[2], dsys);
  HIPCHK(hipGetLastError());
  long launched = 0;
  int K = 8;
  for (;;) {
    for (int j = 0; j < K; ++j) {
      hipLaunchKernelGGL((k_pcg_A<double, PREC, KIND>), dim3(nb[0]), dim3(MC_BLOCK), 0, s, dp,
                         dt[0], dsys);
      hipLaunchKernelGGL((k_pcg_B<double, PREC, KIND>), dim3(nb[1]), dim3(MC_BLOCK), 0, s, dp,
                         dt[1], dsys);
      if (schur)
        hipLaunchKernelGGL(k_schur<double>, dim3(nb[2]), dim3(MC_BLOCK), 0, s, dp, dt[2], dsys);
    }
    HIPCHK(hipGetLastError());
    launched += K;
    HIPCHK(hipMemcpyAsync(&hs, dsys, sizeof(SysState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hs.done) return;
    // iterations launched after convergence return at once, so overshooting costs launches
    if (launched > (long)max_iter + 1)
      throw Error{MC_EDEVICE, "PCG did not report completion within max_iter iterations"};
    K = (int)std::min<long>(std::min(2 * K, 64), (long)max_iter + 2 - launched);
    K = std::max(K, 1);
  }
}

static mc_status solve_noalloc(mc_problem* P, int c, const double* rhs, double* x,
                               mc_report* rep) {
  Exec& X = P->X;
  if (X.opt.precision == MC_MIXED)
    throw Error{MC_EINVAL, "the no-allocation solve is FP64; set precision MC_FP64"};
  if (X.opt.precond == MC_MG)
    throw Error{MC_EINVAL, "the no-allocation solve takes Jacobi or block IC(0) (MC_JACOBI, "
                           "MC_BIC0); the V-cycle's level vectors do not fit its workspace"};
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != P->device)
    throw Error{MC_EINVAL, "the problem's device (" + std::to_string(P->device) +
                               ") must be current for the no-allocation solve"};
  const Cont& C = P->cont[c];
  const bool bic0 = X.opt.precond == MC_BIC0;
  PartD q = base_part(P, c, 0, 0, 0, false);   // system record 0, slots from 0
  const PartTiling til = tiling_of(P, c);
  std::vector<Tile> tl[3];
  const bool xcd = env_flag("MCDEC_XCD", true);
  for (int f = 0; f < 3; ++f) part_tiles(q, 0, til, f, xcd, tl[f]);
  const size_t need = noalloc_bytes(P, c, tl);
  if (need > (size_t)MC_NOALLOC_BYTES)
    throw Error{MC_EINVAL, "continuum " + std::to_string(c) + " (" + std::to_string(C.n) +
                               " unknowns) needs " + std::to_string(need) +
                               " bytes of workspace; the no-allocation solve has " +
                               std::to_string((long)MC_NOALLOC_BYTES)};
  Carve cv{scratch_on(dev)};
  SysState* dsys = cv.take<SysState>(1);
  PartD* dpart = cv.take<PartD>(1);
  Tile* dt[3];
  for (int f = 0; f < 3; ++f) dt[f] = cv.take<Tile>(tl[f].size());
  double* slotA = cv.take<double>((size_t)C.blocks[0] * MC_SLOT);
  double* slotB = cv.take<double>((size_t)(C.blocks[1] + C.blocks[2]) * MC_SLOT);
  double* vec[5];
  for (int v = 0; v < 5; ++v) vec[v] = cv.take<double>(C.n);
  q.x = x;
  q.x64 = x;
  q.b = const_cast<double*>(rhs);
  q.r = vec[0];
  q.r64 = vec[0];
  q.p = vec[1];
  q.p2 = vec[2];
  q.q = vec[3];
  q.z = vec[4];
  if (C.K > 0) {
    q.gX = cv.take<double>(C.K);
    q.zX = cv.take<double>(C.K);
  }
  // the record: solve parameters, a fresh start, and the slots of this call's tiling
  SysState hs;
  std::memset(&hs, 0, sizeof(hs));
  sys_params(X, hs, X.opt.tol, false);
  hs.status = ST_RUN;
  hs.outer_status = ST_RUN;
  hs.nslotsA = C.blocks[0];
  hs.nslotsB = C.blocks[1] + C.blocks[2];
  hs.partA = slotA;
  hs.partB = slotB;
  const hipStream_t s = X.stream;
  HIPCHK(hipMemcpyAsync(dsys, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dpart, &q, sizeof(q), hipMemcpyHostToDevice, s));
  int nb[3];
  for (int f = 0; f < 3; ++f) {
    nb[f] = (int)tl[f].size();
    if (nb[f])
      HIPCHK(hipMemcpyAsync(dt[f], tl[f].data(), tl[f].size() * sizeof(Tile),
                            hipMemcpyHostToDevice, s));
  }
  const int mi = X.opt.max_iter;
  if (q.kind == PART_GRID) {
    if (bic0) noalloc_iterate<PREC_BIC0, PART_GRID>(s, dpart, dt, nb, dsys, hs, mi);
    else noalloc_iterate<PREC_JACOBI, PART_GRID>(s, dpart, dt, nb, dsys, hs, mi);
  } else {
    if (bic0) noalloc_iterate<PREC_BIC0, PART_GRAPH>(s, dpart, dt, nb, dsys, hs, mi);
    else noalloc_iterate<PREC_JACOBI, PART_GRAPH>(s, dpart, dt, nb, dsys, hs, mi);
  }
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->n_cont = P->ncont;
    rep->failed = -1;
    rep->step = P->step_count;
    if (c < 3) {
      rep->iters[c] = hs.iter;
      rep->converged[c] = hs.status == ST_CONV;
      rep->relres[c] = hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : std::sqrt(hs.rr);
    }
  }
  if (hs.status != ST_CONV) {
    if (rep) rep->failed = c;
    return hs.status == ST_NOCONV ? MC_ENOCONV : MC_EBREAKDOWN;
  }
  return MC_OK;
}

void spd_inverse(double* S, int K, hipStream_t s, int lda) { invert_spd(S, K, s, lda); }

void fine_view(const mc_problem* P, FineView& v) {
  if (P->nz > 1) throw std::invalid_argument("the coarse-grid path is defined for 2-D grids");
  if (P->X.opt.scheme == MC_SCHEME_EX)
    throw std::invalid_argument("the coarse-grid path needs a problem whose diagonals include "
                                "the transfer (any scheme but MC_SCHEME_EX)");
  v.nx = P->d.nx;
  v.ny = P->d.ny;
  v.nz = P->nz;
  v.n_omega = P->n_omega;
  v.nf = P->nf;
  v.ncont = P->ncont;
  v.scheme = P->X.opt.scheme;
  v.ncell = P->ncell;
  v.h = P->d.h;
  v.tau = P->d.tau;
  v.s12 = P->n_omega == 2 ? omega_transfer(P) : 0.0;
  for (int c = 0; c < P->ncont; ++c) {
    const Cont& C = P->cont[c];
    v.diag[c] = C.diag;
    v.F[c] = C.F;
    v.state[c] = C.ps[P->cur];
    if (c < P->n_omega) {
      v.mtau[c] = C.mtau;
      v.c[c] = P->d.omega[c].c;
      v.has_t[c] = C.has_t;
      v.tconst[c] = C.tconst;
      v.tx[c] = C.tx;
      v.ty[c] = C.ty;
    } else {
      v.mt = C.mt;
      v.val = C.val;
    }
  }
  v.flen = P->flen;
  v.aperture = P->d.aperture;
  v.c_f = P->d.c_f;
  v.rowptr = P->rowptr;
  v.col = P->col;
  v.host = P->host;
  v.hptr = P->hptr;
  v.hidx = P->hidx;
  v.sigma_f = P->sigma_f;
  v.stream = P->X.stream;
  v.device = P->device;
  v.h_host = P->host_h;
  v.h_rowptr = P->gh.rowptr;
  v.h_col = P->gh.col;
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
  if (P->X.stream) (void)hipStreamSynchronize(P->X.stream);
  mc::clear_tables(P);
  mc::exec_release(P->X);   // every stream idle before the memory goes back
  P->mem.release();
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
  if (P->X.opt.precision == MC_MIXED)
    throw mc::Error{MC_EINVAL, "mc_solve_continuum solves in FP64; set precision MC_FP64"};
  auto t0 = std::chrono::steady_clock::now();
  std::vector<PartD> parts = mc::decoupled_parts(P, {alpha}, false);
  parts[0].x = x;
  parts[0].x64 = x;
  parts[0].b = const_cast<double*>(rhs);
  mc::Table& T = mc::upload_table(P, "solve" + std::to_string(alpha), parts);
  mc::set_sys_params(P->X, alpha, alpha + 1, P->X.opt.tol, false);
  mc::solve_table(P->X, T, alpha, alpha + 1, false, false, false);
  mc_report r;
  std::memset(&r, 0, sizeof(r));
  r.n_cont = P->ncont;
  mc_status st = mc::fill_report(P->X, {alpha}, {alpha}, &r, false);
  r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  r.step = P->step_count;
  if (rep) *rep = r;
  return st;
  ABI_END(P)
}

mc_status mc_solve_continuum_noalloc(mc_problem* P, int32_t alpha, const double* rhs,
                                     double* x, mc_report* rep) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (alpha < 0 || alpha >= P->ncont) throw mc::Error{MC_EINVAL, "alpha out of range"};
  if (!rhs || !x) throw mc::Error{MC_EINVAL, "rhs and x must be device pointers"};
  auto t0 = std::chrono::steady_clock::now();
  mc_report r;
  mc_status st = mc::solve_noalloc(P, alpha, rhs, x, &r);
  r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = r;
  if (st != MC_OK) P->err = "no-allocation solve of continuum " + std::to_string(alpha) + " failed";
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
  mc::launch_all(P->X.stream, T, 0, mc::k_apply<PART_GRID>, mc::k_apply<PART_GRAPH>);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(P->X.stream));
  return MC_OK;
  ABI_END(P)
}

mc_status mc_apply_coupled(mc_problem* P, const double* x, double* y) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (!x || !y) throw mc::Error{MC_EINVAL, "x and y must be device pointers"};
  std::vector<PartD> parts = mc::coupled_parts(P, P->ncont, 0);
  long off = 0;
  for (int c = 0; c < P->ncont; ++c) {
    parts[c].x = const_cast<double*>(x) + off;
    parts[c].q = y + off;
    off += P->cont[c].n;
  }
  mc::Table& T = mc::upload_table(P, "applyc", parts);
  mc::launch_all(P->X.stream, T, 0, mc::k_apply<PART_GRID>, mc::k_apply<PART_GRAPH>);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(P->X.stream));
  return MC_OK;
  ABI_END(P)
}

mc_status mc_apply_precond(mc_problem* P, int32_t alpha, const double* r, double* z) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (alpha < 0 || alpha >= P->ncont) throw mc::Error{MC_EINVAL, "alpha out of range"};
  if (!r || !z) throw mc::Error{MC_EINVAL, "r and z must be device pointers"};
  std::vector<PartD> parts = mc::decoupled_parts(P, {alpha}, false);
  parts[0].r = const_cast<double*>(r);
  parts[0].z = z;
  mc::Table& T = mc::upload_table(P, "prec" + std::to_string(alpha), parts);
  if (mc::ic_precond(P->X.opt.precond)) {
    mc::launch_all(P->X.stream, T, 1, mc::k_precond<PREC_BIC0, PART_GRID>,
                   mc::k_precond<PREC_BIC0, PART_GRAPH>);
    mc::launch_vcycle<double>(T, P->X.stream, nullptr, false);
    if (T.nblk[2][PART_GRAPH]) {   // fracture: crossing cells, then z = y + block responses
      hipLaunchKernelGGL(mc::k_schur_apply, dim3(T.nblk[2][PART_GRAPH]), dim3(MC_BLOCK), 0,
                         P->X.stream, T.parts, T.tiles[2][PART_GRAPH]);
      hipLaunchKernelGGL(mc::k_schur_finish, dim3(T.nblk[1][PART_GRAPH]), dim3(MC_BLOCK), 0,
                         P->X.stream, T.parts, T.tiles[1][PART_GRAPH]);
    }
  }
  else
    mc::launch_all(P->X.stream, T, 1, mc::k_precond<PREC_JACOBI, PART_GRID>,
                   mc::k_precond<PREC_JACOBI, PART_GRAPH>);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(P->X.stream));
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
  parts[0].extrap = WS_PREVIOUS;      // (no history kept or read)
  parts[0].coupled = 0;
  mc::Table& T = mc::upload_table(P, "rhs" + std::to_string(alpha), parts);
  mc::launch_all(P->X.stream, T, 0, mc::k_rhs<PART_GRID>, mc::k_rhs<PART_GRAPH>, P->X.sys);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(P->X.stream));
  return MC_OK;
  ABI_END(P)
}

mc_status mc_get_state(mc_problem* P, int32_t alpha, double* out) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (alpha < 0 || alpha >= P->ncont || !out) throw mc::Error{MC_EINVAL, "bad argument"};
  HIPCHK(hipMemcpyAsync(out, P->cont[alpha].ps[P->cur], P->cont[alpha].n * sizeof(double),
                        hipMemcpyDeviceToHost, P->X.stream));
  HIPCHK(hipStreamSynchronize(P->X.stream));
  return MC_OK;
  ABI_END(P)
}

mc_status mc_set_state(mc_problem* P, int32_t alpha, const double* in) {
  if (!P) return MC_EINVAL;
  ABI_BEGIN
  if (alpha < 0 || alpha >= P->ncont || !in) throw mc::Error{MC_EINVAL, "bad argument"};
  P->hist = 0;   // the layer history no longer describes the state
  HIPCHK(hipMemcpyAsync(P->cont[alpha].ps[P->cur], in, P->cont[alpha].n * sizeof(double),
                        hipMemcpyHostToDevice, P->X.stream));
  HIPCHK(hipStreamSynchronize(P->X.stream));
  return MC_OK;
  ABI_END(P)
}

mc_status mc_set_options(mc_problem* P, const mc_options* o) {
  if (!P || !o) return MC_EINVAL;
  ABI_BEGIN
  std::string m = mc::validate_options(*o);
  if (!m.empty()) throw mc::Error{MC_EINVAL, m};
  if (o->stream && o->stream != (void*)P->X.stream)
    throw mc::Error{MC_EINVAL, "the stream cannot change after creation"};
  if (P->nz > 1 && o->precond == MC_MG)
    throw mc::Error{MC_EINVAL, "the multigrid preconditioner needs a 2-D grid (nz <= 1)"};
  const mc_options& cur = P->X.opt;
  const bool rebuild = (o->scheme == MC_SCHEME_EX) != (cur.scheme == MC_SCHEME_EX) ||
                       (o->precision != cur.precision) || (o->precond != cur.precond);
  if (o->warm_start != cur.warm_start) P->hist = 0;   // the history is kept per mode
  P->X.opt = *o;
  P->X.opt.stream = P->X.stream;
  mc::ensure_history(P);
  if (rebuild) mc::build_coefficients(P);
  mc::clear_tables(P);
  // the update tiling depends on the preconditioner: refresh the slot counts
  const size_t nb = (P->ncont + 1) * sizeof(SysState);
  HIPCHK(hipMemcpy(P->X.h_sys, P->X.sys, nb, hipMemcpyDeviceToHost));
  mc::set_slot_counts(P, P->X.h_sys);
  HIPCHK(hipMemcpy(P->X.sys, P->X.h_sys, nb, hipMemcpyHostToDevice));
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
  if (P->ncont > P->n_omega) {
    const Cont& F = P->cont[P->n_omega];
    info->n_crossing = F.fblocks ? 0 : F.K;
    info->n_frac_blocks = F.fblocks ? F.K : 0;
  }
  for (int c = 0; c < P->ncont && c < 3; ++c) {
    info->tiles[c] = P->cont[c].tiles;
    info->blocks[c][0] = P->cont[c].blocks[0];
    info->blocks[c][1] = P->cont[c].blocks[1];
    info->mg_levels[c] = P->cont[c].mg_on ? (int32_t)P->cont[c].mg.size() : 0;
    if (P->cont[c].mg_on) {   // a last level above the tail: smoothed once or twice
      const mc::MgLevel& last = P->cont[c].mg.back();
      if (!last.coarsest && last.n > mc::mg_tail_cells()) {
        const int f = mc::env_int("MCDEC_MG_STOP_ONCE", -1);
        info->mg_stop_sweeps[c] = (f < 0 ? last.smooth_once : f != 0) ? 1 : 2;
      }
    }
  }
  return MC_OK;
}

const char* mc_last_error(const mc_problem* P) {
  if (P) return P->err.c_str();
  return mc::g_thread_error.c_str();
}

static mc_status exec_profile(mc::Exec& X, int32_t enable) {
  HIPCHK(hipStreamSynchronize(X.stream));
  mc::prof_harvest(X);
  X.prof = enable != 0;
  if (enable) {
    for (int k = 0; k < mc::Exec::NPROF; ++k) {
      X.prof_launch[k] = 0;
      X.prof_ms[k] = 0;
      X.prof_count[k] = 0;
      X.prof_samples[k].clear();
    }
    X.prof_every = enable;
  }
  return MC_OK;
}

static mc_status exec_profile_read(mc::Exec& X, int32_t which, int64_t* sampled,
                                   double* sampled_ms, int64_t* issued) {
  if (which < 0 || which >= mc::Exec::NPROF) return MC_EINVAL;
  HIPCHK(hipStreamSynchronize(X.stream));
  mc::prof_harvest(X);
  if (sampled) *sampled = X.prof_launch[which];
  if (sampled_ms) *sampled_ms = X.prof_ms[which];
  if (issued) *issued = X.prof_count[which];
  return MC_OK;
}

static mc_status exec_profile_read_above(mc::Exec& X, int32_t which, double min_ms,
                                        int64_t* sampled, double* sampled_ms) {
  if (which < 0 || which >= mc::Exec::NPROF) return MC_EINVAL;
  HIPCHK(hipStreamSynchronize(X.stream));
  mc::prof_harvest(X);
  int64_t n = 0;
  double sum = 0.0;
  for (float ms : X.prof_samples[which])
    if (ms >= min_ms) {
      n += 1;
      sum += ms;
    }
  if (sampled) *sampled = n;
  if (sampled_ms) *sampled_ms = sum;
  return MC_OK;
}

mc_status mc_profile(mc_problem* P, int32_t enable) {
  if (!P || enable < 0) return MC_EINVAL;
  ABI_BEGIN
  return exec_profile(P->X, enable);
  ABI_END(P)
}

mc_status mc_profile_read(mc_problem* P, int32_t which, int64_t* sampled, double* sampled_ms,
                          int64_t* issued) {
  if (!P || which < 0 || which >= mc::Exec::NPROF) return MC_EINVAL;
  ABI_BEGIN
  return exec_profile_read(P->X, which, sampled, sampled_ms, issued);
  ABI_END(P)
}

mc_status mc_profile_read_above(mc_problem* P, int32_t which, double min_ms, int64_t* sampled,
                                double* sampled_ms) {
  if (!P || which < 0 || which >= mc::Exec::NPROF) return MC_EINVAL;
  ABI_BEGIN
  return exec_profile_read_above(P->X, which, min_ms, sampled, sampled_ms);
  ABI_END(P)
}

mc_status mc_footprint(const mc_problem_desc* d, const mc_options* o, int64_t* bytes) {
  if (!d || !bytes) return MC_EINVAL;
  mc_options od;
  mc_options_default(&od);
  if (o) od = *o;
  *bytes = mc::footprint(*d, od);
  return MC_OK;
}

mc_status mc_autotune(mc_problem* const* probs, int32_t n, int32_t iters) {
  if (!probs || n < 1) return MC_EINVAL;
  ABI_BEGIN
  for (int i = 0; i < n; ++i)
    if (!probs[i]) throw mc::Error{MC_EINVAL, "problem " + std::to_string(i) + " is NULL"};
  if (iters < 1) iters = 20;
  mc::autotune(probs, n, iters);
  return MC_OK;
  ABI_END(probs[0])
}

mc_status mc_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(mc::g_tune_mu);
  mc::g_tune.clear();
  return MC_OK;
}

// ---- batches -------------------------------------------------------------------------
mc_status mc_batch_create(const mc_options* o, mc_batch** out) {
  if (!out) {
    mc::g_thread_error = "out is NULL";
    return MC_EINVAL;
  }
  *out = nullptr;
  mc_options od;
  mc_options_default(&od);
  if (o) od = *o;
  std::string m = mc::validate_options(od);
  if (!m.empty()) {
    mc::g_thread_error = m;
    return MC_EINVAL;
  }
  if (od.scheme == MC_SCHEME_L || od.scheme == MC_SCHEME_U) {
    mc::g_thread_error = "the L- and U-schemes are not batched";
    return MC_EINVAL;
  }
  mc_batch* B = new mc_batch();
  try {
    B->X.opt = od;
    B->mem.use_hooks(od);
    mc::exec_init(B->X, od.stream);
    B->X.opt.stream = B->X.stream;
  } catch (const mc::Error& e) {
    mc::g_thread_error = e.msg;
    mc_batch_destroy(B);
    return e.st;
  }
  *out = B;
  return MC_OK;
}

mc_status mc_batch_destroy(mc_batch* B) {
  if (!B) return MC_OK;
  if (B->X.stream) (void)hipStreamSynchronize(B->X.stream);
  for (auto& t : B->tab) mc::drop_graphs(t);
  mc::exec_release(B->X);
  B->mem.release();
  delete B;
  return MC_OK;
}

mc_status mc_batch_step(mc_batch* B, mc_problem* const* probs, int32_t n, int32_t n_steps,
                        mc_report* reps) {
  if (!B) return MC_EINVAL;
  ABI_BEGIN
  if (n_steps < 1) throw mc::Error{MC_EINVAL, "n_steps must be >= 1"};
  mc::batch_check(B, probs, n);
  auto t0 = std::chrono::steady_clock::now();
  mc_status st = MC_OK;
  for (int k = 0; k < n_steps && st == MC_OK; ++k) st = mc::batch_step_once(B, probs, n, reps);
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (reps)
    for (int i = 0; i < n; ++i) reps[i].seconds = sec;
  return st;
  ABI_END(B)
}

const char* mc_batch_last_error(const mc_batch* B) {
  if (B) return B->err.c_str();
  return mc::g_thread_error.c_str();
}

mc_status mc_batch_profile(mc_batch* B, int32_t enable) {
  if (!B || enable < 0) return MC_EINVAL;
  ABI_BEGIN
  return exec_profile(B->X, enable);
  ABI_END(B)
}

mc_status mc_batch_profile_read(mc_batch* B, int32_t which, int64_t* sampled,
                                double* sampled_ms, int64_t* issued) {
  if (!B || which < 0 || which >= mc::Exec::NPROF) return MC_EINVAL;
  ABI_BEGIN
  return exec_profile_read(B->X, which, sampled, sampled_ms, issued);
  ABI_END(B)
}

mc_status mc_batch_profile_read_above(mc_batch* B, int32_t which, double min_ms,
                                      int64_t* sampled, double* sampled_ms) {
  if (!B || which < 0 || which >= mc::Exec::NPROF) return MC_EINVAL;
  ABI_BEGIN
  return exec_profile_read_above(B->X, which, min_ms, sampled, sampled_ms);
  ABI_END(B)
}

}  // extern "C"
