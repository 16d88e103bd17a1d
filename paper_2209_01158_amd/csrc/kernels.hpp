// HIP kernels for gfx950 (wave64).  Included once, by engine.hip.
//
// Memory layout: every Omega-continuum vector is an ny x nx row-major array; every fracture
// vector is [nf].  A grid tile is 64 consecutive cells of a row (one wavefront, coalesced
// 512-byte FP64 rows) times `ty` rows; a workgroup of 4 waves covers it with each wave taking
// every 4th row.  A graph tile is 256 consecutive fracture rows.
#pragma once
#include <hip/hip_runtime.h>
#include "common.hpp"

namespace mc {

// ------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------
template <class T> __device__ __forceinline__ const T* pick(const double* d, const float* f);
template <> __device__ __forceinline__ const double* pick<double>(const double* d, const float*) { return d; }
template <> __device__ __forceinline__ const float* pick<float>(const double*, const float* f) { return f; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic block reduction of NV values; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*red)[NV]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[w][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
  __syncthreads();
}

__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every block of a system deposits its NV partial sums in its slot; the block that arrives
// last sums all slots in slot order (so the result does not depend on arrival order or on
// other systems in the launch) and returns true with the totals in tot (all threads).
template <int NV>
__device__ bool arrive(SysState& S, int slot, double (&v)[NV], int kc, double (&tot)[NV]) {
  __shared__ double red[4][NV];
  __shared__ int last;
  __shared__ double bc[NV];
  block_sum<NV>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) st_agent(&S.partials[slot * MC_SLOT + k], v[k]);
    unsigned prev = __hip_atomic_fetch_add(&S.cnt[kc], 1u, __ATOMIC_ACQ_REL,
                                           __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == (unsigned)(S.nslots - 1));
  }
  __syncthreads();
  if (!last) return false;
  double a[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) a[k] = 0.0;
  for (int s = threadIdx.x; s < S.nslots; s += MC_BLOCK) {
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] += ld_agent(&S.partials[s * MC_SLOT + k]);
  }
  block_sum<NV>(a, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) bc[k] = a[k];
    __hip_atomic_store(&S.cnt[kc], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) tot[k] = bc[k];
  return true;
}

__device__ __forceinline__ void finish(SysState& S, int status) {
  S.done = 1;
  S.status = status;
  __hip_atomic_fetch_add(S.active, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool finite(double v) { return v == v && v - v == 0.0; }

// ------------------------------------------------------------------------------------
// coefficient setup (once per problem / per option change)
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double harm(double a, double b) {
  double s = a + b;
  return s > 0.0 ? 2.0 * a * b / s : 0.0;
}

struct GridSetup {
  int nx, ny;
  const double* k;  // may be null
  double kc, c, h, tau, s12;
  int bc_type[4];
  double bc_value[4];
  const double* src;
  const int* hptr;
  const int* hidx;
  const double* hsig;
  int ex;
  double *diag, *tx, *ty, *F;
};

// Storage c h^2 / tau, harmonic-mean face conductances, half-cell Dirichlet faces (2 k),
// transfer row sums S (sigma_omega h^2 plus the sigma of every fracture cell hosted here).
__global__ void k_setup_grid(GridSetup g) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)g.nx * g.ny;
  if (i >= n) return;
  const int x = (int)(i % g.nx), y = (int)(i / g.nx);
  auto K = [&](long j) { return g.k ? g.k[j] : g.kc; };
  const double kc = K(i);
  double tE = x + 1 < g.nx ? harm(kc, K(i + 1)) : 0.0;
  double tN = y + 1 < g.ny ? harm(kc, K(i + g.nx)) : 0.0;
  double tW = x > 0 ? harm(K(i - 1), kc) : 0.0;
  double tS = y > 0 ? harm(K(i - g.nx), kc) : 0.0;
  double tb = 0.0, fb = 0.0;
  const bool side[4] = {x == 0, x == g.nx - 1, y == 0, y == g.ny - 1};
  for (int s = 0; s < 4; ++s)
    if (side[s] && g.bc_type[s] == 1) {
      tb += 2.0 * kc;
      fb += 2.0 * kc * g.bc_value[s];
    }
  double S = g.s12;
  if (g.hptr)
    for (int j = g.hptr[i]; j < g.hptr[i + 1]; ++j) S += g.hsig[g.hidx[j]];
  double d = g.c * g.h * g.h / g.tau + ((tE + tW) + (tN + tS)) + tb;
  if (!g.ex) d += S;
  g.diag[i] = d;
  g.tx[i] = tE;
  g.ty[i] = tN;
  g.F[i] = fb + (g.src ? g.src[i] * g.h * g.h : 0.0);
}

struct GraphSetup {
  int nf, n_omega;
  const int* rowptr;
  const int* eidx;     // CSR entry -> connection index
  const double* edge_d;
  const double* flen;
  const double* sig0;
  const double* sig1;
  const double* src;
  double k_f, c_f, aperture, tau;
  int ex;
  double *val, *diag, *mt, *F;
};

__global__ void k_setup_graph(GraphSetup g) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= g.nf) return;
  double s = 0.0;
  for (int j = g.rowptr[l]; j < g.rowptr[l + 1]; ++j) {
    double t = g.k_f * g.aperture / g.edge_d[g.eidx[j]];
    g.val[j] = t;
    s += t;
  }
  const double meas = g.aperture * g.flen[l];
  const double mt = g.c_f * meas / g.tau;
  double S = g.sig0[l] + (g.n_omega > 1 ? g.sig1[l] : 0.0);
  g.mt[l] = mt;
  g.diag[l] = mt + s + (g.ex ? 0.0 : S);
  g.F[l] = g.src ? g.src[l] * meas : 0.0;
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void k_copy64(const double* __restrict__ a, double* __restrict__ b, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// ------------------------------------------------------------------------------------
// operator application
// ------------------------------------------------------------------------------------
// (A v)_i for grid cell i = (x, y):  diag_i v_i - sum over existing faces T v_nbr.
template <class T, class V>
__device__ __forceinline__ T grid_Av(const PartD& P, int x, int y, long i, T vi, const V& v) {
  const T* d = pick<T>(P.diag, P.diag32);
  T acc = d[i] * vi;
  const int nx = P.nx;
  if (P.has_t) {
    const T* tx = pick<T>(P.tx, P.tx32);
    const T* ty = pick<T>(P.ty, P.ty32);
    if (x > 0) acc -= tx[i - 1] * v(i - 1);
    if (x + 1 < nx) acc -= tx[i] * v(i + 1);
    if (y > 0) acc -= ty[i - nx] * v(i - nx);
    if (y + 1 < P.ny) acc -= ty[i] * v(i + nx);
  } else {
    const T t = (T)P.tconst;
    T s = (T)0;
    if (x > 0) s += v(i - 1);
    if (x + 1 < nx) s += v(i + 1);
    if (y > 0) s += v(i - nx);
    if (y + 1 < P.ny) s += v(i + nx);
    acc -= t * s;
  }
  return acc;
}

template <class T, class V>
__device__ __forceinline__ T graph_Av(const PartD& P, int l, T vl, const V& v) {
  const T* d = pick<T>(P.diag, P.diag32);
  const T* val = pick<T>(P.val, P.val32);
  T acc = d[l] * vl;
  for (int j = P.rowptr[l]; j < P.rowptr[l + 1]; ++j) acc -= val[j] * v(P.col[j]);
  return acc;
}

// Off-diagonal transfer blocks of the coupled operator (FP64): -Q_ab v_b.
template <class VP>
__device__ __forceinline__ double grid_coupling(const PartD* parts, const PartD& P, long i,
                                                const VP& vpart) {
  double acc = 0.0;
  if (P.other >= 0) acc -= P.s12 * vpart(P.other, i);
  if (P.frac >= 0 && P.hptr)
    for (int j = P.hptr[i]; j < P.hptr[i + 1]; ++j) {
      const int l = P.hidx[j];
      acc -= P.hsig[l] * vpart(P.frac, (long)l);
    }
  return acc;
}

template <class VP>
__device__ __forceinline__ double graph_coupling(const PartD& P, int l, const VP& vpart) {
  double acc = 0.0;
  const long h = P.host[l];
  if (P.omg[0] >= 0) acc -= P.fsig0[l] * vpart(P.omg[0], h);
  if (P.n_omega > 1 && P.omg[1] >= 0) acc -= P.fsig1[l] * vpart(P.omg[1], h);
  return acc;
}

// ------------------------------------------------------------------------------------
// right-hand side assembly (transfer lagged / taken from tsrc), always FP64
// b = M/tau p_old + F + sum_b Q_ab p_b (decoupled) [- S p_old for EX];  coupled: no transfer
// x = p_old (warm start)
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(MC_BLOCK) k_rhs(const PartD* __restrict__ parts,
                                                  const Tile* __restrict__ tiles) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;   // padding of the XCD-aware launch order
  const PartD& P = parts[t.part];
  double* x = P.x64;   // the FP64 iterate (the same buffer as P.x in FP64 solves)
  if (P.kind == PART_GRID) {
    const int x0 = (t.tile % P.tiles_x) * MC_TX, y0 = (t.tile / P.tiles_x) * P.trows;
    const int cx = x0 + (threadIdx.x & 63);
    if (cx >= P.nx) return;
    for (int r = threadIdx.x >> 6; r < P.trows; r += 4) {
      const int cy = y0 + r;
      if (cy >= P.ny) break;
      const long i = (long)cy * P.nx + cx;
      const double po = P.pold[i];
      double b = P.mtau * po + (P.F ? P.F[i] : 0.0);
      if (!P.coupled) {
        double tr = 0.0, S = 0.0;
        if (P.s12 != 0.0 && P.tsrc[1 - P.cont]) {
          tr += P.s12 * P.tsrc[1 - P.cont][i];
          S += P.s12;
        }
        if (P.hptr) {
          const double* pf = P.tsrc[P.n_omega];
          for (int j = P.hptr[i]; j < P.hptr[i + 1]; ++j) {
            const int l = P.hidx[j];
            tr += P.hsig[l] * pf[l];
            S += P.hsig[l];
          }
        }
        b += tr;
        if (P.ex) b -= S * po;
      }
      P.b[i] = b;
      x[i] = po;
    }
  } else {
    const int l = t.tile * MC_GRAPH_ROWS + threadIdx.x;
    if (l >= P.n) return;
    const double po = P.pold[l];
    double b = P.mt[l] * po + (P.F ? P.F[l] : 0.0);
    if (!P.coupled) {
      const long h = P.host[l];
      double tr = P.fsig0[l] * P.tsrc[0][h];
      double S = P.fsig0[l];
      if (P.n_omega > 1) {
        tr += P.fsig1[l] * P.tsrc[1][h];
        S += P.fsig1[l];
      }
      b += tr;
      if (P.ex) b -= S * po;
    }
    P.b[l] = b;
    x[l] = po;
  }
}

// ------------------------------------------------------------------------------------
// PCG (templated on the vector/coefficient type T; reductions always FP64)
// ------------------------------------------------------------------------------------
template <class T, int PREC>
__device__ __forceinline__ T zval(const PartD& P, long i) {
  if (PREC == PREC_JACOBI) {
    const T* r = (const T*)P.r;
    const T* d = pick<T>(P.diag, P.diag32);
    return r[i] / d[i];
  } else {
    return ((const T*)P.z)[i];
  }
}

// Iterate a grid tile: calls f(cx, cy, i) for every cell of the tile owned by this thread.
template <class F>
__device__ __forceinline__ void for_tile_cells(const PartD& P, int tile, const F& f) {
  const int x0 = (tile % P.tiles_x) * MC_TX, y0 = (tile / P.tiles_x) * P.trows;
  const int cx = x0 + (threadIdx.x & 63);
  if (cx >= P.nx) return;
  const int yend = min(y0 + P.trows, P.ny);
  for (int cy = y0 + (threadIdx.x >> 6); cy < yend; cy += 4) f(cx, cy, (long)cy * P.nx + cx);
}

// initial residual r = b - A x (FP64); partial (r,z), (b,b), (r,r)
template <int PREC>
__global__ void __launch_bounds__(MC_BLOCK) k_init(const PartD* __restrict__ parts,
                                                   const Tile* __restrict__ tiles,
                                                   SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;   // padding of the XCD-aware launch order
  const PartD& P = parts[t.part];
  SysState& S = sys[P.sys];
  double v[3] = {0.0, 0.0, 0.0};
  const double* x = (const double*)P.x;
  double* r = (double*)P.r;
  auto xpart = [&](int pi, long j) { return ((const double*)parts[pi].x)[j]; };
  auto xs = [&](long j) { return x[j]; };
  auto body = [&](long i, double ax) {
    const double b = P.b[i];
    const double ri = b - ax;
    r[i] = ri;
    if (PREC == PREC_JACOBI) v[0] += ri * (ri / P.diag[i]);
    v[1] += b * b;
    v[2] += ri * ri;
  };
  if (P.kind == PART_GRID) {
    for_tile_cells(P, t.tile, [&](int cx, int cy, long i) {
      double ax = grid_Av<double>(P, cx, cy, i, x[i], xs);
      if (P.coupled) ax += grid_coupling(parts, P, i, xpart);
      body(i, ax);
    });
  } else {
    const int l = t.tile * MC_GRAPH_ROWS + threadIdx.x;
    if (l < P.n) {
      double ax = graph_Av<double>(P, l, x[l], xs);
      if (P.coupled) ax += graph_coupling(P, l, xpart);
      body(l, ax);
    }
  }
  double tot[3];
  if (arrive<3>(S, P.slot0 + t.tile, v, KC_INIT, tot) && threadIdx.x == 0) {
    S.rz = tot[0];
    S.bb = tot[1];
    S.rr = tot[2];
    S.rr0 = tot[2];
    S.iter = 0;
    S.first = 1;
    S.beta = 0.0;
    S.done = 0;
    S.status = ST_RUN;
    if (S.rr <= S.tol2 * S.bb) finish(S, ST_CONV);
    else if (!finite(S.rz) || !finite(S.rr)) finish(S, ST_BREAK);
  }
}

// q = A p_new, p_new = z + beta p_old (z recomputed where a neighbour needs it); the new
// direction goes to the other buffer; partial (p_new, q); finalize alpha = (r,z)/(p,q).
template <class T, int PREC>
__global__ void __launch_bounds__(MC_BLOCK) k_pcg_A(const PartD* __restrict__ parts,
                                                    const Tile* __restrict__ tiles,
                                                    SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;   // padding of the XCD-aware launch order
  const PartD& P = parts[t.part];
  SysState& S = sys[P.sys];
  if (S.done) return;
  const T beta = (T)S.beta;
  const bool first = S.first != 0;
  const int par = S.iter & 1;
  auto pold = [&](const PartD& Q) { return (const T*)(par ? Q.p2 : Q.p); };
  auto pn_of = [&](const PartD& Q, long j) -> T {
    const T z = zval<T, PREC>(Q, j);
    return first ? z : z + beta * pold(Q)[j];
  };
  T* pnew = (T*)(par ? P.p : P.p2);
  T* q = (T*)P.q;
  double v[1] = {0.0};
  auto pself = [&](long j) { return pn_of(P, j); };
  auto body = [&](long i, T pi, T ax) {
    if (P.coupled) {
      auto vp = [&](int pj, long j) { return (double)pn_of(parts[pj], j); };
      ax = (T)((double)ax + (P.kind == PART_GRID ? grid_coupling(parts, P, i, vp)
                                                 : graph_coupling(P, (int)i, vp)));
    }
    q[i] = ax;
    pnew[i] = pi;
    v[0] += (double)pi * (double)ax;
  };
  if (P.kind == PART_GRID) {
    for_tile_cells(P, t.tile, [&](int cx, int cy, long i) {
      const T pi = pn_of(P, i);
      body(i, pi, grid_Av<T>(P, cx, cy, i, pi, pself));
    });
  } else {
    const int l = t.tile * MC_GRAPH_ROWS + threadIdx.x;
    if (l < P.n) {
      const T pl = pn_of(P, l);
      body(l, pl, graph_Av<T>(P, l, pl, pself));
    }
  }
  double tot[1];
  if (arrive<1>(S, P.slot0 + t.tile, v, KC_A, tot) && threadIdx.x == 0) {
    S.pq = tot[0];
    if (!(S.pq > 0.0) || !finite(S.pq)) finish(S, ST_BREAK);
    else S.alpha = S.rz / S.pq;
  }
}

// x += alpha p, r -= alpha q, z = M^-1 r; partial (r,z), (r,r); finalize beta and the
// stopping test ||r||^2 <= tol^2 ||b||^2.
template <class T, int PREC>
__global__ void __launch_bounds__(MC_BLOCK) k_pcg_B(const PartD* __restrict__ parts,
                                                    const Tile* __restrict__ tiles,
                                                    SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;   // padding of the XCD-aware launch order
  const PartD& P = parts[t.part];
  SysState& S = sys[P.sys];
  if (S.done) return;
  const T alpha = (T)S.alpha;
  const int par = S.iter & 1;
  const T* p = (const T*)(par ? P.p : P.p2);   // the buffer k_pcg_A just wrote
  const T* q = (const T*)P.q;
  T* x = (T*)P.x;
  T* r = (T*)P.r;
  const T* d = pick<T>(P.diag, P.diag32);
  double v[2] = {0.0, 0.0};
  auto body = [&](long i) {
    x[i] = x[i] + alpha * p[i];
    const T ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (PREC == PREC_JACOBI) v[0] += (double)ri * (double)(ri / d[i]);
    v[1] += (double)ri * (double)ri;
  };
  if (P.kind == PART_GRID) {
    for_tile_cells(P, t.tile, [&](int, int, long i) { body(i); });
  } else {
    const int l = t.tile * MC_GRAPH_ROWS + threadIdx.x;
    if (l < P.n) body(l);
  }
  double tot[2];
  if (arrive<2>(S, P.slot0 + t.tile, v, KC_B, tot) && threadIdx.x == 0) {
    const double rz = tot[0];
    S.rr = tot[1];
    S.iter += 1;
    S.total_iter += 1;
    if (S.rr <= S.tol2 * S.bb) finish(S, ST_CONV);
    else if (!finite(rz) || !finite(S.rr) || !(rz > 0.0)) finish(S, ST_BREAK);
    else if (S.iter >= S.max_iter) finish(S, ST_NOCONV);
    else {
      S.beta = rz / S.rz;
      S.rz = rz;
      S.first = 0;
    }
  }
}

// ------------------------------------------------------------------------------------
// mixed precision: FP64 residual of the FP64 iterate, handed to the FP32 inner solve
// ------------------------------------------------------------------------------------
// r64 = b - A64 x64; inner r32 = (float) r64, inner x32 = 0; partial (r64,r64), (r32,z32),
// (r32,r32).  Finalize: outer test ||r64|| <= outer_tol ||b||; otherwise (re)start the inner
// PCG with tolerance inner_tol relative to ||r32||.
__global__ void __launch_bounds__(MC_BLOCK) k_residual(const PartD* __restrict__ parts,
                                                       const Tile* __restrict__ tiles,
                                                       SysState* __restrict__ sys,
                                                       double inner_tol2) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;   // padding of the XCD-aware launch order
  const PartD& P = parts[t.part];
  SysState& S = sys[P.sys];
  if (S.outer_done) return;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const double* x = P.x64;
  float* r32 = (float*)P.r;
  float* x32 = (float*)P.x;
  auto xs = [&](long j) { return x[j]; };
  auto xpart = [&](int pi, long j) { return parts[pi].x64[j]; };
  auto body = [&](long i, double ax) {
    const double bi = P.b[i];
    const double ri = bi - ax;
    const float rf = (float)ri;
    r32[i] = rf;
    x32[i] = 0.0f;
    v[0] += ri * ri;
    v[1] += (double)rf * (double)(rf / P.diag32[i]);
    v[2] += (double)rf * (double)rf;
    v[3] += bi * bi;
  };
  if (P.kind == PART_GRID) {
    for_tile_cells(P, t.tile, [&](int cx, int cy, long i) {
      double ax = grid_Av<double>(P, cx, cy, i, x[i], xs);
      if (P.coupled) ax += grid_coupling(parts, P, i, xpart);
      body(i, ax);
    });
  } else {
    const int l = t.tile * MC_GRAPH_ROWS + threadIdx.x;
    if (l < P.n) {
      double ax = graph_Av<double>(P, l, x[l], xs);
      if (P.coupled) ax += graph_coupling(P, l, xpart);
      body(l, ax);
    }
  }
  double tot[4];
  if (arrive<4>(S, P.slot0 + t.tile, v, KC_RES, tot) && threadIdx.x == 0) {
    S.orr = tot[0];
    if (S.outer == 0) S.obb = tot[3];
    bool stop = true;
    if (S.orr <= S.otol2 * S.obb) S.outer_status = ST_CONV;
    else if (!finite(S.orr)) S.outer_status = ST_BREAK;
    else if (S.outer >= S.max_outer) S.outer_status = ST_NOCONV;
    else stop = false;
    if (stop) {
      S.outer_done = 1;
      __hip_atomic_fetch_add(S.oactive, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      S.done = 1;
      S.status = S.outer_status;
    } else {
      S.rz = tot[1];
      S.rr = tot[2];
      S.bb = tot[2];          // inner stop is relative to the residual it starts from
      S.tol2 = inner_tol2;
      S.iter = 0;
      S.first = 1;
      S.beta = 0.0;
      S.done = 0;
      S.status = ST_RUN;
      __hip_atomic_fetch_add(S.active, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!(S.rz > 0.0)) finish(S, ST_BREAK);
    }
  }
}

// x64 += (double) x32 for systems still refining; counts the pass.
__global__ void __launch_bounds__(MC_BLOCK) k_correct(const PartD* __restrict__ parts,
                                                      const Tile* __restrict__ tiles,
                                                      SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;   // padding of the XCD-aware launch order
  const PartD& P = parts[t.part];
  SysState& S = sys[P.sys];
  if (S.outer_done) return;
  const float* d = (const float*)P.x;
  double* x = P.x64;
  if (P.kind == PART_GRID) {
    for_tile_cells(P, t.tile, [&](int, int, long i) { x[i] += (double)d[i]; });
  } else {
    const int l = t.tile * MC_GRAPH_ROWS + threadIdx.x;
    if (l < P.n) x[l] += (double)d[l];
  }
}

// y = A x (same operator code as the solver; FP64), y in P.q, x in P.x
__global__ void __launch_bounds__(MC_BLOCK) k_apply(const PartD* __restrict__ parts,
                                                    const Tile* __restrict__ tiles) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;   // padding of the XCD-aware launch order
  const PartD& P = parts[t.part];
  const double* x = (const double*)P.x;
  double* y = (double*)P.q;
  auto xs = [&](long j) { return x[j]; };
  auto xpart = [&](int pi, long j) { return ((const double*)parts[pi].x)[j]; };
  if (P.kind == PART_GRID) {
    for_tile_cells(P, t.tile, [&](int cx, int cy, long i) {
      double ax = grid_Av<double>(P, cx, cy, i, x[i], xs);
      if (P.coupled) ax += grid_coupling(parts, P, i, xpart);
      y[i] = ax;
    });
  } else {
    const int l = t.tile * MC_GRAPH_ROWS + threadIdx.x;
    if (l < P.n) {
      double ax = graph_Av<double>(P, l, x[l], xs);
      if (P.coupled) ax += graph_coupling(P, l, xpart);
      y[l] = ax;
    }
  }
}

// Reset of the shared counters and per-system scalars before a solve phase (a kernel, not a
// memset, so that the sequence stays capturable).
__global__ void k_reset(SysState* sys, int nsys, int* counters, int active, int oactive,
                        int outer_mode) {
  // FP64 solves start with every system active; refinement starts with every outer loop
  // active and the inner solves are activated one by one by k_residual.
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) {
    counters[0] = active;
    counters[1] = oactive;
  }
  if (s < nsys) {
    SysState& S = sys[s];
    for (int k = 0; k < KC_N; ++k) S.cnt[k] = 0u;
    S.done = 0;
    S.status = ST_RUN;
    S.total_iter = 0;
    if (outer_mode) {
      S.outer = 0;
      S.outer_done = 0;
      S.outer_status = ST_RUN;
    }
  }
}

// outer bookkeeping for refinement: count a pass for systems still refining
__global__ void k_outer_count(SysState* sys, int nsys) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsys && !sys[s].outer_done) sys[s].outer += 1;
}

}  // namespace mc
