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

// Pointers read from descriptors are generic; these casts let the compiler emit global
// (not flat) memory instructions, which keep the LDS counter out of the memory waits.
template <class T>
using gconst = const __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gconst<T> gc(const T* p) {
  return (gconst<T>)p;
}
template <class T>
using gmut = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gmut<T> gm(T* p) {
  return (gmut<T>)p;
}

// Cache policy.  One PCG iteration streams several times the capacity of the L2 and the
// memory-side cache, and most vectors are written by one kernel and read by the next (p and
// q from the operator to the update, r and z_p from the update to the V-cycle, z from the
// V-cycle to the operator).  Streams whose next reader is a whole iteration away -- the
// operator and factor coefficients, and x and q in the update -- are read (x also written)
// with non-temporal accesses, so that they do not displace those vectors.

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

// Partial sums are stored component-major: component k of slot s at part[k * nslots + s],
// so that a wavefront reads 64 consecutive slots of one component and a reader loads only
// the components it uses.  Every slot s < nslots of a record is written before it is read.

// Sum of all partial slots of a system, in slot order.  Every workgroup of the system runs
// the same loads and the same reduction tree, so all obtain the identical value.  Must be
// reached by all threads of the workgroup.  Only the first `nv` components are loaded (the
// others come back 0).
template <int NV>
__device__ __forceinline__ void reduce_slots(const double* __restrict__ part, int nslots,
                                             double (&tot)[NV], int nv = NV) {
  __shared__ double red[4][NV];
  __shared__ double bc[NV];
  double a[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) a[k] = 0.0;
  for (int s = threadIdx.x; s < nslots; s += MC_BLOCK) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nv) a[k] += part[(long)k * nslots + s];
  }
  block_sum<NV>(a, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) bc[k] = a[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) tot[k] = bc[k];
}

// Reduce this workgroup's NV values and store them in its slot.
template <int NV>
__device__ __forceinline__ void write_slot(double* __restrict__ part, int nslots, int slot,
                                           double (&v)[NV]) {
  __shared__ double red[4][NV];
  block_sum<NV>(v, red);
  if (threadIdx.x == 0 && slot < nslots) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part[(long)k * nslots + slot] = v[k];
  }
}

// The done flag is written by workgroup 0 of a kernel while other workgroups of the same
// kernel may read it; every workgroup reaches the same decision from the same reduction, so
// either value it observes leads to the same behaviour.  Relaxed atomics keep it race-free.
__device__ __forceinline__ int ld_flag(int* f) {
  return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(int* f, int v) {
  __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
  int nx, ny, nz;   // ny rows per plane, nz planes (1: the 2-D model)
  const double* k;  // may be null
  double kc, c, h, tau, s12;
  int bc_type[4];
  double bc_value[4];
  const double* src;
  const int* hptr;
  const int* hidx;
  const double* hsig;
  int bc_type_z[2];    // (3-D) bottom, top
  double bc_value_z[2];
  int ex;
  double *diag, *tx, *ty, *tz, *F;   // tz: 3-D only
};

// Storage c |cell| / tau, harmonic-mean face conductances, half-cell Dirichlet faces,
// transfer row sums S (sigma_omega |cell| plus the sigma of every fracture cell hosted here).
// 2-D: |cell| = h^2 and a face's |E| / d = 1.  3-D (nz > 1, planes stacked in z): |cell| = h^3,
// |E| / d = h; ty is 0 on the last row of every plane (the plane above is not a north
// neighbour) and tz couples a cell to the one above it.
__global__ void k_setup_grid(GridSetup g) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long plane = (long)g.nx * g.ny;
  const long n = plane * g.nz;
  if (i >= n) return;
  const int x = (int)(i % g.nx);
  const int y = (int)((i / g.nx) % g.ny), z = (int)(i / plane);
  const bool d3 = g.nz > 1;
  const double fac = d3 ? g.h : 1.0;   // |E| / d of a face
  auto K = [&](long j) { return g.k ? g.k[j] : g.kc; };
  const double kc = K(i);
  double tE = x + 1 < g.nx ? fac * harm(kc, K(i + 1)) : 0.0;
  double tN = y + 1 < g.ny ? fac * harm(kc, K(i + g.nx)) : 0.0;
  double tW = x > 0 ? fac * harm(K(i - 1), kc) : 0.0;
  double tS = y > 0 ? fac * harm(K(i - g.nx), kc) : 0.0;
  double tb = 0.0, fb = 0.0;
  const bool side[6] = {x == 0, x == g.nx - 1, y == 0, y == g.ny - 1, d3 && z == 0,
                        d3 && z == g.nz - 1};
  for (int s = 0; s < 6; ++s) {
    const int bt = s < 4 ? g.bc_type[s] : g.bc_type_z[s - 4];
    if (side[s] && bt == 1) {
      const double bv = s < 4 ? g.bc_value[s] : g.bc_value_z[s - 4];
      tb += 2.0 * kc * fac;
      fb += 2.0 * kc * fac * bv;
    }
  }
  double S = g.s12;
  if (g.hptr)
    for (int j = g.hptr[i]; j < g.hptr[i + 1]; ++j) S += g.hsig[g.hidx[j]];
  double faces = (tE + tW) + (tN + tS);
  double tU = 0.0;
  if (d3) {
    tU = z + 1 < g.nz ? fac * harm(kc, K(i + plane)) : 0.0;
    const double tD = z > 0 ? fac * harm(K(i - plane), kc) : 0.0;
    faces += tU + tD;
  }
  double d = (d3 ? g.c * g.h * g.h * g.h : g.c * g.h * g.h) / g.tau + faces + tb;
  if (!g.ex) d += S;
  g.diag[i] = d;
  g.tx[i] = tE;
  g.ty[i] = tN;
  if (d3) g.tz[i] = tU;
  g.F[i] = fb + (g.src ? (d3 ? g.src[i] * g.h * g.h * g.h : g.src[i] * g.h * g.h) : 0.0);
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
  const double* wq;    // well q_w per unit measure, or null
  const double* wp;    // well pressure p_w, or null
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
  // a well q_w (p_w - p) is implicit in every scheme: q_w |iota_l| on the diagonal
  const double w = g.wq ? g.wq[l] * meas : 0.0;
  g.mt[l] = mt;
  g.diag[l] = mt + s + w + (g.ex ? 0.0 : S);
  g.F[l] = (g.src ? g.src[l] * meas : 0.0) + (g.wp ? w * g.wp[l] : 0.0);
}

// Copies the lower triangle of a column-major K x K matrix to its upper triangle.
__global__ void k_symmetrize(double* __restrict__ a, int K, int lda) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)K * K) return;
  const int r = (int)(idx % K), c = (int)(idx / K);
  if (r < c) a[(long)c * lda + r] = a[(long)r * lda + c];
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
    if (P.plane) {   // 3-D: the cells below and above (ty is 0 across a plane boundary)
      const T* tz = pick<T>(P.tz, P.tz32);
      if (i >= P.plane) acc -= tz[i - P.plane] * v(i - P.plane);
      if (i + P.plane < (long)P.n) acc -= tz[i] * v(i + P.plane);
    }
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
// block incomplete Cholesky, zero fill (IC(0) in natural order inside each block)
//   M = (D + E) D^-1 (D + E^T),  E = strictly lower part of A restricted to the block,
//   d_i = a_ii - sum_{j<i, j~i in block} a_ij^2 / d_j;  we store dinv_i = 1/d_i.
// Grid blocks are the 64 x MC_TY tiles; fracture blocks are the chains (tridiagonal, so
// IC(0) is their exact Cholesky factorization).
// ------------------------------------------------------------------------------------
struct GridIC0Setup {
  int nx, ny, tiles_x, ntiles;
  int rows;       // block height: MC_ICY (a continuum) or MC_ICYC (a coarse level)
  const double* diag;
  const double* tx;
  const double* ty;
  double* dinv;   // first holds d, then 1/d
};

// One thread per IC(0) block (64 columns x g.rows rows): pivots in natural order (row by
// row, west to east) with the west and south couplings that stay inside the block.
__global__ void k_setup_grid_ic0(GridIC0Setup g) {
  const int per = MC_TY / g.rows;   // blocks per tile
  const int unit = blockIdx.x * blockDim.x + threadIdx.x;
  if (unit >= g.ntiles * per) return;
  const int tile = unit / per;
  const int x0 = (tile % g.tiles_x) * MC_TX;
  const int y0 = (tile / g.tiles_x) * MC_TY + (unit % per) * g.rows;
  const int x1 = min(x0 + MC_TX, g.nx), y1 = min(y0 + g.rows, g.ny);
  if (y0 >= g.ny) return;
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x) {
      const long i = (long)y * g.nx + x;
      double d = g.diag[i];
      if (x > x0) {
        const double t = g.tx[i - 1];
        d -= t * t / g.dinv[i - 1];
      }
      if (y > y0) {
        const double t = g.ty[i - g.nx];
        d -= t * t / g.dinv[i - g.nx];
      }
      g.dinv[i] = d;
    }
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x) {
      const long i = (long)y * g.nx + x;
      g.dinv[i] = 1.0 / g.dinv[i];
    }
}

// ---- wave-level scans of affine maps u -> A + B u ------------------------------------
// DPP moves on 32-bit halves.  A lane whose source is outside the row (or whose row is
// masked) keeps `old`, which we set to the identity map (A = 0, B = 1).
template <int CTRL, int ROWM>
__device__ __forceinline__ double dpp_d(double old, double src) {
  const long long o = __builtin_bit_cast(long long, old), s = __builtin_bit_cast(long long, src);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, CTRL, ROWM, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), CTRL, ROWM, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL, int ROWM>
__device__ __forceinline__ float dpp_d(float old, float src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                __builtin_bit_cast(int, src),
                                                                CTRL, ROWM, 0xF, false));
}
template <int CTRL, int ROWM, class T>
__device__ __forceinline__ void combine_dpp(T& A, T& B) {
  const T Ap = dpp_d<CTRL, ROWM>((T)0, A);
  const T Bp = dpp_d<CTRL, ROWM>((T)1, B);
  A = A + B * Ap;
  B = B * Bp;
}
// value of lane l (wave-uniform result)
__device__ __forceinline__ double readlane_t(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float readlane_t(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Inclusive prefix over the 64 lanes, lane 0 applied first: row_shr 1,2,4,8 inside each
// row of 16 lanes, then row_bcast:15 (rows 1, 3 take the end of the row before) and
// row_bcast:31 (rows 2, 3 take lane 31).
template <class T>
__device__ __forceinline__ void scan_maps_up(T& A, T& B) {
  combine_dpp<0x111, 0xF>(A, B);
  combine_dpp<0x112, 0xF>(A, B);
  combine_dpp<0x114, 0xF>(A, B);
  combine_dpp<0x118, 0xF>(A, B);
  combine_dpp<0x142, 0xA>(A, B);
  combine_dpp<0x143, 0xC>(A, B);
}
// Inclusive prefix with lane 63 applied first: row_shl 1,2,4,8 inside rows, then rows 0 and
// 2 take the first lane of the row after them, then rows 0 and 1 take lane 32.
template <class T>
__device__ __forceinline__ void scan_maps_down(T& A, T& B) {
  combine_dpp<0x101, 0xF>(A, B);
  combine_dpp<0x102, 0xF>(A, B);
  combine_dpp<0x104, 0xF>(A, B);
  combine_dpp<0x108, 0xF>(A, B);
  const int lane = threadIdx.x & 63, row = lane >> 4;
  // the values crossing rows come from single lanes (16, 48, then 32): lane reads into
  // scalar registers; the lanes that take no value combine with the identity
  {
    const T A16 = readlane_t(A, 16), B16 = readlane_t(B, 16);
    const T A48 = readlane_t(A, 48), B48 = readlane_t(B, 48);
    const T Ap = row == 0 ? A16 : (row == 2 ? A48 : (T)0);
    const T Bp = row == 0 ? B16 : (row == 2 ? B48 : (T)1);
    A = A + B * Ap;
    B = B * Bp;
  }
  {
    const bool take = row < 2;
    const T A32 = readlane_t(A, 32), B32 = readlane_t(B, 32);
    const T Ap = take ? A32 : (T)0;
    const T Bp = take ? B32 : (T)1;
    A = A + B * Ap;
    B = B * Bp;
  }
}

// z = M^-1 r on one fracture chain [l0, l1) by one wavefront.  Forward u_l = (r_l + T_l
// u_{l-1}) / d_l and backward z_l = u_l + T_{l+1} z_{l+1} / d_l are first-order affine
// recurrences: each lane composes the maps of CH consecutive cells, a 64-lane scan gives
// every lane its incoming value, and each lane then runs its cells.
template <class T>
__device__ void chain_solve(const T* __restrict__ rin, T* __restrict__ z,
                            const T* __restrict__ dinvin, const T* __restrict__ cTin, int l0,
                            int l1) {
  constexpr int CH = 4;
  const gconst<T> r = gc(rin);
  const gconst<T> dinv = gc(dinvin);
  const gconst<T> cT = gc(cTin);
  const int lane = threadIdx.x & 63;
  T carry = (T)0;
  for (int base = l0; base < l1; base += 64 * CH) {
    const int s = base + lane * CH;
    T A = (T)0, B = (T)1;
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int l = s + j;
      if (l < l1) {
        const T di = dinv[l];
        A = r[l] * di + (cT[l] * di) * A;
        B = (cT[l] * di) * B;
      }
    }
    scan_maps_up(A, B);
    T Ae = __shfl_up(A, 1, 64), Be = __shfl_up(B, 1, 64);
    if (lane == 0) {
      Ae = (T)0;
      Be = (T)1;
    }
    T u = Ae + Be * carry;
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int l = s + j;
      if (l < l1) {
        const T di = dinv[l];
        u = r[l] * di + (cT[l] * di) * u;
        z[l] = u;
      }
    }
    carry = __shfl(A + B * carry, 63, 64);
  }
  __threadfence_block();   // the backward pass reads u written by other lanes
  carry = (T)0;
  for (int top = l1; top > l0; top -= 64 * CH) {
    const int lo = max(l0, top - 64 * CH);
    const int e = top - lane * CH;   // this lane: cells e-1 down to e-CH (>= lo)
    T A = (T)0, B = (T)1;
#pragma unroll
    for (int j = 1; j <= CH; ++j) {
      const int l = e - j;
      if (l >= lo) {
        const T c = l + 1 < l1 ? cT[l + 1] * dinv[l] : (T)0;
        A = z[l] + c * A;
        B = c * B;
      }
    }
    scan_maps_up(A, B);
    T Ae = __shfl_up(A, 1, 64), Be = __shfl_up(B, 1, 64);
    if (lane == 0) {
      Ae = (T)0;
      Be = (T)1;
    }
    T zz = Ae + Be * carry;
#pragma unroll
    for (int j = 1; j <= CH; ++j) {
      const int l = e - j;
      if (l >= lo) {
        const T c = l + 1 < l1 ? cT[l + 1] * dinv[l] : (T)0;
        zz = z[l] + c * zz;
        z[l] = zz;
      }
    }
    carry = __shfl(A + B * carry, 63, 64);
    __threadfence_block();
  }
}

// One block of the grid block IC(0) preconditioner as seen by one wavefront: 64 columns
// (lane = column) by R rows (MC_ICY on a continuum, MC_ICYC on the coarse levels of a
// V-cycle).  cell(y) is a valid cell index for every lane (clamped to the grid), act(y)
// says whether this lane's cell of row y exists.
template <int R>
struct IcBlkR {
  static constexpr int rows = R;
  int cx, cxs, y0, nx, ny;
  bool colact;
  __device__ IcBlkR(const PartD& P, int unit) {
    constexpr int per = MC_TY / R;   // unit = IC(0) block: tile and its band of R rows
    const int tile = unit / per;
    nx = P.nx;
    ny = P.ny;
    cx = (tile % P.tiles_x) * MC_TX + (int)(threadIdx.x & 63);
    cxs = min(cx, nx - 1);
    y0 = (tile / P.tiles_x) * MC_TY + (unit % per) * R;
    colact = cx < nx;
  }
  __device__ bool act(int y) const { return colact && y0 + y < ny; }
  __device__ long cell(int y) const { return (long)min(y0 + y, ny - 1) * nx + cxs; }
};
using IcBlk = IcBlkR<MC_ICY>;

// Block IC(0) solve on one grid block by one wavefront, entirely in registers.  rv holds
// this lane's residual in the block's rows (0 for cells outside the grid); the caller loads
// it for all rows before the sweep, so every memory access of the block is issued before
// the first dependent step.  The inverse pivots and face conductances are read once, as
// FP32 copies (a preconditioner needs no more; PCG still converges to the FP64 solution).
// Rows are swept in order; inside a row the west (forward) or east (backward) coupling is a
// first-order recurrence across lanes, solved by a 64-lane scan.  z is stored to zout.
// Dot products: with M = (D + E) D^-1 (D + E^T), the forward values u = (D + E)^-1 r and
// z = M^-1 r satisfy (D + E^T) z = D u, hence (r, z) = (M z, z) = sum_i d_i u_i^2: both
// (r,z) and (r,r) are complete after the forward sweep, so r never has to stay live.
// Factor values of a block as the sweep uses them: inverse pivots dv, east and north
// conductances te, tn, zero outside the grid and tn zero on the block's last row (couplings
// inside the block only).  ex / nx_: this lane's east and north face conductances per row
// when the caller has them already (HAS_T), else they are loaded.
template <bool HAS_T, int R, bool LOADED = false>
__device__ __forceinline__ void ic0_coefs(const PartD& P, const IcBlkR<R>& B, float (&dv)[R],
                                          float (&te)[R], float (&tn)[R],
                                          const float* ex = nullptr, const float* nx_ = nullptr) {
  const gconst<float> dinv = gc(P.fdinv32);
  const gconst<float> tx = gc(P.tx32);
  const gconst<float> ty = gc(P.ty32);
  const float tc = (float)P.tconst;
#pragma unroll
  for (int y = 0; y < R; ++y) {
    const bool act = B.act(y);
    const long i = B.cell(y);
    const float d = __builtin_nontemporal_load(&dinv[i]);   // (cache policy above)
    float e, n;
    if constexpr (HAS_T) {
      e = LOADED ? ex[y] : __builtin_nontemporal_load(&tx[i]);
      n = LOADED ? nx_[y] : __builtin_nontemporal_load(&ty[i]);
    } else {
      e = B.cx + 1 < B.nx ? tc : 0.0f;
      n = B.y0 + y + 1 < B.ny ? tc : 0.0f;
    }
    dv[y] = act ? d : 0.0f;
    te[y] = act ? e : 0.0f;
    tn[y] = act && y + 1 < R ? n : 0.0f;   // couplings inside the block only
  }
}

// The sweep on factor values prepared by ic0_coefs.
template <class T, int R, class EZ>
__device__ __forceinline__ void ic0_sweep_core(const IcBlkR<R>& B, const T (&rv)[R],
                                               const float (&dv)[R], const float (&te)[R],
                                               const float (&tn)[R], const EZ& emit_z,
                                               double& rz, double& rr) {
  const int lane = threadIdx.x & 63;
  T u[R];
  T uprev = (T)0;
#pragma unroll
  for (int y = 0; y < R; ++y) {
    const T ri = rv[y];
    const T di = (T)dv[y];
    // west conductance = east conductance of the lane to the left (0 for lane 0)
    const float tw = __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, te[y]), 0x138, 0xF, 0xF,
                                           false));
    const T ts = y > 0 ? (T)tn[y - 1] : (T)0;
    T a = (ri + ts * uprev) * di;
    T b = (T)tw * di;
    scan_maps_up(a, b);
    u[y] = a;
    uprev = a;
    rr += (double)ri * (double)ri;
    if (B.act(y)) rz += (double)a * (double)a / (double)dv[y];
  }
  T zabove = (T)0;
#pragma unroll
  for (int y = R - 1; y >= 0; --y) {
    const T di = (T)dv[y];
    const T e = lane < 63 ? (T)te[y] : (T)0;
    T a = u[y] + (T)tn[y] * zabove * di;
    T b = e * di;
    scan_maps_down(a, b);
    zabove = a;
    emit_z(y, a);
  }
}

template <class T, bool HAS_T, int R, class EZ>
__device__ __forceinline__ void ic0_sweep(const PartD& P, const IcBlkR<R>& B,
                                          const T (&rv)[R], const EZ& emit_z,
                                          double& rz, double& rr) {
  float dv[R], te[R], tn[R];
  ic0_coefs<HAS_T, R>(P, B, dv, te, tn);
  ic0_sweep_core<T, R>(B, rv, dv, te, tn, emit_z, rz, rr);
}

// z = M^-1 r on one block, handing each z value to emit_z(row, value)
template <class T, int R, class EZ>
__device__ __forceinline__ void ic0_block_f(const PartD& P, const IcBlkR<R>& B,
                                            const T (&rv)[R], const EZ& emit_z, double& rz,
                                            double& rr) {
  if (P.has_t) ic0_sweep<T, true, R>(P, B, rv, emit_z, rz, rr);
  else ic0_sweep<T, false, R>(P, B, rv, emit_z, rz, rr);
}

template <class T, int R>
__device__ __forceinline__ void ic0_block(const PartD& P, const IcBlkR<R>& B, const T (&rv)[R],
                                          T* __restrict__ zout, double& rz, double& rr) {
  ic0_block_f<T, R>(P, B, rv, [&](int y, T a) {
    if (B.act(y)) zout[B.cell(y)] = a;
  }, rz, rr);
}

// The finest pre-smoothing of a V-cycle, z_p = M^-1 r on one block (as ic0_block), fused with
// the block's share of the restriction into level 1: r_c += P^T (r - A_B z_p), where A_B
// keeps the operator's couplings inside the block.  The couplings to the neighbouring blocks
// are added by the level-1 kernel (k_mg_fix_smooth): from the block edges recorded here (z_p
// of the first and last column, the east face of the last column, per row) and from the rows
// next to the block's first and last row.  The fine residual is formed in the launch
// precision and summed in FP64, as in the unfused restriction.  Without `fuse` this is
// ic0_block storing z to zout (one copy of the sweep serves both).  For the residual pass
// after the sweep, z_p waits in the wavefront's LDS slice `zs` (MC_ICY rows of 64), the
// operator's FP32 diagonal is loaded straight into `ds` (global_load_lds: no registers; it
// lands with the factor loads) and r is read back from rg, where this thread stored it
// before the sweep.  Every lane reads only its own LDS entries (the west and east values come
// by DPP).
template <class T, bool HAS_T>
__device__ __forceinline__ void ic0_block_restrict(const PartD* __restrict__ parts,
                                                   const PartD& P, const IcBlk& B,
                                                   const T (&rv)[MC_ICY], const T* rg,
                                                   T* __restrict__ zout, bool fuse, T* zs,
                                                   float* ds, double& rz, double& rr) {
  constexpr int R = MC_ICY;
  const int lane = threadIdx.x & 63;
  float dv[R], te[R], tn[R];
  ic0_coefs<HAS_T, R>(P, B, dv, te, tn);
  if (fuse) {
#pragma unroll
    for (int y = 0; y < R; ++y)   // (a lane outside the grid loads a clamped in-grid cell)
      __builtin_amdgcn_global_load_lds((const void*)(P.diag32 + B.cell(y)),
                                       (__attribute__((address_space(3))) void*)(ds + y * 64),
                                       4, 0, 0);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  }
  const gmut<T> zo = gm(zout);   // (global, not flat, accesses: no LDS counter in their waits)
  ic0_sweep_core<T, R>(B, rv, dv, te, tn, [&](int y, T a) {
    if (B.act(y)) zo[B.cell(y)] = a;
    if (fuse) zs[y * 64 + lane] = a;
  }, rz, rr);
  if (!fuse) return;
  T rb[R];
#pragma unroll
  for (int y = 0; y < R; ++y) rb[y] = B.act(y) ? gc(rg)[B.cell(y)] : (T)0;
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
  // block edges: z_p of the first and last column, the last column's east face
  const gmut<T> edz = gm((T*)P.mg_edz);
  const gmut<float> edt = gm(P.mg_edt);
  const long e0 = (long)((B.cx - lane) / MC_TX) * P.ny + B.y0;
  if (lane == 0 || lane == 63) {
#pragma unroll
    for (int y = 0; y < R; ++y)
      if (B.y0 + y < P.ny) {
        edz[(e0 + y) * 2 + (lane == 63)] = zs[y * 64 + lane];
        if (lane == 63) edt[e0 + y] = te[y];
      }
  }
  // residual pass: r - A_B z_p row by row, 2 x 2 sums into r_c
  const PartD& C = parts[P.mg_next];
  const gmut<T> rc = gm((T*)C.mg_r);
  double sprev = 0.0;
#pragma unroll
  for (int y = 0; y < R; ++y) {
    const float tw = dpp_d<0x138, 0xF>(0.0f, te[y]);   // lane 0: no west coupling
    const T zc = zs[y * 64 + lane];
    const T zw = lane > 0 ? zs[y * 64 + lane - 1] : (T)0;
    const T ze = lane < 63 ? zs[y * 64 + lane + 1] : (T)0;
    T a = (T)ds[y * 64 + lane] * zc;
    a -= (T)tw * zw;
    if (lane < 63) a -= (T)te[y] * ze;
    if (y > 0) a -= (T)tn[y - 1] * zs[(y - 1) * 64 + lane];
    if (y + 1 < R) a -= (T)tn[y] * zs[(y + 1) * 64 + lane];   // tn = 0 on the last row
    const double sv = B.act(y) ? (double)rb[y] - (double)a : 0.0;
    if (!(y & 1)) {
      sprev = sv;
      continue;
    }
    double v = sprev + sv;
    v += dpp_d<0xB1, 0xF>(0.0, v);
    if (!(lane & 1) && B.act(y - 1))
      rc[(long)((B.y0 + y) >> 1) * C.nx + (B.cx >> 1)] = (T)v;
  }
}

template <class T>
__device__ __forceinline__ void ic0_block_restrict_any(const PartD* __restrict__ parts,
                                                       const PartD& P, const IcBlk& B,
                                                       const T (&rv)[MC_ICY], const T* rg,
                                                       T* __restrict__ zout, bool fuse, T* zs,
                                                       float* ds, double& rz, double& rr) {
  if (P.has_t) ic0_block_restrict<T, true>(parts, P, B, rv, rg, zout, fuse, zs, ds, rz, rr);
  else ic0_block_restrict<T, false>(parts, P, B, rv, rg, zout, fuse, zs, ds, rz, rr);
}

// Runs f(unit) for the IC(0) blocks of the workgroup's tile run, one wavefront per block.
template <class F>
__device__ __forceinline__ void for_wave_tiles(const Tile& t, const F& f) {
  for (int unit = t.t0 * MC_ICB + (int)(threadIdx.x >> 6); unit < t.t1 * MC_ICB; unit += 4)
    f(unit);
}

// ------------------------------------------------------------------------------------
// work iteration: a workgroup walks the tiles [t0, t1) of its part
// ------------------------------------------------------------------------------------
template <class F>
__device__ __forceinline__ void grid_cells(const PartD& P, int tile, const F& f) {
  const int x0 = (tile % P.tiles_x) * MC_TX, y0 = (tile / P.tiles_x) * MC_TY;
  const int cx = x0 + (threadIdx.x & 63);
  if (cx >= P.nx) return;
  const int yend = min(y0 + MC_TY, P.ny);
  for (int cy = y0 + (threadIdx.x >> 6); cy < yend; cy += 4) f(cx, cy, (long)cy * P.nx + cx);
}

template <int KIND, class FG, class FF>
__device__ __forceinline__ void for_cells(const PartD& P, const Tile& t, const FG& fg,
                                          const FF& ff) {
  for (int tile = t.t0; tile < t.t1; ++tile) {
    if constexpr (KIND == PART_GRID) {
      grid_cells(P, tile, fg);
    } else {
      const int l0 = P.chain_ptr[P.gtile[tile]], l1 = P.chain_ptr[P.gtile[tile + 1]];
      for (int l = l0 + (int)threadIdx.x; l < l1; l += MC_BLOCK) ff(l);
    }
  }
}

// Two-level block preconditioner of a fracture graph (PartD::blocks): one wavefront per block
// of at most 64 cells.  Each lane takes one cell's residual from `rval(l)` (which also does
// that cell's own pointwise work), the block's dense inverse gives y_b = B_b^-1 r_b (the
// residuals broadcast through LDS, the inverse read one coalesced column per step), and the
// block sum g_b = sum of r_b is the coarse right-hand side that the crossing-cell kernel
// solves; (r, y) and (r, r) accumulate into rz, rr.
template <class T, class RV>
__device__ __forceinline__ void block_precond(const PartD& P, const Tile& t, T* __restrict__ z,
                                              const RV& rval, double& rz, double& rr) {
  __shared__ T rsh[MC_BLOCK];
  const int lane = threadIdx.x & 63;
  T* rw = rsh + (threadIdx.x & ~63);
  T* g = (T*)P.gX;
  for (int tile = t.t0; tile < t.t1; ++tile) {
    const int b1 = P.xtile[tile + 1];
    for (int b = P.xtile[tile] + (int)(threadIdx.x >> 6); b < b1; b += MC_BLOCK / 64) {
      const int l = P.bnode[(long)b * 64 + lane];
      const T rl = l >= 0 ? rval(l) : (T)0;
      rw[lane] = rl;
      __threadfence_block();   // the block's residuals are read by every lane
      __builtin_amdgcn_wave_barrier();
      const gconst<float> Bi = gc(P.binv + (long)b * 4096);
      T y = (T)0;
#pragma unroll
      for (int j = 0; j < 64; ++j) y += (T)Bi[j * 64 + lane] * rw[j];
      if (l >= 0) z[l] = y;
      rz += (double)rl * (double)y;
      rr += (double)rl * (double)rl;
      const double gs = wave_sum((double)rl);
      if (lane == 0) g[b] = (T)gs;
      __builtin_amdgcn_wave_barrier();   // rw is written again for the next block
    }
  }
}

// z = M^-1 r at cell i.  Jacobi: r / diag.  Block IC(0): the stored z; on a fracture graph
// with crossing cells the stored vector is y = A_II^-1 r (0 on crossing cells) and the
// crossing solution z_X enters through the responses of each block to its end cells.
template <class T, int PREC>
__device__ __forceinline__ T zval(const PartD& P, long i) {
  if (PREC == PREC_JACOBI) {
    const T* r = (const T*)P.r;
    const T* d = pick<T>(P.diag, P.diag32);
    return r[i] / d[i];
  } else {
    T z = ((const T*)P.z)[i];
    if (P.K > 0) {
      const T* zX = (const T*)P.zX;
      if (P.blocks) return z + zX[P.xlr[2 * i]];   // the coarse value of the cell's block
      const int xl = P.xlr[2 * i], xr = P.xlr[2 * i + 1];
      if (xl >= 0) z += pick<T>(P.cl, P.cl32)[i] * zX[xl];
      if (xr >= 0) z += pick<T>(P.cr, P.cr32)[i] * zX[xr];
    }
    return z;
  }
}

// g_k = r_x + c_(x,x-1) y_(x-1) + c_(x,x+1) y_(x+1) for the crossing cells x of a work tile
// (their chain neighbours are in the same tile, and y vanishes on crossing cells).
template <class T>
__device__ __forceinline__ void schur_gather(const PartD& P, int tile, const T* r, const T* y) {
  T* g = (T*)P.gX;
  for (int k = P.xtile[tile] + (int)threadIdx.x; k < P.xtile[tile + 1]; k += MC_BLOCK) {
    const int x = P.xcells[k];
    T v = r[x];
    if (P.cxl[k] != 0.0) v += (T)P.cxl[k] * y[x - 1];
    if (P.cxr[k] != 0.0) v += (T)P.cxr[k] * y[x + 1];
    g[k] = v;
  }
}

// ------------------------------------------------------------------------------------
// right-hand side assembly, always FP64 (Section 3.3, D-scheme; Section 3.2, coupled):
// decoupled  b = M/tau p_old + F + sum_b Q_ab p_b   [EX: - S p_old]
// coupled    b = M/tau p_old + F
// and the warm start of the layer's PCG (x holds p^{n-2} on entry).  The warm start changes
// iteration counts only, never the tolerance the solution meets.
// ------------------------------------------------------------------------------------
// Polynomial extrapolation of order k from the history g[0] = p^{n-1}, g[1] = p^{n-2}, ...
__device__ __forceinline__ double extrapolate(int k, double g0, double g1, double g2,
                                              double g3) {
  switch (k) {
    case 1: return 2.0 * g0 - g1;
    case 2: return 3.0 * g0 - 3.0 * g1 + g2;
    case 3: return 4.0 * g0 - 6.0 * g1 + 4.0 * g2 - g3;
    default: return g0;
  }
}

// Adaptive warm start (WS_ADAPTIVE), first pass: how well each extrapolation order k = 0 ..
// min(hist - 1, 3) predicts the previous layer p^{n-1} from the layers before it,
// sum (p^{n-1} - E_k(p^{n-2}, ...))^2 per system -> partA slots (4 components).  k_rhs picks
// the order with the least error (the lower order on ties): high orders win once the
// solution varies smoothly in time and lose in the first layers after a jump.
template <int KIND>
__global__ void __launch_bounds__(MC_BLOCK) k_extrap_err(const PartD* __restrict__ parts,
                                                         const Tile* __restrict__ tiles,
                                                         SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  const PartD& P = parts[t.part];
  SysState& S = sys[P.sys];
  if (P.extrap != WS_ADAPTIVE || S.hist < 2) return;   // uniform over the system
  const int kmax = min(S.hist - 1, 3);
  const double* x = P.x64;   // p^{n-2}
  double e[4] = {0.0, 0.0, 0.0, 0.0};
  auto cell = [&](long i) {
    const double g0 = P.pold[i], g1 = x[i];
    const double g2 = kmax >= 1 ? P.hx[0][i] : 0.0;
    const double g3 = kmax >= 2 ? P.hx[1][i] : 0.0;
    const double g4 = kmax >= 3 ? P.hx[2][i] : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k <= kmax) {
        const double d = g0 - extrapolate(k, g1, g2, g3, g4);
        e[k] += d * d;
      }
  };
  for_cells<KIND>(P, t, [&](int, int, long i) { cell(i); }, [&](int l) { cell(l); });
  write_slot<4>(S.partA, S.nslotsA, t.slot, e);
}

template <int KIND>
__global__ void __launch_bounds__(MC_BLOCK) k_rhs(const PartD* __restrict__ parts,
                                                  const Tile* __restrict__ tiles,
                                                  SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  const PartD& P = parts[t.part];
  SysState& Sy = sys[P.sys];
  // the warm start's order: every workgroup of the system reaches the same one
  const int hist = Sy.hist;
  int order = 0;
  if (P.extrap == WS_LINEAR || (P.extrap == WS_ADAPTIVE && hist == 1)) order = hist >= 1;
  if (P.extrap == WS_ADAPTIVE && hist >= 2) {
    const int kmax = min(hist - 1, 3);
    double e[4];
    reduce_slots<4>(Sy.partA, Sy.nslotsA, e, kmax + 1);
    for (int k = 1; k <= kmax; ++k)
      if (e[k] < e[order]) order = k;
  }
  if (t.slot == 0 && threadIdx.x == 0) Sy.wsorder = order;
  // the adaptive warm start keeps the history: p^{n-3..n-5} <- p^{n-2..n-4}
  const bool shift = P.extrap == WS_ADAPTIVE;
  double* x = P.x64;
  auto guess = [&](long i, double po) {
    const double g1 = x[i];
    const double g2 = shift || order >= 2 ? P.hx[0][i] : 0.0;
    const double g3 = shift || order >= 3 ? P.hx[1][i] : 0.0;
    x[i] = extrapolate(order, po, g1, g2, g3);
    if (shift) {
      P.hx[2][i] = g3;
      P.hx[1][i] = g2;
      P.hx[0][i] = g1;
    }
  };
  for_cells<KIND>(
      P, t,
      [&](int, int, long i) {
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
        guess(i, po);
      },
      [&](int l) {
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
        guess(l, po);
      });
}

// ------------------------------------------------------------------------------------
// PCG.  Iteration k is the launch pair (k_pcg_A, k_pcg_B); k lives in the system record.
//   init   r = b - A x                               -> partB (rz, rr, bb)
//   A(k)   from partB: stop test, beta; p_new = z + beta p_old; q = A p_new -> partA (pq)
//   B(k)   from partA: alpha; x += alpha p; r -= alpha q; z = M^-1 r        -> partB (rz, rr)
// ------------------------------------------------------------------------------------
// FP64 residual b - A x of one cell (grid: res(cx, cy, i); graph: resg(l)), including the
// transfer blocks of the coupled operator.
struct Residual64 {
  const PartD* parts;
  const PartD& P;
  const double* x;
  bool use_x64;   // coupled parts read the other parts' x64 (else their x)
  __device__ double xpart(int pi, long j) const {
    return use_x64 ? parts[pi].x64[j] : ((const double*)parts[pi].x)[j];
  }
  __device__ double res(int cx, int cy, long i) const {
    auto xs = [&](long j) { return x[j]; };
    auto xp = [&](int pi, long j) { return xpart(pi, j); };
    double ax = grid_Av<double>(P, cx, cy, i, x[i], xs);
    if (P.coupled) ax += grid_coupling(parts, P, i, xp);
    return P.b[i] - ax;
  }
  __device__ double resg(int l) const {
    auto xs = [&](long j) { return x[j]; };
    auto xp = [&](int pi, long j) { return xpart(pi, j); };
    double ax = graph_Av<double>(P, l, x[l], xs);
    if (P.coupled) ax += graph_coupling(P, l, xp);
    return P.b[l] - ax;
  }
  // The residuals of a whole IC(0) block at this lane's column (uncoupled 2-D grid parts;
  // false otherwise): x, the coefficients and b are loaded once per half block -- the rows
  // above and below from the same column, the west and east neighbours from the adjacent
  // lanes -- and the operator is applied in grid_Av's order, so the values are the same.
  template <int R>
  __device__ bool block_res(const IcBlkR<R>& B, double (&out)[R]) const {
    if (P.coupled || P.plane) return false;
    constexpr int H = R / 2;
    static_assert(R % 2 == 0, "whole half blocks");
    const int nx = P.nx, ny = P.ny, lane = (int)(threadIdx.x & 63);
    const int x0 = B.cx - lane;
    const int hx = lane == 0 ? max(x0 - 1, 0) : (lane == 63 ? min(x0 + MC_TX, nx - 1) : B.cxs);
    auto row = [&](int j) { return (long)min(max(B.y0 + j, 0), ny - 1) * nx; };
    const bool has_t = P.has_t;
    const double tc = P.tconst;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j0 = h * H;
      double xv[H + 2], xh[H], dv[H], te[H], th[H], tn[H + 1], bv[H];
#pragma unroll
      for (int j = 0; j < H + 2; ++j) xv[j] = x[row(j0 + j - 1) + B.cxs];
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const long o = row(j0 + j);
        xh[j] = x[o + hx];
        dv[j] = P.diag[o + B.cxs];
        bv[j] = P.b[o + B.cxs];
        te[j] = has_t ? P.tx[o + B.cxs] : 0.0;
        th[j] = has_t ? P.tx[o + hx] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < H + 1; ++j) tn[j] = has_t ? P.ty[row(j0 + j - 1) + B.cxs] : 0.0;
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const int y = B.y0 + j0 + j;
        const double vw = dpp_d<0x138, 0xF>(xh[j], xv[j + 1]);   // lane 0 keeps its halo
        const double ve = dpp_d<0x130, 0xF>(xh[j], xv[j + 1]);   // lane 63 keeps its halo
        const double tw = dpp_d<0x138, 0xF>(th[j], te[j]);
        double acc = dv[j] * xv[j + 1];
        if (has_t) {
          if (B.cx > 0) acc -= tw * vw;
          if (B.cx + 1 < nx) acc -= te[j] * ve;
          if (y > 0) acc -= tn[j] * xv[j];
          if (y + 1 < ny) acc -= tn[j + 1] * xv[j + 2];
        } else {
          double s = 0.0;
          if (B.cx > 0) s += vw;
          if (B.cx + 1 < nx) s += ve;
          if (y > 0) s += xv[j];
          if (y + 1 < ny) s += xv[j + 2];
          acc -= tc * s;
        }
        out[j0 + j] = B.act(j0 + j) ? bv[j] - acc : 0.0;
      }
    }
    return true;
  }
};

// Shared by the FP64 initial residual and the refinement residual: takes the FP64 residual
// of every cell from `R` (R.res(cx, cy, i) / R.resg(l)), hands it to `emit(i, r, b)` which
// stores it in the solve's precision and returns the stored value, then applies the
// preconditioner to the stored residuals and accumulates (r,z), (r,r) into v[0], v[1].
template <class T, int PREC, int KIND, class R, class Emit>
__device__ __forceinline__ void residual_and_precond(const PartD& P, const Tile& t, const R& Rs,
                                                     T* __restrict__ rs, T* __restrict__ z,
                                                     const Emit& emit, double (&v)[5]) {
  auto res = [&](int cx, int cy, long i) { return Rs.res(cx, cy, i); };
  auto resg = [&](int l) { return Rs.resg(l); };
  const T* d = pick<T>(P.diag, P.diag32);
  if constexpr (PREC == PREC_BIC0 && KIND == PART_GRID) {
    for_wave_tiles(t, [&](int unit) {
      const IcBlk B(P, unit);
      double r64[MC_ICY];
      if (!Rs.block_res(B, r64)) {
#pragma unroll
        for (int y = 0; y < MC_ICY; ++y)   // loads only: all rows in flight together
          r64[y] = B.act(y) ? res(B.cxs, min(B.y0 + y, B.ny - 1), B.cell(y)) : 0.0;
      }
      T rs_[MC_ICY];
#pragma unroll
      for (int y = 0; y < MC_ICY; ++y)
        rs_[y] = B.act(y) ? emit(B.cell(y), r64[y], P.b[B.cell(y)]) : (T)0;
      // under a V-cycle this is the pre-smoothing of the finest level
      ic0_block<T>(P, B, rs_, P.mg_next >= 0 ? (T*)P.mg_zp : z, v[0], v[1]);
    });
    if (P.mg_next >= 0) v[0] = 0.0;   // (r, z) comes from the final smoothing
  } else if constexpr (PREC == PREC_BIC0 && KIND == PART_GRAPH) {
    const T* dinv = pick<T>(P.fdinv, P.fdinv32);
    const T* cT = pick<T>(P.cT, P.cT32);
    if (P.blocks)
      block_precond<T>(P, t, z, [&](int l) { return emit(l, resg(l), P.b[l]); }, v[0], v[1]);
    for (int tile = t.t0; tile < t.t1 && !P.blocks; ++tile) {
      const int c0 = P.gtile[tile], c1 = P.gtile[tile + 1];
      const int l0 = P.chain_ptr[c0], l1 = P.chain_ptr[c1];
      for (int l = l0 + (int)threadIdx.x; l < l1; l += MC_BLOCK) emit(l, resg(l), P.b[l]);
      __syncthreads();
      for (int c = c0 + (int)(threadIdx.x >> 6); c < c1; c += 4)
        chain_solve<T>(rs, z, dinv, cT, P.chain_ptr[c], P.chain_ptr[c + 1]);
      __syncthreads();
      if (P.K > 0) schur_gather<T>(P, tile, rs, z);
      for (int l = l0 + (int)threadIdx.x; l < l1; l += MC_BLOCK) {
        v[0] += (double)rs[l] * (double)z[l];   // (r_I, y_I); the Schur kernel adds g . z_X
        v[1] += (double)rs[l] * (double)rs[l];
      }
    }
  } else {
    for_cells<KIND>(
        P, t,
        [&](int cx, int cy, long i) {
          const T rn = emit(i, res(cx, cy, i), P.b[i]);
          v[0] += (double)rn * (double)(rn / d[i]);
          v[1] += (double)rn * (double)rn;
        },
        [&](int l) {
          const T rn = emit(l, resg(l), P.b[l]);
          v[0] += (double)rn * (double)(rn / d[l]);
          v[1] += (double)rn * (double)rn;
        });
  }
}

// initial residual r = b - A x (FP64) and z = M^-1 r  -> partB (rz, rr, bb)
template <int PREC, int KIND>
__global__ void __launch_bounds__(MC_BLOCK) __attribute__((amdgpu_waves_per_eu(2))) k_init(const PartD* __restrict__ parts,
                                                   const Tile* __restrict__ tiles,
                                                   SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  const PartD& P = parts[t.part];
  SysState& S = sys[P.sys];
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double* r = (double*)P.r;
  auto emit = [&](long i, double ri, double b) {
    r[i] = ri;
    v[2] += b * b;
    return ri;
  };
  const Residual64 R{parts, P, (const double*)P.x, false};
  residual_and_precond<double, PREC, KIND>(P, t, R, r, (double*)P.z, emit, v);
  write_slot<5>(S.partB, S.nslotsB, t.slot, v);
}

template <class T, int PREC, int KIND>
__global__ void __launch_bounds__(MC_BLOCK) k_pcg_A(const PartD* __restrict__ parts,
                                                    const Tile* __restrict__ tiles,
                                                    SysState* __restrict__ sys) {
  constexpr int W = MC_TX + 2, H = MC_TY + 2;
  __shared__ T sp[KIND == PART_GRID ? W * H : 1];
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  SysState& S = sys[t.sys];
  if (ld_flag(&S.done)) return;
  const PartD& P = parts[t.part];
  const int k = S.ka;
  const bool outer_check = S.mixed && k == 0;   // first inner iteration after a residual
  // one thread writes the record (total_iter is a read-modify-write)
  const bool w0 = t.slot == 0 && threadIdx.x == 0;
  if (w0) S.kb = k;
  double v[5];   // (r,z), (r,r); (b,b) at k = 0; the FP64 norms after a refinement residual
  reduce_slots<5>(S.partB, S.nslotsB, v, outer_check ? 5 : (k == 0 ? 3 : 2));
  if (outer_check) {   // first inner iteration after an FP64 residual: refinement test
    const double orr = v[3];
    const double obb = S.outer == 0 ? v[4] : S.obb;
    int ost = ST_RUN;
    if (orr <= S.otol2 * obb) ost = ST_CONV;
    else if (!finite(orr)) ost = ST_BREAK;
    else if (S.outer >= S.max_outer) ost = ST_NOCONV;
    if (w0) {
      S.orr = orr;
      if (S.outer == 0) S.obb = obb;
    }
    if (ost != ST_RUN) {
      if (w0) {
        S.outer_done = 1;
        S.outer_status = ost;
        S.status = ost;
        S.iter = 0;
        st_flag(&S.done, 1);
      }
      return;
    }
  }
  const double rz = v[0], rr = v[1];
  const double bb = k == 0 ? v[2] : S.bb;
  int st = ST_RUN;
  if (rr <= S.tol2 * bb) st = ST_CONV;
  else if (!finite(rz) || !finite(rr) || !(rz > 0.0)) st = ST_BREAK;
  else if (k >= S.max_iter) st = ST_NOCONV;
  if (w0) {
    S.rzh[k & 1] = rz;
    S.rr = rr;
    S.iter = k;
    if (k == 0) {
      S.bb = bb;
      S.rr0 = rr;
    }
  }
  if (st != ST_RUN) {
    if (w0) {
      S.status = st;
      S.total_iter += k;
      st_flag(&S.done, 1);
    }
    return;
  }
  const bool first = k == 0;
  const T beta = first ? (T)0 : (T)(rz / S.rzh[(k - 1) & 1]);
  const int par = k & 1;   // p_old in (par ? p2 : p), p_new to the other buffer
  auto pn_of = [&](const PartD& Q, long j) -> T {
    const T z = zval<T, PREC>(Q, j);
    return first ? z : z + beta * ((const T*)(par ? Q.p2 : Q.p))[j];
  };
  T* pnew = (T*)(par ? P.p : P.p2);
  T* q = (T*)P.q;
  double pq = 0.0;
  if constexpr (KIND == PART_GRID) {
    constexpr int WR = MC_TY / 4;                          // consecutive rows per wave
    constexpr int NE = (W * H + MC_BLOCK - 1) / MC_BLOCK;  // staged cells per thread
    const int nx = P.nx, ny = P.ny;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const gconst<T> d = gc(pick<T>(P.diag, P.diag32));
    const gconst<T> tx = gc(pick<T>(P.tx, P.tx32));
    const gconst<T> ty = gc(pick<T>(P.ty, P.ty32));
    const gconst<T> zsrc = gc((const T*)(PREC == PREC_JACOBI ? P.r : P.z));
    const gconst<T> pold = gc((const T*)(par ? P.p2 : P.p));
    const T tc = (T)P.tconst;
    // 3-D grid whose planes hold whole tile rows: consecutive tile rows in launch order go
    // through the planes (z fastest), so the tiles above and below, whose z and p_old the
    // z-couplings read again, are read by workgroups in flight at the same time
    int rp = 0, nzp = 0;
    if (P.plane) {
      const int rows = (int)(P.plane / nx);
      if (rows % MC_TY == 0) {
        rp = rows / MC_TY;
        nzp = ny / rows;
      }
    }
    for (int tile = t.t0; tile < t.t1; ++tile) {
      int trow = tile / P.tiles_x;
      if (rp) trow = (trow % nzp) * rp + trow / nzp;
      const int x0 = (tile % P.tiles_x) * MC_TX, y0 = trow * MC_TY;
      const int cx = x0 + lane, cxs = min(cx, nx - 1);
      const int r0 = y0 + wv * WR;   // first row of this wave
      // every load of the tile is issued before the first dependent step: the wave's
      // operator coefficients, then z (or r, diag) and p_old on the tile and its halo
      T dv[WR], te[WR], tn[WR], tw[WR];
      T ts0 = (T)0;
#pragma unroll
      for (int r = 0; r < WR; ++r) {
        const long i = (long)min(r0 + r, ny - 1) * nx + cxs;
        dv[r] = __builtin_nontemporal_load(&d[i]);   // coefficients: non-temporal
        if (P.has_t) {
          te[r] = __builtin_nontemporal_load(&tx[i]);
          tn[r] = __builtin_nontemporal_load(&ty[i]);
          tw[r] = cx > 0 && cx < nx ? tx[i - 1] : (T)0;
        }
      }
      if (P.has_t && r0 > 0) ts0 = ty[(long)min(r0 - 1, ny - 1) * nx + cxs];
      T sz[NE], sd[NE], so[NE];
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        const int e = min((int)threadIdx.x + k * MC_BLOCK, W * H - 1);
        const int gx = min(max(x0 + e % W - 1, 0), nx - 1);
        const int gy = min(max(y0 + e / W - 1, 0), ny - 1);
        const long j = (long)gy * nx + gx;
        sz[k] = zsrc[j];
        if (PREC == PREC_JACOBI) sd[k] = d[j];
        so[k] = first ? (T)0 : pold[j];
      }
      // stage p_new = z + beta p_old on the tile and its one-cell halo (zero outside)
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        const int e = (int)threadIdx.x + k * MC_BLOCK;
        if (e < W * H) {
          const int gx = x0 + e % W - 1, gy = y0 + e / W - 1;
          const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
          const T z = PREC == PREC_JACOBI ? sz[k] / sd[k] : sz[k];
          sp[e] = in ? (first ? z : z + beta * so[k]) : (T)0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < WR; ++r) {
        const int cy = r0 + r;
        const int c = (r0 - y0 + r + 1) * W + lane + 1;
        const T pc = sp[c];
        T acc = dv[r] * pc;
        if (P.has_t) {
          // tx = 0 on the last column and ty = 0 on the last row, where the halo is 0 too
          const T ts = r > 0 ? tn[r - 1] : ts0;
          acc -= te[r] * sp[c + 1];
          acc -= tw[r] * sp[c - 1];
          acc -= tn[r] * sp[c + W];
          acc -= ts * sp[c - W];
        } else {
          acc -= tc * ((sp[c - 1] + sp[c + 1]) + (sp[c - W] + sp[c + W]));
        }
        if (cx < nx && cy < ny) {
          const long i = (long)cy * nx + cx;
          if (P.plane) {   // 3-D: the cells below and above, outside the plane's tile
            const gconst<T> tz = gc(pick<T>(P.tz, P.tz32));
            if (i >= P.plane) acc -= tz[i - P.plane] * pn_of(P, i - P.plane);
            if (i + P.plane < (long)P.n) acc -= tz[i] * pn_of(P, i + P.plane);
          }
          if (P.coupled) {
            auto vp = [&](int pj, long j) { return (double)pn_of(parts[pj], j); };
            acc = (T)((double)acc + grid_coupling(parts, P, i, vp));
          }
          q[i] = acc;
          pnew[i] = pc;
          pq += (double)pc * (double)acc;
        }
      }
      __syncthreads();
    }
  } else {
    auto pself = [&](long j) { return pn_of(P, j); };
    for (int tile = t.t0; tile < t.t1; ++tile) {
      const int l0 = P.chain_ptr[P.gtile[tile]], l1 = P.chain_ptr[P.gtile[tile + 1]];
      for (int l = l0 + (int)threadIdx.x; l < l1; l += MC_BLOCK) {
        const T pl = pn_of(P, l);
        T acc = graph_Av<T>(P, l, pl, pself);
        if (P.coupled) {
          auto vp = [&](int pj, long j) { return (double)pn_of(parts[pj], j); };
          acc = (T)((double)acc + graph_coupling(P, l, vp));
        }
        q[l] = acc;
        pnew[l] = pl;
        pq += (double)pl * (double)acc;
      }
    }
  }
  double o[1] = {pq};
  write_slot<1>(S.partA, S.nslotsA, t.slot, o);
}

template <class T, int PREC, int KIND>
__global__ void __launch_bounds__(MC_BLOCK) __attribute__((amdgpu_waves_per_eu(2))) k_pcg_B(const PartD* __restrict__ parts,
                                                    const Tile* __restrict__ tiles,
                                                    SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  SysState& S = sys[t.sys];
  if (ld_flag(&S.done)) return;
  const PartD& P = parts[t.part];
  const int k = S.kb;
  if (t.slot == 0 && threadIdx.x == 0) S.ka = k + 1;
  double v1[1];
  reduce_slots<1>(S.partA, S.nslotsA, v1);
  const double pq = v1[0];
  double o[2] = {0.0, 0.0};
  if (!(pq > 0.0) || !finite(pq)) {
    // breakdown: every workgroup sees it; the NaN stops the system in the next A
    o[0] = __builtin_nan("");
    write_slot<2>(S.partB, S.nslotsB, t.slot, o);
    return;
  }
  const T alpha = (T)(S.rzh[k & 1] / pq);
  const int par = k & 1;
  const T* p = (const T*)(par ? P.p : P.p2);   // the buffer A(k) wrote
  const T* q = (const T*)P.q;
  T* x = (T*)P.x;
  T* r = (T*)P.r;
  T* z = (T*)P.z;
  const T* d = pick<T>(P.diag, P.diag32);
  if constexpr (PREC == PREC_BIC0 && KIND == PART_GRID) {
    // one wavefront per IC(0) block: every load of the block is issued first, then x and r
    // are updated and stored, then the sweep runs on r held in registers
    const gconst<T> xg = gc((const T*)x);
    const gconst<T> pg = gc(p);
    const gconst<T> rg = gc((const T*)r);
    const gconst<T> qg = gc(q);
    // each wavefront's z_p rows and FP32 diagonal rows (fused restriction)
    __shared__ T zstash[4 * MC_ICY * 64];
    __shared__ float dstash[4 * MC_ICY * 64];
    for_wave_tiles(t, [&](int unit) {
      const IcBlk B(P, unit);
      T xv[MC_ICY], pv[MC_ICY], rv[MC_ICY], qv[MC_ICY];
#pragma unroll
      for (int y = 0; y < MC_ICY; ++y) {
        const long i = B.cell(y);
        xv[y] = __builtin_nontemporal_load(&xg[i]);   // x and q: non-temporal
        pv[y] = pg[i];
        rv[y] = rg[i];
        qv[y] = __builtin_nontemporal_load(&qg[i]);
      }
#pragma unroll
      for (int y = 0; y < MC_ICY; ++y) {
        const T xn = xv[y] + alpha * pv[y];
        const T rn = rv[y] - alpha * qv[y];
        if (B.act(y)) {
          __builtin_nontemporal_store(xn, &gm(x)[B.cell(y)]);
          gm(r)[B.cell(y)] = rn;
        }
        rv[y] = B.act(y) ? rn : (T)0;
      }
      __builtin_amdgcn_sched_barrier(0);
      // under a V-cycle this is the pre-smoothing of the finest level (with the block's
      // share of the restriction into level 1, when that level is not in the small tail)
      ic0_block_restrict_any<T>(parts, P, B, rv, (const T*)r,
                                P.mg_next >= 0 ? (T*)P.mg_zp : z,
                                P.mg_fuse != 0 && P.mg_next >= 0,
                                zstash + (threadIdx.x >> 6) * MC_ICY * 64,
                                dstash + (threadIdx.x >> 6) * MC_ICY * 64,
                                o[0], o[1]);
    });
    if (P.mg_next >= 0) o[0] = 0.0;   // (r, z) comes from the final smoothing
  } else if constexpr (PREC == PREC_BIC0 && KIND == PART_GRAPH) {
    const T* dinv = pick<T>(P.fdinv, P.fdinv32);
    const T* cT = pick<T>(P.cT, P.cT32);
    if (P.blocks) {   // the update of each cell is done by the lane that holds it in a block
      block_precond<T>(P, t, z, [&](int l) {
        x[l] = x[l] + alpha * p[l];
        const T rn = r[l] - alpha * q[l];
        r[l] = rn;
        return rn;
      }, o[0], o[1]);
    }
    for (int tile = t.t0; tile < t.t1 && !P.blocks; ++tile) {
      const int c0 = P.gtile[tile], c1 = P.gtile[tile + 1];
      const int l0 = P.chain_ptr[c0], l1 = P.chain_ptr[c1];
      for (int l = l0 + (int)threadIdx.x; l < l1; l += MC_BLOCK) {
        x[l] = x[l] + alpha * p[l];
        r[l] = r[l] - alpha * q[l];
      }
      __syncthreads();
      for (int c = c0 + (int)(threadIdx.x >> 6); c < c1; c += 4)
        chain_solve<T>(r, z, dinv, cT, P.chain_ptr[c], P.chain_ptr[c + 1]);
      __syncthreads();
      if (P.K > 0) schur_gather<T>(P, tile, (const T*)r, (const T*)z);
      for (int l = l0 + (int)threadIdx.x; l < l1; l += MC_BLOCK) {
        o[0] += (double)r[l] * (double)z[l];
        o[1] += (double)r[l] * (double)r[l];
      }
    }
  } else {
    auto body = [&](long i) {
      x[i] = x[i] + alpha * p[i];
      const T ri = r[i] - alpha * q[i];
      r[i] = ri;
      o[0] += (double)ri * (double)(ri / d[i]);
      o[1] += (double)ri * (double)ri;
    };
    for_cells<KIND>(P, t, [&](int, int, long i) { body(i); }, [&](int l) { body(l); });
  }
  write_slot<2>(S.partB, S.nslotsB, t.slot, o);
}

// ------------------------------------------------------------------------------------
// mixed precision: FP64 residual of the FP64 iterate handed to the FP32 inner PCG
//   k_residual64  r64 = b - A64 x64 (FP64)                         -> partA (rr64, bb)
//   k_residual    s = 2^-e with 2^e ~ rms(r64); r32 = (float)(s r64); x32 = 0;
//                 z32 = M^-1 r32                                    -> partB (rz, rr, rr, rr64, bb)
//   ... inner PCG on A d = s r64 ...
//   k_correct     x64 += d / s
// The scale keeps the FP32 residual near unit size whatever the magnitude of the FP64 one
// (residuals far below FP32's normal range would otherwise round to zero); a power of two
// makes scaling and unscaling exact.
// ------------------------------------------------------------------------------------
template <int KIND>
__global__ void __launch_bounds__(MC_BLOCK) k_residual64(const PartD* __restrict__ parts,
                                                         const Tile* __restrict__ tiles,
                                                         SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  const PartD& P = parts[t.part];
  SysState& S = sys[P.sys];
  if (S.outer_done) return;
  const Residual64 R{parts, P, P.x64, true};
  double* r64 = P.r64;
  double v[2] = {0.0, 0.0};
  for_cells<KIND>(
      P, t,
      [&](int cx, int cy, long i) {
        const double ri = R.res(cx, cy, i);
        r64[i] = ri;
        v[0] += ri * ri;
        v[1] += P.b[i] * P.b[i];
      },
      [&](int l) {
        const double ri = R.resg(l);
        r64[l] = ri;
        v[0] += ri * ri;
        v[1] += P.b[l] * P.b[l];
      });
  write_slot<2>(S.partA, S.nslotsA, t.slot, v);
}

template <int PREC, int KIND>
__global__ void __launch_bounds__(MC_BLOCK) __attribute__((amdgpu_waves_per_eu(2))) k_residual(const PartD* __restrict__ parts,
                                                       const Tile* __restrict__ tiles,
                                                       SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  const PartD& P = parts[t.part];
  SysState& S = sys[P.sys];
  if (S.outer_done) return;
  double tot[2];
  reduce_slots<2>(S.partA, S.nslotsA, tot);
  const double orr = tot[0], obb = tot[1];
  double sc = 1.0;
  if (orr > 0.0 && finite(orr) && P.n > 0) {
    int e = 0;
    (void)frexp(sqrt(orr / (double)P.n), &e);
    sc = ldexp(1.0, -e);
  }
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  float* r32 = (float*)P.r;
  float* x32 = (float*)P.x;
  const double* r64 = P.r64;
  struct Scaled {
    const double* r64;
    double sc;
    __device__ double res(int, int, long i) const { return sc * r64[i]; }
    __device__ double resg(int l) const { return sc * r64[l]; }
    __device__ bool block_res(const IcBlk&, double (&)[MC_ICY]) const { return false; }
  } R{r64, sc};
  auto emit = [&](long i, double ri, double) {
    const float rf = (float)ri;
    r32[i] = rf;
    x32[i] = 0.0f;
    return rf;
  };
  residual_and_precond<float, PREC, KIND>(P, t, R, r32, (float*)P.z, emit, v);
  v[2] = v[1];
  const bool w0 = t.slot == 0 && threadIdx.x == 0;
  v[3] = w0 ? orr : 0.0;   // the FP64 norms, once per system
  v[4] = w0 ? obb : 0.0;
  write_slot<5>(S.partB, S.nslotsB, t.slot, v);
  if (w0) {   // a new inner solve starts
    S.rscale = sc;
    S.ka = 0;
    st_flag(&S.done, 0);
  }
}

// x64 += (double) x32 / s for systems still refining; workgroup 0 counts the pass.
template <int KIND>
__global__ void __launch_bounds__(MC_BLOCK) k_correct(const PartD* __restrict__ parts,
                                                      const Tile* __restrict__ tiles,
                                                      SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  const PartD& P = parts[t.part];
  SysState& S = sys[P.sys];
  if (S.outer_done) return;
  const double inv = 1.0 / S.rscale;   // exact: a power of two
  const float* d = (const float*)P.x;
  double* x = P.x64;
  for_cells<KIND>(P, t, [&](int, int, long i) { x[i] += (double)d[i] * inv; },
                  [&](int l) { x[l] += (double)d[l] * inv; });
  if (t.slot == 0 && threadIdx.x == 0) S.outer += 1;
}

// y = A x (FP64, the operator the solver inverts); y in P.q, x in P.x
template <int KIND>
__global__ void __launch_bounds__(MC_BLOCK) k_apply(const PartD* __restrict__ parts,
                                                    const Tile* __restrict__ tiles) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  const PartD& P = parts[t.part];
  const double* x = (const double*)P.x;
  double* y = (double*)P.q;
  auto xs = [&](long j) { return x[j]; };
  auto xpart = [&](int pi, long j) { return ((const double*)parts[pi].x)[j]; };
  for_cells<KIND>(
      P, t,
      [&](int cx, int cy, long i) {
        double ax = grid_Av<double>(P, cx, cy, i, x[i], xs);
        if (P.coupled) ax += grid_coupling(parts, P, i, xpart);
        y[i] = ax;
      },
      [&](int l) {
        double ax = graph_Av<double>(P, l, x[l], xs);
        if (P.coupled) ax += graph_coupling(P, l, xpart);
        y[l] = ax;
      });
}

// z = M^-1 r with the solver's preconditioner (FP64), r in P.r, z in P.z
template <int PREC, int KIND>
__global__ void __launch_bounds__(MC_BLOCK) __attribute__((amdgpu_waves_per_eu(2))) k_precond(const PartD* __restrict__ parts,
                                                      const Tile* __restrict__ tiles) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  const PartD& P = parts[t.part];
  const double* r = (const double*)P.r;
  double* z = (double*)P.z;
  if constexpr (PREC == PREC_BIC0 && KIND == PART_GRID) {
    double dz = 0.0, dr = 0.0;
    for_wave_tiles(t, [&](int unit) {
      const IcBlk B(P, unit);
      double rv[MC_ICY];
#pragma unroll
      for (int y = 0; y < MC_ICY; ++y) rv[y] = B.act(y) ? r[B.cell(y)] : 0.0;
      ic0_block<double>(P, B, rv, P.mg_next >= 0 ? (double*)P.mg_zp : z, dz, dr);
    });
  } else if constexpr (PREC == PREC_BIC0 && KIND == PART_GRAPH) {
    double rz = 0.0, rr = 0.0;
    if (P.blocks) block_precond<double>(P, t, z, [&](int l) { return r[l]; }, rz, rr);
    for (int tile = t.t0; tile < t.t1 && !P.blocks; ++tile) {
      const int c0 = P.gtile[tile], c1 = P.gtile[tile + 1];
      for (int c = c0 + (int)(threadIdx.x >> 6); c < c1; c += 4)
        chain_solve<double>(r, z, P.fdinv, P.cT, P.chain_ptr[c], P.chain_ptr[c + 1]);
      __syncthreads();
      if (P.K > 0) schur_gather<double>(P, tile, r, z);
    }
  } else {
    for_cells<KIND>(P, t, [&](int, int, long i) { z[i] = r[i] / P.diag[i]; },
                    [&](int l) { z[l] = r[l] / P.diag[l]; });
  }
}

// ------------------------------------------------------------------------------------
// crossing cells of a fracture graph: z_X = S^-1 g (dense, symmetric), one workgroup per
// MC_SCHUR_ROWS rows; in a PCG launch the partial g . z_X completes (r, z) in the update
// slots that follow the graph update kernel's own.
// ------------------------------------------------------------------------------------
template <class T, class M, bool PCG>
__device__ __forceinline__ void schur_rows_m(const PartD& P, const Tile& t, const gconst<T> gs,
                                             const gconst<M> Sv, double& gz) {
  const int K = P.K;
  T* zX = (T*)P.zX;
  const int lane = threadIdx.x & 63;
  const int k1 = min(t.t1 * MC_SCHUR_ROWS, K);
  for (int k = t.t0 * MC_SCHUR_ROWS + (int)(threadIdx.x >> 6); k < k1; k += 4) {
    const long row = (long)k * K;
    // four partial sums over interleaved columns: independent loads stay in flight
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = lane;
#pragma unroll 2
    for (; j + 192 < K; j += 256) {
      a0 += (double)Sv[row + j] * (double)gs[j];
      a1 += (double)Sv[row + j + 64] * (double)gs[j + 64];
      a2 += (double)Sv[row + j + 128] * (double)gs[j + 128];
      a3 += (double)Sv[row + j + 192] * (double)gs[j + 192];
    }
    for (; j < K; j += 64) a0 += (double)Sv[row + j] * (double)gs[j];
    const double acc = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) {
      const T zk = (T)acc;
      zX[k] = zk;
      if (PCG) gz += (double)gs[k] * (double)zk;
    }
  }
}

template <class T, bool PCG>
__device__ __forceinline__ void schur_rows(const PartD& P, const Tile& t, double& gz) {
  // g (at most 6144 values) is read by every row of every workgroup: it stays in L1 / L2,
  // so it is read in place rather than first copied to LDS behind a barrier
  const gconst<T> gs = gc((const T*)P.gX);
  // the coarse inverse of the two-level block preconditioner is read in FP32 (symmetric as
  // stored, so the preconditioner stays symmetric); the exact solve's Schur inverse in the
  // solve's precision
  if (P.blocks && sizeof(T) == 8) schur_rows_m<T, float, PCG>(P, t, gs, gc(P.sinv32), gz);
  else schur_rows_m<T, T, PCG>(P, t, gs, gc(pick<T>(P.sinv, P.sinv32)), gz);
}

template <class T>
__global__ void __launch_bounds__(MC_BLOCK) k_schur(const PartD* __restrict__ parts,
                                                    const Tile* __restrict__ tiles,
                                                    SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  SysState& S = sys[t.sys];
  if (ld_flag(&S.done)) return;
  const PartD& P = parts[t.part];
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  schur_rows<T, true>(P, t, v[0]);
  write_slot<5>(S.partB, S.nslotsB, t.slot, v);
}

// boundary call z = M^-1 r: the crossing solution, then z = y + block responses in place
__global__ void __launch_bounds__(MC_BLOCK) k_schur_apply(const PartD* __restrict__ parts,
                                                          const Tile* __restrict__ tiles) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  double gz = 0.0;
  schur_rows<double, false>(parts[t.part], t, gz);
}

__global__ void __launch_bounds__(MC_BLOCK) k_schur_finish(const PartD* __restrict__ parts,
                                                           const Tile* __restrict__ tiles) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  const PartD& P = parts[t.part];
  if (P.K == 0) return;
  double* z = (double*)P.z;
  for_cells<PART_GRAPH>(P, t, [&](int, int, long) {}, [&](int l) {
    z[l] = zval<double, PREC_BIC0>(P, l);
  });
}

// ------------------------------------------------------------------------------------
// multigrid V-cycle on a grid continuum (preconditioner option MC_MG)
//   levels: 2 x 2 aggregates of cells (ragged at odd sizes); coarse operator = P^T A P with
//   P piecewise constant, again a 5-point operator with face conductances; the coarsest level
//   (at most MC_MG_COARSE cells) is solved by its dense inverse.
//   V(r): z_p = M^-1 r (block IC(0)); r_c = P^T (r - A z_p); e = V_c(r_c);
//         z = (z_p + P e) + M^-1 (r - A (z_p + P e)).   Symmetric, as PCG needs.
// ------------------------------------------------------------------------------------
struct CoarsenSetup {
  int nx, ny, cnx, cny;      // fine and coarse grid
  const double* diag;        // fine operator
  const double* tx;
  const double* ty;
  double* cdiag;             // coarse operator
  double* ctx;
  double* cty;
};

// Coarse operator for 2 x 2 aggregates: the Galerkin product P^T A P (the diagonal sums the
// aggregate's diagonal entries and subtracts twice its internal face conductances; a coarse
// face sums the fine faces it covers) with its face conductances halved and the diagonal
// lowered by the same amount, which keeps the row sums (storage and transfer) exact.  The
// Galerkin faces of piecewise-constant aggregates are twice those of a cell of side 2h.
__global__ void k_mg_coarsen(CoarsenSetup g) {
  const long I = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= (long)g.cnx * g.cny) return;
  const int X = (int)(I % g.cnx), Y = (int)(I / g.cnx);
  double d = 0.0, e = 0.0, n = 0.0;
  for (int b = 0; b < 2; ++b) {
    const int y = 2 * Y + b;
    if (y >= g.ny) continue;
    for (int a = 0; a < 2; ++a) {
      const int x = 2 * X + a;
      if (x >= g.nx) continue;
      const long i = (long)y * g.nx + x;
      d += g.diag[i];
      if (a == 0 && x + 1 < g.nx) d -= 2.0 * g.tx[i];   // face inside the aggregate
      if (b == 0 && y + 1 < g.ny) d -= 2.0 * g.ty[i];
      if (a == 1 || x + 1 == g.nx) e += g.tx[i];        // east faces of the aggregate
      if (b == 1 || y + 1 == g.ny) n += g.ty[i];        // north faces
    }
  }
  double w = 0.0, s = 0.0;   // west and south faces (the neighbours' east / north faces)
  for (int b = 0; b < 2 && X > 0; ++b)
    if (2 * Y + b < g.ny) w += g.tx[(long)(2 * Y + b) * g.nx + 2 * X - 1];
  for (int a = 0; a < 2 && Y > 0; ++a)
    if (2 * X + a < g.nx) s += g.ty[(long)(2 * Y - 1) * g.nx + 2 * X + a];
  e = X + 1 < g.cnx ? e : 0.0;
  n = Y + 1 < g.cny ? n : 0.0;
  g.cdiag[I] = d - 0.5 * ((e + w) + (n + s));
  g.ctx[I] = 0.5 * e;
  g.cty[I] = 0.5 * n;
}

// Dense symmetric matrix of a 5-point operator (n = nx * ny, leading dimension ld >= n; a
// must be zero on entry).
__global__ void k_mg_dense_fill(const double* __restrict__ diag, const double* __restrict__ tx,
                                const double* __restrict__ ty, int nx, int ny, int ld,
                                double* __restrict__ a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)nx * ny;
  if (i >= n) return;
  const int x = (int)(i % nx), y = (int)(i / nx);
  a[i * ld + i] = diag[i];
  if (x + 1 < nx) {
    a[i * ld + i + 1] = -tx[i];
    a[(i + 1) * ld + i] = -tx[i];
  }
  if (y + 1 < ny) {
    a[i * ld + i + nx] = -ty[i];
    a[(i + nx) * ld + i] = -ty[i];
  }
}

// Diagonal dominance of a level operator: per workgroup, the sums over its cells of the
// row sum (diagonal minus the face conductances: storage, transfer and Dirichlet terms) and
// of the face conductances -> part[2 b], part[2 b + 1] (grid-stride loop, fixed order).
__global__ void __launch_bounds__(256) k_mg_dominance(int nx, int ny,
                                                      const double* __restrict__ diag,
                                                      const double* __restrict__ tx,
                                                      const double* __restrict__ ty,
                                                      double* __restrict__ part) {
  __shared__ double sh[2][256];
  const long n = (long)nx * ny;
  double rs = 0.0, fs = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx), y = (int)(i / nx);
    double f = tx[i] + ty[i];
    if (x > 0) f += tx[i - 1];
    if (y > 0) f += ty[i - nx];
    rs += diag[i] - f;
    fs += f;
  }
  sh[0][threadIdx.x] = rs;
  sh[1][threadIdx.x] = fs;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0];
    part[2 * blockIdx.x + 1] = sh[1][0];
  }
}

__global__ void k_fill0(double* __restrict__ a, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

// Row-wise 5-point product on a wavefront whose lane l holds column x = x0 + l of one row
// (the operator's FP32 copies: inside the preconditioner they need no more):
// (A v)_x with the west / east values of v from the neighbouring lanes and, at lanes 0 and
// 63, from `vh` (the lane's halo value: column x0 - 1 at lane 0, x0 + 64 at lane 63).
// te: this column's east face conductance; th: the halo column's (lane 0 takes it as its
// west face); ts / tn: south / north faces.  Without a conductance field every face is tc.
// Every lane must call it (the lane moves are wave-wide).
template <class T, bool HAS_T>
__device__ __forceinline__ T row_Av(int x, int nx, bool south, bool north, float d, T vc, T vh,
                                    T vs, T vn, float te, float th, float ts, float tn, T tc) {
  const T vw = dpp_d<0x138, 0xF>(vh, vc);   // wave_shr:1, lane 0 keeps vh
  const T ve = dpp_d<0x130, 0xF>(vh, vc);   // wave_shl:1, lane 63 keeps vh
  T acc = (T)d * vc;
  if constexpr (HAS_T) {
    const float tw = dpp_d<0x138, 0xF>(th, te);
    if (x > 0) acc -= (T)tw * vw;
    if (x + 1 < nx) acc -= (T)te * ve;
    if (south) acc -= (T)ts * vs;
    if (north) acc -= (T)tn * vn;
  } else {
    T sum = (T)0;
    if (x > 0) sum += vw;
    if (x + 1 < nx) sum += ve;
    if (south) sum += vs;
    if (north) sum += vn;
    acc -= tc * sum;
  }
  return acc;
}

// r_c = P^T (r - A z_p) of the finer level F on one band of R fine rows of fine tile `tile`
// (band 0..MC_TY/R-1), by one wavefront (lane = fine column): every value it needs is loaded
// first, then the fine residuals are formed and each 2 x 2 aggregate is summed over a row
// pair and a lane pair (tiles and bands start at even columns and rows, so no aggregate
// straddles two wavefronts).
template <class T, bool HAS_T, int R>
__device__ __forceinline__ void restrict_band(const PartD& C, int tile, int band) {
  static_assert(R % 2 == 0 && MC_TY % R == 0, "bands of whole row pairs");
  const int nx = C.mg_fnx, ny = C.mg_fny, cnx = C.nx, lane = threadIdx.x & 63;
  const int x0 = (tile % C.mg_ftiles_x) * MC_TX;
  const int ya = (tile / C.mg_ftiles_x) * MC_TY + band * R;
  if (ya >= ny) return;   // wave-uniform
  const T* rf = (const T*)C.mg_fr;   // the finer level's right-hand side (level 0: PCG r)
  const T* zf = (const T*)C.mg_fzp;
  T* rc = (T*)C.mg_r;
  const float* d = C.mg_fd32;
  const float* txp = C.mg_ftx32;
  const float* typ = C.mg_fty32;
  const T tc = (T)C.mg_ftc;
  const int x = x0 + lane, xs = min(x, nx - 1);
  const int hx = lane == 0 ? max(x0 - 1, 0) : (lane == 63 ? min(x0 + MC_TX, nx - 1) : xs);
  auto row = [&](int j) { return (long)min(max(ya + j, 0), ny - 1) * nx; };
  T z[R + 2], zh[R], rv[R];
  float dv[R], te[R], th[R], ty[R + 1];
#pragma unroll
  for (int j = 0; j < R + 2; ++j) z[j] = zf[row(j - 1) + xs];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const long o = row(j);
    zh[j] = zf[o + hx];
    rv[j] = rf[o + xs];
    dv[j] = d[o + xs];
    te[j] = HAS_T ? txp[o + xs] : 0.0f;
    th[j] = HAS_T ? txp[o + hx] : 0.0f;
  }
#pragma unroll
  for (int j = 0; j < R + 1; ++j) ty[j] = HAS_T ? typ[row(j - 1) + xs] : 0.0f;
  double s[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int y = ya + j;
    const T a = row_Av<T, HAS_T>(x, nx, y > 0, y + 1 < ny, dv[j], z[j + 1], zh[j], z[j],
                                 z[j + 2], te[j], th[j], ty[j], ty[j + 1], tc);
    s[j] = (x < nx && y < ny) ? (double)rv[j] - (double)a : 0.0;
  }
#pragma unroll
  for (int j = 0; j < R; j += 2) {
    double v = s[j] + s[j + 1];
    v += __shfl_xor(v, 1, 64);
    if (!(lane & 1) && x < nx && ya + j < ny) rc[(long)((ya + j) >> 1) * cnx + (x >> 1)] = (T)v;
  }
}

template <class T, int R>
__device__ __forceinline__ void restrict_band_any(const PartD& C, int tile, int band) {
  if (C.mg_fhas_t) restrict_band<T, true, R>(C, tile, band);
  else restrict_band<T, false, R>(C, tile, band);
}

// z_p = M^-1 r on IC(0) block `unit` of a coarse level (one wavefront)
template <class T>
__device__ __forceinline__ void smooth_unit(const PartD& P, int unit) {
  const T* r = (const T*)P.mg_r;
  const IcBlkR<MC_ICYC> B(P, unit);
  T rv[MC_ICYC];
#pragma unroll
  for (int y = 0; y < MC_ICYC; ++y) rv[y] = B.act(y) ? r[B.cell(y)] : (T)0;
  double dz = 0.0, dr = 0.0;
  ic0_block<T>(P, B, rv, (T*)P.mg_zp, dz, dr);
}

// z = (z_p + P e) + M^-1 (r - A (z_p + P e)) on IC(0) block `unit`, e the coarser level's
// solution, by one wavefront: z_p + P e on the block's rows and the rows above and below
// (west / east values from the neighbouring lanes, the band's edge columns loaded by lanes
// 0 and 63), the residual of each half of the block from values loaded first, then the
// sweep.  At the finest level of a PCG solve (FINAL) the result is the PCG vector z and
// (r, z) is added to rz.
template <class T, bool FINAL, bool HAS_T, int R, bool HAS_E = true>
__device__ __forceinline__ void post_unit(const PartD* __restrict__ parts, const PartD& P,
                                          int unit, double& rz) {
  const T* zp = (const T*)P.mg_zp;
  const T* e = (const T*)P.mg_e;   // the coarser level's solution
  const T* r = (const T*)(P.mg_level == 0 ? P.r : P.mg_r);   // level 0: the PCG vectors
  T* out = (T*)(P.mg_level == 0 ? P.z : P.mg_z);
  const float* d = P.diag32;
  const float* txp = P.tx32;
  const float* typ = P.ty32;
  const T tc = (T)P.tconst;
  const int nx = P.nx, ny = P.ny, cnx = P.mg_cnx, lane = threadIdx.x & 63;
  const IcBlkR<R> B(P, unit);
  const int x0 = B.cx - lane;
  const int hx = lane == 0 ? max(x0 - 1, 0) : (lane == 63 ? min(x0 + MC_TX, nx - 1) : B.cxs);
  auto rowy = [&](int j) { return min(max(B.y0 + j, 0), ny - 1); };
  // the last level of a truncated hierarchy has no coarser correction (e = 0, !HAS_E)
  auto zfull = [&](int y, int x) {
    if constexpr (HAS_E) return zp[(long)y * nx + x] + e[(long)(y >> 1) * cnx + (x >> 1)];
    else return zp[(long)y * nx + x];
  };
  T zo[R + 2];
#pragma unroll
  for (int j = 0; j < R + 2; ++j) zo[j] = zfull(rowy(j - 1), B.cxs);
  T rl[R], rv[R];
  float ef[R], nf[R];   // this lane's east / north faces, handed on to the sweep
  constexpr int H = R / 2;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    T zh[H], rr[H];
    float dv[H], te[H], th[H], ty[H + 1];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int y = rowy(h * H + j);
      const long o = (long)y * nx;
      zh[j] = zfull(y, hx);
      rr[j] = r[o + B.cxs];
      dv[j] = __builtin_nontemporal_load(&d[o + B.cxs]);
      te[j] = HAS_T ? __builtin_nontemporal_load(&txp[o + B.cxs]) : 0.0f;
      th[j] = HAS_T ? txp[o + hx] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < H + 1; ++j)
      ty[j] = HAS_T ? __builtin_nontemporal_load(&typ[(long)rowy(h * H + j - 1) * nx + B.cxs])
                    : 0.0f;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int jj = h * H + j, y = B.y0 + jj;
      const T a = row_Av<T, HAS_T>(B.cx, nx, y > 0, y + 1 < ny, dv[j], zo[jj + 1], zh[j],
                                   zo[jj], zo[jj + 2], te[j], th[j], ty[j], ty[j + 1], tc);
      rl[jj] = rr[j];
      rv[jj] = B.act(jj) ? rr[j] - a : (T)0;
      ef[jj] = te[j];
      nf[jj] = ty[j + 1];
    }
  }
  double dz = 0.0, dr = 0.0;
  float dv[R], te[R], tn[R];
  ic0_coefs<HAS_T, R, true>(P, B, dv, te, tn, ef, nf);
  ic0_sweep_core<T, R>(B, rv, dv, te, tn, [&](int y, T a) {
    if (B.act(y)) {
      const T zf = zo[y + 1] + a;
      out[B.cell(y)] = zf;
      if (FINAL) rz += (double)rl[y] * (double)zf;
    }
  }, dz, dr);
}

template <class T, bool FINAL, int R>
__device__ __forceinline__ void post_unit_any(const PartD* __restrict__ parts, const PartD& P,
                                              int unit, double& rz) {
  if (!P.mg_e) {   // truncated hierarchy: its last level (always with face arrays)
    post_unit<T, FINAL, true, R, false>(parts, P, unit, rz);
    return;
  }
  if (P.has_t) post_unit<T, FINAL, true, R>(parts, P, unit, rz);
  else post_unit<T, FINAL, false, R>(parts, P, unit, rz);
}

// Restriction into coarse level C and its pre-smoothing in one pass, on IC(0) block `unit`
// of C (64 coarse columns x MC_ICYC coarse rows; one wavefront, lane = coarse column X).
// The lane forms the fine residual r - A z_p of its two fine columns 2X, 2X+1 over the
// block's 2 * MC_ICYC fine rows (the west / east fine neighbours come from the neighbouring
// lanes, the band's edge columns are loaded by lanes 0 and 63), sums each 2 x 2 aggregate in
// registers, stores r_c and sweeps it at once: z_p = M^-1 r_c.  Half of the fine rows at a
// time keeps the registers bounded.
template <class T, bool HAS_T>
__device__ __forceinline__ void restrict_smooth_unit(const PartD& C, int unit) {
  constexpr int R = MC_ICYC, FR = 2 * R, H = FR / 2;   // coarse rows, fine rows, half
  const IcBlkR<R> B(C, unit);
  const int lane = threadIdx.x & 63;
  const int nx = C.mg_fnx, ny = C.mg_fny;   // the finer level (copied fields)
  const T* rf = (const T*)C.mg_fr;
  const T* zf = (const T*)C.mg_fzp;
  const float* d = C.mg_fd32;
  const float* txp = C.mg_ftx32;
  const float* typ = C.mg_fty32;
  const T tc = (T)C.mg_ftc;
  const int X = B.cx;                       // coarse column (may be past the grid)
  const int fx0 = min(2 * X, nx - 1), fx1 = min(2 * X + 1, nx - 1);
  const bool c0 = 2 * X < nx, c1 = 2 * X + 1 < nx;
  const int fxb = 2 * (B.cx - lane);        // first fine column of the band
  const int hx = lane == 0 ? max(fxb - 1, 0) : (lane == 63 ? min(fxb + 2 * MC_TX, nx - 1) : fx0);
  const int fy0 = 2 * B.y0;                 // first fine row of the block
  auto row = [&](int j) { return (long)min(max(fy0 + j, 0), ny - 1) * nx; };
  double rc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) rc[k] = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j0 = h * H;
    T z0[H + 2], z1[H + 2], zh[H], r0[H], r1[H];
    float d0[H], d1[H], e0[H], e1[H], eh[H], n0[H + 1], n1[H + 1];
#pragma unroll
    for (int j = 0; j < H + 2; ++j) {
      const long o = row(j0 + j - 1);
      z0[j] = zf[o + fx0];
      z1[j] = zf[o + fx1];
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const long o = row(j0 + j);
      zh[j] = zf[o + hx];
      r0[j] = rf[o + fx0];
      r1[j] = rf[o + fx1];
      d0[j] = __builtin_nontemporal_load(&d[o + fx0]);
      d1[j] = __builtin_nontemporal_load(&d[o + fx1]);
      e0[j] = HAS_T ? __builtin_nontemporal_load(&txp[o + fx0]) : 0.0f;
      e1[j] = HAS_T ? __builtin_nontemporal_load(&txp[o + fx1]) : 0.0f;
      eh[j] = HAS_T ? txp[o + hx] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < H + 1; ++j) {
      const long o = row(j0 + j - 1);
      n0[j] = HAS_T ? __builtin_nontemporal_load(&typ[o + fx0]) : 0.0f;
      n1[j] = HAS_T ? __builtin_nontemporal_load(&typ[o + fx1]) : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int fy = fy0 + j0 + j;
      const bool south = fy > 0, north = fy + 1 < ny;
      // west of column 2X is column 2X-1 (the left lane's second column); east of 2X+1 is
      // 2X+2 (the right lane's first column)
      const T zw = dpp_d<0x138, 0xF>(zh[j], z1[j + 1]);
      const T ze = dpp_d<0x130, 0xF>(zh[j], z0[j + 1]);
      T a0 = (T)d0[j] * z0[j + 1], a1 = (T)d1[j] * z1[j + 1];
      if constexpr (HAS_T) {
        const float tw = dpp_d<0x138, 0xF>(eh[j], e1[j]);   // face between 2X-1 and 2X
        if (2 * X > 0) a0 -= (T)tw * zw;
        if (c1) {                                            // face between 2X and 2X+1
          a0 -= (T)e0[j] * z1[j + 1];
          a1 -= (T)e0[j] * z0[j + 1];
        }
        if (2 * X + 2 < nx) a1 -= (T)e1[j] * ze;
        if (south) {
          a0 -= (T)n0[j] * z0[j];
          a1 -= (T)n1[j] * z1[j];
        }
        if (north) {
          a0 -= (T)n0[j + 1] * z0[j + 2];
          a1 -= (T)n1[j + 1] * z1[j + 2];
        }
      } else {
        T s0 = (T)0, s1 = (T)0;
        if (2 * X > 0) s0 += zw;
        if (c1) {
          s0 += z1[j + 1];
          s1 += z0[j + 1];
        }
        if (2 * X + 2 < nx) s1 += ze;
        if (south) {
          s0 += z0[j];
          s1 += z1[j];
        }
        if (north) {
          s0 += z0[j + 2];
          s1 += z1[j + 2];
        }
        a0 -= tc * s0;
        a1 -= tc * s1;
      }
      const bool in = fy < ny;
      double v = 0.0;
      if (in && c0) v += (double)r0[j] - (double)a0;
      if (in && c1) v += (double)r1[j] - (double)a1;
      rc[(j0 + j) >> 1] += v;
    }
  }
  T* rcp = (T*)C.mg_r;
  T rv[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    rv[k] = B.act(k) ? (T)rc[k] : (T)0;
    if (B.act(k)) rcp[B.cell(k)] = rv[k];
  }
  double dz = 0.0, dr = 0.0;
  ic0_block<T, R>(C, B, rv, (T*)C.mg_zp, dz, dr);
}

// Level 1 after a fused finest pre-smoothing (ic0_block_restrict): completes r_c = P^T (r -
// A z_p) with the couplings across the edges of the finest IC(0) blocks (64 x MC_ICY), whose
// in-block part the update kernel has summed into r_c already, then pre-smooths z_p = M^-1
// r_c, on IC(0) block `unit` of level 1 (one wavefront, lane = coarse column X over fine
// columns 2X, 2X+1; fine rows 2 y0 .. 2 y0 + 2 MC_ICYC - 1).  The band's fine columns start
// at a multiple of 128, so block edges fall at lanes 0 / 31 / 32 / 63, and its fine rows
// start at a multiple of 8, so it holds either the first or the last row of a block row.
// A fine cell next to an edge gets t z_p of the cell across it (r - A z_p has +t z_p there).
template <class T, bool HAS_T>
__device__ __forceinline__ void fix_smooth_unit(const PartD& C, int unit) {
  static_assert(2 * MC_ICYC <= MC_ICY && MC_ICY % (2 * MC_ICYC) == 0 && 2 * MC_TX == 128,
                "a level-1 block covers whole halves of finest IC(0) blocks");
  constexpr int R = MC_ICYC, FR = 2 * R;
  const IcBlkR<R> B(C, unit);
  const int lane = threadIdx.x & 63;
  const int nx = C.mg_fnx, ny = C.mg_fny;
  const T* zf = (const T*)C.mg_fzp;
  const T* edz = (const T*)C.mg_fedz;
  const float* edt = C.mg_fedt;
  T* rcp = (T*)C.mg_r;
  const int fxb = 2 * (B.cx - lane);   // the band's first fine column
  const int fy0 = 2 * B.y0;            // its first fine row
  const int kb = fxb / MC_TX;          // IC(0) block column of fxb
  double rc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) rc[k] = B.act(k) ? (double)rcp[B.cell(k)] : 0.0;
  // vertical edges: (block across, its column 0 / 1 = first / last, face's block)
  int kz = -1, cz = 0, kt = 0;
  if (lane == 0 && kb >= 1 && fxb < nx) kz = kb - 1, cz = 1, kt = kb - 1;
  if (lane == 31 && fxb + MC_TX < nx) kz = kb + 1, cz = 0, kt = kb;
  if (lane == 32 && fxb + MC_TX < nx) kz = kb, cz = 1, kt = kb;
  if (lane == 63 && fxb + 2 * MC_TX < nx) kz = kb + 2, cz = 0, kt = kb + 1;
  if (kz >= 0) {
#pragma unroll
    for (int j = 0; j < FR; ++j) {
      const int fy = fy0 + j;
      if (fy < ny)
        rc[j >> 1] += (double)edt[(long)kt * ny + fy] * (double)edz[((long)kz * ny + fy) * 2 + cz];
    }
  }
  // horizontal edge: the band's first fine row is a block's first row (south neighbour
  // across), or its last fine row is a block's last row (north neighbour across)
  const bool south = (fy0 % MC_ICY) == 0;
  const int fyc = south ? fy0 : fy0 + FR - 1;    // the fine row next to the edge
  const int fya = south ? fy0 - 1 : fy0 + FR;    // the row across it
  const int fyt = south ? fy0 - 1 : fy0 + FR - 1;  // the row whose north face it is
  const int k = south ? 0 : R - 1;
  if (fya >= 0 && fya < ny && fyc < ny) {
    const T tc = (T)C.mg_ftc;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int fx = 2 * B.cx + c;
      if (fx < nx) {
        const double t = HAS_T ? (double)C.mg_fty32[(long)fyt * nx + fx] : (double)tc;
        rc[k] += t * (double)zf[(long)fya * nx + fx];
      }
    }
  }
  T rv[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    rv[q] = B.act(q) ? (T)rc[q] : (T)0;
    if (B.act(q)) rcp[B.cell(q)] = rv[q];
  }
  double dz = 0.0, dr = 0.0;
  ic0_block<T, R>(C, B, rv, (T*)C.mg_zp, dz, dr);
}

// (Every V-cycle kernel skips systems whose solve has ended: the iterations launched past
// convergence in a replayed chunk then cost only their launches.  The done flag is found
// from the tile alone.  `sys` is null for a plain application of the preconditioner.)

// restriction into a level: the workgroup's tiles of the finer level, one band per wavefront
template <class T>
__global__ void __launch_bounds__(MC_BLOCK) k_mg_restrict(const PartD* __restrict__ parts,
                                                          const Tile* __restrict__ tiles,
                                                          SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  if (sys && ld_flag(&sys[t.sys].done)) return;
  const PartD& C = parts[t.part];
  for (int tile = t.t0; tile < t.t1; ++tile)
    restrict_band_any<T, MC_TY / 4>(C, tile, (int)(threadIdx.x >> 6));
}

// restriction into a coarse level fused with its pre-smoothing (ranges of the coarse
// level's IC(0) blocks, one per wavefront)
template <class T>
__global__ void __launch_bounds__(MC_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_mg_restrict_smooth(const PartD* __restrict__ parts, const Tile* __restrict__ tiles,
                     SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  if (sys && ld_flag(&sys[t.sys].done)) return;
  const PartD& C = parts[t.part];
  for (int u = t.t0 + (int)(threadIdx.x >> 6); u < t.t1; u += 4) {
    if (C.mg_fhas_t) restrict_smooth_unit<T, true>(C, u);
    else restrict_smooth_unit<T, false>(C, u);
  }
}

// completion of the restriction into level 1 and its pre-smoothing, after a fused finest
// pre-smoothing (the same level-1 IC(0) blocks as k_mg_restrict_smooth)
template <class T>
__global__ void __launch_bounds__(MC_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_mg_fix_smooth(const PartD* __restrict__ parts, const Tile* __restrict__ tiles,
                SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  if (sys && ld_flag(&sys[t.sys].done)) return;
  const PartD& C = parts[t.part];
  for (int u = t.t0 + (int)(threadIdx.x >> 6); u < t.t1; u += 4) {
    if (C.mg_fhas_t) fix_smooth_unit<T, true>(C, u);
    else fix_smooth_unit<T, false>(C, u);
  }
}

// coarse correction and post-smoothing on a coarse level; the list entry holds a range of
// IC(0) blocks (units), one per wavefront
template <class T>
__global__ void __launch_bounds__(MC_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_mg_post_c(const PartD* __restrict__ parts, const Tile* __restrict__ tiles,
            SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  if (sys && ld_flag(&sys[t.sys].done)) return;
  const PartD& P = parts[t.part];
  double unused = 0.0;
  for (int u = t.t0 + (int)(threadIdx.x >> 6); u < t.t1; u += 4)
    post_unit_any<T, false, MC_ICYC>(parts, P, u, unused);
}

// coarse correction and post-smoothing on the finest level (tile ranges of the continuum's
// update tiling); FINAL (inside a PCG solve) adds (r, z) to the workgroup's partial slot
template <class T, bool FINAL>
__global__ void __launch_bounds__(MC_BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
k_mg_post(const PartD* __restrict__ parts, const Tile* __restrict__ tiles,
          SysState* __restrict__ sys) {
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  if (sys && ld_flag(&sys[t.sys].done)) return;
  const PartD& P = parts[t.part];
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for_wave_tiles(t, [&](int unit) { post_unit_any<T, FINAL, MC_ICY>(parts, P, unit, v[0]); });
  if (FINAL) write_slot<5>(sys[P.sys].partB, sys[P.sys].nslotsB, t.slot, v);
}

// The small levels of a V-cycle in one workgroup: starting at level part t.part (whose
// right-hand side is in place), smoothing and restriction down to the coarsest level, its
// dense solve, then the corrections and post-smoothing back up to the starting level.  The
// phases are separated by workgroup barriers instead of kernel boundaries.
template <class T>
__global__ void __launch_bounds__(MC_TAIL_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
k_mg_tail(const PartD* __restrict__ parts, const Tile* __restrict__ tiles,
          SysState* __restrict__ sys) {
  constexpr int NW = MC_TAIL_THREADS / 64;
  const Tile t = tiles[blockIdx.x];
  if (t.part < 0) return;
  if (sys && ld_flag(&sys[t.sys].done)) return;
  const PartD* P0 = &parts[t.part];
  static_assert(MC_TAIL_THREADS % (MC_MG_COARSE / 2) == 0, "tail threads: whole row pairs");
  const int wave = (int)(threadIdx.x >> 6);
  const PartD* P = P0;
  while (P->mg_next >= 0) {
    const int ntiles = (int)(((P->nx + MC_TX - 1) / MC_TX) * ((P->ny + MC_TY - 1) / MC_TY));
    for (int u = wave; u < ntiles * (MC_TY / MC_ICYC); u += NW) smooth_unit<T>(*P, u);
    __syncthreads();
    const PartD& C = parts[P->mg_next];
    for (int k = wave; k < ntiles * 8; k += NW) restrict_band_any<T, MC_TY / 8>(C, k >> 3, k & 7);
    __syncthreads();
    P = &C;
  }
  {   // coarsest: z = A^-1 r by the FP32 copy of the dense (symmetric) inverse, stored with
      // an even leading dimension ld (zero padding): thread (pair p, chunk c) reads rows 2p,
      // 2p+1 of column j (one 2-wide load, consecutive across threads) for the chunk's j; the
      // chunks' FP64 sums meet in LDS.
    constexpr int NP = MC_MG_COARSE / 2, H = MC_TAIL_THREADS / NP;
    __shared__ double part[2][MC_TAIL_THREADS];
    const int n = P->n, ld = n + (n & 1);
    const T* r = (const T*)P->mg_r;
    const float2* inv = (const float2*)P->mg_inv32;   // FP32 copy: half the bytes
    T* z = (T*)P->mg_z;
    const int pr = (int)threadIdx.x % NP, c = (int)threadIdx.x / NP;
    const int j0 = c * n / H, j1 = (c + 1) * n / H;
    double a0 = 0.0, a1 = 0.0;
    if (2 * pr < n) {
#pragma unroll 8
      for (int j = j0; j < j1; ++j) {
        const float2 w = inv[(long)j * (ld / 2) + pr];
        const double rj = (double)r[j];
        a0 += (double)w.x * rj;
        a1 += (double)w.y * rj;
      }
    }
    part[0][threadIdx.x] = a0;
    part[1][threadIdx.x] = a1;
    __syncthreads();
    if (c == 0 && 2 * pr < n) {
      double s0 = part[0][pr], s1 = part[1][pr];
      for (int q = 1; q < H; ++q) {
        s0 += part[0][q * NP + pr];
        s1 += part[1][q * NP + pr];
      }
      z[2 * pr] = (T)s0;
      if (2 * pr + 1 < n) z[2 * pr + 1] = (T)s1;
    }
    __syncthreads();
  }
  while (P != P0) {
    P = &parts[P->mg_prev];
    const int ntiles = (int)(((P->nx + MC_TX - 1) / MC_TX) * ((P->ny + MC_TY - 1) / MC_TY));
    double unused = 0.0;
    for (int u = wave; u < ntiles * (MC_TY / MC_ICYC); u += NW)
      post_unit_any<T, false, MC_ICYC>(parts, *P, u, unused);
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------
// small systems: one workgroup runs a whole Jacobi-PCG solve (FP64)
// ------------------------------------------------------------------------------------
// Workgroup b solves the decoupled system of part part0 + b (its record sys[P.sys] holds the
// tolerance and iteration limit; b and the warm start x come from k_rhs).  The vectors stay
// in global memory (L2-resident at these sizes); every dot product is a fixed-order
// workgroup reduction, so every thread sees the same scalars.  Same stopping test as the
// general path: ||r||^2 <= tol^2 ||b||^2 on the recursive residual, or max_iter.
// Wave total by a DPP inclusive scan (row_shr 1, 2, 4, 8 within rows of 16 lanes, then
// row_bcast:15 and row_bcast:31 across rows; lanes without a source add the identity 0):
// lane 63 ends with the sum of all 64 lanes, read back into every lane.
__device__ __forceinline__ double wave_total_dpp(double v) {
  v += dpp_d<0x111, 0xF>(0.0, v);
  v += dpp_d<0x112, 0xF>(0.0, v);
  v += dpp_d<0x114, 0xF>(0.0, v);
  v += dpp_d<0x118, 0xF>(0.0, v);
  v += dpp_d<0x142, 0xA>(0.0, v);
  v += dpp_d<0x143, 0xC>(0.0, v);
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int NT>
__device__ __forceinline__ void small_sum(double (&v)[3], double (*buf)[3]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = wave_total_dpp(v[k]);
  if (lane == 0)
    for (int k = 0; k < 3; ++k) buf[wv][k] = v[k];
  __syncthreads();
  for (int k = 0; k < 3; ++k) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += buf[w][k];
    v[k] = t;
  }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_small_pcg(const PartD* __restrict__ parts, int part0,
                                                  SysState* __restrict__ sys) {
  __shared__ double red[2][NT / 64][3];   // two buffers: a reduction never reuses the last
  const PartD& P = parts[part0 + blockIdx.x];
  SysState& S = sys[P.sys];
  const long n = P.n;
  const int tid = threadIdx.x;
  double* x = (double*)P.x;
  double* r = (double*)P.r;
  double* p = (double*)P.p;
  double* q = (double*)P.q;
  const double* b = P.b;
  const double* d = P.diag;
  const bool grid = P.kind == PART_GRID;
  auto Av = [&](long i, const double* v) {
    auto vs = [&](long j) { return v[j]; };
    if (grid) return grid_Av<double>(P, (int)(i % P.nx), (int)(i / P.nx), i, v[i], vs);
    return graph_Av<double>(P, (int)i, v[i], vs);
  };
  int rb = 0;
  double v[3] = {0.0, 0.0, 0.0};
  for (long i = tid; i < n; i += NT) {      // r = b - A x, p = z = r / diag
    const double ri = b[i] - Av(i, x);
    const double zi = ri / d[i];
    r[i] = ri;
    p[i] = zi;
    v[0] += ri * zi;
    v[1] += ri * ri;
    v[2] += b[i] * b[i];
  }
  small_sum<NT>(v, red[rb]);
  rb ^= 1;
  double rz = v[0], rr = v[1];
  const double bb = v[2], tol2 = S.tol2;
  const int max_iter = S.max_iter;
  int k = 0, st = ST_RUN;
  for (;;) {
    if (rr <= tol2 * bb) st = ST_CONV;
    else if (!finite(rz) || !finite(rr) || !(rz > 0.0)) st = ST_BREAK;
    else if (k >= max_iter) st = ST_NOCONV;
    if (st != ST_RUN) break;
    __syncthreads();                        // p complete before A p
    double w[3] = {0.0, 0.0, 0.0};
    for (long i = tid; i < n; i += NT) {
      const double qi = Av(i, p);
      q[i] = qi;
      w[0] += p[i] * qi;
    }
    small_sum<NT>(w, red[rb]);
    rb ^= 1;
    const double pq = w[0];
    if (!(pq > 0.0) || !finite(pq)) {
      st = ST_BREAK;
      break;
    }
    const double alpha = rz / pq;
    double u[3] = {0.0, 0.0, 0.0};
    for (long i = tid; i < n; i += NT) {
      x[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      r[i] = ri;
      const double zi = ri / d[i];
      u[0] += ri * zi;
      u[1] += ri * ri;
    }
    small_sum<NT>(u, red[rb]);
    rb ^= 1;
    const double beta = u[0] / rz;
    rz = u[0];
    rr = u[1];
    for (long i = tid; i < n; i += NT) p[i] = r[i] / d[i] + beta * p[i];
    ++k;
  }
  if (tid == 0) {
    S.bb = bb;
    S.rr = rr;
    S.iter = k;
    S.total_iter = k;
    S.status = st;
    S.done = 1;
  }
}

// The same solve with the search direction p in LDS and every cell's coefficients and x,
// r, q in registers (thread t owns cells t, t + NT, ...; at most CPT each): one workgroup per
// 2-D grid system of at most NT * CPT cells, or per fracture system whose CSR also fits the
// LDS.  LDS layout: p [n]; for a fracture system then val [nnz], col [nnz], rowptr [n + 1].
template <int NT, int CPT>
__global__ void __launch_bounds__(NT) k_small_pcg_lds(const PartD* __restrict__ parts,
                                                      SysState* __restrict__ sys) {
  extern __shared__ double lds[];
  __shared__ double red[2][NT / 64][3];
  const PartD& P = parts[blockIdx.x];
  SysState& S = sys[P.sys];
  const int n = P.n, tid = threadIdx.x, nx = P.nx;
  const bool grid = P.kind == PART_GRID;
  double* pl = lds;
  double* vall = lds + n;
  int nnz = 0;
  if (!grid) nnz = P.rowptr[n];
  int* coll = (int*)(vall + nnz);
  int* rpl = coll + nnz;
  if (!grid) {
    for (int j = tid; j < nnz; j += NT) {
      vall[j] = P.val[j];
      coll[j] = P.col[j];
    }
    for (int j = tid; j <= n; j += NT) rpl[j] = P.rowptr[j];
  }
  double dg[CPT], tw[CPT], te[CPT], ts[CPT], tn[CPT], x[CPT], r[CPT], q[CPT];
  const double* xg = (const double*)P.x;
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int i = tid + k * NT;
    dg[k] = 1.0;
    tw[k] = te[k] = ts[k] = tn[k] = x[k] = 0.0;
    if (i < n) {
      dg[k] = P.diag[i];
      x[k] = xg[i];
      if (grid) {
        const int cx = i % nx, cy = i / nx;
        const double tc = P.tconst;
        if (cx > 0) tw[k] = P.has_t ? P.tx[i - 1] : tc;
        if (cx + 1 < nx) te[k] = P.has_t ? P.tx[i] : tc;
        if (cy > 0) ts[k] = P.has_t ? P.ty[i - nx] : tc;
        if (cy + 1 < P.ny) tn[k] = P.has_t ? P.ty[i] : tc;
      }
    }
  }
  // (A v)_i from v in LDS: the grid's 5-point operator (faces of missing neighbours are 0)
  // or the fracture CSR
  auto Av = [&](int k, const double* v) {
    const int i = tid + k * NT;
    double acc = dg[k] * v[i];
    if (grid) {
      if (tw[k] != 0.0) acc -= tw[k] * v[i - 1];
      if (te[k] != 0.0) acc -= te[k] * v[i + 1];
      if (ts[k] != 0.0) acc -= ts[k] * v[i - nx];
      if (tn[k] != 0.0) acc -= tn[k] * v[i + nx];
    } else {
      for (int j = rpl[i]; j < rpl[i + 1]; ++j) acc -= vall[j] * v[coll[j]];
    }
    return acc;
  };
  // r = b - A x and p = z = r / diag: x goes through the LDS once
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int i = tid + k * NT;
    if (i < n) pl[i] = x[k];
  }
  __syncthreads();
  int rb = 0;
  double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int i = tid + k * NT;
    r[k] = 0.0;
    if (i < n) {
      const double bi = P.b[i];
      r[k] = bi - Av(k, pl);
      const double zi = r[k] / dg[k];
      v[0] += r[k] * zi;
      v[1] += r[k] * r[k];
      v[2] += bi * bi;
    }
  }
  small_sum<NT>(v, red[rb]);   // its barrier also ends every read of x from the LDS
  rb ^= 1;
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int i = tid + k * NT;
    if (i < n) pl[i] = r[k] / dg[k];
  }
  double rz = v[0], rr = v[1];
  const double bb = v[2], tol2 = S.tol2;
  const int max_iter = S.max_iter;
  int it = 0, st = ST_RUN;
  for (;;) {
    if (rr <= tol2 * bb) st = ST_CONV;
    else if (!finite(rz) || !finite(rr) || !(rz > 0.0)) st = ST_BREAK;
    else if (it >= max_iter) st = ST_NOCONV;
    if (st != ST_RUN) break;
    __syncthreads();                        // p complete before A p
    double w[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int i = tid + k * NT;
      q[k] = 0.0;
      if (i < n) {
        q[k] = Av(k, pl);
        w[0] += pl[i] * q[k];
      }
    }
    small_sum<NT>(w, red[rb]);
    rb ^= 1;
    const double pq = w[0];
    if (!(pq > 0.0) || !finite(pq)) {
      st = ST_BREAK;
      break;
    }
    const double alpha = rz / pq;
    double u[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int i = tid + k * NT;
      if (i < n) {
        x[k] += alpha * pl[i];
        r[k] -= alpha * q[k];
        const double zi = r[k] / dg[k];
        u[0] += r[k] * zi;
        u[1] += r[k] * r[k];
      }
    }
    small_sum<NT>(u, red[rb]);   // its barrier also ends every read of p in this iteration
    rb ^= 1;
    const double beta = u[0] / rz;
    rz = u[0];
    rr = u[1];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int i = tid + k * NT;
      if (i < n) pl[i] = r[k] / dg[k] + beta * pl[i];
    }
    ++it;
  }
  double* xo = (double*)P.x;
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int i = tid + k * NT;
    if (i < n) xo[i] = x[k];
  }
  if (tid == 0) {
    S.bb = bb;
    S.rr = rr;
    S.iter = it;
    S.total_iter = it;
    S.status = st;
    S.done = 1;
  }
}

// Solve parameters of the system records [s0, s1)
__global__ void k_set_params(SysState* sys, int s0, int s1, double tol2, double otol2,
                             int max_iter, int max_outer, int mixed, int hist) {
  const int s = s0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (s < s1) {
    SysState& S = sys[s];
    S.tol2 = tol2;
    S.otol2 = otol2;
    S.max_iter = max_iter;
    S.max_outer = max_outer;
    S.mixed = mixed;
    S.hist = hist;
  }
}

// Per-solve reset of the system records [s0, s1) (a kernel, so the sequence stays free of
// memset nodes).
__global__ void k_reset(SysState* sys, int s0, int s1) {
  const int s = s0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (s < s1) {
    SysState& S = sys[s];
    S.done = 0;
    S.status = ST_RUN;
    S.iter = 0;
    S.total_iter = 0;
    S.outer = 0;
    S.outer_done = 0;
    S.outer_status = ST_RUN;
    S.ka = 0;
    S.kb = 0;
  }
}

}  // namespace mc
