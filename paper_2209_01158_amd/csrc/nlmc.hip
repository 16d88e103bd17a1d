// Coarse-grid schemes of the nonlocal multicontinuum (NLMC) method (Section 4) on the GPU.
//
// Setup, from a fine problem already on the device:
//   * for every coarse cell i, the local operator A_loc of the oversampled region K_i^+ (the
//     principal block of the fine A = D + Q over the region's unknowns: zero values outside)
//     in a banded ordering, factored A_loc = L L^T by one workgroup per region;
//   * the constrained energy minimizers of eq. eq:basis through the constraint Schur
//     complement: Z = L^-1 C^T, S = C A_loc^-1 C^T = Z^T Z, and for each unit centred on
//     K_i the basis function psi = L^-T Z S^-1 e_unit (the Lagrange multipliers are
//     -S^-1 e_unit);
//   * A_bar from psi_v^T A psi_u over the overlapping supports (the nonlocal
//     transmissibilities), symmetrized, with a diagonal that makes every row sum equal the
//     unit's summed fine row sums; M_bar and F_bar summed over each unit's fine cells;
//   * the dense inverses of the coarse systems of each scheme (rocSOLVER at setup).
// Stepping: each layer of eq. is-nlmc (coupled) or eq. si-nlmc (D, L, U) is a right-hand
// side kernel and a dense product with the inverse of the block being solved, per block in
// the scheme's order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mcdec.h"
#include "fine_view.hpp"
#include "nlmc_host.hpp"

namespace mc {
namespace nl {

#define NL_CHECK(x)                                                                        \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) throw NlError{MC_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

struct NlError {
  mc_status st;
  std::string msg;
};

constexpr int NL_BLOCK = 256;
constexpr int NL_FWD_COLS = 64;   // constraint columns per workgroup of the forward solve
constexpr int NL_TILE = 16;       // S = Z^T Z tile edge

// A region's shape and offsets (device copy of NlRegion).
struct RegionD {
  int x0, y0, W, H;        // K_i^+ as fine cells
  int ex0, ey0, eW, eH;    // grown by one cell
  int n, w, m, ncenter;
  int center_local[3];
  int center_unit[3];
  long start_off, ext_off, row_off, unit_off, band_off, z_off, s_off;
  long psi_off[3];         // basis function of each centre unit (box ordering)
};

// Pieces of the fine operator A = D + Q (+ wells), by value.
struct FineD {
  int nx, ny, n_omega, nf;
  long ncell;
  double s12, h2, aperture, c_f;
  double mtau[2], c[2], tconst[2];
  int has_t[2];
  const double* diag[3];
  const double* tx[2];
  const double* ty[2];
  const double* F[3];
  const double* state[3];
  const double *mt, *val, *sigma_f, *flen;
  const int *rowptr, *col, *host, *hptr;
};

__device__ inline double east_T(const FineD& f, int a, long g, int x) {
  if (x + 1 >= f.nx) return 0.0;
  return f.has_t[a] ? f.tx[a][g] : f.tconst[a];
}
__device__ inline double north_T(const FineD& f, int a, long g, int y) {
  if (y + 1 >= f.ny) return 0.0;
  return f.has_t[a] ? f.ty[a][g] : f.tconst[a];
}
// diagonal of A (the system diagonal without the storage term)
__device__ inline double diagA_grid(const FineD& f, int a, long g) {
  return f.diag[a][g] - f.mtau[a];
}
__device__ inline double diagA_frac(const FineD& f, int l) {
  return f.diag[f.n_omega][l] - f.mt[l];
}

// Local row of box cell (x, y) slot s, or -1 outside the box.
__device__ inline int box_row(const int* start, int x0, int y0, int W, int H, int x, int y,
                              int s) {
  if (x < x0 || y < y0 || x >= x0 + W || y >= y0 + H) return -1;
  return start[(y - y0) * W + (x - x0)] + s;
}

// ---------------------------------------------------------------------------------------
// fine vectors and unit sums
// ---------------------------------------------------------------------------------------
// kind 0: (A 1) per fine unknown; 1: storage m (c h^2, c_f a l); 2: F; 3: measure (h^2,
// a l); 4: measure x current state.  Concatenated continuum order.
__global__ void k_nl_fine_vec(FineD f, int kind, double* __restrict__ out) {
  const long N = f.n_omega * f.ncell + f.nf;
  const long G = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= N) return;
  double v = 0.0;
  if (G < f.n_omega * f.ncell) {
    const int a = (int)(G / f.ncell);
    const long g = G % f.ncell;
    const int x = (int)(g % f.nx), y = (int)(g / f.nx);
    if (kind == 0) {
      double s = diagA_grid(f, a, g) - east_T(f, a, g, x) - north_T(f, a, g, y);
      if (x > 0) s -= east_T(f, a, g - 1, x - 1);
      if (y > 0) s -= north_T(f, a, g - f.nx, y - 1);
      if (f.n_omega == 2) s -= f.s12;
      v = s;   // the transfer to hosted fracture cells: k_nl_a1_transfer
    } else if (kind == 1) {
      v = f.c[a] * f.h2;
    } else if (kind == 2) {
      v = f.F[a][g];
    } else if (kind == 3) {
      v = f.h2;
    } else {
      v = f.h2 * f.state[a][g];
    }
  } else {
    const int l = (int)(G - f.n_omega * f.ncell);
    const double meas = f.aperture * f.flen[l];
    if (kind == 0) {
      double s = diagA_frac(f, l);
      for (int k = f.rowptr[l]; k < f.rowptr[l + 1]; ++k) s -= f.val[k];
      for (int a = 0; a < f.n_omega; ++a) s -= f.sigma_f[(long)a * f.nf + l];
      v = s;
    } else if (kind == 1) {
      v = f.c_f * meas;
    } else if (kind == 2) {
      v = f.F[f.n_omega][l];
    } else if (kind == 3) {
      v = meas;
    } else {
      v = meas * f.state[f.n_omega][l];
    }
  }
  out[G] = v;
}

// Transfer part of (A 1) on the grid rows: minus the sum of sigma_{a,l} over the fracture
// cells l hosted by each cell (one thread per grid cell, in host order).
__global__ void k_nl_a1_transfer(FineD f, const int* __restrict__ hidx, double* __restrict__ out) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= f.ncell || f.nf == 0) return;
  for (int a = 0; a < f.n_omega; ++a) {
    double s = 0.0;
    for (int k = f.hptr[g]; k < f.hptr[g + 1]; ++k) s += f.sigma_f[(long)a * f.nf + hidx[k]];
    out[a * f.ncell + g] -= s;
  }
}

// out[u] = sum of v over unit u's cells (in the unit's cell order); one wavefront per unit.
__global__ void k_nl_unit_sum(const int* __restrict__ uptr, const int* __restrict__ ucell,
                              const double* __restrict__ v, int nunits,
                              double* __restrict__ out) {
  const int u = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (u >= nunits) return;
  double s = 0.0;
  for (int k = uptr[u] + lane; k < uptr[u + 1]; k += 64) s += v[ucell[k]];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) out[u] = s;
}

__global__ void k_nl_div(const double* __restrict__ a, const double* __restrict__ b, int n,
                         double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] / b[i];
}

// ---------------------------------------------------------------------------------------
// local operators and their band Cholesky factors
// ---------------------------------------------------------------------------------------
// band[r * (w + 1) + d] = A_loc[r][r - d] (lower band, zero-filled beforehand); rw[r] =
// measure of row r's cell over its unit's measure (the constraint weights).
__global__ void __launch_bounds__(NL_BLOCK) k_nl_band(const RegionD* __restrict__ regs,
                                                      FineD f, const int* __restrict__ starts,
                                                      const int* __restrict__ row_g,
                                                      const int* __restrict__ row_unit,
                                                      const int* __restrict__ reg_units,
                                                      const int* __restrict__ rank,
                                                      const double* __restrict__ unit_meas,
                                                      double* __restrict__ band,
                                                      double* __restrict__ rw) {
  const RegionD R = regs[blockIdx.x];
  const int* st = starts + R.start_off;
  const int ld = R.w + 1;
  for (int r = threadIdx.x; r < R.n; r += blockDim.x) {
    const int G = row_g[R.row_off + r];
    double* Br = band + R.band_off + (long)r * ld;
    double meas;
    if (G < f.n_omega * f.ncell) {
      const int a = (int)(G / f.ncell);
      const long g = G % f.ncell;
      const int x = (int)(g % f.nx), y = (int)(g / f.nx);
      Br[0] = diagA_grid(f, a, g);
      const int rw_ = box_row(st, R.x0, R.y0, R.W, R.H, x - 1, y, a);
      if (rw_ >= 0) Br[r - rw_] = -east_T(f, a, g - 1, x - 1);
      const int rs_ = box_row(st, R.x0, R.y0, R.W, R.H, x, y - 1, a);
      if (rs_ >= 0) Br[r - rs_] = -north_T(f, a, g - f.nx, y - 1);
      if (a == 1) Br[1] = -f.s12;
      meas = f.h2;
    } else {
      const int l = G - f.n_omega * (int)f.ncell;
      const int gh = f.host[l];
      const int x = gh % f.nx, y = gh / f.nx;
      Br[0] = diagA_frac(f, l);
      for (int a = 0; a < f.n_omega; ++a) {
        const int r2 = box_row(st, R.x0, R.y0, R.W, R.H, x, y, a);
        Br[r - r2] = -f.sigma_f[(long)a * f.nf + l];
      }
      for (int k = f.rowptr[l]; k < f.rowptr[l + 1]; ++k) {
        const int l2 = f.col[k];
        const int g2 = f.host[l2];
        const int r2 = box_row(st, R.x0, R.y0, R.W, R.H, g2 % f.nx, g2 / f.nx,
                               f.n_omega + rank[l2]);
        if (r2 >= 0 && r2 < r) Br[r - r2] -= f.val[k];
      }
      meas = f.aperture * f.flen[l];
    }
    rw[R.row_off + r] = meas / unit_meas[reg_units[R.unit_off + row_unit[R.row_off + r]]];
  }
}

// In place: band -> its Cholesky factor L (L[r][r] at d = 0, L[r][r-d] at d); a non-positive
// pivot sets *bad (the local operator is not positive definite).
__global__ void __launch_bounds__(NL_BLOCK) k_nl_chol(const RegionD* __restrict__ regs,
                                                      double* __restrict__ band,
                                                      int* __restrict__ bad) {
  const RegionD R = regs[blockIdx.x];
  double* B = band + R.band_off;
  const int n = R.n, w = R.w, ld = w + 1;
  __shared__ double s_inv;
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      const double piv = B[(long)k * ld];
      s_bad = !(piv > 0.0);
      const double lkk = s_bad ? 1.0 : sqrt(piv);
      B[(long)k * ld] = lkk;
      s_inv = 1.0 / lkk;
    }
    __syncthreads();
    if (s_bad) {
      if (tid == 0) atomicMax(bad, 1);
      return;
    }
    const double inv = s_inv;
    const int tmax = min(w, n - 1 - k);
    for (int t = 1 + tid; t <= tmax; t += blockDim.x) B[(long)(k + t) * ld + t] *= inv;
    __syncthreads();
    // rows k+t, columns k+s (1 <= s <= t): A[k+t][k+s] -= L[k+t][k] L[k+s][k]
    for (int t = 1 + (tid >> 5); t <= tmax; t += blockDim.x >> 5) {
      double* Bt = B + (long)(k + t) * ld;
      const double lt = Bt[t];
      if (lt == 0.0) continue;
      for (int s = 1 + (tid & 31); s <= t; s += 32) Bt[t - s] -= lt * B[(long)(k + s) * ld + s];
    }
    __syncthreads();
  }
}

// Z[:, c0 + j] = L^-1 C^T[:, c0 + j] for NL_FWD_COLS constraint columns: column k of C^T is
// rw on the rows of the region's k-th unit.  Lane = column; the four wavefronts split the
// band sum; the last w rows of Z live in an LDS ring.
__global__ void __launch_bounds__(NL_BLOCK) k_nl_fwd(const RegionD* __restrict__ regs,
                                                     const double* __restrict__ band,
                                                     const int* __restrict__ row_unit,
                                                     const double* __restrict__ rw,
                                                     double* __restrict__ Z) {
  extern __shared__ double sm[];
  const RegionD R = regs[blockIdx.x];
  const int c0 = blockIdx.y * NL_FWD_COLS;
  if (c0 >= R.m) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = c0 + lane;
  const int ld = R.w + 1;
  double* ring = sm;                  // [ld][64]
  double* part = sm + (long)ld * 64;  // [4][64]
  const double* B = band + R.band_off;
  double* Zr = Z + R.z_off;
  int pos = 0;                        // r mod ld
  for (int r = 0; r < R.n; ++r) {
    const double* Lr = B + (long)r * ld;
    const int dmax = min(R.w, r);
    double acc = 0.0;
    for (int d = 1 + wv; d <= dmax; d += 4) {
      int q = pos - d;
      if (q < 0) q += ld;
      acc += Lr[d] * ring[q * 64 + lane];
    }
    part[wv * 64 + lane] = acc;
    __syncthreads();
    if (wv == 0) {
      const double b = row_unit[R.row_off + r] == col ? rw[R.row_off + r] : 0.0;
      const double z = (b - (part[lane] + part[64 + lane] + part[128 + lane] + part[192 + lane])) /
                       Lr[0];
      ring[pos * 64 + lane] = z;
      if (col < R.m) Zr[(long)r * R.m + col] = z;
    }
    __syncthreads();
    pos = pos + 1 == ld ? 0 : pos + 1;
  }
}

// S = Z^T Z (lower triangle, row-major m x m): workgroup (region, tile pair) computes a
// 16 x 16 tile, staging 16 rows of both column panels per pass.
__global__ void __launch_bounds__(NL_BLOCK) k_nl_gram(const RegionD* __restrict__ regs,
                                                      const double* __restrict__ Z,
                                                      double* __restrict__ S) {
  const RegionD R = regs[blockIdx.x];
  const int nt = (R.m + NL_TILE - 1) / NL_TILE;
  // tile pair (ti >= tj) from blockIdx.y
  int ti = 0, rem = blockIdx.y;
  while (rem > ti) {
    rem -= ti + 1;
    ++ti;
  }
  const int tj = rem;
  if (ti >= nt) return;
  __shared__ double pa[NL_TILE][NL_TILE + 1], pb[NL_TILE][NL_TILE + 1];
  const int i = threadIdx.x / NL_TILE, j = threadIdx.x % NL_TILE;
  const int u = ti * NL_TILE + i, v = tj * NL_TILE + j;
  const double* Zr = Z + R.z_off;
  double acc = 0.0;
  for (int r0 = 0; r0 < R.n; r0 += NL_TILE) {
    // thread (i, j) loads row r0 + i, columns ti*16 + j and tj*16 + j
    const int r = r0 + i;
    const int ca = ti * NL_TILE + j, cb = tj * NL_TILE + j;
    pa[i][j] = (r < R.n && ca < R.m) ? Zr[(long)r * R.m + ca] : 0.0;
    pb[i][j] = (r < R.n && cb < R.m) ? Zr[(long)r * R.m + cb] : 0.0;
    __syncthreads();
    for (int k = 0; k < NL_TILE; ++k) acc += pa[k][i] * pb[k][j];
    __syncthreads();
  }
  if (u < R.m && v < R.m && v <= u) S[R.s_off + (long)u * R.m + v] = acc;
}

// Per region: S = G G^T (dense Cholesky, in place, lower), then for each centre unit c:
// lambda = S^-1 e_c and y = Z lambda, written where the basis function goes (the band back
// substitution turns it into psi).
__global__ void __launch_bounds__(NL_BLOCK) k_nl_lambda(const RegionD* __restrict__ regs,
                                                        double* __restrict__ S,
                                                        const double* __restrict__ Z,
                                                        double* __restrict__ psi,
                                                        int* __restrict__ bad) {
  extern __shared__ double lam[];   // [m]
  const RegionD R = regs[blockIdx.x];
  const int m = R.m, tid = threadIdx.x;
  double* Sr = S + R.s_off;
  __shared__ double s_inv;
  __shared__ int s_bad;
  for (int k = 0; k < m; ++k) {
    if (tid == 0) {
      const double piv = Sr[(long)k * m + k];
      s_bad = !(piv > 0.0);
      const double lkk = s_bad ? 1.0 : sqrt(piv);
      Sr[(long)k * m + k] = lkk;
      s_inv = 1.0 / lkk;
    }
    __syncthreads();
    if (s_bad) {
      if (tid == 0) atomicMax(bad, 2);
      return;
    }
    for (int i = k + 1 + tid; i < m; i += blockDim.x) Sr[(long)i * m + k] *= s_inv;
    __syncthreads();
    const int rows = m - k - 1;
    for (int e = tid; e < rows * rows; e += blockDim.x) {
      const int i = k + 1 + e / rows, j = k + 1 + e % rows;
      if (j <= i) Sr[(long)i * m + j] -= Sr[(long)i * m + k] * Sr[(long)j * m + k];
    }
    __syncthreads();
  }
  for (int c = 0; c < R.ncenter; ++c) {
    // forward: G y = e_c ; backward: G^T lambda = y  (thread 0: m is small)
    if (tid == 0) {
      const int e = R.center_local[c];
      for (int i = 0; i < m; ++i) {
        double s = i == e ? 1.0 : 0.0;
        for (int j = 0; j < i; ++j) s -= Sr[(long)i * m + j] * lam[j];
        lam[i] = s / Sr[(long)i * m + i];
      }
      for (int i = m - 1; i >= 0; --i) {
        double s = lam[i];
        for (int j = i + 1; j < m; ++j) s -= Sr[(long)j * m + i] * lam[j];
        lam[i] = s / Sr[(long)i * m + i];
      }
    }
    __syncthreads();
    const double* Zr = Z + R.z_off;
    double* y = psi + R.psi_off[c];
    for (int r = tid; r < R.n; r += blockDim.x) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += Zr[(long)r * m + k] * lam[k];
      y[r] = s;
    }
    __syncthreads();
  }
}

// psi = L^-T y in place, one wavefront per centre unit (lanes split the band sum; the last
// w values of psi in an LDS ring).
__global__ void __launch_bounds__(64) k_nl_back(const RegionD* __restrict__ regs,
                                                const int* __restrict__ unit_region,
                                                const int* __restrict__ unit_center,
                                                const double* __restrict__ band,
                                                double* __restrict__ psi) {
  extern __shared__ double ring[];   // [w + 1]
  const int u = blockIdx.x;
  const RegionD R = regs[unit_region[u]];
  const int c = unit_center[u];
  const int lane = threadIdx.x;
  const int ld = R.w + 1;
  const double* B = band + R.band_off;
  double* x = psi + R.psi_off[c];
  int pos = (R.n - 1) % ld;   // ring slot of row r: r mod ld
  for (int r = R.n - 1; r >= 0; --r) {
    const int dmax = min(R.w, R.n - 1 - r);
    double acc = 0.0;
    for (int d = 1 + lane; d <= dmax; d += 64) {
      int q = pos + d;
      if (q >= ld) q -= ld;
      acc += B[(long)(r + d) * ld + d] * ring[q];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    const double v = (x[r] - acc) / B[(long)r * ld];
    __syncthreads();
    if (lane == 0) {
      ring[pos] = v;
      x[r] = v;
    }
    __syncthreads();
    pos = pos == 0 ? ld - 1 : pos - 1;
  }
}

// t_u = A psi_u on the extended box of u's region (zero values of psi outside its box).
__global__ void __launch_bounds__(NL_BLOCK) k_nl_apply(const RegionD* __restrict__ regs,
                                                       FineD f, const int* __restrict__ starts,
                                                       const int* __restrict__ unit_region,
                                                       const int* __restrict__ unit_center,
                                                       const int* __restrict__ hidx,
                                                       const int* __restrict__ rank,
                                                       const double* __restrict__ psi,
                                                       const long* __restrict__ t_off,
                                                       double* __restrict__ t) {
  const int u = blockIdx.x;
  const RegionD R = regs[unit_region[u]];
  const double* ps = psi + R.psi_off[unit_center[u]];
  const int* st = starts + R.start_off;
  const int* es = starts + R.ext_off;
  double* tu = t + t_off[u];
  auto P = [&](int x, int y, int s) {
    const int r = box_row(st, R.x0, R.y0, R.W, R.H, x, y, s);
    return r < 0 ? 0.0 : ps[r];
  };
  const int ncells = R.eW * R.eH;
  for (int ce = threadIdx.x; ce < ncells; ce += blockDim.x) {
    const int x = R.ex0 + ce % R.eW, y = R.ey0 + ce / R.eW;
    const long g = (long)y * f.nx + x;
    const int r0 = es[ce];
    for (int a = 0; a < f.n_omega; ++a) {
      double v = diagA_grid(f, a, g) * P(x, y, a);
      v -= east_T(f, a, g, x) * P(x + 1, y, a);
      v -= north_T(f, a, g, y) * P(x, y + 1, a);
      if (x > 0) v -= east_T(f, a, g - 1, x - 1) * P(x - 1, y, a);
      if (y > 0) v -= north_T(f, a, g - f.nx, y - 1) * P(x, y - 1, a);
      if (f.n_omega == 2) v -= f.s12 * P(x, y, 1 - a);
      if (f.nf)
        for (int k = f.hptr[g]; k < f.hptr[g + 1]; ++k) {
          const int l = hidx[k];
          v -= f.sigma_f[(long)a * f.nf + l] * P(x, y, f.n_omega + (k - f.hptr[g]));
        }
      tu[r0 + a] = v;
    }
    if (f.nf)
      for (int k = f.hptr[g]; k < f.hptr[g + 1]; ++k) {
        const int l = hidx[k];
        const int s = f.n_omega + (k - f.hptr[g]);
        double v = diagA_frac(f, l) * P(x, y, s);
        for (int e = f.rowptr[l]; e < f.rowptr[l + 1]; ++e) {
          const int l2 = f.col[e];
          const int g2 = f.host[l2];
          v -= f.val[e] * P(g2 % f.nx, g2 / f.nx, f.n_omega + rank[l2]);
        }
        for (int a = 0; a < f.n_omega; ++a) v -= f.sigma_f[(long)a * f.nf + l] * P(x, y, a);
        tu[r0 + s] = v;
      }
  }
}

// A_bar[u][v] = psi_v . t_u over the cells of v's box inside u's extended box; one wavefront
// per pair (u, v).
__global__ void __launch_bounds__(NL_BLOCK) k_nl_pairs(const RegionD* __restrict__ regs,
                                                       const int* __restrict__ starts,
                                                       const int* __restrict__ unit_region,
                                                       const int* __restrict__ unit_center,
                                                       const int* __restrict__ pu,
                                                       const int* __restrict__ pv, long npairs,
                                                       const double* __restrict__ psi,
                                                       const double* __restrict__ t,
                                                       const long* __restrict__ t_off, int nh,
                                                       double* __restrict__ Abar) {
  const long p = (long)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (p >= npairs) return;
  const int u = pu[p], v = pv[p];
  const RegionD Ru = regs[unit_region[u]];
  const RegionD Rv = regs[unit_region[v]];
  const int* es = starts + Ru.ext_off;
  const int* bs = starts + Rv.start_off;
  const double* tu = t + t_off[u];
  const double* pvv = psi + Rv.psi_off[unit_center[v]];
  const int x0 = max(Ru.ex0, Rv.x0), x1 = min(Ru.ex0 + Ru.eW, Rv.x0 + Rv.W);
  const int y0 = max(Ru.ey0, Rv.y0), y1 = min(Ru.ey0 + Ru.eH, Rv.y0 + Rv.H);
  double acc = 0.0;
  const int wx = x1 - x0;
  const int cells = wx > 0 && y1 > y0 ? wx * (y1 - y0) : 0;
  for (int c = lane; c < cells; c += 64) {
    const int x = x0 + c % wx, y = y0 + c / wx;
    const int cb = (y - Rv.y0) * Rv.W + (x - Rv.x0);
    const int ce = (y - Ru.ey0) * Ru.eW + (x - Ru.ex0);
    const int rb = bs[cb], cnt = bs[cb + 1] - rb, re = es[ce];
    for (int s = 0; s < cnt; ++s) acc += pvv[rb + s] * tu[re + s];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) Abar[(long)u * nh + v] = acc;
}

// A_bar <- (A_bar + A_bar^T) / 2 off the diagonal
__global__ void k_nl_sym(double* __restrict__ A, int nh) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)nh * nh) return;
  const int u = (int)(e / nh), v = (int)(e % nh);
  if (v <= u) return;
  const double s = 0.5 * (A[(long)u * nh + v] + A[(long)v * nh + u]);
  A[(long)u * nh + v] = s;
  A[(long)v * nh + u] = s;
}

// diagonal: row u sums to rs[u]; one wavefront per row
__global__ void k_nl_diag(double* __restrict__ A, int nh, const double* __restrict__ rs) {
  const int u = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (u >= nh) return;
  double s = 0.0;
  for (int v = lane; v < nh; v += 64)
    if (v != u) s += A[(long)u * nh + v];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) A[(long)u * nh + u] = rs[u] - s;
}

// K = diag(mt) + A_bar on the units [r0, r0 + n) (column-major = row-major: symmetric)
__global__ void k_nl_block(const double* __restrict__ A, int nh, const double* __restrict__ mt,
                           int r0, int n, double* __restrict__ K) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  K[e] = A[(long)(r0 + i) * nh + (r0 + j)] + (i == j ? mt[r0 + i] : 0.0);
}

// ---------------------------------------------------------------------------------------
// stepping
// ---------------------------------------------------------------------------------------
// rhs[u] = mt[u] x[u] + F[u] - sum_{v outside [b0, b1)} A_bar[u][v] x[v] for rows
// u in [r0, r1), where x holds the newest values of every block (the right-hand side of
// eqs. is-nlmc / si-nlmc for the block [b0, b1)); one wavefront per row.
__global__ void k_nl_rhs(const double* __restrict__ A, int nh, const double* __restrict__ mt,
                         const double* __restrict__ F, const double* __restrict__ x, int r0,
                         int r1, int b0, int b1, double* __restrict__ rhs) {
  const int u = r0 + blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (u >= r1) return;
  double s = 0.0;
  const double* Au = A + (long)u * nh;
  for (int v = lane; v < nh; v += 64)
    if (v < b0 || v >= b1) s += Au[v] * x[v];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) rhs[u] = mt[u] * x[u] + F[u] - s;
}

// x[r0 + i] = sum_j Kinv[i][j] rhs[j]; one wavefront per row.  Block-diagonal solves of the
// D-scheme pass a table of blocks (unit -> its block's inverse and offset).
__global__ void k_nl_mv(const double* __restrict__ Kinv, const long* __restrict__ koff,
                        const int* __restrict__ blk_of, const int* __restrict__ blk_r0,
                        const int* __restrict__ blk_n, int r0, int r1,
                        const double* __restrict__ rhs, double* __restrict__ x) {
  const int u = r0 + blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (u >= r1) return;
  const int b = blk_of[u];
  const int n = blk_n[b], b0 = blk_r0[b];
  const double* Ki = Kinv + koff[b] + (long)(u - b0) * n;
  const double* rb = rhs + b0;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += Ki[j] * rb[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) x[u] = s;
}


// ---------------------------------------------------------------------------------------
// host object
// ---------------------------------------------------------------------------------------
static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

struct Arena {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  template <class T>
  T* alloc(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      throw NlError{MC_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed"};
    }
    ptrs.push_back(p);
    bytes += n * sizeof(T);
    return (T*)p;
  }
  template <class T>
  T* upload(const std::vector<T>& h, hipStream_t s) {
    T* d = alloc<T>(h.size());
    if (!h.empty()) NL_CHECK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
};

}  // namespace nl
}  // namespace mc

using namespace mc::nl;

struct mc_nlmc {
  int nh = 0, ncont = 0;
  int sizes[3] = {0, 0, 0};
  int n_omega = 0;
  double tau = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  Arena mem;
  mc::NlPlan plan;
  double* A = nullptr;     // [nh * nh] coarse operator
  double* mbar = nullptr;  // [nh] coarse storage M_bar (diagonal)
  double* mt = nullptr;    // [nh] M_bar / tau
  double* F = nullptr;     // [nh] coarse right-hand side
  double* x = nullptr;     // [nh] coarse state
  double* x0 = nullptr;    // [nh] unit means of the fine state at creation
  double* rhs = nullptr;   // [nh]
  int* blk_of = nullptr;   // [nh] continuum block of each unit
  // per scheme (0 coupled, 1 blocks): inverses of the systems solved each layer
  double* kinv[2] = {nullptr, nullptr};
  long* koff[2] = {nullptr, nullptr};
  int* kblk_of[2] = {nullptr, nullptr};
  int* kb0[2] = {nullptr, nullptr};
  int* kbn[2] = {nullptr, nullptr};
  double setup_ms[4] = {0, 0, 0, 0};
  long steps = 0;
  std::string err;
};

namespace {

thread_local std::string g_nl_error;

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  NL_CHECK(hipEventElapsedTime(&ms, a, b));
  return ms;
}

// inverse of diag(mt) + A_bar on [r0, r0 + n) into K (n x n)
void block_inverse(mc_nlmc* N, int r0, int n, double* K) {
  hipLaunchKernelGGL(k_nl_block, dim3(cdiv((long)n * n, 256)), dim3(256), 0, N->stream, N->A,
                     N->nh, N->mt, r0, n, K);
  NL_CHECK(hipGetLastError());
  try {
    mc::spd_inverse(K, n, N->stream, n);
  } catch (...) {
    throw NlError{MC_EDEVICE, "inverse of a coarse system failed (not positive definite?)"};
  }
}

void build(mc_nlmc* N, mc_problem* fine, int bx, int by, int layers) {
  mc::FineView v;
  try {
    mc::fine_view(fine, v);
  } catch (const std::exception& e) {
    throw NlError{MC_EINVAL, e.what()};
  } catch (...) {
    throw NlError{MC_EINVAL, "the fine problem cannot serve the coarse-grid path"};
  }
  int dev = -1;
  NL_CHECK(hipGetDevice(&dev));
  if (dev != v.device) throw NlError{MC_EINVAL, "the fine problem's device must be current"};
  N->device = dev;
  N->stream = v.stream;
  N->tau = v.tau;
  N->n_omega = v.n_omega;
  const hipStream_t s = v.stream;
  try {
    N->plan = mc::build_nl_plan(v.nx, v.ny, v.n_omega, v.nf, v.h_host.data(), v.h_rowptr.data(),
                                v.h_col.data(), bx, by, layers);
  } catch (const std::exception& e) {
    throw NlError{MC_EINVAL, e.what()};
  }
  const mc::NlPlan& P = N->plan;
  N->nh = P.nunits;
  N->ncont = (int)P.usize.size();
  for (int a = 0; a < N->ncont && a < 3; ++a) N->sizes[a] = P.usize[a];
  Arena& M = N->mem;
  // fine operator view
  FineD f;
  std::memset(&f, 0, sizeof(f));
  f.nx = v.nx;
  f.ny = v.ny;
  f.n_omega = v.n_omega;
  f.nf = v.nf;
  f.ncell = v.ncell;
  f.s12 = v.s12;
  f.h2 = v.h * v.h;
  f.aperture = v.aperture;
  f.c_f = v.c_f;
  for (int a = 0; a < 2; ++a) {
    f.mtau[a] = v.mtau[a];
    f.c[a] = v.c[a];
    f.tconst[a] = v.tconst[a];
    f.has_t[a] = v.has_t[a];
    f.tx[a] = v.tx[a];
    f.ty[a] = v.ty[a];
  }
  for (int c = 0; c < 3; ++c) {
    f.diag[c] = v.diag[c];
    f.F[c] = v.F[c];
    f.state[c] = v.state[c];
  }
  f.mt = v.mt;
  f.val = v.val;
  f.sigma_f = v.sigma_f;
  f.flen = v.flen;
  f.rowptr = v.rowptr;
  f.col = v.col;
  f.host = v.host;
  f.hptr = v.hptr;
  // regions to the device
  std::vector<RegionD> hr(P.reg.size());
  std::vector<long> cpsi;
  for (size_t i = 0; i < P.reg.size(); ++i) {
    const mc::NlRegion& R = P.reg[i];
    RegionD& d = hr[i];
    std::memset(&d, 0, sizeof(d));
    d.x0 = R.box.x0;
    d.y0 = R.box.y0;
    d.W = R.box.W;
    d.H = R.box.H;
    d.ex0 = R.ext.x0;
    d.ey0 = R.ext.y0;
    d.eW = R.ext.W;
    d.eH = R.ext.H;
    d.n = R.n;
    d.w = R.w;
    d.m = R.m;
    d.ncenter = R.ncenter;
    for (int c = 0; c < 3; ++c) {
      d.center_local[c] = R.center_local[c];
      d.center_unit[c] = R.center_unit[c];
      d.psi_off[c] = c < R.ncenter ? P.psi_off[R.center_unit[c]] : 0;
    }
    d.start_off = R.start_off;
    d.ext_off = R.ext_off;
    d.row_off = R.row_off;
    d.unit_off = R.unit_off;
    d.band_off = R.band_off;
    d.z_off = R.z_off;
    d.s_off = R.s_off;
  }
  const int nreg = (int)hr.size();
  const int nh = N->nh;
  RegionD* regs = M.upload(hr, s);
  int* starts = M.upload(P.starts, s);
  int* row_g = M.upload(P.row_g, s);
  int* row_unit = M.upload(P.row_unit, s);
  int* reg_units = M.upload(P.reg_units, s);
  int* rank = M.upload(P.rank, s);
  int* uptr = M.upload(P.uptr, s);
  int* ucell = M.upload(P.ucell, s);
  int* unit_region = M.upload(P.unit_region, s);
  int* unit_center = M.upload(P.unit_center, s);
  long* t_off = M.upload(P.t_off, s);
  std::vector<int> pu;
  for (int u = 0; u < nh; ++u)
    for (int k = P.pair_ptr[u]; k < P.pair_ptr[u + 1]; ++k) pu.push_back(u);
  int* d_pu = M.upload(pu, s);
  int* d_pv = M.upload(P.pair_v, s);
  const long npairs = (long)pu.size();
  int* bad = M.alloc<int>(1);
  NL_CHECK(hipMemsetAsync(bad, 0, sizeof(int), s));
  // fine vectors and unit sums
  const long nfine = (long)v.n_omega * v.ncell + v.nf;
  double* fv = M.alloc<double>(nfine);
  double* unit_meas = M.alloc<double>(nh);
  double* rs = M.alloc<double>(nh);
  N->mbar = M.alloc<double>(nh);
  N->mt = M.alloc<double>(nh);
  N->F = M.alloc<double>(nh);
  N->x = M.alloc<double>(nh);
  N->x0 = M.alloc<double>(nh);
  N->rhs = M.alloc<double>(nh);
  double* tmp = M.alloc<double>(nh);
  auto fine_sum = [&](int kind, double* out) {
    hipLaunchKernelGGL(k_nl_fine_vec, dim3(cdiv(nfine, 256)), dim3(256), 0, s, f, kind, fv);
    if (kind == 0 && v.nf)
      hipLaunchKernelGGL(k_nl_a1_transfer, dim3(cdiv(v.ncell, 256)), dim3(256), 0, s, f,
                         v.hidx, fv);
    hipLaunchKernelGGL(k_nl_unit_sum, dim3(cdiv(nh, 4)), dim3(256), 0, s, uptr, ucell, fv, nh,
                       out);
    NL_CHECK(hipGetLastError());
  };
  hipEvent_t ev[5];
  for (auto& e : ev) NL_CHECK(hipEventCreate(&e));
  NL_CHECK(hipEventRecord(ev[0], s));
  fine_sum(3, unit_meas);
  fine_sum(0, rs);
  fine_sum(1, N->mbar);
  fine_sum(2, N->F);
  fine_sum(4, tmp);
  hipLaunchKernelGGL(k_nl_div, dim3(cdiv(nh, 256)), dim3(256), 0, s, tmp, unit_meas, nh, N->x0);
  std::vector<double> htau(nh, v.tau);
  double* dtau = M.upload(htau, s);
  hipLaunchKernelGGL(k_nl_div, dim3(cdiv(nh, 256)), dim3(256), 0, s, N->mbar, dtau, nh, N->mt);
  NL_CHECK(hipMemcpyAsync(N->x, N->x0, nh * sizeof(double), hipMemcpyDeviceToDevice, s));
  // local operators, their factors and the basis functions
  double* band = M.alloc<double>(P.band);
  double* rw = M.alloc<double>(P.rows);
  double* Z = M.alloc<double>(P.zsize);
  double* S = M.alloc<double>(P.ssize);
  double* psi = M.alloc<double>(P.psi_size);
  double* t = M.alloc<double>(P.t_size);
  NL_CHECK(hipMemsetAsync(band, 0, P.band * sizeof(double), s));
  hipLaunchKernelGGL(k_nl_band, dim3(nreg), dim3(NL_BLOCK), 0, s, regs, f, starts, row_g,
                     row_unit, reg_units, rank, unit_meas, band, rw);
  hipLaunchKernelGGL(k_nl_chol, dim3(nreg), dim3(NL_BLOCK), 0, s, regs, band, bad);
  NL_CHECK(hipGetLastError());
  NL_CHECK(hipEventRecord(ev[1], s));
  const size_t fwd_lds = ((size_t)(P.max_w + 1) * 64 + 4 * 64) * sizeof(double);
  if (fwd_lds > 160 * 1024)
    throw NlError{MC_EINVAL, "local band width " + std::to_string(P.max_w) +
                                 " exceeds the forward solve's LDS ring; use smaller coarse "
                                 "cells or fewer oversampling layers"};
  if (fwd_lds > 64 * 1024)
    NL_CHECK(hipFuncSetAttribute((const void*)k_nl_fwd,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)fwd_lds));
  hipLaunchKernelGGL(k_nl_fwd, dim3(nreg, cdiv(P.max_m, NL_FWD_COLS)), dim3(NL_BLOCK), fwd_lds,
                     s, regs, band, row_unit, rw, Z);
  const int nt = (int)cdiv(P.max_m, NL_TILE);
  hipLaunchKernelGGL(k_nl_gram, dim3(nreg, nt * (nt + 1) / 2), dim3(NL_BLOCK), 0, s, regs, Z, S);
  hipLaunchKernelGGL(k_nl_lambda, dim3(nreg), dim3(NL_BLOCK), P.max_m * sizeof(double), s, regs,
                     S, Z, psi, bad);
  hipLaunchKernelGGL(k_nl_back, dim3(nh), dim3(64), (P.max_w + 1) * sizeof(double), s, regs,
                     unit_region, unit_center, band, psi);
  NL_CHECK(hipGetLastError());
  NL_CHECK(hipEventRecord(ev[2], s));
  // coarse operator
  N->A = M.alloc<double>((size_t)nh * nh);
  NL_CHECK(hipMemsetAsync(N->A, 0, (size_t)nh * nh * sizeof(double), s));
  hipLaunchKernelGGL(k_nl_apply, dim3(nh), dim3(NL_BLOCK), 0, s, regs, f, starts, unit_region,
                     unit_center, v.hidx, rank, psi, t_off, t);
  if (npairs)
    hipLaunchKernelGGL(k_nl_pairs, dim3(cdiv(npairs, 4)), dim3(256), 0, s, regs, starts,
                       unit_region, unit_center, d_pu, d_pv, npairs, psi, t, t_off, nh, N->A);
  hipLaunchKernelGGL(k_nl_sym, dim3(cdiv((long)nh * nh, 256)), dim3(256), 0, s, N->A, nh);
  hipLaunchKernelGGL(k_nl_diag, dim3(cdiv(nh, 4)), dim3(256), 0, s, N->A, nh, rs);
  NL_CHECK(hipGetLastError());
  NL_CHECK(hipEventRecord(ev[3], s));
  // inverses: [0] the coupled system, [1] the continuum blocks
  std::vector<int> b0(N->ncont), bn(N->ncont), blk(nh);
  int off = 0;
  for (int a = 0; a < N->ncont; ++a) {
    b0[a] = off;
    bn[a] = P.usize[a];
    for (int u = off; u < off + bn[a]; ++u) blk[u] = a;
    off += bn[a];
  }
  N->blk_of = M.upload(blk, s);
  {
    std::vector<long> ko{0};
    std::vector<int> z0{0}, zn{nh}, zb(nh, 0);
    N->kinv[0] = M.alloc<double>((size_t)nh * nh);
    block_inverse(N, 0, nh, N->kinv[0]);
    N->koff[0] = M.upload(ko, s);
    N->kblk_of[0] = M.upload(zb, s);
    N->kb0[0] = M.upload(z0, s);
    N->kbn[0] = M.upload(zn, s);
  }
  {
    std::vector<long> ko;
    long tot = 0;
    for (int a = 0; a < N->ncont; ++a) {
      ko.push_back(tot);
      tot += (long)bn[a] * bn[a];
    }
    N->kinv[1] = M.alloc<double>(tot);
    for (int a = 0; a < N->ncont; ++a) block_inverse(N, b0[a], bn[a], N->kinv[1] + ko[a]);
    N->koff[1] = M.upload(ko, s);
    N->kblk_of[1] = M.upload(blk, s);
    N->kb0[1] = M.upload(b0, s);
    N->kbn[1] = M.upload(bn, s);
  }
  NL_CHECK(hipEventRecord(ev[4], s));
  int hbad = 0;
  NL_CHECK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  NL_CHECK(hipStreamSynchronize(s));
  for (int k = 0; k < 4; ++k) N->setup_ms[k] = elapsed_ms(ev[k], ev[k + 1]);
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (hbad == 1)
    throw NlError{MC_EBREAKDOWN, "a local operator of an oversampled region is not positive "
                                 "definite (a region without Dirichlet values, wells or a "
                                 "boundary inside the domain?)"};
  if (hbad == 2) throw NlError{MC_EBREAKDOWN, "a constraint Schur complement is not positive definite"};
  // the scratch of the basis construction is no longer needed
  for (void* p : {(void*)band, (void*)Z, (void*)S, (void*)t, (void*)psi, (void*)rw, (void*)fv}) {
    auto it = std::find(M.ptrs.begin(), M.ptrs.end(), p);
    if (it != M.ptrs.end()) {
      (void)hipFree(p);
      M.ptrs.erase(it);
    }
  }
}

// one layer of the scheme on the state N->x
void layer(mc_nlmc* N, int scheme) {
  const hipStream_t s = N->stream;
  const int nh = N->nh;
  auto rhs = [&](int r0, int r1, int b0, int b1) {
    hipLaunchKernelGGL(k_nl_rhs, dim3(cdiv(r1 - r0, 4)), dim3(256), 0, s, N->A, nh, N->mt, N->F,
                       N->x, r0, r1, b0, b1, N->rhs);
  };
  auto mv = [&](int k, int r0, int r1) {
    hipLaunchKernelGGL(k_nl_mv, dim3(cdiv(r1 - r0, 4)), dim3(256), 0, s, N->kinv[k], N->koff[k],
                       N->kblk_of[k], N->kb0[k], N->kbn[k], r0, r1, N->rhs, N->x);
  };
  if (scheme == MC_SCHEME_COUPLED) {
    rhs(0, nh, 0, nh);
    mv(0, 0, nh);
  } else if (scheme == MC_SCHEME_D) {
    // every block's right-hand side from the previous layer, then the block solves
    int off = 0;
    for (int a = 0; a < N->ncont; ++a) {
      rhs(off, off + N->sizes[a], off, off + N->sizes[a]);
      off += N->sizes[a];
    }
    mv(1, 0, nh);
  } else {
    // L: ascending continua, U: descending; solved blocks enter with their new values
    std::vector<int> order;
    for (int a = 0; a < N->ncont; ++a) order.push_back(a);
    if (scheme == MC_SCHEME_U) std::reverse(order.begin(), order.end());
    for (int a : order) {
      int off = 0;
      for (int b = 0; b < a; ++b) off += N->sizes[b];
      rhs(off, off + N->sizes[a], off, off + N->sizes[a]);
      mv(1, off, off + N->sizes[a]);
    }
  }
  NL_CHECK(hipGetLastError());
}

}  // namespace

#define NL_BEGIN try {
#define NL_END(N)                                                                       \
  }                                                                                     \
  catch (const NlError& e) {                                                            \
    if (N) (N)->err = e.msg; else g_nl_error = e.msg;                                   \
    return e.st;                                                                        \
  }                                                                                     \
  catch (const std::exception& e) {                                                     \
    if (N) (N)->err = e.what(); else g_nl_error = e.what();                             \
    return MC_EDEVICE;                                                                  \
  }

extern "C" {

mc_status mc_nlmc_create(mc_problem* fine, int32_t bx, int32_t by, int32_t layers,
                         mc_nlmc** out) {
  if (!out) return MC_EINVAL;
  *out = nullptr;
  if (!fine) {
    g_nl_error = "fine problem is NULL";
    return MC_EINVAL;
  }
  mc_nlmc* N = new mc_nlmc();
  try {
    build(N, fine, bx, by, layers);
  } catch (const NlError& e) {
    g_nl_error = e.msg;
    mc_nlmc_destroy(N);
    return e.st;
  } catch (const std::exception& e) {
    g_nl_error = e.what();
    mc_nlmc_destroy(N);
    return MC_EDEVICE;
  }
  *out = N;
  return MC_OK;
}

mc_status mc_nlmc_destroy(mc_nlmc* N) {
  if (!N) return MC_OK;
  if (N->stream) (void)hipStreamSynchronize(N->stream);
  N->mem.release();
  delete N;
  return MC_OK;
}

mc_status mc_nlmc_get_info(const mc_nlmc* N, mc_nlmc_info* info) {
  if (!N || !info) return MC_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->n_units = N->nh;
  info->n_cont = N->ncont;
  for (int a = 0; a < 3; ++a) info->sizes[a] = N->sizes[a];
  info->n_regions = (int32_t)N->plan.reg.size();
  info->max_region_unknowns = N->plan.max_n;
  info->max_band = N->plan.max_w;
  info->max_constraints = N->plan.max_m;
  info->n_pairs = (int64_t)N->plan.pair_v.size();
  info->device_bytes = (int64_t)N->mem.bytes;
  for (int k = 0; k < 4; ++k) info->setup_ms[k] = N->setup_ms[k];
  info->steps = N->steps;
  return MC_OK;
}

mc_status mc_nlmc_get_system(mc_nlmc* N, double* A_host, double* M_host, double* F_host) {
  if (!N) return MC_EINVAL;
  NL_BEGIN
  const size_t nh = (size_t)N->nh;
  if (A_host) NL_CHECK(hipMemcpyAsync(A_host, N->A, nh * nh * sizeof(double), hipMemcpyDeviceToHost, N->stream));
  if (M_host) NL_CHECK(hipMemcpyAsync(M_host, N->mbar, nh * sizeof(double), hipMemcpyDeviceToHost, N->stream));
  if (F_host) NL_CHECK(hipMemcpyAsync(F_host, N->F, nh * sizeof(double), hipMemcpyDeviceToHost, N->stream));
  NL_CHECK(hipStreamSynchronize(N->stream));
  return MC_OK;
  NL_END(N)
}

mc_status mc_nlmc_set_state(mc_nlmc* N, const double* host_in) {
  if (!N) return MC_EINVAL;
  NL_BEGIN
  if (host_in)
    NL_CHECK(hipMemcpyAsync(N->x, host_in, N->nh * sizeof(double), hipMemcpyHostToDevice, N->stream));
  else
    NL_CHECK(hipMemcpyAsync(N->x, N->x0, N->nh * sizeof(double), hipMemcpyDeviceToDevice, N->stream));
  NL_CHECK(hipStreamSynchronize(N->stream));
  N->steps = 0;
  return MC_OK;
  NL_END(N)
}

mc_status mc_nlmc_get_state(mc_nlmc* N, double* host_out) {
  if (!N || !host_out) return MC_EINVAL;
  NL_BEGIN
  NL_CHECK(hipMemcpyAsync(host_out, N->x, N->nh * sizeof(double), hipMemcpyDeviceToHost, N->stream));
  NL_CHECK(hipStreamSynchronize(N->stream));
  return MC_OK;
  NL_END(N)
}

mc_status mc_nlmc_step(mc_nlmc* N, int32_t scheme, int32_t n_steps) {
  if (!N) return MC_EINVAL;
  NL_BEGIN
  if (n_steps < 1) throw NlError{MC_EINVAL, "n_steps must be >= 1"};
  if (scheme != MC_SCHEME_COUPLED && scheme != MC_SCHEME_D && scheme != MC_SCHEME_L &&
      scheme != MC_SCHEME_U)
    throw NlError{MC_EINVAL, "the coarse schemes are coupled, D, L and U"};
  for (int k = 0; k < n_steps; ++k) layer(N, scheme);
  NL_CHECK(hipStreamSynchronize(N->stream));
  N->steps += n_steps;
  return MC_OK;
  NL_END(N)
}

const char* mc_nlmc_last_error(const mc_nlmc* N) {
  if (N) return N->err.c_str();
  return g_nl_error.c_str();
}

}  // extern "C"
