#include "host_setup.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace mc {

namespace {
bool fin(double v) { return std::isfinite(v); }

std::string fmt(const char* f, long a = 0, long b = 0) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), f, a, b);
  return buf;
}
}  // namespace

std::string validate_desc(const mc_problem_desc& d) {
  if (d.nx < 1 || d.ny < 1) return "nx and ny must be >= 1";
  if (d.nz < 0) return "nz must be >= 0 (0 or 1: a 2-D grid)";
  const long nzp = d.nz > 1 ? d.nz : 1;
  if ((long)d.nx * (long)d.ny * nzp > (1L << 31) - 2) return "grid too large for 32-bit cell indices";
  if (!(d.h > 0) || !fin(d.h)) return "h must be finite and > 0";
  if (!(d.tau > 0) || !fin(d.tau)) return "tau must be finite and > 0";
  if (d.n_omega != 1 && d.n_omega != 2) return "n_omega must be 1 or 2";
  const long nc = (long)d.nx * d.ny * nzp;
  for (int a = 0; a < d.n_omega; ++a) {
    const mc_omega_desc& o = d.omega[a];
    if (!(o.c > 0) || !fin(o.c)) return fmt("omega[%ld].c must be finite and > 0", a);
    if (o.k) {
      for (long i = 0; i < nc; ++i)
        if (!(o.k[i] >= 0) || !fin(o.k[i])) return fmt("omega[%ld].k[%ld] invalid", a, i);
    } else if (!(o.k_const >= 0) || !fin(o.k_const)) {
      return fmt("omega[%ld].k_const must be finite and >= 0", a);
    }
    if (o.src)
      for (long i = 0; i < nc; ++i)
        if (!fin(o.src[i])) return fmt("omega[%ld].src[%ld] not finite", a, i);
    if (o.p0)
      for (long i = 0; i < nc; ++i)
        if (!fin(o.p0[i])) return fmt("omega[%ld].p0[%ld] not finite", a, i);
  }
  if (!(d.sigma_omega >= 0) || !fin(d.sigma_omega)) return "sigma_omega must be finite and >= 0";
  for (int s = 0; s < 4; ++s) {
    if (d.bc_type[s] != 0 && d.bc_type[s] != 1) return fmt("bc_type[%ld] must be 0 or 1", s);
    if (d.bc_type[s] == 1 && !fin(d.bc_value[s])) return fmt("bc_value[%ld] not finite", s);
  }
  if (nzp > 1)
    for (int s = 0; s < 2; ++s) {
      if (d.bc_type_z[s] != 0 && d.bc_type_z[s] != 1) return fmt("bc_type_z[%ld] must be 0 or 1", s);
      if (d.bc_type_z[s] == 1 && !fin(d.bc_value_z[s])) return fmt("bc_value_z[%ld] not finite", s);
    }
  if (d.nf < 0) return "nf must be >= 0";
  if (d.nf > 0) {
    if (!d.host || !d.flen || !d.sigma_f) return "host, flen and sigma_f are required when nf > 0";
    if (!(d.k_f >= 0) || !fin(d.k_f)) return "k_f must be finite and >= 0";
    if (!(d.c_f > 0) || !fin(d.c_f)) return "c_f must be finite and > 0";
    if (!(d.aperture > 0) || !fin(d.aperture)) return "aperture must be finite and > 0";
    for (int l = 0; l < d.nf; ++l) {
      if (d.host[l] < 0 || d.host[l] >= nc) return fmt("host[%ld] = %ld out of range", l, d.host[l]);
      if (!(d.flen[l] > 0) || !fin(d.flen[l])) return fmt("flen[%ld] must be > 0", l);
    }
    for (long j = 0; j < (long)d.n_omega * d.nf; ++j)
      if (!(d.sigma_f[j] >= 0) || !fin(d.sigma_f[j])) return fmt("sigma_f[%ld] invalid", j);
    if (d.src_f)
      for (int l = 0; l < d.nf; ++l)
        if (!fin(d.src_f[l])) return fmt("src_f[%ld] not finite", l);
    if (d.p0_f)
      for (int l = 0; l < d.nf; ++l)
        if (!fin(d.p0_f[l])) return fmt("p0_f[%ld] not finite", l);
    if (d.well_q)
      for (int l = 0; l < d.nf; ++l)
        if (!(d.well_q[l] >= 0) || !fin(d.well_q[l])) return fmt("well_q[%ld] must be finite and >= 0", l);
    if (d.well_p)
      for (int l = 0; l < d.nf; ++l)
        if (!fin(d.well_p[l])) return fmt("well_p[%ld] not finite", l);
  }
  if (d.ne < 0) return "ne must be >= 0";
  if (d.ne > 0) {
    if (d.nf == 0 || !d.edges || !d.edge_d) return "edges and edge_d are required when ne > 0";
    for (int e = 0; e < d.ne; ++e) {
      int a = d.edges[2 * e], b = d.edges[2 * e + 1];
      if (a < 0 || a >= d.nf || b < 0 || b >= d.nf) return fmt("edge %ld endpoint out of range", e);
      if (a == b) return fmt("edge %ld joins a cell to itself", e);
      if (!(d.edge_d[e] > 0) || !fin(d.edge_d[e])) return fmt("edge_d[%ld] must be > 0", e);
    }
  }
  return "";
}

std::string validate_options(const mc_options& o) {
  if (o.scheme < MC_SCHEME_D || o.scheme > MC_SCHEME_EX) return "unknown scheme";
  if (o.precision != MC_FP64 && o.precision != MC_MIXED) return "unknown precision";
  if (o.precond != MC_JACOBI && o.precond != MC_BIC0 && o.precond != MC_MG)
    return "unknown preconditioner";
  if (!(o.tol > 0 && o.tol < 1)) return "tol must be in (0, 1)";
  if (o.max_iter < 1) return "max_iter must be >= 1";
  if (o.precision == MC_MIXED) {
    if (!(o.outer_tol > 0 && o.outer_tol < 1)) return "outer_tol must be in (0, 1)";
    if (!(o.inner_tol > 0 && o.inner_tol < 1)) return "inner_tol must be in (0, 1)";
    if (o.max_outer < 1) return "max_outer must be >= 1";
    if (o.scheme == MC_SCHEME_COUPLED) return "the coupled scheme runs in FP64 only";
  }
  if (o.check_every < 0) return "check_every must be >= 0";
  if (o.tile_rows != 0 && o.tile_rows != 32)
    return "tile_rows must be 0 (default) or 32 in this build";
  if (o.warm_start < 0 || o.warm_start > 2)
    return "warm_start must be 0 (linear extrapolation), 1 (previous layer) or 2 (adaptive "
           "extrapolation)";
  if (o.small_max < 0) return "small_max must be >= 0";
  if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr))
    return "dev_alloc and dev_free must be given together (or neither)";
  return "";
}

GraphCSR build_graph(int nf, int ne, const int32_t* edges) {
  GraphCSR g;
  g.rowptr.assign(nf + 1, 0);
  for (int e = 0; e < ne; ++e) {
    g.rowptr[edges[2 * e] + 1]++;
    g.rowptr[edges[2 * e + 1] + 1]++;
  }
  for (int l = 0; l < nf; ++l) g.rowptr[l + 1] += g.rowptr[l];
  std::vector<std::pair<int, int>> ent(g.rowptr[nf]);
  std::vector<int> fill(g.rowptr.begin(), g.rowptr.end() - 1);
  for (int e = 0; e < ne; ++e) {
    int a = edges[2 * e], b = edges[2 * e + 1];
    ent[fill[a]++] = {b, e};
    ent[fill[b]++] = {a, e};
  }
  for (int l = 0; l < nf; ++l)
    std::sort(ent.begin() + g.rowptr[l], ent.begin() + g.rowptr[l + 1]);
  g.col.resize(ent.size());
  g.eidx.resize(ent.size());
  for (size_t j = 0; j < ent.size(); ++j) {
    g.col[j] = ent[j].first;
    g.eidx[j] = ent[j].second;
  }
  return g;
}

HostMap build_host_map(int ncell, int nf, const int32_t* host) {
  HostMap m;
  m.hptr.assign((size_t)ncell + 1, 0);
  for (int l = 0; l < nf; ++l) m.hptr[(size_t)host[l] + 1]++;
  for (long i = 0; i < ncell; ++i) m.hptr[i + 1] += m.hptr[i];
  m.hidx.resize(nf);
  std::vector<int> fill(m.hptr.begin(), m.hptr.end() - 1);
  for (int l = 0; l < nf; ++l) m.hidx[fill[host[l]]++] = l;   // ascending l within a host
  return m;
}

std::vector<int> build_chains(int nf, const GraphCSR& g) {
  std::vector<int> ptr{0};
  for (int l = 0; l + 1 < nf; ++l) {
    bool linked = false;
    for (int j = g.rowptr[l]; j < g.rowptr[l + 1]; ++j)
      if (g.col[j] == l + 1) linked = true;
    if (!linked) ptr.push_back(l + 1);
  }
  if (nf > 0) ptr.push_back(nf);
  return ptr;
}

std::vector<int> build_graph_tiles(const std::vector<int>& chain_ptr, int target) {
  std::vector<int> t{0};
  const int nch = (int)chain_ptr.size() - 1;
  int cells = 0;
  for (int c = 0; c < nch; ++c) {
    cells += chain_ptr[c + 1] - chain_ptr[c];
    if (cells >= target) {
      t.push_back(c + 1);
      cells = 0;
    }
  }
  if (t.back() != nch) t.push_back(nch);
  return t;
}

int count_crossing_cells(int nf, int ne, const int32_t* edges) {
  std::vector<char> x(nf > 0 ? nf : 1, 0);
  int K = 0;
  for (int e = 0; e < ne; ++e) {
    const int a = edges[2 * e], b = edges[2 * e + 1];
    if (a - b == 1 || b - a == 1) continue;
    if (!x[a]) x[a] = 1, ++K;
    if (!x[b]) x[b] = 1, ++K;
  }
  return K;
}

SchurHost build_schur(int nf, const GraphCSR& g, const std::vector<int>& chain_ptr,
                      const std::vector<int>& gtile, const double* diag, const double* val,
                      int kmax) {
  SchurHost H;
  // conductance between l and l + 1 inside a chain (sum over parallel connections)
  std::vector<char> start(nf + 1, 0);
  for (size_t c = 0; c + 1 < chain_ptr.size(); ++c) start[chain_ptr[c]] = 1;
  start[nf] = 1;
  std::vector<double> link(nf, 0.0);
  std::vector<int> xidx(nf, -1);
  for (int l = 0; l < nf; ++l)
    for (int j = g.rowptr[l]; j < g.rowptr[l + 1]; ++j) {
      const int m = g.col[j];
      if (m == l + 1 && !start[l + 1]) link[l] += val[j];
      else if (m != l - 1 && m != l + 1) xidx[l] = 0;   // a crossing cell
    }
  for (int l = 0; l < nf; ++l)
    if (xidx[l] == 0) H.K_all += 1;
  const bool schur = H.K_all > 0 && H.K_all <= kmax;
  int K = 0;
  for (int l = 0; l < nf; ++l) {
    if (schur && xidx[l] == 0) {
      xidx[l] = K++;
      H.xcells.push_back(l);
    } else {
      xidx[l] = -1;
    }
  }
  H.K = K;
  H.dinv.assign(nf, 0.0);
  H.cT.assign(nf, 0.0);
  H.cl.assign(nf, 0.0);
  H.cr.assign(nf, 0.0);
  H.xl.assign(nf, -1);
  H.xr.assign(nf, -1);
  H.cxl.assign(K, 0.0);
  H.cxr.assign(K, 0.0);
  H.S.assign((size_t)K * K, 0.0);
  auto Sref = [&](int r, int c) -> double& { return H.S[(size_t)c * K + r]; };
  // A_XX
  for (int k = 0; k < K; ++k) {
    const int x = H.xcells[k];
    Sref(k, k) += diag[x];
    for (int j = g.rowptr[x]; j < g.rowptr[x + 1]; ++j) {
      const int m = xidx[g.col[j]];
      if (m >= 0) Sref(k, m) -= val[j];
    }
    H.cxl[k] = x > 0 && !start[x] ? link[x - 1] : 0.0;
    H.cxr[k] = !start[x + 1] ? link[x] : 0.0;
    H.xl[x] = k;
    H.cl[x] = 1.0;
  }
  // sub-chain blocks: tridiagonal factor, responses, and their share of S
  std::vector<double> u, v;
  for (size_t c = 0; c + 1 < chain_ptr.size(); ++c) {
    const int c0 = chain_ptr[c], c1 = chain_ptr[c + 1];
    int a = c0;
    while (a < c1) {
      if (xidx[a] >= 0) {
        ++a;
        continue;
      }
      int b = a;
      while (b + 1 < c1 && xidx[b + 1] < 0) ++b;
      // factor of the block [a, b]: d_a = a_aa, d_l = a_ll - c^2 / d_{l-1}
      H.cT[a] = 0.0;
      H.dinv[a] = 1.0 / diag[a];
      for (int l = a + 1; l <= b; ++l) {
        H.cT[l] = link[l - 1];
        H.dinv[l] = 1.0 / (diag[l] - H.cT[l] * H.cT[l] * H.dinv[l - 1]);
      }
      // T^-1 e_s by the same factor: forward u_l = (e_s + cT_l u_{l-1}) dinv_l, backward
      // z_l = u_l + cT_{l+1} dinv_l z_{l+1}
      auto col = [&](int s, std::vector<double>& z) {
        z.assign(b - a + 1, 0.0);
        double w = 0.0;
        for (int l = a; l <= b; ++l) {
          w = ((l == s ? 1.0 : 0.0) + (l > a ? H.cT[l] * w : 0.0)) * H.dinv[l];
          z[l - a] = w;
        }
        for (int l = b - 1; l >= a; --l) z[l - a] += H.cT[l + 1] * H.dinv[l] * z[l + 1 - a];
      };
      const int kl = a > c0 ? xidx[a - 1] : -1;     // a block starts at a chain start or after X
      const int kr = b + 1 < c1 ? xidx[b + 1] : -1;
      const double clk = kl >= 0 ? link[a - 1] : 0.0, crk = kr >= 0 ? link[b] : 0.0;
      if (kl >= 0) col(a, u);
      if (kr >= 0) col(b, v);
      for (int l = a; l <= b; ++l) {
        if (kl >= 0) {
          H.xl[l] = kl;
          H.cl[l] = clk * u[l - a];
        }
        if (kr >= 0) {
          H.xr[l] = kr;
          H.cr[l] = crk * v[l - a];
        }
      }
      if (kl >= 0) Sref(kl, kl) -= clk * clk * u[0];
      if (kr >= 0) Sref(kr, kr) -= crk * crk * v[b - a];
      if (kl >= 0 && kr >= 0) {
        Sref(kl, kr) -= clk * crk * u[b - a];
        Sref(kr, kl) -= clk * crk * u[b - a];
      }
      a = b + 1;
    }
  }
  // crossing cells of every work tile (tiles are contiguous runs of whole chains)
  const int nt = (int)gtile.size() - 1;
  H.xtile.assign(nt + 1, 0);
  for (int t = 0; t <= nt; ++t) {
    const int l0 = chain_ptr[gtile[t]];
    H.xtile[t] = (int)(std::lower_bound(H.xcells.begin(), H.xcells.end(), l0) - H.xcells.begin());
  }
  return H;
}

int build_blocks(int nf, const GraphCSR& g, std::vector<int>& node, std::vector<int>& blk) {
  blk.assign(nf, -1);
  node.clear();
  std::vector<int> queue;
  queue.reserve(kBlockCells);
  int nb = 0;
  for (int s = 0; s < nf; ++s) {
    if (blk[s] >= 0) continue;
    // breadth-first from s over unassigned cells until the block is full or closed
    queue.clear();
    queue.push_back(s);
    blk[s] = nb;
    for (size_t h = 0; h < queue.size() && (int)queue.size() < kBlockCells; ++h) {
      const int u = queue[h];
      for (int j = g.rowptr[u]; j < g.rowptr[u + 1] && (int)queue.size() < kBlockCells; ++j) {
        const int v = g.col[j];
        if (blk[v] < 0) {
          blk[v] = nb;
          queue.push_back(v);
        }
      }
    }
    node.insert(node.end(), queue.begin(), queue.end());
    node.insert(node.end(), kBlockCells - queue.size(), -1);
    ++nb;
  }
  return nb;
}

BlockHost build_block_solve(int nf, const GraphCSR& g, int ntiles, const double* diag,
                            const double* val, int nbmax) {
  BlockHost H;
  const int nb = build_blocks(nf, g, H.node, H.blk);
  if (nb > nbmax || nb == 0) {
    H = BlockHost{};
    return H;
  }
  H.nb = nb;
  constexpr int W = kBlockCells;
  H.binv.assign((size_t)nb * W * W, 0.0f);
  H.Ac.assign((size_t)nb * nb, 0.0);
  std::vector<int> pos(nf, -1);   // position of a cell inside its block
  std::vector<double> a(W * W), L(W * W), inv(W * W);
  for (int b = 0; b < nb; ++b) {
    const int* nd = &H.node[(size_t)b * W];
    int m = 0;
    while (m < W && nd[m] >= 0) pos[nd[m]] = m, ++m;
    // block matrix: the diagonal and minus the conductances inside the block
    std::fill(a.begin(), a.end(), 0.0);
    for (int i = 0; i < m; ++i) {
      const int l = nd[i];
      a[i * W + i] = diag[l];
      for (int j = g.rowptr[l]; j < g.rowptr[l + 1]; ++j)
        if (H.blk[g.col[j]] == b) a[i * W + pos[g.col[j]]] -= val[j];
    }
    // Cholesky a = L L^T (lower), then the inverse column by column from L
    std::fill(L.begin(), L.end(), 0.0);
    for (int j = 0; j < m; ++j) {
      double d = a[j * W + j];
      for (int k = 0; k < j; ++k) d -= L[j * W + k] * L[j * W + k];
      if (!(d > 0.0)) {
        H.ok = false;
        return H;
      }
      L[j * W + j] = std::sqrt(d);
      for (int i = j + 1; i < m; ++i) {
        double v = a[i * W + j];
        for (int k = 0; k < j; ++k) v -= L[i * W + k] * L[j * W + k];
        L[i * W + j] = v / L[j * W + j];
      }
    }
    for (int c = 0; c < m; ++c) {   // solve L L^T x = e_c
      std::vector<double> w(m, 0.0);
      for (int i = 0; i < m; ++i) {
        double v = i == c ? 1.0 : 0.0;
        for (int k = 0; k < i; ++k) v -= L[i * W + k] * w[k];
        w[i] = v / L[i * W + i];
      }
      for (int i = m - 1; i >= 0; --i) {
        double v = w[i];
        for (int k = i + 1; k < m; ++k) v -= L[k * W + i] * inv[c * W + k];
        inv[c * W + i] = v / L[i * W + i];
      }
    }
    float* bo = &H.binv[(size_t)b * W * W];
    for (int i = 0; i < m; ++i)      // symmetric by construction: store the mean of (i,j), (j,i)
      for (int j = 0; j < m; ++j) bo[j * W + i] = (float)(0.5 * (inv[j * W + i] + inv[i * W + j]));
  }
  // coarse operator: sum of the fracture matrix over pairs of blocks
  for (int l = 0; l < nf; ++l) {
    const int bl = H.blk[l];
    H.Ac[(size_t)bl * nb + bl] += diag[l];
    for (int j = g.rowptr[l]; j < g.rowptr[l + 1]; ++j)
      H.Ac[(size_t)H.blk[g.col[j]] * nb + bl] -= val[j];
  }
  H.xtile.resize(ntiles + 1);
  for (int t = 0; t <= ntiles; ++t) H.xtile[t] = (int)((long)t * nb / ntiles);
  return H;
}

std::vector<int> xcd_order(int n, int nxcd) {
  if (nxcd <= 1 || n < 2 * nxcd) {
    std::vector<int> o(n);
    std::iota(o.begin(), o.end(), 0);
    return o;
  }
  const int per = (n + nxcd - 1) / nxcd;
  std::vector<int> o((size_t)per * nxcd, -1);
  for (int b = 0; b < per * nxcd; ++b) {
    const int j = b % nxcd, k = b / nxcd;
    const int idx = j * per + k;
    o[b] = idx < n ? idx : -1;
  }
  return o;
}

}  // namespace mc
