// Host-side bookkeeping of the coarse-grid (NLMC) builder; see nlmc_host.hpp.
#include "nlmc_host.hpp"

#include <algorithm>
#include <stdexcept>

namespace mc {

namespace {

// hosted[g]: fracture cells hosted by grid cell g (ascending l); built once
struct Hosted {
  std::vector<int> ptr, idx;
};

Hosted hosted_cells(long ncell, int nf, const int* host) {
  Hosted h;
  h.ptr.assign(ncell + 1, 0);
  for (int l = 0; l < nf; ++l) h.ptr[host[l] + 1]++;
  for (long g = 0; g < ncell; ++g) h.ptr[g + 1] += h.ptr[g];
  h.idx.resize(nf);
  std::vector<int> fill(h.ptr.begin(), h.ptr.end() - 1);
  for (int l = 0; l < nf; ++l) h.idx[fill[host[l]]++] = l;   // ascending l within a host
  return h;
}

NlBox make_box(int x0, int y0, int x1, int y1, int nx, int n_omega, const Hosted& hc) {
  NlBox b;
  b.x0 = x0;
  b.y0 = y0;
  b.W = x1 - x0;
  b.H = y1 - y0;
  b.start.resize((size_t)b.W * b.H + 1);
  int r = 0;
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x) {
      const long g = (long)y * nx + x;
      b.start[(size_t)(y - y0) * b.W + (x - x0)] = r;
      r += n_omega + (hc.ptr[g + 1] - hc.ptr[g]);
    }
  b.start[(size_t)b.W * b.H] = r;
  return b;
}

}  // namespace

NlPlan build_nl_plan(int nx, int ny, int n_omega, int nf, const int* host, const int* rowptr,
                     const int* col, int bx, int by, int layers) {
  if (nx < 1 || ny < 1 || n_omega < 1 || n_omega > 2 || nf < 0)
    throw std::runtime_error("bad grid shape or continuum count");
  if (bx < 1 || by < 1 || nx % bx != 0 || ny % by != 0)
    throw std::runtime_error("coarse cells of bx x by fine cells must tile the grid exactly");
  if (layers < 0) throw std::runtime_error("oversampling layers must be >= 0");
  NlPlan P;
  P.nx = nx;
  P.ny = ny;
  P.n_omega = n_omega;
  P.nf = nf;
  P.bx = bx;
  P.by = by;
  P.layers = layers;
  P.ncx = nx / bx;
  P.ncy = ny / by;
  P.ncell = (long)nx * ny;
  const long ncell = P.ncell;
  const int nco = P.ncx * P.ncy;
  for (int l = 0; l < nf; ++l)
    if (host[l] < 0 || host[l] >= ncell) throw std::runtime_error("fracture host out of range");
  // fracture neighbours must be hosted at most one cell apart (the one-cell ring around a
  // region then holds every row where A psi can be non-zero)
  for (int l = 0; l < nf; ++l)
    for (int k = rowptr[l]; k < rowptr[l + 1]; ++k) {
      const int a = host[l], b = host[col[k]];
      if (std::abs(a % nx - b % nx) > 1 || std::abs(a / nx - b / nx) > 1)
        throw std::runtime_error("fracture cells " + std::to_string(l) + " and " +
                                 std::to_string(col[k]) +
                                 " are joined across more than one grid cell; the coarse-grid "
                                 "path needs neighbouring hosts");
    }
  const Hosted hc = hosted_cells(ncell, nf, host);
  P.rank.assign(nf, 0);
  for (long g = 0; g < ncell; ++g)
    for (int k = hc.ptr[g]; k < hc.ptr[g + 1]; ++k) P.rank[hc.idx[k]] = k - hc.ptr[g];
  auto coarse_of = [&](long g) { return (int)((g / nx) / by) * P.ncx + (int)((g % nx) / bx); };
  // units
  P.uptr.push_back(0);
  for (int a = 0; a < n_omega; ++a) {
    for (int j = 0; j < nco; ++j) {
      P.ucont.push_back(a);
      P.ucoarse.push_back(j);
      const int cy = j / P.ncx, cx = j % P.ncx;
      for (int y = cy * by; y < (cy + 1) * by; ++y)
        for (int x = cx * bx; x < (cx + 1) * bx; ++x)
          P.ucell.push_back((int)(a * ncell + (long)y * nx + x));
      P.uptr.push_back((int)P.ucell.size());
    }
    P.usize.push_back(nco);
  }
  P.frac_unit.assign(nco, -1);
  if (nf > 0) {
    std::vector<std::vector<int>> fl(nco);
    for (int l = 0; l < nf; ++l) fl[coarse_of(host[l])].push_back(l);
    int k = 0;
    for (int j = 0; j < nco; ++j) {
      if (fl[j].empty()) continue;
      P.frac_unit[j] = (int)P.ucont.size();
      P.ucont.push_back(n_omega);
      P.ucoarse.push_back(j);
      for (int l : fl[j]) P.ucell.push_back((int)(n_omega * ncell + l));
      P.uptr.push_back((int)P.ucell.size());
      ++k;
    }
    P.usize.push_back(k);
  }
  P.nunits = (int)P.ucont.size();
  auto unit_of = [&](int a, int j) { return a < n_omega ? a * nco + j : P.frac_unit[j]; };
  // regions
  P.unit_region.assign(P.nunits, -1);
  P.unit_center.assign(P.nunits, -1);
  P.reg.resize(nco);
  for (int i = 0; i < nco; ++i) {
    NlRegion& R = P.reg[i];
    R.ci = i;
    const int cy = i / P.ncx, cx = i % P.ncx;
    const int cx0 = std::max(0, cx - layers), cx1 = std::min(P.ncx, cx + layers + 1);
    const int cy0 = std::max(0, cy - layers), cy1 = std::min(P.ncy, cy + layers + 1);
    const int x0 = cx0 * bx, x1 = cx1 * bx, y0 = cy0 * by, y1 = cy1 * by;
    R.box = make_box(x0, y0, x1, y1, nx, n_omega, hc);
    R.ext = make_box(std::max(0, x0 - 1), std::max(0, y0 - 1), std::min(nx, x1 + 1),
                     std::min(ny, y1 + 1), nx, n_omega, hc);
    R.n = R.box.start.back();
    // units of K_i^+, ascending
    std::vector<int> us;
    for (int a = 0; a <= n_omega; ++a)
      for (int yy = cy0; yy < cy1; ++yy)
        for (int xx = cx0; xx < cx1; ++xx) {
          const int j = yy * P.ncx + xx;
          if (a == n_omega && (nf == 0 || P.frac_unit[j] < 0)) continue;
          us.push_back(unit_of(a, j));
        }
    std::sort(us.begin(), us.end());
    R.m = (int)us.size();
    auto local = [&](int u) {
      return (int)(std::lower_bound(us.begin(), us.end(), u) - us.begin());
    };
    for (int a = 0; a <= n_omega; ++a) {
      if (a == n_omega && (nf == 0 || P.frac_unit[i] < 0)) continue;
      const int u = unit_of(a, i);
      R.center_unit[R.ncenter] = u;
      R.center_local[R.ncenter] = local(u);
      P.unit_region[u] = i;
      P.unit_center[u] = R.ncenter;
      ++R.ncenter;
    }
    // rows and band width
    R.start_off = (long)P.starts.size();
    P.starts.insert(P.starts.end(), R.box.start.begin(), R.box.start.end());
    R.ext_off = (long)P.starts.size();
    P.starts.insert(P.starts.end(), R.ext.start.begin(), R.ext.start.end());
    R.row_off = P.rows;
    R.unit_off = (long)P.reg_units.size();
    P.reg_units.insert(P.reg_units.end(), us.begin(), us.end());
    const int W = R.box.W;
    int w = 0;
    for (int y = y0; y < y1; ++y)
      for (int x = x0; x < x1; ++x) {
        const long g = (long)y * nx + x;
        const int c = (y - y0) * W + (x - x0);
        const int s0 = R.box.start[c];
        const int j = coarse_of(g);
        for (int a = 0; a < n_omega; ++a) {
          P.row_g.push_back((int)(a * ncell + g));
          P.row_unit.push_back(local(unit_of(a, j)));
          const int r = s0 + a;
          if (x > x0) w = std::max(w, r - (R.box.start[c - 1] + a));
          if (y > y0) w = std::max(w, r - (R.box.start[c - W] + a));
          if (a > 0) w = std::max(w, a);
        }
        for (int k = hc.ptr[g]; k < hc.ptr[g + 1]; ++k) {
          const int l = hc.idx[k];
          P.row_g.push_back((int)(n_omega * ncell + l));
          P.row_unit.push_back(local(P.frac_unit[j]));
          const int r = s0 + n_omega + (k - hc.ptr[g]);
          w = std::max(w, r - s0);   // its host's grid unknowns
          for (int e = rowptr[l]; e < rowptr[l + 1]; ++e) {
            const int l2 = col[e];
            const long g2 = host[l2];
            const int x2 = (int)(g2 % nx), y2 = (int)(g2 / nx);
            if (x2 < x0 || x2 >= x1 || y2 < y0 || y2 >= y1) continue;
            const int r2 = R.box.start[(y2 - y0) * W + (x2 - x0)] + n_omega + P.rank[l2];
            if (r2 < r) w = std::max(w, r - r2);
          }
        }
      }
    R.w = w;
    P.rows += R.n;
    R.band_off = P.band;
    P.band += (long)R.n * (w + 1);
    R.z_off = P.zsize;
    P.zsize += (long)R.n * R.m;
    R.s_off = P.ssize;
    P.ssize += (long)R.m * R.m;
    P.max_w = std::max(P.max_w, w);
    P.max_m = std::max(P.max_m, R.m);
    P.max_n = std::max(P.max_n, R.n);
  }
  // basis functions (box ordering of their region) and A psi (ext ordering)
  P.psi_off.assign(P.nunits, 0);
  P.t_off.assign(P.nunits, 0);
  for (int u = 0; u < P.nunits; ++u) {
    const NlRegion& R = P.reg[P.unit_region[u]];
    P.psi_off[u] = P.psi_size;
    P.psi_size += R.n;
    P.t_off[u] = P.t_size;
    P.t_size += R.ext.start.back();
  }
  // pairs: v whose region box meets the extended box of u's region
  P.pair_ptr.push_back(0);
  for (int u = 0; u < P.nunits; ++u) {
    const NlRegion& R = P.reg[P.unit_region[u]];
    const NlBox& E = R.ext;
    const int cy = R.ci / P.ncx, cx = R.ci % P.ncx;
    const int span = 2 * layers + 1;
    for (int yy = std::max(0, cy - span); yy <= std::min(P.ncy - 1, cy + span); ++yy)
      for (int xx = std::max(0, cx - span); xx <= std::min(P.ncx - 1, cx + span); ++xx) {
        const int j = yy * P.ncx + xx;
        const NlBox& B = P.reg[j].box;
        if (B.x0 >= E.x0 + E.W || E.x0 >= B.x0 + B.W || B.y0 >= E.y0 + E.H ||
            E.y0 >= B.y0 + B.H)
          continue;
        for (int a = 0; a <= n_omega; ++a) {
          if (a == n_omega && (nf == 0 || P.frac_unit[j] < 0)) continue;
          const int v = unit_of(a, j);
          if (v != u) P.pair_v.push_back(v);
        }
      }
    P.pair_ptr.push_back((int)P.pair_v.size());
  }
  return P;
}

}  // namespace mc
