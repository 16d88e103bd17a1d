// CPU self-test of the NLMC host bookkeeping (coarse units, oversampled regions, their banded
// local orderings, unit pairs).  Built and run by tests/test_nlmc_plan.py with g++; every
// property is checked against a brute-force recount from the inputs.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <stdexcept>
#include <vector>

#include "../paper_2209_01158_amd/csrc/nlmc_host.hpp"

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);          \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

// a random fracture network on an nx x ny grid: chains of cells whose hosts step by at most
// one cell, plus a few crossings between cells sharing a host
struct Net {
  std::vector<int> host, rowptr, col;
};

static Net random_net(int nx, int ny, int nchains, std::mt19937& rng) {
  Net N;
  std::vector<std::pair<int, int>> edges;
  for (int c = 0; c < nchains; ++c) {
    int x = rng() % nx, y = rng() % ny;
    const int len = 2 + rng() % 12;
    const int first = (int)N.host.size();
    for (int k = 0; k < len; ++k) {
      N.host.push_back(y * nx + x);
      if (k > 0) edges.push_back({first + k - 1, first + k});
      x = std::min(nx - 1, std::max(0, x + (int)(rng() % 3) - 1));
      y = std::min(ny - 1, std::max(0, y + (int)(rng() % 3) - 1));
    }
  }
  const int nf = (int)N.host.size();
  for (int a = 0; a < nf; ++a)
    for (int b = a + 1; b < nf; ++b)
      if (N.host[a] == N.host[b] && rng() % 2) edges.push_back({a, b});
  std::vector<std::vector<int>> adj(nf);
  for (auto& e : edges) {
    adj[e.first].push_back(e.second);
    adj[e.second].push_back(e.first);
  }
  N.rowptr.push_back(0);
  for (int l = 0; l < nf; ++l) {
    std::sort(adj[l].begin(), adj[l].end());
    adj[l].erase(std::unique(adj[l].begin(), adj[l].end()), adj[l].end());
    for (int v : adj[l]) N.col.push_back(v);
    N.rowptr.push_back((int)N.col.size());
  }
  return N;
}

static void check_plan(int nx, int ny, int no, int bx, int by, int layers, const Net& N) {
  const int nf = (int)N.host.size();
  const mc::NlPlan P = mc::build_nl_plan(nx, ny, no, nf, N.host.data(), N.rowptr.data(),
                                         N.col.data(), bx, by, layers);
  const long ncell = (long)nx * ny;
  const int ncx = nx / bx, ncy = ny / by, nco = ncx * ncy;
  auto coarse_of = [&](long g) { return (int)((g / nx) / by) * ncx + (int)((g % nx) / bx); };
  // units: every fine unknown in exactly one unit; grid units are whole coarse cells
  std::vector<int> owner(no * ncell + nf, -1);
  for (int u = 0; u < P.nunits; ++u)
    for (int k = P.uptr[u]; k < P.uptr[u + 1]; ++k) {
      const int G = P.ucell[k];
      CHECK(owner[G] == -1);
      owner[G] = u;
      const int a = G < no * ncell ? (int)(G / ncell) : no;
      CHECK(P.ucont[u] == a);
      const long g = a < no ? G % ncell : N.host[G - no * ncell];
      CHECK(coarse_of(g) == P.ucoarse[u]);
    }
  for (int G : owner) CHECK(G >= 0);
  // regions: box = K_i grown by `layers` coarse cells (clipped); rows are the box's
  // unknowns; the band width is the largest row distance of a coupling inside the box
  CHECK((int)P.reg.size() == nco);
  for (int i = 0; i < nco; ++i) {
    const mc::NlRegion& R = P.reg[i];
    const int cx = i % ncx, cy = i / ncx;
    const int x0 = std::max(0, cx - layers) * bx, y0 = std::max(0, cy - layers) * by;
    const int x1 = std::min(ncx, cx + layers + 1) * bx, y1 = std::min(ncy, cy + layers + 1) * by;
    CHECK(R.box.x0 == x0 && R.box.y0 == y0 && R.box.W == x1 - x0 && R.box.H == y1 - y0);
    std::vector<int> loc(no * ncell + nf, -1);
    for (int r = 0; r < R.n; ++r) {
      const int G = P.row_g[R.row_off + r];
      CHECK(loc[G] == -1);
      loc[G] = r;
      // the row's unit is the region unit list entry it names
      CHECK(P.reg_units[R.unit_off + P.row_unit[R.row_off + r]] == owner[G]);
    }
    int nin = 0;   // unknowns whose cell (host) lies in the box
    for (long G = 0; G < no * ncell + nf; ++G) {
      const long g = G < no * ncell ? G % ncell : N.host[G - no * ncell];
      const int x = (int)(g % nx), y = (int)(g / nx);
      const bool in = x >= x0 && x < x1 && y >= y0 && y < y1;
      CHECK(in == (loc[G] >= 0));
      nin += in;
    }
    CHECK(nin == R.n);
    int w = 0;
    auto couple = [&](long Ga, long Gb) {
      if (loc[Ga] >= 0 && loc[Gb] >= 0) w = std::max(w, std::abs(loc[Ga] - loc[Gb]));
    };
    for (int a = 0; a < no; ++a)
      for (long g = 0; g < ncell; ++g) {
        if ((g % nx) + 1 < nx) couple(a * ncell + g, a * ncell + g + 1);
        if ((g / nx) + 1 < ny) couple(a * ncell + g, a * ncell + g + nx);
        if (a == 1) couple(g, ncell + g);
      }
    for (int l = 0; l < nf; ++l) {
      for (int a = 0; a < no; ++a) couple(no * ncell + l, a * ncell + N.host[l]);
      for (int k = N.rowptr[l]; k < N.rowptr[l + 1]; ++k)
        couple(no * ncell + l, no * ncell + N.col[k]);
    }
    CHECK(R.w == w);
    // the region's units: those of the coarse cells in K_i^+, ascending
    std::vector<int> us(P.reg_units.begin() + R.unit_off, P.reg_units.begin() + R.unit_off + R.m);
    CHECK(std::is_sorted(us.begin(), us.end()));
    std::set<int> want;
    for (int G = 0; G < (int)owner.size(); ++G)
      if (loc[G] >= 0) want.insert(owner[G]);
    CHECK(std::set<int>(us.begin(), us.end()) == want);
    for (int c = 0; c < R.ncenter; ++c) {
      CHECK(P.ucoarse[R.center_unit[c]] == i);
      CHECK(us[R.center_local[c]] == R.center_unit[c]);
      CHECK(P.unit_region[R.center_unit[c]] == i);
    }
  }
  // pairs: v listed for u exactly when v's box meets u's box grown by one cell
  for (int u = 0; u < P.nunits; ++u) {
    const mc::NlBox& E = P.reg[P.unit_region[u]].ext;
    std::set<int> got(P.pair_v.begin() + P.pair_ptr[u], P.pair_v.begin() + P.pair_ptr[u + 1]);
    CHECK((int)got.size() == P.pair_ptr[u + 1] - P.pair_ptr[u]);
    for (int v = 0; v < P.nunits; ++v) {
      const mc::NlBox& B = P.reg[P.unit_region[v]].box;
      const bool meet = B.x0 < E.x0 + E.W && E.x0 < B.x0 + B.W && B.y0 < E.y0 + E.H &&
                        E.y0 < B.y0 + B.H;
      CHECK((meet && v != u) == (got.count(v) == 1));
    }
  }
}

int main() {
  std::mt19937 rng(7);
  const int shapes[][6] = {{12, 12, 1, 3, 3, 1}, {12, 8, 2, 4, 2, 1}, {16, 16, 1, 4, 4, 2},
                           {10, 15, 2, 5, 3, 3}, {9, 9, 1, 1, 1, 1}, {8, 6, 2, 8, 6, 2}};
  for (auto& s : shapes)
    for (int rep = 0; rep < 3; ++rep) {
      Net N = random_net(s[0], s[1], 1 + rng() % 6, rng);
      check_plan(s[0], s[1], s[2], s[3], s[4], s[5], N);
    }
  Net none;
  none.rowptr.push_back(0);
  check_plan(12, 12, 2, 4, 4, 1, none);   // no fracture continuum
  // refusals: coarse cells that do not tile the grid; connections across non-neighbour hosts
  bool threw = false;
  try {
    mc::build_nl_plan(10, 10, 1, 0, nullptr, none.rowptr.data(), nullptr, 3, 5, 1);
  } catch (const std::exception&) {
    threw = true;
  }
  CHECK(threw);
  Net far;
  far.host = {0, 5};
  far.rowptr = {0, 1, 2};
  far.col = {1, 0};
  threw = false;
  try {
    mc::build_nl_plan(10, 10, 1, 2, far.host.data(), far.rowptr.data(), far.col.data(), 5, 5, 1);
  } catch (const std::exception&) {
    threw = true;
  }
  CHECK(threw);
  std::printf(failures ? "FAILED %d\n" : "OK\n", failures);
  return failures ? 1 : 0;
}
