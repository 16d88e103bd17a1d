// CPU self-test of the host construction of the exact fracture solve (build_schur): on random
// fracture graphs (chains of consecutive cells plus crossing connections) the solve
//   y = A_II^-1 r_I,  g = r_X - A_XI y,  z_X = S^-1 g,  z_l = y_l + cl_l z_X[xl_l] + cr_l z_X[xr_l]
// must equal the dense Gaussian-elimination solution of A z = r, and (r, z) must equal
// (r_I, y_I) + g . z_X.  Built and run by tests/test_schur_host.py.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_2209_01158_amd/csrc/host_setup.hpp"

static int failures = 0;
#define CHECK(c, ...)                                                      \
  do {                                                                     \
    if (!(c)) {                                                            \
      std::printf("FAIL %s:%d: %s ", __FILE__, __LINE__, #c);              \
      std::printf(__VA_ARGS__);                                            \
      std::printf("\n");                                                   \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

// dense solve with partial pivoting (row-major n x n), in place on a copy
static std::vector<double> dense_solve(std::vector<double> M, std::vector<double> b, int n) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(M[(size_t)i * n + k]) > std::fabs(M[(size_t)p * n + k])) p = i;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(M[(size_t)k * n + j], M[(size_t)p * n + j]);
      std::swap(b[k], b[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = M[(size_t)i * n + k] / M[(size_t)k * n + k];
      if (f == 0.0) continue;
      for (int j = k; j < n; ++j) M[(size_t)i * n + j] -= f * M[(size_t)k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= M[(size_t)k * n + j] * b[j];
    b[k] = s / M[(size_t)k * n + k];
  }
  return b;
}

static void one_case(unsigned seed, int kmax) {
  std::mt19937_64 rng(seed);
  std::uniform_int_distribution<int> nchain(1, 12), clen(1, 15);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  // cells of random chains, consecutive cells linked
  std::vector<int> edges;
  int nf = 0;
  const int nc = nchain(rng);
  for (int c = 0; c < nc; ++c) {
    const int L = clen(rng);
    for (int j = 0; j + 1 < L; ++j) edges.insert(edges.end(), {nf + j, nf + j + 1});
    nf += L;
  }
  // crossing connections between non-consecutive cells (some parallel to others)
  const int nx = (int)(U(rng) * 2 * nf / 3);
  for (int e = 0; e < nx; ++e) {
    int a = (int)(U(rng) * nf), b = (int)(U(rng) * nf);
    if (a == b || a - b == 1 || b - a == 1) continue;
    edges.insert(edges.end(), {a, b});
  }
  const int ne = (int)edges.size() / 2;
  mc::GraphCSR g = mc::build_graph(nf, ne, edges.data());
  std::vector<int> chains = mc::build_chains(nf, g);
  std::vector<int> tiles = mc::build_graph_tiles(chains, 7);
  // conductances (wide range, as in a fracture network) and an SPD diagonal
  std::vector<double> T(ne), val(2 * ne), diag(nf);
  for (int e = 0; e < ne; ++e) T[e] = std::exp(std::log(1e-3) + U(rng) * std::log(1e6));
  for (size_t j = 0; j < g.col.size(); ++j) val[j] = T[g.eidx[j]];
  std::vector<double> A((size_t)nf * nf, 0.0);
  for (int l = 0; l < nf; ++l) {
    double s = 1e-4 + U(rng) * 1e-2;   // storage over tau plus transfer
    for (int j = g.rowptr[l]; j < g.rowptr[l + 1]; ++j) {
      s += val[j];
      A[(size_t)l * nf + g.col[j]] -= val[j];
    }
    diag[l] = s;
    A[(size_t)l * nf + l] = s;
  }
  mc::SchurHost H = mc::build_schur(nf, g, chains, tiles, diag.data(), val.data(), kmax);
  CHECK((int)H.xcells.size() == H.K, "seed %u", seed);
  CHECK((int)H.xtile.size() == (int)tiles.size(), "seed %u", seed);
  // S symmetric
  for (int i = 0; i < H.K; ++i)
    for (int j = 0; j < H.K; ++j)
      CHECK(std::fabs(H.S[(size_t)j * H.K + i] - H.S[(size_t)i * H.K + j]) <=
                1e-12 * std::fabs(H.S[(size_t)i * H.K + i]),
            "seed %u S not symmetric", seed);
  std::vector<double> r(nf);
  for (auto& x : r) x = U(rng) - 0.5;
  // y = A_II^-1 r by the block factor (the recurrences the device chain solve runs)
  std::vector<double> y(nf, 0.0), w(nf, 0.0);
  for (size_t c = 0; c + 1 < chains.size(); ++c) {
    const int c0 = chains[c], c1 = chains[c + 1];
    double u = 0.0;
    for (int l = c0; l < c1; ++l) {
      u = (r[l] + (l > c0 ? H.cT[l] * u : 0.0)) * H.dinv[l];
      w[l] = u;
    }
    double z = 0.0;
    for (int l = c1 - 1; l >= c0; --l) {
      z = w[l] + (l + 1 < c1 ? H.cT[l + 1] * H.dinv[l] * z : 0.0);
      y[l] = z;
    }
  }
  std::vector<double> gx(H.K), Sd((size_t)H.K * H.K);
  for (int k = 0; k < H.K; ++k) {
    const int x = H.xcells[k];
    CHECK(y[x] == 0.0, "seed %u y at crossing cell", seed);
    gx[k] = r[x] + H.cxl[k] * (x > 0 ? y[x - 1] : 0.0) + H.cxr[k] * (x + 1 < nf ? y[x + 1] : 0.0);
  }
  for (int i = 0; i < H.K; ++i)
    for (int j = 0; j < H.K; ++j) Sd[(size_t)i * H.K + j] = H.S[(size_t)j * H.K + i];
  std::vector<double> zX = H.K ? dense_solve(Sd, gx, H.K) : std::vector<double>();
  std::vector<double> z(nf);
  for (int l = 0; l < nf; ++l)
    z[l] = y[l] + (H.xl[l] >= 0 ? H.cl[l] * zX[H.xl[l]] : 0.0) +
           (H.xr[l] >= 0 ? H.cr[l] * zX[H.xr[l]] : 0.0);
  if (H.K == H.K_all) {   // exact
    std::vector<double> ref = dense_solve(A, r, nf);
    double num = 0, den = 0;
    for (int l = 0; l < nf; ++l) {
      num += (z[l] - ref[l]) * (z[l] - ref[l]);
      den += ref[l] * ref[l];
    }
    CHECK(std::sqrt(num / den) < 1e-9, "seed %u nf %d K %d err %.3e", seed, nf, H.K,
          std::sqrt(num / den));
    double rz = 0, ry = 0, gz = 0;
    for (int l = 0; l < nf; ++l) {
      rz += r[l] * z[l];
      ry += r[l] * y[l];
    }
    for (int k = 0; k < H.K; ++k) gz += gx[k] * zX[k];
    CHECK(std::fabs(rz - (ry + gz)) <= 1e-9 * std::fabs(rz), "seed %u (r,z) identity", seed);
  } else {                // too many crossing cells: whole chains, crossings left out
    CHECK(H.K == 0, "seed %u", seed);
    for (int l = 0; l < nf; ++l) CHECK(H.xl[l] < 0 && H.xr[l] < 0, "seed %u", seed);
  }
}

int main() {
  for (unsigned s = 1; s <= 300; ++s) one_case(s, 1 << 20);
  for (unsigned s = 1; s <= 50; ++s) one_case(s, 2);   // fallback when K exceeds kmax
  if (failures) {
    std::printf("%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
