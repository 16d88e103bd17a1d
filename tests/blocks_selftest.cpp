// CPU self-test of the host construction of the two-level block preconditioner of a fracture
// graph (build_blocks / build_block_solve).  On random fracture graphs (chains with crossing
// connections, and rectangular planes of cells joined where planes meet):
//   - every cell is in exactly one block of at most 64 cells, listed first in its block's row
//     of the cell table (padding -1 after), and every block is connected;
//   - blocks are grown breadth-first until full: a block of fewer than 64 cells has no
//     neighbour in a later block (any such neighbour was still unassigned when it grew);
//   - the stored block inverse times the block's matrix is the identity (FP32 rounding);
//   - the coarse operator equals P^T A P formed densely;
//   - work tiles split the blocks in order, and more blocks than nbmax gives nb = 0.
// Built and run by tests/test_schur_host.py.
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

static void check_graph(unsigned seed, int nf, const std::vector<int>& edges, std::mt19937_64& rng) {
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const int ne = (int)edges.size() / 2;
  const mc::GraphCSR g = mc::build_graph(nf, ne, edges.data());
  std::vector<double> T(ne), val(g.col.size()), diag(nf);
  for (int e = 0; e < ne; ++e) T[e] = std::exp(std::log(1e-3) + U(rng) * std::log(1e4));
  for (size_t j = 0; j < g.col.size(); ++j) val[j] = T[g.eidx[j]];
  std::vector<double> A((size_t)nf * nf, 0.0);   // row-major
  for (int l = 0; l < nf; ++l) {
    double s = 1e-6 + U(rng) * 1e-5;
    for (int j = g.rowptr[l]; j < g.rowptr[l + 1]; ++j) {
      s += val[j];
      A[(size_t)l * nf + g.col[j]] -= val[j];
    }
    diag[l] = s;
    A[(size_t)l * nf + l] = s;
  }
  const int ntiles = 1 + (int)(U(rng) * 9);
  const mc::BlockHost H = mc::build_block_solve(nf, g, ntiles, diag.data(), val.data(), 1 << 20);
  const int nb = H.nb, W = mc::kBlockCells;
  CHECK(H.ok, "seed %u", seed);
  CHECK(nb > 0 && (int)H.node.size() == nb * W && (int)H.blk.size() == nf, "seed %u", seed);
  // cells once, listed first, blk consistent
  std::vector<int> seen(nf, 0), size(nb, 0);
  for (int b = 0; b < nb; ++b) {
    bool pad = false;
    for (int i = 0; i < W; ++i) {
      const int l = H.node[(size_t)b * W + i];
      if (l < 0) {
        pad = true;
        continue;
      }
      CHECK(!pad, "seed %u block %d: a cell after padding", seed, b);
      CHECK(l < nf && H.blk[l] == b, "seed %u block %d cell %d", seed, b, l);
      seen[l]++;
      size[b]++;
    }
    CHECK(size[b] >= 1, "seed %u empty block %d", seed, b);
  }
  for (int l = 0; l < nf; ++l) CHECK(seen[l] == 1, "seed %u cell %d in %d blocks", seed, l, seen[l]);
  // connected blocks; a block that is not full has no neighbour in a later block
  for (int b = 0; b < nb; ++b) {
    const int* nd = &H.node[(size_t)b * W];
    std::vector<int> reach(1, nd[0]);
    std::vector<char> in(nf, 0);
    in[nd[0]] = 1;
    for (size_t h = 0; h < reach.size(); ++h)
      for (int j = g.rowptr[reach[h]]; j < g.rowptr[reach[h] + 1]; ++j) {
        const int v = g.col[j];
        if (H.blk[v] == b && !in[v]) in[v] = 1, reach.push_back(v);
      }
    CHECK((int)reach.size() == size[b], "seed %u block %d not connected", seed, b);
    if (size[b] < W)
      for (int i = 0; i < size[b]; ++i)
        for (int j = g.rowptr[nd[i]]; j < g.rowptr[nd[i] + 1]; ++j)
          CHECK(H.blk[g.col[j]] <= b, "seed %u block %d (not full) touches later block %d",
                seed, b, H.blk[g.col[j]]);
  }
  // block inverse times block matrix
  for (int b = 0; b < nb; ++b) {
    const int* nd = &H.node[(size_t)b * W];
    const float* bi = &H.binv[(size_t)b * W * W];
    const int m = size[b];
    double worst = 0.0;
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < m; ++k) {
        double s = 0.0, sa = 0.0;
        for (int j = 0; j < m; ++j) {
          const double t = (double)bi[j * W + i] * A[(size_t)nd[j] * nf + nd[k]];
          s += t;
          sa += std::fabs(t);
        }
        worst = std::fmax(worst, std::fabs(s - (i == k ? 1.0 : 0.0)) / std::fmax(sa, 1.0));
      }
    CHECK(worst < 1e-5, "seed %u block %d |B^-1 B - I| %.3e", seed, b, worst);
    for (int i = m; i < W; ++i)
      for (int j = 0; j < W; ++j)
        CHECK(bi[j * W + i] == 0.0f && bi[i * W + j] == 0.0f, "seed %u padding", seed);
  }
  // coarse operator
  std::vector<double> Ac((size_t)nb * nb, 0.0), mag((size_t)nb * nb, 0.0);
  for (int l = 0; l < nf; ++l)
    for (int m = 0; m < nf; ++m) {
      Ac[(size_t)H.blk[m] * nb + H.blk[l]] += A[(size_t)l * nf + m];
      mag[(size_t)H.blk[m] * nb + H.blk[l]] += std::fabs(A[(size_t)l * nf + m]);
    }
  for (size_t k = 0; k < Ac.size(); ++k)   // rounding of sums with cancellation
    CHECK(std::fabs(Ac[k] - H.Ac[k]) <= 1e-14 * mag[k],
          "seed %u coarse entry %zu: %.6e vs %.6e", seed, k, Ac[k], H.Ac[k]);
  // tiles
  CHECK((int)H.xtile.size() == ntiles + 1 && H.xtile[0] == 0 && H.xtile[ntiles] == nb, "seed %u", seed);
  for (int t = 0; t < ntiles; ++t) CHECK(H.xtile[t] <= H.xtile[t + 1], "seed %u", seed);
  // more blocks than allowed
  const mc::BlockHost F = mc::build_block_solve(nf, g, ntiles, diag.data(), val.data(), nb - 1);
  CHECK(F.nb == 0 && F.binv.empty() && F.Ac.empty(), "seed %u nbmax", seed);
}

int main() {
  for (unsigned seed = 1; seed <= 40; ++seed) {
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::vector<int> edges;
    int nf = 0;
    if (seed % 2) {   // chains with crossing connections
      const int nc = 1 + (int)(U(rng) * 10);
      for (int c = 0; c < nc; ++c) {
        const int L = 1 + (int)(U(rng) * 90);
        for (int j = 0; j + 1 < L; ++j) edges.insert(edges.end(), {nf + j, nf + j + 1});
        nf += L;
      }
      const int nx = (int)(U(rng) * nf / 2);
      for (int e = 0; e < nx; ++e) {
        const int a = (int)(U(rng) * nf), b = (int)(U(rng) * nf);
        if (a != b) edges.insert(edges.end(), {a, b});
      }
    } else {          // rectangular planes numbered row by row, joined at random cells
      const int np = 1 + (int)(U(rng) * 4);
      std::vector<int> start;
      for (int p = 0; p < np; ++p) {
        const int rows = 1 + (int)(U(rng) * 20), cols = 1 + (int)(U(rng) * 20);
        start.push_back(nf);
        for (int i = 0; i < rows; ++i)
          for (int j = 0; j < cols; ++j) {
            const int c = nf + i * cols + j;
            if (j + 1 < cols) edges.insert(edges.end(), {c, c + 1});
            if (i + 1 < rows) edges.insert(edges.end(), {c, c + cols});
          }
        nf += rows * cols;
      }
      for (int p = 1; p < np; ++p)
        for (int k = 0; k < 5; ++k) {
          const int a = start[p - 1] + (int)(U(rng) * (start[p] - start[p - 1]));
          const int b = start[p] + (int)(U(rng) * ((p + 1 < np ? start[p + 1] : nf) - start[p]));
          edges.insert(edges.end(), {a, b});
        }
    }
    check_graph(seed, nf, edges, rng);
  }
  if (failures) {
    std::printf("%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
