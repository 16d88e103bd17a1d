// Host-side integer bookkeeping of a problem: descriptor validation, the fracture graph in
// CSR form, the host-cell -> fracture-cell map, the fracture chains (blocks of the fracture
// preconditioner) and the launch tile tables.  Plain C++ (no HIP), so it also builds with g++
// for sanitizer tests.  No floating-point arithmetic of the method happens here.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mcdec.h"

namespace mc {

// Empty string if the descriptor is valid, else the first violation found.
std::string validate_desc(const mc_problem_desc& d);
std::string validate_options(const mc_options& o);

struct GraphCSR {
  std::vector<int> rowptr;  // [nf+1]
  std::vector<int> col;     // [2*ne] neighbour per entry, ascending within a row
  std::vector<int> eidx;    // [2*ne] connection index per entry
};
GraphCSR build_graph(int nf, int ne, const int32_t* edges);

struct HostMap {
  std::vector<int> hptr;  // [ncell+1]
  std::vector<int> hidx;  // [nf] fracture cells grouped by host, ascending within a host
};
HostMap build_host_map(int ncell, int nf, const int32_t* host);

// Chains: maximal runs of consecutive fracture cells l, l+1 joined by a connection.
std::vector<int> build_chains(int nf, const GraphCSR& g);

// Fracture work tiles: consecutive whole chains packed until a tile holds at least
// `target` cells.  Returns chain boundaries of the tiles, [ntiles+1].
std::vector<int> build_graph_tiles(const std::vector<int>& chain_ptr, int target);

// Exact fracture solve by a Schur complement on the crossing cells.
//
// Cells with a connection to a cell other than their chain neighbours l-1, l+1 are the
// crossing cells X (K of them); every other cell belongs to a sub-chain block I (a run of
// a chain between crossing cells), whose matrix is tridiagonal.  With
//   A = [A_II A_IX; A_XI A_XX],  S = A_XX - A_XI A_II^-1 A_IX  (K x K, SPD),
// a solve A z = r is  y = A_II^-1 r_I  (y = 0 on X),  g = r_X - A_XI y,  z_X = S^-1 g,
// z_I = y + A_II^-1 (-A_IX) z_X.  The last term is non-zero only on blocks next to a crossing
// cell: z_l = y_l + cl_l z_X[xl_l] + cr_l z_X[xr_l], with cl, cr the responses of the block to
// its left and right crossing neighbours.  Written so that a crossing cell x also fits:
// y_x = 0, xl_x = its own index, cl_x = 1.
struct SchurHost {
  int K = 0;                       // crossing cells used (0 if none or more than kmax)
  int K_all = 0;                   // crossing cells present
  std::vector<int> xcells;         // [K] ascending
  std::vector<double> dinv, cT;    // [nf] block factor: inverse pivots; coupling to l-1 (0 at block starts)
  std::vector<double> cl, cr;      // [nf] responses to the left / right crossing neighbour
  std::vector<int> xl, xr;         // [nf] their crossing indices, or -1
  std::vector<double> cxl, cxr;    // [K] conductance of crossing cell k to its chain neighbours l-1, l+1
  std::vector<int> xtile;          // [ntiles + 1] range of xcells in each fracture work tile
  std::vector<double> S;           // [K * K] Schur complement, column-major
};

// diag: [nf] full diagonal of the fracture system; val: [2*ne] conductance of every CSR entry
// of g.  Above kmax crossing cells no Schur complement is formed: the blocks are then the
// whole chains and the crossing couplings are left out (an approximate inverse).
SchurHost build_schur(int nf, const GraphCSR& g, const std::vector<int>& chain_ptr,
                      const std::vector<int>& gtile, const double* diag, const double* val,
                      int kmax);

// Number of crossing cells of a connection list (cells joined to a cell other than l-1, l+1).
int count_crossing_cells(int nf, int ne, const int32_t* edges);

// Two-level block preconditioner of a fracture graph with more crossing cells than the exact
// solve takes (fracture planes, dense networks).  The cells are grouped into connected blocks
// of at most kBlockCells = 64 cells, grown breadth-first from the lowest unassigned cell;
// with B the block diagonal of the fracture matrix A and P the block indicator (P_lb = 1 if
// cell l is in block b),
//   z = B^-1 r + P A_c^-1 P^T r,   A_c = P^T A P,
// symmetric positive definite as PCG needs.  The coarse solve A_c^-1 runs in the crossing-cell
// kernels (K = nb rows, e = A_c^-1 g with g = P^T r), and the response of cell l is e of its
// own block (xl = block, cl = 1).
constexpr int kBlockCells = 64;
struct BlockHost {
  int nb = 0;                  // blocks
  std::vector<int> node;       // [nb * 64] cells of each block, ascending BFS order; -1 padding
  std::vector<int> blk;        // [nf] block of each cell
  std::vector<float> binv;     // [nb * 64 * 64] inverse of each block's matrix (symmetric,
                               // entry (i, j) at j * 64 + i; 0 on padding rows and columns)
  std::vector<double> Ac;      // [nb * nb] coarse operator P^T A P, column-major
  std::vector<int> xtile;      // [ntiles + 1] first block of each fracture work tile
  bool ok = true;              // false if a block matrix was not positive definite
};

// Blocks only (cell lists and the block of each cell); returns the number of blocks.
int build_blocks(int nf, const GraphCSR& g, std::vector<int>& node, std::vector<int>& blk);

// diag, val as for build_schur; the blocks are spread evenly over `ntiles` work tiles.
// Returns nb = 0 (and nothing else) when more than nbmax blocks would be needed.
BlockHost build_block_solve(int nf, const GraphCSR& g, int ntiles, const double* diag,
                            const double* val, int nbmax);

// Launch order of `n` work items such that hardware round-robin dispatch over `nxcd`
// compute dies gives die j a contiguous range of items.  Entries of -1 are padding.
std::vector<int> xcd_order(int n, int nxcd);

}  // namespace mc
