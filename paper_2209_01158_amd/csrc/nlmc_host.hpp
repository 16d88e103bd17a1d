// Host-side integer bookkeeping of the coarse-grid (NLMC) builder: coarse units, the
// oversampled regions K_i^+ with their local orderings and band widths, and the pairs of
// units whose basis functions overlap.  Plain C++ (no HIP, no floating-point arithmetic of
// the method).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace mc {

// Local ordering of a rectangle of grid cells (row-major): every cell contributes its
// n_omega grid unknowns, then the fracture cells it hosts (ascending).  start[c] is the
// first local row of box cell c, start[W*H] the number of rows.
struct NlBox {
  int x0 = 0, y0 = 0, W = 0, H = 0;
  std::vector<int> start;
};

struct NlRegion {
  int ci = 0;          // coarse cell the region is centred on
  NlBox box;           // K_i^+ as fine cells
  NlBox ext;           // the box grown by one cell on each side (clipped to the grid)
  int n = 0;           // local unknowns (rows of box)
  int w = 0;           // lower band width of the local operator in this ordering
  int m = 0;           // units inside K_i^+ (its constraints)
  int ncenter = 0;     // units centred on ci (their basis functions are built here)
  int center_local[3] = {0, 0, 0};   // their indices in the region's unit list
  int center_unit[3] = {0, 0, 0};    // their global unit ids
  // offsets into the concatenated device arrays
  long start_off = 0, ext_off = 0;   // start tables
  long row_off = 0;                  // per-row arrays (n)
  long unit_off = 0;                 // region unit list (m)
  long band_off = 0;                 // band (n * (w + 1))
  long z_off = 0;                      // L^-1 C^T (n * m, row-major)
  long s_off = 0;                      // S = C A^-1 C^T (m * m)
};

struct NlPlan {
  int nx = 0, ny = 0, n_omega = 0, nf = 0, bx = 0, by = 0, layers = 0;
  int ncx = 0, ncy = 0;
  long ncell = 0;
  // coarse units: continuum by continuum, coarse cells row-major; fracture units only where
  // a coarse cell hosts fracture cells
  int nunits = 0;
  std::vector<int> ucont, ucoarse;   // [nunits]
  std::vector<int> usize;            // [n_omega + 1] units per continuum (fracture last)
  std::vector<int> uptr, ucell;      // CSR: concatenated fine indices of every unit's cells
  std::vector<int> frac_unit;        // [ncx*ncy] fracture unit of a coarse cell or -1
  std::vector<int> rank;             // [nf] position of a fracture cell among its host's
  std::vector<NlRegion> reg;         // one per coarse cell
  std::vector<int> unit_region;      // [nunits] region building the unit's basis function
  std::vector<int> unit_center;      // [nunits] its index among that region's centre units
  // concatenated per-region arrays
  std::vector<int> starts;           // box and ext start tables
  std::vector<int> row_g;            // per row: concatenated fine index of the unknown
  std::vector<int> row_unit;         // per row: index of its unit in the region's unit list
  std::vector<int> reg_units;        // per region: global unit ids (ascending)
  long rows = 0, band = 0, zsize = 0, ssize = 0;
  long psi_size = 0, t_size = 0;     // basis functions (box ordering) and A psi (ext ordering)
  std::vector<long> psi_off, t_off;  // [nunits]
  // unit pairs (u, v) with supp psi_v meeting the extended box of u, grouped by u
  std::vector<int> pair_ptr, pair_v; // CSR over u
  int max_w = 0, max_m = 0, max_n = 0;
};

// Builds the plan; throws std::runtime_error with a message on inputs it cannot serve.
// host: [nf] host cell per fracture cell; rowptr/col: fracture CSR (both host copies).
NlPlan build_nl_plan(int nx, int ny, int n_omega, int nf, const int* host, const int* rowptr,
                     const int* col, int bx, int by, int layers);

}  // namespace mc
