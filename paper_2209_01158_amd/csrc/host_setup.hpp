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

// For every fracture cell l that is not the first of its chain, the CSR entry of its
// connection to l-1; -1 for chain starts.
std::vector<int> chain_prev_entry(int nf, const GraphCSR& g, const std::vector<int>& chain_ptr);

// Launch order of `n` work items such that hardware round-robin dispatch over `nxcd`
// compute dies gives die j a contiguous range of items.  Entries of -1 are padding.
std::vector<int> xcd_order(int n, int nxcd);

}  // namespace mc
