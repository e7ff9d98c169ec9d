// internal.h - host-side types shared by the front-end, the packer, the
// runtime and the C ABI of the decomposer library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mpld.h"

namespace mpld {

// Error carrying an ABI code; caught at the ABI boundary.
struct Error {
  int32_t code;
  std::string what;
};
[[noreturn]] void fail(int32_t code, const std::string& what);

// Sets the thread-local detail string returned by mpld_last_error().
void set_last_error(const std::string& s);

// Layout graph in CSR form (Sec. 2.1): adjacency over conflict edges,
// ascending per node; partner[v] = stitch partner or -1.
struct Graph {
  int32_t n = 0;
  std::vector<int64_t> ptr;      // n + 1
  std::vector<int32_t> adj;      // 2 * |CE|
  std::vector<int32_t> partner;  // n
  int64_t num_ce = 0;
};

// Validates a caller's graph and builds the CSR form.  Throws MPLD_E_INVALID
// on ids out of range, self loops, duplicates, two stitch partners for one
// node or a pair that is both stitch and conflict.
Graph make_graph(const mpld_graph& g);

// Simplification and sub-graph split (Sec. 2.2 and Algorithm 1).
struct Split {
  std::vector<int32_t> removal;    // removal order (FIFO)
  std::vector<int32_t> comp_of;    // component of each node, -1 if removed
  std::vector<int32_t> order;      // core nodes, grouped by component, local order
  std::vector<int32_t> comp_ptr;   // components + 1
  std::vector<int32_t> local;      // local index of each core node, -1 if removed
};
Split simplify_and_split(const Graph& g, int32_t k, bool simplify);

// Local conflict pairs (i < j) of component c, in ascending (i, j) order.
void local_edges(const Graph& g, const Split& s, int32_t c,
                 std::vector<int32_t>& out_pairs);

// Recovery of removed nodes (reverse removal order) and the Eq. 1 tallies.
void recover(const Graph& g, const Split& s, int32_t k, std::vector<int8_t>& colors);
void tallies(const Graph& g, const std::vector<int8_t>& colors, int64_t* stitches,
             int64_t* conflicts, int64_t* uncolored);

// Rectangles -> layout graph (grid neighbour search, several threads).
struct OwnedGraph {
  int32_t num_nodes = 0;
  std::vector<int32_t> ce;   // pairs u < v, sorted
  std::vector<int32_t> se;   // pairs
};
// threads = 0: host_threads().
void build_layout_graph(const mpld_rect* rects, int32_t n, int32_t dmin,
                        int32_t split_len, OwnedGraph& out, int threads = 0);

// Validation, midpoint stitch split and search grid of a layout, shared by
// the host and the device graph builders: nd = node boxes (split halves
// consecutive, lower/left first), partner[v] = stitch partner or -1, se =
// stitch pairs; grid of gx x gy square cells of side `cell` from (minx,
// miny), cell > largest box extent + d_min, so that every conflict pair has
// its lower-left corners in the same or adjacent cells.
struct LayoutPrep {
  std::vector<mpld_rect> nd;
  std::vector<int32_t> partner, se;
  int64_t minx = 0, miny = 0, cell = 1, gx = 1, gy = 1;
};
void prepare_layout(const mpld_rect* rects, int32_t n, int32_t dmin, int32_t split_len,
                    LayoutPrep& lp);

int host_threads();

}  // namespace mpld

struct mpld_owned_graph {
  mpld::OwnedGraph g;
};

struct mpld_result {
  std::vector<int8_t> colors;
  std::vector<int32_t> comp_of;
  std::vector<mpld_comp_record> comps;
  int64_t stitches = 0, conflicts = 0, uncolored = 0;
  double queue_us = 0, total_us = 0;   // serving timing
};
