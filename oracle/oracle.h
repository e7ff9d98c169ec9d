/*
 * oracle.h - plain, slow, single-threaded CPU reference of the exact-cover
 * layout decomposition path.  TEST INFRASTRUCTURE ONLY: it is linked by the
 * tests and by the benchmark's CPU-baseline leg, never by the product
 * library, and it shares no code with it.
 *
 * Everything is integer arithmetic.  Each function cites the passage of the
 * paper it follows ("GPU-Accelerated Matrix Cover Algorithm for Multiple
 * Patterning Layout Decomposition", Chen, Yang, Yu, 2023):
 *   - Sec. 2.1: layout graph G = (V, CE u SE), colors x_i, conflicts and
 *     stitches (Eq. 1).
 *   - Sec. 2.2: flow - layout graph, simplification with stitch insertion,
 *     coloring solver, recovery of removed nodes.
 *   - Sec. 2.3: exact-cover matrix of the no-stitch graph, dancing-links
 *     cover/uncover (Eq. 2), Algorithm 1 (sub-graphs, column choice, row
 *     loop, first solution ends the search).
 * Where the paper is silent the readings used are stated at each function.
 */
#ifndef MPLD_ORACLE_H
#define MPLD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FEASIBLE = 0, ORC_INFEASIBLE = 1, ORC_BUDGET = 2 };
enum { ORC_SIMPLIFY = 1, ORC_MARK = 2, ORC_STITCH = 4, ORC_MINIMIZE = 8 };
/* ORC_MINIMIZE applies to components of at most this many nodes. */
enum { ORC_MINIMIZE_MAX_N = 64 };

typedef struct { int32_t x0, y0, x1, y1; } orc_rect;

/* Per component record of the pipeline. */
typedef struct {
  int32_t size;          /* nodes in the component                     */
  int32_t status;        /* ORC_FEASIBLE / ORC_INFEASIBLE / ORC_BUDGET */
  int64_t nodes;         /* search nodes counted                       */
  uint64_t trace_hash;   /* fingerprint of the node trace (oracle.c)   */
  int32_t depth_at_stop; /* rows in the partial solution at the stop   */
  int32_t stitches;      /* SE pairs inside, colored differently; -1 unless colored */
  int32_t first_node;    /* smallest original node id                  */
  int32_t num_edges;     /* conflict edges inside                      */
  int32_t conflicts;     /* conflict edges inside whose ends share a color */
  int32_t min_nodes;     /* ORC_MINIMIZE: branch-and-bound nodes, negated when its
                            budget stopped it (least cost not proven); 0 = not run */
} orc_comp;

/* Builds the node list and conflict/stitch edges of a rectangle layout.
 * split_len > 0 splits every rectangle whose long side exceeds split_len at
 * floor(L/2) into two nodes (lower/left first) joined by a stitch edge.
 * Conflict edge iff the Euclidean gap of the closed boxes is < dmin.
 * Outputs are malloc'ed (free with orc_free): ce and se hold pairs (u < v),
 * ce sorted lexicographically.  Returns 0 or negative on error. */
int32_t orc_build_graph(const orc_rect* rects, int32_t n, int32_t dmin,
                        int32_t split_len, int32_t* num_nodes,
                        int64_t* num_ce, int32_t** ce, int64_t* num_se,
                        int32_t** se);

/* Full decomposition of a graph.  flags: ORC_SIMPLIFY, ORC_MARK (components
 * the search leaves without a solution are colored by orc_mark_conflicts),
 * ORC_STITCH (stitch-aware row order, orc_solve_component_stitch, with each
 * node's stitch partner when the partner is in the same component),
 * ORC_MINIMIZE (implies ORC_MARK for unsolved components; then every
 * component of at most ORC_MINIMIZE_MAX_N nodes whose coloring has a
 * positive Eq. 1 cost goes through orc_minimize_component with min_budget
 * nodes, stitch partners inside the component included).
 * colors (num_nodes, -1 = uncolored) and
 * comp_of (num_nodes, -1 = removed by simplification) are caller-allocated;
 * *comps is malloc'ed (free with orc_free).  Totals may be NULL. */
int32_t orc_decompose(int32_t num_nodes, int64_t num_ce, const int32_t* ce,
                      int64_t num_se, const int32_t* se, int32_t k,
                      int64_t budget, int64_t min_budget, uint32_t flags, int8_t* colors,
                      int32_t* comp_of, int32_t* num_comps, orc_comp** comps,
                      int64_t* total_stitches, int64_t* total_conflicts,
                      int64_t* total_uncolored);

/* Simplification and sub-graph split only (no search), for inspection:
 * removal_order (num_nodes), comp_of (num_nodes), bfs_order (num_nodes; core
 * nodes grouped by component in local order) and comp_ptr (num_nodes + 1)
 * are caller-allocated. */
int32_t orc_simplify(int32_t num_nodes, int64_t num_ce, const int32_t* ce,
                     int32_t k, uint32_t flags, int32_t* removal_order,
                     int32_t* num_removed, int32_t* comp_of, int32_t* bfs_order,
                     int32_t* comp_ptr, int32_t* num_comps);

/* Solves one component given in local numbering (edges are local pairs,
 * any order, no duplicates).  colors (n) caller-allocated. */
int32_t orc_solve_component(int32_t n, int64_t m, const int32_t* edges,
                            int32_t k, int64_t budget, int8_t* colors,
                            int32_t* status, int64_t* nodes,
                            uint64_t* trace_hash, int32_t* depth_at_stop);

/* The same search with a stitch-aware row order (Eq. 1 counts a stitch for
 * each pair of split halves colored differently): when the chosen column's
 * node has a stitch partner (partner[v], local id, -1 none; symmetric) that
 * is already colored on the current path and the row of that color is
 * still present, that row is tried first, the others follow in ascending
 * order.  partner = NULL is orc_solve_component. */
int32_t orc_solve_component_stitch(int32_t n, int64_t m, const int32_t* edges,
                                   int32_t k, int64_t budget, const int32_t* partner,
                                   int8_t* colors, int32_t* status, int64_t* nodes,
                                   uint64_t* trace_hash, int32_t* depth_at_stop);

/* Conflict marking of Algorithm 1 for one component in local numbering:
 * the no-backtracking descent of the search in which a column left with
 * no row takes the row it lost last (a marked conflict).  colors (n) are
 * caller-allocated; every node is colored. */
int32_t orc_mark_conflicts(int32_t n, int64_t m, const int32_t* edges, int32_t k,
                           int8_t* colors);

/* Eq. 1 minimisation of one component (local numbering) from a complete
 * incumbent coloring `colors` (in/out): a depth-first branch and bound over
 * the relaxed exact cover in which a row may be taken over covered
 * secondary columns at one conflict each; cost = 10 conflicts + stitches
 * (alpha = 0.1 scaled by 10).  partner: local stitch partners (-1 none) or
 * NULL.  *cost: the incumbent's cost in, the best cost out; *nodes: nodes
 * counted (budget tested before counting); *stopped: 1 when the budget
 * ended it.  An incumbent of cost 0 returns at once with 0 nodes. */
int32_t orc_minimize_component(int32_t n, int64_t m, const int32_t* edges, int32_t k,
                               const int32_t* partner, int64_t budget, int8_t* colors,
                               int64_t* nodes, int32_t* stopped, int32_t* cost);

/* Solves many components (concatenated local edge lists) on `threads`
 * threads, each component independently with orc_solve_component's
 * semantics, and repeats the whole set `passes` times in the same call
 * (the threads stay alive across passes).  The outputs hold the first
 * pass; *total_nodes (may be NULL) is the search-node sum over every pass.
 * threads == 1 runs on the calling thread.  Used only to time the oracle
 * on the host cores. */
int32_t orc_solve_many(int32_t count, const int32_t* sizes,
                       const int64_t* edge_counts, const int32_t* edges,
                       int32_t k, int64_t budget, int32_t threads, int32_t passes,
                       int8_t* colors, int32_t* status, int64_t* nodes,
                       uint64_t* trace_hash, int64_t* total_nodes);

/* Builds the exact-cover matrix of a component (for inspection in tests):
 * rows R = n*k, columns C = n + m*k; returns CSR over rows (row_ptr R+1,
 * col_idx) malloc'ed.  Row r = v*k + c has a 1 in primary column v and in
 * secondary column n + e*k + c for each local edge e (sorted pairs u < w)
 * incident to v. */
int32_t orc_ec_matrix(int32_t n, int64_t m, const int32_t* edges, int32_t k,
                      int64_t** row_ptr, int32_t** col_idx);

void orc_free(void* p);

#ifdef __cplusplus
}
#endif
#endif
