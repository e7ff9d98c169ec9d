/*
 * mpld.h - C ABI of the MI355X exact-cover layout decomposer.
 *
 * What it computes (Chen, Yang, Yu, "GPU-Accelerated Matrix Cover Algorithm
 * for Multiple Patterning Layout Decomposition", 2023):
 *   Sec. 2.1  A layout graph G = (V, CE u SE) and a mask count k go in; a
 *             color x_i in {0..k-1} per node comes out, with the conflict
 *             count (conflict-edge ends colored alike) and the stitch count
 *             (stitch-edge ends colored differently) of Eq. 1.
 *   Sec. 2.2  Flow: layout graph -> simplification (removal of nodes the
 *             coloring can always extend to) -> sub-graphs -> coloring
 *             solver -> recovery of the removed nodes.
 *   Sec. 2.3  The solver is exact cover on the 0/1 matrix with one row per
 *             (node, color), one primary column per node and one secondary
 *             column per (conflict edge, color), searched with Algorithm X
 *             (Algorithm 1); the dancing-links cover/uncover of Eq. 2 is
 *             replaced by data-parallel bitset operations on the GPU.
 *
 * Readings where the paper is silent (all deterministic, so the GPU result
 * is reproducible bit for bit):
 *   - simplification: first-in first-out removal of nodes with conflict
 *     degree < k (queue seeded in ascending id, neighbours visited in
 *     ascending id); recovery in reverse removal order: the stitch partner's
 *     color if free, else the lowest color free among colored conflict
 *     neighbours;
 *   - sub-graphs: connected components of the remaining nodes, ordered by
 *     smallest id; local index = BFS order from that node (neighbours in
 *     ascending id);
 *   - column choice (Algorithm 1, column selection: a column with a single
 *     related row first, else BFS order): the uncovered primary column with
 *     the fewest rows, lowest local index on ties; rows tried in ascending color; the first exact cover ends the
 *     search; an empty column is a dead end (no conflict-candidate marking);
 *   - a search node is one entry into the search that passes the budget
 *     test (budget tested before counting), so nodes <= budget always and
 *     BUDGET_EXHAUSTED implies nodes == budget;
 *   - trace hash (a fingerprint of the search order; the method defines
 *     none): each search node contributes x = FNV-1a 64 of its 16 bytes -
 *     depth, entering row (v*k + c; 0xFFFFFFFF at the root), chosen column
 *     (0xFFFFFFFF at a solution), its row count; u32 little-endian each -
 *     from the offset basis, and N nodes in search order give
 *     sum x_i * B^(N-i) mod 2^64, B = 0x100000001B3 (h = h*B + x per node
 *     from 0).  A trace followed by another of n nodes has h1 * B^n + h2,
 *     so subtrees searched apart combine exactly.
 *
 * Conventions:
 *   - Return codes are int32: 0 = ok, negative = error (enum below).  No
 *     C++ exception crosses the ABI.  mpld_last_error() gives a thread-local
 *     detail string valid until the next call on that thread.
 *   - Inputs are caller-owned, read-only and copied before return.
 *   - Outputs (mpld_result, mpld_owned_graph, mpld_batch, mpld_server) are
 *     library-owned; free them with their *_free call.  Accessors return
 *     borrowed pointers valid until that free.
 *   - A context owns one device, one HIP stream and its device memory.  One
 *     thread per context, or external locking.  After MPLD_E_DEVICE the
 *     context is unusable and must be destroyed.
 *   - Every device step is HIP code; there is no host fallback: a missing
 *     device returns MPLD_E_DEVICE.
 *
 * Surface, against a plainer sketch of it (generate / submit / poll / wait
 * / free on the context): no layout generator here - synthetic layouts come
 * from a separate input library, so that the checking code and this library
 * share nothing but their inputs, and a user brings their own rectangles;
 * serving is a server object on a context (mpld_server_*), so that one
 * context can host servers with arenas of their own; every owned object
 * has a typed free (mpld_result_free, mpld_owned_graph_free,
 * mpld_batch_free, mpld_server_destroy) rather than one generic free.
 */
#ifndef MPLD_H
#define MPLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPLD_ABI_VERSION 3u
#define MPLD_MAX_K 8

enum {
  MPLD_OK = 0,
  MPLD_E_INVALID = -1,     /* bad argument: k, ids, self loop, duplicate, CE n SE, budget */
  MPLD_E_NOMEM = -2,       /* host or device allocation failed / larger than the arena */
  MPLD_E_DEVICE = -3,      /* HIP error; the context is unusable */
  MPLD_E_NOT_READY = -4,   /* serving: ticket not finished yet */
  MPLD_E_CANCELLED = -5,   /* serving: server shut down before the ticket ran */
  MPLD_E_INTERNAL = -6,    /* broken invariant (a bug) */
  MPLD_E_UNSUPPORTED = -7  /* a forced tier cannot take this component */
};

/* per component status */
enum { MPLD_FEASIBLE = 0, MPLD_INFEASIBLE = 1, MPLD_BUDGET_EXHAUSTED = 2 };

/* option flags */
enum {
  MPLD_SIMPLIFY = 1u << 0,     /* degree < k removal + recovery (default on) */
  MPLD_TRACE_HASH = 1u << 1,   /* accumulate the per-component trace hash      */
  MPLD_PLAIN = 1u << 2,        /* one kernel launch per component (comparison) */
  MPLD_FORCE_WAVE = 1u << 3,   /* force the register tier (n <= 64)           */
  MPLD_FORCE_LDS = 1u << 4,    /* force the LDS tier                          */
  MPLD_FORCE_GLOBAL = 1u << 5, /* force the big tier: level headers and undo
                                  log in global memory, the lists in LDS on
                                  one wave or in global memory on a workgroup
                                  (mpld_tune.big_one_wave)                    */
  MPLD_DIRECT = 1u << 6,       /* batched solve: launch the kernels directly
                                  instead of replaying the captured HIP graph */
  MPLD_FORCE_DEVICE = 1u << 7, /* force the device-wide tier: one component at a
                                  time over every CU, columns split across
                                  workgroups, a device-wide min-count reduction
                                  per search node                              */
  MPLD_SPLIT_HEAVY = 1u << 8,  /* register-tier components still searching after
                                  a first capped pass are searched in parallel
                                  subtrees by many wavefronts; the sequential
                                  status, node count, depth, colors and trace
                                  hash are recomputed exactly from the
                                  subtrees' counts and hashes in search order
                                  (each subtree's hash appended with the
                                  concatenation rule of the trace hash; a
                                  component cut by its budget is re-run
                                  sequentially).  LDS-tier and big-tier
                                  components are searched as k subtree tasks,
                                  one per root row (the root column is node
                                  0), each on its own wave or workgroup; their
                                  counts and hashes are added in row order,
                                  and a budget crossed inside a later row's
                                  subtree is found by searching that subtree
                                  again with the budget left.  Makes
                                  mpld_batch_solve wait.  mpld_decompose and
                                  mpld_solve_components, which wait anyway,
                                  use it for every solve whether or not the
                                  flag is given. */
  MPLD_UNTIMED = 1u << 9,      /* mpld_batch_solve: record no HIP events around
                                  the search (last_search_ms keeps the value of
                                  the last timed solve); for callers timing
                                  many back-to-back solves themselves */
  MPLD_MARK_CONFLICTS = 1u << 10, /* conflict marking (Algorithm 1, a column
                                  left with no related row is a conflict
                                  candidate): a component whose search ends
                                  INFEASIBLE or BUDGET_EXHAUSTED is still
                                  colored, by one descent of the search that
                                  never backtracks, in which such a column
                                  takes the color of the row it lost last.
                                  Status, node count, hash and depth stay the
                                  search's; `conflicts` and `stitches` are
                                  counted on the colors.  Decompose, batches,
                                  mpld_solve_components and servers (a served
                                  component is marked when its search ends). */
  MPLD_STITCH_ORDER = 1u << 11, /* stitch-aware row order (Eq. 1 counts a stitch
                                  for each pair of split halves colored
                                  differently): when the chosen column's node
                                  has its stitch partner in the component and
                                  already colored on the path, the row of the
                                  partner's color (if open) is tried first,
                                  the others follow ascending.  Register, LDS
                                  and big tiers (the CSR blocks of the LDS
                                  tiers then end with each node's partner); a
                                  forced device-wide tier gives
                                  MPLD_E_UNSUPPORTED; with MPLD_SPLIT_HEAVY
                                  the subtree tasks rebuild each path's row
                                  order (device-resident rounds only; the
                                  root-row tasks of the LDS tiers start where
                                  no partner is colored yet); servers take it
                                  (the partner registers are part of the
                                  resumable state). */
  MPLD_ROUNDTRIP = 1u << 12,   /* mpld_batch_solve: the whole device solve -
                                  copy of the packed image from page-locked
                                  host memory to the device, the search, copy
                                  of the records and local colors back to
                                  page-locked host memory - enqueued between
                                  two HIP events; mpld_batch_info's
                                  last_roundtrip_ms reads their distance.  The
                                  result is the same as without the flag. */
  MPLD_MINIMIZE = 1u << 13     /* Eq. 1 minimisation: after the search (and the
                                  conflict marking, which this flag implies),
                                  every component of the register tier (at
                                  most 64 nodes) whose coloring costs anything
                                  - cost = 10 x conflicts + stitches, Eq. 1
                                  with alpha = 0.1 scaled by 10 - is searched
                                  again by a depth-first branch and bound over
                                  the exact cover relaxed so that a row may be
                                  taken over covered (edge, color) columns at
                                  one conflict each: penalty of (u, c) = 10 x
                                  colored neighbours of color c + 1 when u's
                                  stitch partner has another color; bound =
                                  cost + sum of the uncolored nodes' least
                                  penalties; branch on the uncolored node with
                                  the fewest conflict-free colors (lowest
                                  index on ties), colors ascending, a color
                                  skipped when its child bound reaches the
                                  incumbent's cost; at most
                                  mpld_options.min_budget nodes per component.
                                  The best coloring replaces the incumbent;
                                  status, nodes, hash and depth stay the
                                  search's; mpld_comp_record.min_nodes tells
                                  whether least cost was proven.  Decompose,
                                  batches, mpld_solve_components and servers
                                  (a served register-tier component is
                                  minimised by the tick that ends its
                                  search); not with a forced LDS, global or
                                  device tier (MPLD_E_UNSUPPORTED). */
};

typedef struct { int32_t x0, y0, x1, y1; } mpld_rect;  /* nm, closed box */

/* A layout graph (Sec. 2.1).  ce: num_ce pairs (u, v), 0 <= u, v <
 * num_nodes, u != v, no duplicate pair in either orientation.  se: num_se
 * stitch pairs (may be 0 / NULL); each node is in at most one stitch pair
 * and no stitch pair is also a conflict pair.  Caller-owned. */
typedef struct {
  int32_t num_nodes;
  int32_t reserved;
  int64_t num_ce;
  const int32_t* ce;
  int64_t num_se;
  const int32_t* se;
} mpld_graph;

typedef struct {
  uint32_t struct_size;   /* sizeof(mpld_options)                       */
  int32_t k;              /* mask count, 2 .. MPLD_MAX_K                */
  int64_t node_budget;    /* per component, >= 1                        */
  uint32_t flags;         /* MPLD_* flags                               */
  int32_t min_budget;     /* MPLD_MINIMIZE: branch-and-bound nodes per
                             component; 0 = 10000; < 0 is MPLD_E_INVALID */
} mpld_options;

/* Per component record (48 bytes). */
typedef struct {
  int32_t size;           /* nodes                                          */
  int32_t status;         /* MPLD_FEASIBLE / MPLD_INFEASIBLE / MPLD_BUDGET_EXHAUSTED */
  int64_t nodes;          /* search nodes                                   */
  uint64_t trace_hash;    /* trace hash above (0 unless MPLD_TRACE_HASH)    */
  int32_t depth_at_stop;  /* rows in the partial solution when it stopped (0 if infeasible) */
  int32_t stitches;       /* stitch pairs inside colored differently; -1 unless colored
                             (feasible, or marked with MPLD_MARK_CONFLICTS) */
  int32_t first_node;     /* smallest original node id                      */
  int32_t num_edges;      /* conflict edges inside                          */
  int32_t conflicts;      /* conflict edges inside whose ends share a color
                             (0 unless MPLD_MARK_CONFLICTS marked it)        */
  int32_t min_nodes;      /* MPLD_MINIMIZE: branch-and-bound nodes; negated
                             when min_budget stopped it (least cost not
                             proven); 0 when it did not run (cost 0, or more
                             than 64 nodes)                                 */
} mpld_comp_record;

/* One component given directly in its local numbering (no simplification,
 * no renumbering): n nodes, m local pairs. */
typedef struct {
  int32_t n;
  int32_t reserved;
  int64_t m;
  const int32_t* edges;
} mpld_component;

/* Optional device allocator (e.g. a framework's caching allocator).  alloc
 * returns device memory of at least `bytes` bytes aligned to 256, or NULL. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} mpld_allocator;

typedef struct mpld_context mpld_context;
typedef struct mpld_result mpld_result;
typedef struct mpld_owned_graph mpld_owned_graph;
typedef struct mpld_batch mpld_batch;

uint32_t mpld_abi_version(void);
const char* mpld_error_string(int32_t err);   /* static string */
const char* mpld_last_error(void);            /* thread-local detail */

/* ---- host front-end (Sec. 2.1, 2.2) ------------------------------------
 * Layout graph of n rectangles: a conflict edge joins two features whose
 * closed boxes are less than dmin_nm apart (Euclidean gap).  split_len_nm >
 * 0 splits every rectangle whose long side exceeds it at floor(L/2) into
 * two consecutive nodes (lower/left first) joined by a stitch edge and
 * never by a conflict edge.  Conflict pairs come out as (u < v) sorted.
 * Errors: MPLD_E_INVALID for n < 0, dmin < 0, split < 0, a box with
 * x1 < x0 or y1 < y0. */
int32_t mpld_build_graph(const mpld_rect* rects, int32_t n, int32_t dmin_nm,
                         int32_t split_len_nm, mpld_owned_graph** out);
/* The same layout graph (identical pairs, stitch pairs and node count)
 * built on the context's device: the host validates, splits and picks the
 * search grid, the device sorts the nodes into grid cells and tests every
 * node against its 3x3 cell neighbourhood.  For large layouts, where the
 * host pair search dominates.  Synchronous on the context's stream.
 * Errors as mpld_build_graph, plus MPLD_E_DEVICE / MPLD_E_NOMEM. */
int32_t mpld_build_graph_device(mpld_context* ctx, const mpld_rect* rects, int32_t n,
                                int32_t dmin_nm, int32_t split_len_nm, mpld_owned_graph** out);
/* Simplification and sub-graph split (Sec. 2.2; Algorithm 1 splits the
 * graph into sub-graphs) of a layout graph, computed on the context's
 * device: FIFO removal of nodes of conflict degree < k (queue seeded in
 * ascending id, a removed node's neighbours visited in ascending id),
 * connected components of the rest ordered by smallest id, local numbering
 * by BFS from that node with neighbours in ascending id.  flags:
 * MPLD_SIMPLIFY or 0 (no removal).  Outputs are caller-allocated:
 * removal_order (num_nodes; the first *num_removed are used), comp_of
 * (num_nodes; -1 = removed), bfs_order (num_nodes; core nodes grouped by
 * component, each in local order), comp_ptr (num_nodes + 1; component c is
 * bfs_order[comp_ptr[c] .. comp_ptr[c + 1])).  Wide passes (the first peel
 * levels, union-find, numbering) run over the whole device, the small tail
 * of the peeling and the BFS of components above 64 nodes on one workgroup,
 * the BFS of smaller components one wave each.  Synchronous on the
 * context's stream.  Errors: MPLD_E_INVALID
 * for a bad graph (as mpld_decompose), k outside [2, MPLD_MAX_K] or a NULL
 * output; MPLD_E_DEVICE / MPLD_E_NOMEM. */
int32_t mpld_split_graph_device(mpld_context* ctx, const mpld_graph* g, int32_t k, uint32_t flags,
                                int32_t* removal_order, int32_t* num_removed, int32_t* comp_of,
                                int32_t* bfs_order, int32_t* comp_ptr, int32_t* num_comps);
/* Borrowed view of an owned graph (valid until mpld_owned_graph_free). */
int32_t mpld_owned_graph_view(const mpld_owned_graph* g, mpld_graph* view);
void mpld_owned_graph_free(mpld_owned_graph* g);

/* ---- context ----------------------------------------------------------
 * device: HIP ordinal.  alloc: NULL = hipMalloc/hipFree.  hip_stream: a
 * hipStream_t the caller keeps alive (e.g. a framework's current stream),
 * or NULL for a stream the context creates.  Errors: MPLD_E_DEVICE when no
 * such device or it is not gfx950. */
int32_t mpld_context_create(int32_t device, const mpld_allocator* alloc,
                            void* hip_stream, mpld_context** out);
int32_t mpld_context_destroy(mpld_context* ctx);

/* ---- one-shot decomposition (Sec. 2.2 flow, synchronous) --------------- */
int32_t mpld_decompose(mpld_context* ctx, const mpld_graph* g,
                       const mpld_options* opt, mpld_result** out);

/* ---- staged decomposition: device-resident batch -----------------------
 * mpld_batch_create runs the host front-end (simplification, sub-graphs,
 * exact-cover packing) and uploads the packed image to device memory.
 * mpld_batch_solve enqueues the whole device search on the context stream
 * and does not wait: the tiered persistent kernels, launched directly or,
 * when the batch's schedule says so (mpld_tune.use_graph), captured once
 * into a HIP graph and replayed (MPLD_DIRECT in `flags` always launches
 * directly); with MPLD_PLAIN one launch per component.  Queue counters
 * reset themselves at the end of each launch, so no memset is enqueued.
 * Per-component results stay on the device.  mpld_batch_result waits, copies the results back and runs
 * recovery and the Eq. 1 tallies. */
int32_t mpld_batch_create(mpld_context* ctx, const mpld_graph* g,
                          const mpld_options* opt, mpld_batch** out);
int32_t mpld_batch_solve(mpld_batch* b, uint32_t flags);
int32_t mpld_batch_result(mpld_batch* b, mpld_result** out);
/* Batch statistics: components per tier, core nodes, image bytes, and the
 * device time (ms) of the last solve's search launches measured with HIP
 * events recorded on the context stream right around them (read after
 * mpld_batch_result or once the stream has drained; 0 before). */
typedef struct {
  int32_t num_components;
  int32_t num_wave;          /* components on the register tier (n <= 64) */
  int32_t num_lds;           /* components on the LDS tier                */
  int32_t num_global;        /* components on the big tier                */
  int32_t core_nodes;        /* nodes left after simplification           */
  int32_t max_size;
  int64_t image_bytes;       /* packed device image                       */
  int64_t core_edges;
  float last_search_ms;      /* search kernels of the last solve          */
  float last_total_ms;       /* whole enqueued solve of the last solve    */
  int32_t launches;          /* kernel launches of the last solve         */
  int32_t num_device;        /* components on the device-wide tier        */
  int32_t heavy_components;  /* MPLD_SPLIT_HEAVY, last solve: components past
                                the first-pass cap                          */
  int32_t split_rounds;      /* ... task rounds                              */
  int32_t split_tasks;       /* ... subtree tasks run                        */
  int32_t split_reruns;      /* ... components re-run sequentially (budget)  */
  float last_roundtrip_ms;   /* last MPLD_ROUNDTRIP solve: first byte of the
                                image copied to the device .. last result byte
                                back on the host (0 before)                  */
  int32_t big_waves;         /* waves per workgroup of the big tier's
                                workgroup layout; 0: every big component runs
                                on one wave with its lists in LDS            */
} mpld_batch_info;
int32_t mpld_batch_get_info(mpld_batch* b, mpld_batch_info* info);
void mpld_batch_free(mpld_batch* b);

/* ---- launch parameters and the autotuner --------------------------------
 * The tiered launch schedule of a batch: register-tier workgroup size (in
 * waves of 64 lanes) and grid cap, queue order, HIP-graph replay, and whether
 * components of at least giant_min_nodes nodes use the device-wide tier.
 * mpld_batch_autotune times candidate schedules on the batch with HIP
 * events (median of `reps` solves; one solve each for batches whose solve
 * takes over 5 ms, which then only vary the order and the giant tier),
 * checks that every candidate reproduces the default's records and colors
 * (MPLD_E_INTERNAL otherwise), adopts the fastest and, when cache_path (or
 * $MPLD_TUNE_CACHE) names a file, appends it as one JSON line keyed by the
 * device architecture, CU count, k, trace flag and the batch's component
 * count and size (powers of two).  mpld_batch_create applies the last
 * matching cache line.  The schedule never changes a result. */
typedef struct {
  uint32_t struct_size;      /* sizeof(mpld_tune)                              */
  int32_t waves_per_block;   /* 1, 2 or 4                                      */
  int32_t max_blocks;        /* register-tier grid cap; 0 = a wave per component */
  int32_t use_graph;         /* replay a captured HIP graph                    */
  int32_t order;             /* 0 largest component first, 1 smallest first    */
  int32_t giant_device;      /* giants on the device-wide tier                 */
  int32_t giant_min_nodes;   /* what a giant is (>= 65)                        */
  float best_ms;             /* autotune: median device ms of the chosen one   */
  float default_ms;          /* autotune: the same for the default schedule    */
  int32_t candidates;        /* autotune: schedules timed                      */
  int32_t from_cache;        /* get: the schedule came from the cache          */
  int32_t heavy_first_cap;   /* MPLD_SPLIT_HEAVY: first-pass node cap (>= 64)  */
  int32_t heavy_round_cap;   /* MPLD_SPLIT_HEAVY: nodes per subtree task and
                                round (>= 16)                                   */
  int32_t heavy_levels;      /* MPLD_SPLIT_HEAVY: search levels enumerated when
                                a capped task splits (1..4; 0 = 4, 3 or 2 for
                                k <= 3, k = 4, k >= 5)                          */
  int32_t heavy_device;      /* MPLD_SPLIT_HEAVY: 1 chains the rounds on the
                                device (subtasks written by the kernel, the
                                host resolves once at the end); 0 drives every
                                round from the host                             */
  int32_t root_split;        /* 1: register-tier components of at least
                                root_split_min_n nodes get a workgroup each,
                                whose helper waves search the root's rows 1..3
                                beside the owner (no trace hash, no
                                MPLD_SPLIT_HEAVY); 0: off                      */
  int32_t root_split_min_n;  /* smallest component that gets one (>= 2)        */
  int32_t root_split_max;    /* most components that get one; 0 = all         */
  int32_t root_split_chunk;  /* helper nodes between checks of the owner's
                                release (>= 1)                                  */
  int32_t big_one_wave;      /* 1 (default): each component of the big tier
                                that fits runs on one wave with its neighbour
                                lists in LDS (level headers and undo log in
                                global memory; k <= 6, at most 16384 nodes,
                                2m < 2^17, degrees < 2^15, within the
                                workgroup's LDS), the others on a workgroup;
                                0: every one on a workgroup of up to 16 waves
                                sharing the column scan, lists in global
                                memory                                        */
} mpld_tune;
int32_t mpld_batch_autotune(mpld_batch* b, int32_t reps, const char* cache_path, mpld_tune* out);
int32_t mpld_batch_get_tune(mpld_batch* b, mpld_tune* out);
/* Re-packs and re-uploads the batch with the given schedule. */
int32_t mpld_batch_set_tune(mpld_batch* b, const mpld_tune* t);

/* ---- components directly (no simplification, no renumbering) -----------
 * Solves `count` components given in local numbering.  out: count records;
 * colors_out: sum of n entries, component after component (-1 unless
 * feasible).  Synchronous. */
int32_t mpld_solve_components(mpld_context* ctx, const mpld_component* comps,
                              int32_t count, const mpld_options* opt,
                              mpld_comp_record* out, int8_t* colors_out);

/* ---- components without any allocation ---------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * result as mpld_solve_components (records and colors, bit for bit) for
 * components of at most 64 nodes each, flags MPLD_TRACE_HASH and
 * MPLD_MARK_CONFLICTS (others: MPLD_E_UNSUPPORTED).  Every device buffer
 * the call needs - queue counter, records, local colors, packed items -
 * lives in one fixed device array of MPLD_NOALLOC_SCRATCH_BYTES per GPU
 * (held until the process ends), and the host staging in static memory:
 * the call makes no hipMalloc, hipFree or other allocation on success.
 * Limits: at most MPLD_NOALLOC_MAX_COMPONENTS components, and 256 +
 * 24 x count (rounded up to 256) + sum of n (rounded up to 256) +
 * count x (32 + 8 x largest n) bytes within the scratch; beyond either,
 * MPLD_E_INVALID.  Inputs and outputs are the caller's host memory, as in
 * mpld_solve_components.  All calls on one GPU share its array and leave
 * their contents in it; calls overlapping on one GPU race (within one
 * process they are serialised by a lock).  Synchronous on the context's
 * stream. */
#define MPLD_NOALLOC_SCRATCH_BYTES (32u << 20)
#define MPLD_NOALLOC_MAX_COMPONENTS (1 << 18)
int32_t mpld_solve_components_noalloc(mpld_context* ctx, const mpld_component* comps,
                                      int32_t count, const mpld_options* opt,
                                      mpld_comp_record* out, int8_t* colors_out);

/* ---- serving: continuous batching of whole-layout requests --------------
 * A server owns a context's stream from a scheduler thread.  Requests are
 * copied at submit and run through the host front-end on worker threads;
 * the scheduler then admits them in arrival order as soon as their packed
 * image fits the device arena and enough component slots are free (admission
 * by device bytes).  Every tick advances every resident register-tier
 * component by at most `slice_nodes` search nodes from the state it keeps in
 * device memory (larger components run to completion on a second stream,
 * started by the tick that admits them and collected by a later one, so a
 * long one does not hold up the ticks), so requests that arrive while
 * others are on the device join at the next tick and their work shares the
 * same launches.  A request's
 * result depends only on its graph and options - not on arrival time, the
 * mix or the slice.  While a server exists its context must not be used
 * elsewhere.  A request larger than the whole arena (or than all slots)
 * completes with MPLD_E_NOMEM instead of waiting. */
typedef struct mpld_server mpld_server;
typedef struct {
  uint32_t struct_size;    /* sizeof(mpld_server_options)                   */
  int32_t max_components;  /* component slots resident at once; 0 = 65536   */
  int64_t arena_bytes;     /* device bytes for request images; 0 = 256 MiB, at most 2 GiB */
  int64_t slice_nodes;     /* search nodes per component per tick; 0 = 4096 */
  int32_t host_threads;    /* front-end threads; 0 = min(16, host cores)    */
  int32_t graph_builders;  /* device graph builders (own stream each) taken
                              in turn by layout requests of >= 4096 rects;
                              0 = 1, < 0 = none (the host builds every graph) */
  int32_t device_split;    /* >= 0: device-built layouts whose average
                              conflict degree is below k are also simplified
                              and split on the device (mpld_split_graph_device's
                              kernels, behind the pair search; default);
                              < 0: always on the host */
  int32_t reserved;
} mpld_server_options;
typedef struct {
  int64_t submitted, completed, failed, ticks;
  int64_t resident_bytes, resident_components, peak_bytes;
  int64_t search_nodes;     /* of completed requests                       */
  int64_t admission_waits;  /* ticks in which the next request did not fit */
  double device_ms;         /* summed device time of the ticks (HIP events) */
} mpld_server_stats;

int32_t mpld_server_create(mpld_context* ctx, const mpld_server_options* opt,
                           mpld_server** out);
/* Submit a layout graph (copied) or a rectangle layout (copied; the layout
 * graph is built on a worker thread, as mpld_build_graph).  Returns a
 * ticket at once. */
int32_t mpld_server_submit(mpld_server* s, const mpld_graph* g, const mpld_options* opt,
                           uint64_t* ticket);
int32_t mpld_server_submit_layout(mpld_server* s, const mpld_rect* rects, int32_t n,
                                  int32_t dmin_nm, int32_t split_len_nm,
                                  const mpld_options* opt, uint64_t* ticket);
/* The finished result of a ticket (the ticket is consumed), MPLD_E_NOT_READY
 * while it runs, the request's own error code if it failed, MPLD_E_INVALID
 * for an unknown ticket.  wait blocks up to timeout_us (< 0: no limit). */
int32_t mpld_server_poll(mpld_server* s, uint64_t ticket, mpld_result** out);
int32_t mpld_server_wait(mpld_server* s, uint64_t ticket, int64_t timeout_us,
                         mpld_result** out);
int32_t mpld_server_get_stats(mpld_server* s, mpld_server_stats* out);
/* Stops the scheduler after its current tick; requests not finished by then
 * complete with MPLD_E_CANCELLED (their results cannot be fetched). */
int32_t mpld_server_destroy(mpld_server* s);

/* ---- measurement ----------------------------------------------------------
 * The chip's LDS read rate, for the roofline of the LDS-tier kernels (Sec.
 * 2.3 keeps the matrix cover in on-chip shared memory): every CU runs
 * workgroups of 256 lanes that read 32 KB of LDS each with ds_read_b64
 * (bytes_per_lane = 8) or ds_read_b128 (16), iters x 16 reads per lane,
 * contiguous per wave (no bank conflicts); *gbytes_per_s = bytes read over
 * the kernel time of the second of two runs (HIP events on the context
 * stream), *bytes_per_clock_per_cu (may be NULL) the same per CU and cycle
 * of the device's reported clock.  Synchronous.  MPLD_E_INVALID for a
 * NULL pointer, another width or iters outside [1, 2^24]. */
int32_t mpld_measure_lds_read_rate(mpld_context* ctx, int32_t bytes_per_lane, int32_t iters,
                                   double* gbytes_per_s, double* bytes_per_clock_per_cu);
/* The fixed cost of one kernel launch inside a timed step (not a step of
 * the paper's method; it puts the search kernels' times in context): `reps`
 * launches of an empty kernel of `grid` workgroups of `block` lanes, back
 * to back on the context stream after one warm-up launch, timed with two
 * HIP events; *us_per_launch = their distance / reps.  Synchronous.
 * MPLD_E_INVALID for a NULL pointer, grid outside [1, 2^20], block not a
 * multiple of 64 in [64, 1024], or reps outside [1, 100000]. */
int32_t mpld_measure_launch_floor(mpld_context* ctx, int32_t grid, int32_t block, int32_t reps,
                                  double* us_per_launch);
/* As mpld_measure_launch_floor, for a kernel whose every wave reads 64
 * bytes of its own and writes 8 bytes (as a search wave loads its item and
 * stores its record): the fixed cost of a launch that touches device memory
 * both ways.  Device buffers of 72 bytes per wave come from the context's
 * allocator for the call.  Same arguments and errors, plus MPLD_E_NOMEM. */
int32_t mpld_measure_touch_floor(mpld_context* ctx, int32_t grid, int32_t block, int32_t reps,
                                 double* us_per_launch);

/* ---- results ------------------------------------------------------------ */
const int8_t* mpld_result_colors(const mpld_result* r, int32_t* num_nodes);
const int32_t* mpld_result_component_of(const mpld_result* r); /* -1 = removed */
int32_t mpld_result_num_components(const mpld_result* r);
const mpld_comp_record* mpld_result_components(const mpld_result* r);
void mpld_result_totals(const mpld_result* r, int64_t* stitches,
                        int64_t* conflicts, int64_t* uncolored);
/* Serving results: microseconds from submit to admission on the device and
 * from submit to the finished result (0 for results of other calls). */
void mpld_result_timing(const mpld_result* r, double* queue_us, double* total_us);
void mpld_result_free(mpld_result* r);

#ifdef __cplusplus
}
#endif
#endif
