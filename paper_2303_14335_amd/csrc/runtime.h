// runtime.h - device context, device buffers, packed batches and kernel
// launchers of the decomposer library (host side).
#pragma once

#include <hip/hip_runtime_api.h>

#include <memory>
#include <vector>

#include "device_types.h"
#include "internal.h"

namespace mpld {

// kernel launchers (defined with the kernels)
// k: the batch's mask count (every component of a batch shares it).
// wpb: waves per workgroup (1..4); cap < budget stops components after cap
// nodes (status -1, for the heavy-component engine).
// heavy > 0: root split of items 0 .. heavy-1 (cap = ~0, wpb = 4,
// grid >= heavy + ceil((qlen - heavy) / 4)).  mark (cap = ~0 only): a
// component whose search ends without a solution is colored by the
// conflict marking in the same wave.
hipError_t launch_reg_batched(bool trace, int k, int grid, int wpb, RegItems items,
                              int32_t qlen, int32_t* counter, DevRecord* recs, int8_t* colors,
                              uint64_t cap, int32_t heavy, uint32_t chunk, bool mark,
                              hipStream_t s);
// Heavy-component engine: explore / split subtree tasks.
// Task t writes its output block at out + t * kSplitBlockBytes and its
// split items to pool at an offset taken from *pool_count (zero before the
// launch).
hipError_t launch_reg_split(int k, int grid, const SplitTask* tasks, int32_t ntasks,
                            int32_t* counter, RegItems regitems, uint64_t cap,
                            uint32_t levels, uint8_t* out, SplitItem* pool,
                            int32_t* pool_count, hipStream_t s);
// Device-resident heavy engine: move the round window on (one thread), and
// run the current round's tasks (persistent grid; the window comes from
// head).  hc_nodes / hc_limit: per heavy component, explored nodes and the
// limit past which its tasks stop splitting.  trace: tasks and split items
// also carry the trace hashes of their nodes.
hipError_t launch_engine_advance(EngineHead* head, int32_t task_cap, hipStream_t s);
hipError_t launch_engine_round(int k, int grid, EngineHead* head, EngineTask* tasks,
                               int32_t task_cap, uint8_t* blocks, EngineItem* pool,
                               int32_t pool_cap, RegItems regitems,
                               unsigned long long* hc_nodes, const uint64_t* hc_limit,
                               uint64_t cap, uint32_t levels, bool trace, hipStream_t s);
// Scatters `count` resolved heavy components (records and colors).
hipError_t launch_heavy_writeback(const HeavyWrite* w, int32_t count, DevRecord* recs,
                                  int8_t* colors, hipStream_t s);
hipError_t launch_reg_single(bool trace, int k, RegItems items, int32_t item,
                             DevRecord* recs, int8_t* colors, hipStream_t s);
int reg_batched_blocks_per_cu(bool trace);
// Serving tick over register-tier components (see the kernel).
hipError_t launch_reg_tick(bool trace, bool stitch, int k, int grid, const int32_t* list,
                           int32_t len, int32_t* counter, const DevDesc* slot_desc,
                           uint8_t* slot_state, DevRecord* slot_rec, const uint64_t* arena64,
                           int8_t* arena8, const uint8_t* part8, const uint32_t* slot_minb,
                           int32_t* slot_min, uint64_t slice, DevRecord* tick_out, hipStream_t s);
// stitch: the stitch-aware row order (the CSR blocks end with the partners).
hipError_t launch_lds_batched(bool trace, bool big, bool stitch, int waves, int grid,
                              int lds_bytes, const DevDesc* descs, const uint32_t* adj32,
                              int32_t qlen, int32_t* counter, uint64_t* gstack,
                              uint64_t stack_words, DevRecord* recs, int8_t* colors,
                              hipStream_t s);
hipError_t launch_lds_single(bool trace, bool big, bool stitch, int waves, int lds_bytes,
                             const DevDesc* descs, const uint32_t* adj32, int32_t item,
                             uint64_t* gstack, DevRecord* recs, int8_t* colors, hipStream_t s);
// Subtree tasks of LDS-tier (big = false) or big-tier components (trace:
// each task record holds the trace hash of its own nodes).
hipError_t launch_lds_tasks(bool trace, bool big, bool stitch, int waves, int grid, int lds_bytes, const DevDesc* descs,
                            const uint32_t* adj32, const LdsTask* tasks, int32_t ntasks,
                            uint64_t* gstack, uint64_t stack_words, DevRecord* task_recs,
                            int8_t* task_colors, hipStream_t s);
// Writes resolved components' records (rec[i] to recs[comp[i]]) and colors
// (n[i] bytes from src + src_off[i], or -1 when src_off[i] < 0, to colors +
// out_off[i]).
hipError_t launch_csr_writeback(const LdsResolved* w, int32_t count, const int8_t* src,
                                DevRecord* recs, int8_t* colors, hipStream_t s);
// Waves per workgroup for big LDS-tier components of at most max_n nodes.
// The big-tier launchers take waves = 0 for the one-wave wide layout
// (lds_wide_bytes of LDS).
int lds_big_waves(int32_t max_n);
// Conflict marking (MPLD_MARK_CONFLICTS) of the components whose record is
// not FEASIBLE: register-tier items, and CSR components (LDS, big and
// device-wide tiers, one wave each, mark_lds_bytes of LDS).
hipError_t launch_mark_reg(int k, int grid, RegItems items, int32_t qlen, const DevRecord* recs,
                           int8_t* colors, hipStream_t s);
hipError_t launch_mark_lds(int grid, int lds_bytes, const DevDesc* descs, const uint32_t* adj32,
                           int32_t qlen, const DevRecord* recs, int8_t* colors, hipStream_t s);
int64_t mark_lds_bytes(int32_t n, int32_t k);
// Eq. 1 minimisation (MPLD_MINIMIZE) of the register-tier items from the
// incumbent colors in `colors`; partners: stitch partner byte per node
// (indexed like the masks, 0xff none); min_out[comp]: nodes, negated when
// stopped by `budget`, 0 when the incumbent costs nothing.
hipError_t launch_min_reg(int k, int grid, RegItems items, int32_t qlen, const uint8_t* partners,
                          int8_t* colors, int32_t* min_out, uint32_t budget, hipStream_t s);
// LDS bytes of one LDS-tier component (adj_words = n + 1 + 2m) and the
// global stack words of a big one.
int64_t lds_bytes_for(int32_t n, int32_t k, int64_t adj_words, int32_t max_deg, bool big,
                      bool stitch = false);
int64_t lds_stack_words(int32_t n, int32_t k, int64_t adj_words);
// LDS bytes of a big component on one wave with its neighbour lists in LDS
// (the wide layout), or -1 when that layout does not apply to it.
int64_t lds_wide_bytes(int32_t n, int32_t k, int64_t adj_words, int32_t max_deg, bool stitch);
// Device-wide tier (cooperative launch over `grid` workgroups, one per CU).
hipError_t launch_device_tier(bool trace, int grid, int lds_bytes, const DevDesc* desc,
                              const uint32_t* adj32, unsigned long long* keys, uint64_t* stacks,
                              DevRecord* recs, int8_t* colors, hipStream_t s);
int device_tier_lds_bytes(int32_t n, int grid);
int64_t device_tier_stack_words(int32_t n, int32_t max_deg);
// Allows every LDS-tier kernel up to `bytes` of dynamic LDS (once per context).
void lds_configure(int bytes);

void check_hip(hipError_t e, const char* what);

}  // namespace mpld

namespace mpld {
struct GraphBuilder;
}

struct mpld_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  mpld_allocator alloc{};
  bool has_alloc = false;
  int num_cus = 0;
  int reg_blocks_per_cu = 1;
  int lds_per_block = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  mpld::GraphBuilder* graph_builder = nullptr;   // device layout-graph builder (lazy)

  void* dev_alloc(size_t bytes);
  void dev_free(void* p);
};

namespace mpld {

// Device memory owned through the context's allocator.
struct DevBuf {
  mpld_context* ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && ctx) ctx->dev_free(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(mpld_context* c, size_t n) {
    release();
    ctx = c;
    bytes = n ? n : 256;
    p = c->dev_alloc(bytes);
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Page-locked host memory (hipHostMalloc), for small transfers that the
// host waits on.
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  // grows (never shrinks); false if the allocation failed
  bool reserve(size_t n) {
    if (n <= bytes) return true;
    release();
    if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      return false;
    }
    bytes = n;
    return true;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Host-side packed exact-cover image of a set of components.
struct Image {
  std::vector<DevDesc> desc;       // by component id
  std::vector<uint64_t> masks;     // register tier: one neighbour mask per node
  std::vector<uint8_t> partner8;   // register tier: local stitch partner per node (0xff none)
  bool stitch = false;             // MPLD_STITCH_ORDER: items carry the partners
  bool csr_stitch = false;         // MPLD_STITCH_ORDER: CSR blocks end with the partners
  bool minimize = false;           // MPLD_MINIMIZE: partner8 holds the partners
  std::vector<uint32_t> adj32;     // LDS tiers: row offsets, ids, max degree
  std::vector<int32_t> q_reg, q_lds, q_big, q_dev;   // component ids per tier
  int32_t total_nodes = 0;
  int32_t max_size = 0;
  int64_t core_edges = 0;
  int64_t lds_bytes_small = 0;     // largest footprint on the LDS tier
  int64_t lds_bytes_big = 0;       // largest footprint on the big tier
  // per component id, big tier: its LDS bytes in the workgroup layout and
  // in the one-wave layout (-1: that layout does not take it)
  std::vector<int64_t> big_bytes_wg, big_bytes_wide;
  int64_t big_stack_words = 0;     // largest global stack of the big tier
  int32_t big_max_n = 0;           // largest component of the big tier
  int64_t mark_lds = 0;            // LDS of the conflict marking of CSR components
  int64_t dev_stack_words = 0;     // largest per-workgroup stack of the device tier
  int32_t dev_max_n = 0;
};

// LDS byte limit for a component to keep its lists and stack in LDS.
constexpr int64_t kLdsSmallLimit = 64 * 1024;

// Launch parameters of a batch (chosen by the autotuner or defaults).
struct Tune {
  int32_t waves_per_block = 4;   // register tier workgroup = 64 * waves
  int32_t max_blocks = 0;        // register tier grid cap; 0 = one wave per component
  int32_t use_graph = 0;         // replay a captured HIP graph (off: direct launches are cheaper for the usual one or two kernels)
  int32_t order = 0;             // 0 largest first, 1 smallest first
  int32_t giant_device = 0;      // giants on the device-wide tier instead of the big tier
  int32_t giant_min_nodes = 4096;
  int32_t heavy_first_cap = 128;   // heavy-component engine: first-pass node cap
  int32_t heavy_round_cap = 256;   // nodes per subtree task and round
  int32_t heavy_levels = 0;        // levels per split; 0 = by k (4, 3 or 2)
  int32_t heavy_device = 1;        // 1: rounds chained on the device; 0: host-driven rounds
  int32_t root_split = 1;          // root split of the largest register-tier items
  int32_t root_split_min_n = 4;    // smallest item that gets one
  int32_t root_split_max = 0;      // most items that get one; 0 = all
  int32_t root_split_chunk = 16;   // helper nodes between release checks
  int32_t big_one_wave = 1;        // big tier on one wave (wide layout) when every component fits
};

// Adds one component (local numbering, pairs i < j or j < i) to the image.
// Throws MPLD_E_UNSUPPORTED when a forced tier cannot take it or it does
// not fit any tier.
// partner: local stitch partner per node (-1 none), for MPLD_STITCH_ORDER.
void image_add(Image& im, mpld_context* ctx, int32_t n, const int32_t* pairs, int64_t m,
               int32_t k, int64_t budget, uint32_t flags, const int32_t* partner = nullptr);
// Sorts each tier's queue by size (descending, or ascending when order = 1),
// ties by id.
void image_finish(Image& im, int order = 0);

// Device copy of an image plus its outputs and queue counters.
struct DeviceBatch {
  mpld_context* ctx = nullptr;
  DevBuf desc, regitems, adj32, counters, recs, colors, gstack;  // desc in launch order
  uint32_t reg_width = 1;   // masks per register-tier item
  bool reg_stitch = false;  // items carry stitch partners
  bool csr_stitch = false;  // CSR blocks end with stitch partners (LDS and big tiers)
  RegItems reg_items() const {
    const uint32_t pb = reg_stitch ? (reg_width + 7u) & ~7u : 0u;
    return RegItems{regitems.as<uint8_t>(), reg_width, kRegItemHead + 8u * reg_width + pb,
                    reg_stitch ? kRegItemHead + 8u * reg_width : 0u};
  }
  DevBuf dev_keys, dev_stacks;      // device-wide tier
  DevBuf partners, min_out;         // MPLD_MINIMIZE: stitch partners, per-component node counts
  uint32_t min_budget = 10000;      // MPLD_MINIMIZE: nodes per component
  DevBuf sp_tasks, sp_out, sp_pool, sp_writes;      // heavy-component engine
  PinnedBuf sp_host_tasks, sp_host_out, sp_host_pool, sp_host_writes, sp_host_recs;
  DevBuf en_meta, en_tasks, en_blocks, en_pool;     // device-resident rounds
  DevBuf ct_tasks, ct_recs, ct_colors, ct_resolved; // LDS/big-tier subtree tasks
  PinnedBuf ct_host;
  std::vector<uint8_t> sp_host_copy;                // engine results in ordinary memory
  int64_t sp_rounds = 0, sp_tasks_run = 0, sp_heavy = 0, sp_reruns = 0;  // last solve's stats
  Tune tune;
  int32_t n_reg = 0, n_lds = 0, n_big = 0, n_dev = 0;
  // the first n_wide big-tier components take the one-wave layout
  // (lds_wide bytes, grid_wide workgroups), the rest the workgroup layout
  // (lds_big bytes, big_waves waves, grid_big workgroups)
  int32_t n_wide = 0;
  int lds_wide = 0, grid_wide = 1;
  int grid_dev = 1, lds_dev = 0;
  int32_t num_comps = 0, total_nodes = 0;
  int32_t k = 3;
  int grid_reg = 1, grid_lds = 1, grid_big = 1;
  int grid_big_tasks = 1;   // big-tier subtree tasks (stack areas allocated for this many blocks)
  int lds_small = 0, lds_big = 0;
  int big_waves = 1;   // waves per workgroup on the big tier
  int32_t reg_heavy = 0;   // register-tier items (a launch-order prefix) with a root split
  int64_t mark_lds = 0;   // LDS bytes of the CSR conflict marking
  uint64_t big_stack_words = 0;
  float last_search_ms = 0.f, last_total_ms = 0.f;
  int32_t launches = 0;
  hipGraphExec_t graph = nullptr;
  uint32_t graph_flags = 0xffffffffu;
  bool timed = false;               // events of the last solve not read yet
  std::vector<uint8_t> host_items;  // register-tier items as uploaded
  // MPLD_ROUNDTRIP: page-locked copies of the image and the results, and
  // the two events around the whole solve
  PinnedBuf rt_up, rt_down;
  bool rt_ready = false, rt_timed = false;
  hipEvent_t rt_ev[2] = {nullptr, nullptr};
  float last_roundtrip_ms = 0.f;
  std::vector<int32_t> host_queue;  // component ids in launch order (all tiers)
  std::vector<DevDesc> host_desc;   // descriptors in launch order
  ~DeviceBatch();
};

void device_upload(mpld_context* ctx, const Image& im, DeviceBatch& db, const Tune& tune = Tune());
// Enqueues the search of every component on the context stream (no wait).
void device_solve(DeviceBatch& db, uint32_t flags);
// Result of a decomposition from the device records and local colors: maps
// local colors to nodes, fills the component records, recovers the removed
// nodes and computes the Eq. 1 tallies.
void assemble_result(const Graph& g, const Split& s, const Image& im, const mpld_options& opt,
                     const std::vector<DevRecord>& recs, const std::vector<int8_t>& lcol,
                     mpld_result* r, const std::vector<int32_t>* min_nodes = nullptr);

// The whole device solve: image H2D from page-locked memory, the search
// (device_solve with `flags`), records and local colors D2H, between two
// events (read by device_time into last_roundtrip_ms).
void device_roundtrip(DeviceBatch& db, const Image& im, uint32_t flags);
// Reads the last solve's event time if the stream has passed it.
bool device_time(DeviceBatch& db);
// Waits, then copies records and colors back (and, when the batch was
// packed for MPLD_MINIMIZE and min_nodes is given, the minimisation's node
// counts per component: 0 for components off the register tier).
void device_fetch(DeviceBatch& db, std::vector<DevRecord>& recs, std::vector<int8_t>& colors,
                  std::vector<int32_t>* min_nodes = nullptr);

}  // namespace mpld

struct mpld_batch {
  mpld_context* ctx = nullptr;
  mpld::Graph g;
  mpld::Split s;
  mpld_options opt{};
  mpld::Image im;
  mpld::DeviceBatch db;
  bool solved = false;
  bool tuned_from_cache = false;
};

namespace mpld {
// Packs the batch's components with tune `t` (tier of giants, queue order)
// and uploads them (launch geometry).
void batch_pack(mpld_batch* b, const Tune& t);
// Looks the batch's shape up in the tuning cache (path, else $MPLD_TUNE_CACHE);
// true and *t filled on a hit.
bool tune_from_cache(mpld_batch* b, const char* path, Tune* t);
// Device layout-graph builder (graph_device.hip).  own_stream: a stream of
// its own (server front-end workers), else the context's stream.
GraphBuilder* graph_builder_create(mpld_context* ctx, bool own_stream);
void graph_builder_destroy(GraphBuilder* gb);
// Allocates the builder's device and pinned buffers for layouts of up to
// about `nodes` nodes ahead of use (they still grow beyond).
void graph_builder_reserve(GraphBuilder& gb, int32_t nodes);
// Builds the CSR layout graph of `rects` on the device (the host's
// prepare_layout first); se receives the stitch pairs when not null.  With
// `split`, the simplification and sub-graph split (identical to
// simplify_and_split(g, k, simplify)) run on the device too when
// device_split_pays for the graph; returns whether *split was filled.
bool build_layout_graph_device(GraphBuilder& gb, const mpld_rect* rects, int32_t n, int32_t dmin,
                               int32_t split_len, Graph& g, std::vector<int32_t>* se,
                               Split* split = nullptr, int32_t k = 0, bool simplify = true);
// simplify_and_split of a host graph, computed on the device.
void split_graph_device(GraphBuilder& gb, const Graph& g, int32_t k, bool simplify, Split& s);
// Whether the device split is worth it for a graph of n nodes with
// `adj_entries` (= 2 |CE|) adjacency entries: with an average conflict degree
// of at least k most nodes survive the peeling and the components can be
// large, whose BFS runs level by level on one workgroup (a 40k-node
// component: 13.6 ms, against a few ms on the host); below it the peeling
// leaves small components and the device split is about twice as fast.
inline bool device_split_pays(int64_t n, int64_t adj_entries, int32_t k) {
  return adj_entries < (int64_t)k * n;
}

}  // namespace mpld
