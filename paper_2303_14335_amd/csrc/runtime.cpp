// runtime.cpp - device context, exact-cover image packing, upload, tiered
// launches and result download (host side of the decomposer library).
#include "runtime.h"
#include "trace.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

namespace mpld {

void check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  const int32_t code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? MPLD_E_NOMEM
                                                                                   : MPLD_E_DEVICE;
  fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Packing.  Register tier (n <= 64): one uint64 neighbour mask per node.
// LDS tiers: row offsets (n + 1), neighbour ids (2m), largest degree, and
// with the stitch-aware order each node's stitch partner (local id, -1
// none).

void image_add(Image& im, mpld_context* ctx, int32_t n, const int32_t* pairs, int64_t m, int32_t k,
               int64_t budget, uint32_t flags, const int32_t* partner) {
  DevDesc d{};
  d.n = n;
  d.k = k;
  d.budget = budget;
  d.out_off = im.total_nodes;
  const int32_t id = (int32_t)im.desc.size();
  d.comp = id;
  const bool force_lds = flags & MPLD_FORCE_LDS, force_glb = flags & MPLD_FORCE_GLOBAL,
             force_reg = flags & MPLD_FORCE_WAVE, force_dev = flags & MPLD_FORCE_DEVICE;
  const bool stitch = flags & MPLD_STITCH_ORDER;
  const bool minimize = flags & MPLD_MINIMIZE;
  if (minimize && (force_lds || force_glb || force_dev))
    fail(MPLD_E_UNSUPPORTED, "the Eq. 1 minimisation runs on the register tier; a forced LDS, "
                             "global or device tier cannot take it");
  if (minimize) im.minimize = true;
  if (stitch && force_dev)
    fail(MPLD_E_UNSUPPORTED, "the stitch-aware order runs on the register, LDS and big tiers, not "
                             "on the device-wide tier");
  if (n <= 64 && !force_lds && !force_glb && !force_dev) {
    d.nbr_off = (int64_t)im.masks.size();
    im.masks.resize(im.masks.size() + (size_t)n, 0ull);
    im.partner8.resize(im.masks.size(), 0xffu);
    if (stitch) im.stitch = true;
    if (stitch || minimize) {
      if (partner)
        for (int32_t v = 0; v < n; ++v)
          if (partner[v] >= 0) im.partner8[(size_t)d.nbr_off + v] = (uint8_t)partner[v];
    }
    uint64_t* mk = im.masks.data() + d.nbr_off;
    for (int64_t e = 0; e < m; ++e) {
      const int32_t a = pairs[2 * e], b = pairs[2 * e + 1];
      mk[a] |= 1ull << b;
      mk[b] |= 1ull << a;
    }
    im.q_reg.push_back(id);
  } else {
    if (force_reg) fail(MPLD_E_UNSUPPORTED, "register tier takes at most 64 nodes, component has " + std::to_string(n));
    d.nbr_off = (int64_t)im.adj32.size();
    const int64_t adj_words = (int64_t)n + 1 + 2 * m;
    im.adj32.resize(im.adj32.size() + (size_t)adj_words + 1 + (stitch ? (size_t)n : 0u), 0u);
    if (stitch) {
      im.csr_stitch = true;
      uint32_t* pw = im.adj32.data() + d.nbr_off + adj_words + 1;
      for (int32_t v = 0; v < n; ++v) pw[v] = partner && partner[v] >= 0 ? (uint32_t)partner[v] : 0xffffffffu;
    }
    uint32_t* ptr = im.adj32.data() + d.nbr_off;
    uint32_t* ids = ptr + n + 1;
    for (int64_t e = 0; e < m; ++e) {
      ++ptr[pairs[2 * e] + 1];
      ++ptr[pairs[2 * e + 1] + 1];
    }
    uint32_t maxdeg = 0;
    for (int32_t v = 0; v < n; ++v) {
      maxdeg = std::max(maxdeg, ptr[v + 1]);
      ptr[v + 1] += ptr[v];
    }
    std::vector<uint32_t> fill(ptr, ptr + n);
    for (int64_t e = 0; e < m; ++e) {
      const int32_t a = pairs[2 * e], b = pairs[2 * e + 1];
      ids[fill[a]++] = (uint32_t)b;
      ids[fill[b]++] = (uint32_t)a;
    }
    for (int32_t v = 0; v < n; ++v) std::sort(ids + ptr[v], ids + ptr[v + 1]);
    ids[2 * m] = maxdeg;
    const int64_t small = lds_bytes_for(n, k, adj_words, (int32_t)maxdeg, false, stitch);
    const int64_t big = lds_bytes_for(n, k, adj_words, (int32_t)maxdeg, true, stitch);
    const int64_t limit = std::min<int64_t>(kLdsSmallLimit, ctx->lds_per_block);
    im.mark_lds = std::max(im.mark_lds, mark_lds_bytes(n, k));
    if (force_dev) {
      im.dev_stack_words = std::max(im.dev_stack_words, device_tier_stack_words(n, (int32_t)maxdeg));
      im.dev_max_n = std::max(im.dev_max_n, n);
      im.q_dev.push_back(id);
    } else if (!force_glb && small <= limit && n <= kLds1MaxN) {
      im.lds_bytes_small = std::max(im.lds_bytes_small, small);
      im.q_lds.push_back(id);
    } else if (big <= ctx->lds_per_block) {
      im.lds_bytes_big = std::max(im.lds_bytes_big, big);
      const int64_t wide = lds_wide_bytes(n, k, adj_words, (int32_t)maxdeg, stitch);
      if (im.big_bytes_wg.size() <= (size_t)id) {
        im.big_bytes_wg.resize((size_t)id + 1, 0);
        im.big_bytes_wide.resize((size_t)id + 1, -1);
      }
      im.big_bytes_wg[(size_t)id] = big;
      im.big_bytes_wide[(size_t)id] = wide > ctx->lds_per_block ? -1 : wide;
      im.big_stack_words = std::max(im.big_stack_words, lds_stack_words(n, k, adj_words));
      im.big_max_n = std::max(im.big_max_n, n);
      im.q_big.push_back(id);
    } else {
      fail(MPLD_E_UNSUPPORTED, "component of " + std::to_string(n) + " nodes needs " +
                                   std::to_string(big) + " bytes of LDS, more than the " +
                                   std::to_string(ctx->lds_per_block) + " a workgroup gets");
    }
  }
  im.desc.push_back(d);
  im.total_nodes += n;
  im.max_size = std::max(im.max_size, n);
  im.core_edges += m;
}

void image_finish(Image& im, int order) {
  auto by_size = [&](int32_t a, int32_t b) {
    if (im.desc[a].n != im.desc[b].n)
      return order == 1 ? im.desc[a].n < im.desc[b].n : im.desc[a].n > im.desc[b].n;
    return a < b;
  };
  std::sort(im.q_reg.begin(), im.q_reg.end(), by_size);
  std::sort(im.q_lds.begin(), im.q_lds.end(), by_size);
  std::sort(im.q_big.begin(), im.q_big.end(), by_size);
  std::sort(im.q_dev.begin(), im.q_dev.end(), by_size);
}

// ---------------------------------------------------------------------------

DeviceBatch::~DeviceBatch() {
  if (graph) hipGraphExecDestroy(graph);
  for (hipEvent_t e : rt_ev)
    if (e) (void)hipEventDestroy(e);
}

static int blocks_for_lds(mpld_context* ctx, int lds_bytes) {
  // one wave per workgroup: bounded by LDS and by 32 waves per CU
  const int per_cu_lds = 160 * 1024;
  int by_lds = lds_bytes > 0 ? per_cu_lds / lds_bytes : 32;
  by_lds = std::max(1, std::min(by_lds, 32));
  return by_lds * ctx->num_cus;
}

void device_upload(mpld_context* ctx, const Image& im, DeviceBatch& db, const Tune& tune) {
  db.ctx = ctx;
  db.tune = tune;
  if (db.graph) {
    (void)hipGraphExecDestroy(db.graph);
    db.graph = nullptr;
    db.graph_flags = 0xffffffffu;
  }
  db.k = im.desc.empty() ? 3 : im.desc[0].k;
  db.num_comps = (int32_t)im.desc.size();
  db.total_nodes = im.total_nodes;
  db.n_reg = (int32_t)im.q_reg.size();
  db.n_lds = (int32_t)im.q_lds.size();
  db.n_big = (int32_t)im.q_big.size();
  db.n_dev = (int32_t)im.q_dev.size();
  {
    // device-wide tier: each search node costs two grid barriers, whose
    // cost grows with the workgroups (about 3 us at 64, 12 us at 256),
    // while the scan per node shrinks with them: about sqrt(n) / 12
    // workgroups, at least 8 (per node on n = 10^4: 3.6 us at 8, 4.6 at 16,
    // 5.9 at 32, 24.9 at 256), and enough that a block's slice fits in 48 KB
    const int32_t n = std::max(1, im.dev_max_n);
    int grid = std::max(8, (int)std::lround(std::sqrt((double)n) / 12.0));
    while (grid < ctx->num_cus && device_tier_lds_bytes(n, grid) > 48 * 1024) grid *= 2;
    db.grid_dev = std::min(grid, ctx->num_cus);
  }
  db.lds_dev = device_tier_lds_bytes(std::max(1, im.dev_max_n), db.grid_dev);
  db.lds_small = (int)im.lds_bytes_small;
  // big tier: the components whose lists fit LDS run on one wave (the
  // one-wave layout, launched with waves = 0) and come first; the others
  // run on a workgroup sharing the column scan
  std::vector<int32_t> q_big;
  q_big.reserve(im.q_big.size());
  int64_t wide_bytes = 0, wg_bytes = 0;
  int32_t wg_max_n = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int32_t c : im.q_big) {
      const int64_t wb = im.big_bytes_wide[(size_t)c];
      const bool one_wave = tune.big_one_wave && wb >= 0;
      if (one_wave != (pass == 0)) continue;
      q_big.push_back(c);
      if (one_wave) {
        wide_bytes = std::max(wide_bytes, wb);
      } else {
        wg_bytes = std::max(wg_bytes, im.big_bytes_wg[(size_t)c]);
        wg_max_n = std::max(wg_max_n, im.desc[(size_t)c].n);
      }
    }
  db.n_wide = 0;
  for (int32_t c : q_big)
    if (tune.big_one_wave && im.big_bytes_wide[(size_t)c] >= 0) ++db.n_wide;
  db.lds_wide = (int)wide_bytes;
  db.lds_big = (int)wg_bytes;
  db.big_waves = lds_big_waves(std::max(1, wg_max_n));
  db.mark_lds = im.mark_lds;
  db.big_stack_words = (uint64_t)im.big_stack_words;
  {
    const int wpb = std::max(1, std::min(4, tune.waves_per_block));
    const int cap = tune.max_blocks > 0 ? tune.max_blocks : ctx->num_cus * ctx->reg_blocks_per_cu * (4 / wpb);
    db.grid_reg = std::max(1, std::min((db.n_reg + wpb - 1) / wpb, cap));
  }
  db.grid_lds = std::max(1, std::min(db.n_lds, blocks_for_lds(ctx, db.lds_small)));
  {
    const int32_t n_wg = db.n_big - db.n_wide;
    db.grid_wide = std::max(1, std::min(db.n_wide, blocks_for_lds(ctx, db.lds_wide)));
    db.grid_big = std::max(1, std::min(n_wg, blocks_for_lds(ctx, db.lds_big)));
    // subtree tasks: k per big component, each on a workgroup of its own;
    // the stack areas serve the launches of either layout, one at a time
    db.grid_big_tasks = std::max({db.grid_wide, db.grid_big,
                                  std::min(db.k * db.n_wide, blocks_for_lds(ctx, db.lds_wide)),
                                  std::min(db.k * n_wg, blocks_for_lds(ctx, db.lds_big))});
  }

  db.host_queue.clear();
  db.host_queue.insert(db.host_queue.end(), im.q_reg.begin(), im.q_reg.end());
  db.host_queue.insert(db.host_queue.end(), im.q_lds.begin(), im.q_lds.end());
  db.host_queue.insert(db.host_queue.end(), q_big.begin(), q_big.end());
  db.host_queue.insert(db.host_queue.end(), im.q_dev.begin(), im.q_dev.end());

  std::vector<DevDesc>& ordered = db.host_desc;
  ordered.clear();
  ordered.reserve(db.host_queue.size());
  for (int32_t c : db.host_queue) ordered.push_back(im.desc[c]);
  // root split: the largest register-tier items (a prefix of the launch
  // order when it is largest first) get a workgroup each, at most
  // root_split_max of them (0: every item of at least root_split_min_n nodes)
  db.reg_heavy = 0;
  if (db.tune.root_split && db.tune.order == 0 && db.tune.waves_per_block == 4) {
    const int32_t most = db.tune.root_split_max > 0 ? db.tune.root_split_max : db.n_reg;
    while (db.reg_heavy < std::min(most, db.n_reg) &&
           ordered[(size_t)db.reg_heavy].n >= db.tune.root_split_min_n)
      ++db.reg_heavy;
  }
  // register-tier items: descriptor and masks together, in launch order
  int32_t max_reg_n = 0;
  for (int32_t i = 0; i < db.n_reg; ++i) max_reg_n = std::max(max_reg_n, ordered[(size_t)i].n);
  db.reg_width = reg_item_width(max_reg_n);
  db.reg_stitch = im.stitch;
  db.csr_stitch = im.csr_stitch;
  const RegItems shape = db.reg_items();
  const size_t stride = shape.stride;
  std::vector<uint8_t> items(stride * (size_t)db.n_reg, 0);
  for (int32_t i = 0; i < db.n_reg; ++i) {
    uint8_t* it = items.data() + stride * (size_t)i;
    const DevDesc& d = ordered[(size_t)i];
    std::memcpy(it, &d, sizeof(DevDesc));
    std::memcpy(it + kRegItemHead, im.masks.data() + d.nbr_off, sizeof(uint64_t) * (size_t)d.n);
    if (shape.part_off) {
      std::memset(it + shape.part_off, 0xff, db.reg_width);
      std::memcpy(it + shape.part_off, im.partner8.data() + d.nbr_off, (size_t)d.n);
    }
  }

  db.desc.alloc(ctx, sizeof(DevDesc) * ordered.size());
  db.regitems.alloc(ctx, items.size());
  db.adj32.alloc(ctx, sizeof(uint32_t) * im.adj32.size());
  db.counters.alloc(ctx, sizeof(int32_t) * 8);
  db.recs.alloc(ctx, sizeof(DevRecord) * im.desc.size());
  db.colors.alloc(ctx, (size_t)im.total_nodes);
  db.gstack.release();
  db.dev_keys.release();
  db.dev_stacks.release();
  if (db.n_big)
    db.gstack.alloc(ctx, sizeof(uint64_t) * db.big_stack_words * (size_t)db.grid_big_tasks);
  if (db.n_dev) {
    db.dev_keys.alloc(ctx, sizeof(uint64_t) * 4);
    db.dev_stacks.alloc(ctx, sizeof(uint64_t) * (size_t)im.dev_stack_words * (size_t)db.grid_dev);
  }

  hipStream_t s = ctx->stream;
  if (!ordered.empty())
    check_hip(hipMemcpyAsync(db.desc.p, ordered.data(), sizeof(DevDesc) * ordered.size(),
                             hipMemcpyHostToDevice, s), "upload descriptors");
  if (!items.empty())
    check_hip(hipMemcpyAsync(db.regitems.p, items.data(), items.size(),
                             hipMemcpyHostToDevice, s), "upload register items");
  if (!im.adj32.empty())
    check_hip(hipMemcpyAsync(db.adj32.p, im.adj32.data(), sizeof(uint32_t) * im.adj32.size(),
                             hipMemcpyHostToDevice, s), "upload adjacency");
  check_hip(hipMemsetAsync(db.counters.p, 0, sizeof(int32_t) * 8, s), "clear counters");
  if (db.n_dev)
    check_hip(hipMemsetAsync(db.dev_keys.p, 0xff, sizeof(uint64_t) * 4, s), "clear keys");
  check_hip(hipStreamSynchronize(s), "upload");
  db.host_items = std::move(items);
  db.rt_ready = false;
  db.partners.release();
  db.min_out.release();
  if (im.minimize) {
    db.partners.alloc(ctx, std::max<size_t>(im.partner8.size(), 1));
    db.min_out.alloc(ctx, sizeof(int32_t) * std::max<size_t>(im.desc.size(), 1));
    if (!im.partner8.empty())
      check_hip(hipMemcpyAsync(db.partners.p, im.partner8.data(), im.partner8.size(),
                               hipMemcpyHostToDevice, s), "upload stitch partners");
    check_hip(hipStreamSynchronize(s), "upload");
  }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

void device_roundtrip(DeviceBatch& db, const Image& im, uint32_t flags) {
  mpld_context* ctx = db.ctx;
  hipStream_t s = ctx->stream;
  const size_t nd = sizeof(DevDesc) * db.host_desc.size(), ni = db.host_items.size(),
               na = sizeof(uint32_t) * im.adj32.size();
  const size_t nr = sizeof(DevRecord) * (size_t)db.num_comps, nc = (size_t)db.total_nodes;
  if (!db.rt_ready) {
    if (!db.rt_up.reserve(align256(nd) + align256(ni) + align256(na) + 256) ||
        !db.rt_down.reserve(align256(nr) + align256(nc) + 256))
      fail(MPLD_E_NOMEM, "page-locked staging of the round trip");
    auto* up = db.rt_up.as<uint8_t>();
    if (nd) std::memcpy(up, db.host_desc.data(), nd);
    if (ni) std::memcpy(up + align256(nd), db.host_items.data(), ni);
    if (na) std::memcpy(up + align256(nd) + align256(ni), im.adj32.data(), na);
    for (hipEvent_t& e : db.rt_ev)
      if (!e) check_hip(hipEventCreate(&e), "round-trip event");
    db.rt_ready = true;
  }
  const auto* up = db.rt_up.as<uint8_t>();
  auto* down = db.rt_down.as<uint8_t>();
  db.rt_timed = false;
  check_hip(hipEventRecord(db.rt_ev[0], s), "event");
  if (nd) check_hip(hipMemcpyAsync(db.desc.p, up, nd, hipMemcpyHostToDevice, s), "upload descriptors");
  if (ni)
    check_hip(hipMemcpyAsync(db.regitems.p, up + align256(nd), ni, hipMemcpyHostToDevice, s),
              "upload register items");
  if (na)
    check_hip(hipMemcpyAsync(db.adj32.p, up + align256(nd) + align256(ni), na,
                             hipMemcpyHostToDevice, s), "upload adjacency");
  device_solve(db, flags);
  if (nr) check_hip(hipMemcpyAsync(down, db.recs.p, nr, hipMemcpyDeviceToHost, s), "download records");
  if (nc)
    check_hip(hipMemcpyAsync(down + align256(nr), db.colors.p, nc, hipMemcpyDeviceToHost, s),
              "download colors");
  check_hip(hipEventRecord(db.rt_ev[1], s), "event");
  db.rt_timed = true;
}

// split: the LDS and big tiers are left to csr_split (subtree tasks).
// mark: the register-tier kernel also marks the components its search
// leaves without a solution (uncapped launches only).
static void enqueue_batched(DeviceBatch& db, bool trace, uint64_t cap, hipStream_t s,
                            bool split = false, bool mark = false) {
  const auto* desc = db.desc.as<DevDesc>();
  const RegItems items = db.reg_items();
  const auto* adj = db.adj32.as<uint32_t>();
  auto* cnt = db.counters.as<int32_t>();
  auto* recs = db.recs.as<DevRecord>();
  auto* colors = db.colors.as<int8_t>();
  auto* gstack = db.gstack.as<uint64_t>();
  db.launches = 0;
  if (db.n_reg) {
    const int32_t heavy = cap == ~0ull ? db.reg_heavy : 0;
    const int grid = heavy ? heavy + (db.n_reg - heavy + 3) / 4 : db.grid_reg;
    check_hip(launch_reg_batched(trace, db.k, grid, db.tune.waves_per_block, items, db.n_reg, cnt,
                                 recs, colors, cap, heavy, (uint32_t)db.tune.root_split_chunk,
                                 mark && cap == ~0ull, s),
              "register-tier launch");
    ++db.launches;
  }
  if (db.n_lds && !split) {
    check_hip(launch_lds_batched(trace, false, db.csr_stitch, 1, db.grid_lds, db.lds_small, desc + db.n_reg, adj,
                                 db.n_lds, cnt + 1, nullptr, 0, recs, colors, s),
              "LDS-tier launch");
    ++db.launches;
  }
  if (db.n_wide && !split) {   // one-wave layout
    check_hip(launch_lds_batched(trace, true, db.csr_stitch, 0, db.grid_wide, db.lds_wide,
                                 desc + db.n_reg + db.n_lds, adj, db.n_wide, cnt + 3, gstack,
                                 db.big_stack_words, recs, colors, s),
              "big-tier launch (one wave)");
    ++db.launches;
  }
  if (db.n_big > db.n_wide && !split) {   // workgroup layout
    check_hip(launch_lds_batched(trace, true, db.csr_stitch, db.big_waves, db.grid_big, db.lds_big,
                                 desc + db.n_reg + db.n_lds + db.n_wide, adj, db.n_big - db.n_wide,
                                 cnt + 2, gstack, db.big_stack_words, recs, colors, s),
              "big-tier launch (workgroup)");
    ++db.launches;
  }
  for (int32_t i = 0; i < db.n_dev; ++i) {   // one cooperative launch per giant
    check_hip(launch_device_tier(trace, db.grid_dev, db.lds_dev, desc + db.n_reg + db.n_lds + db.n_big + i,
                                 adj, db.dev_keys.as<unsigned long long>(),
                                 db.dev_stacks.as<uint64_t>(), recs, colors, s),
              "device-tier launch");
    ++db.launches;
  }
}

// ---------------------------------------------------------------------------
// Heavy-component engine.  Register-tier components still running after the
// capped first pass are searched as ordered sequences of items: node counts
// (visited in the top levels of a split) and subtree tasks.  Each round runs
// every pending task with a node cap on its own wave; a task that finishes
// reports its exact node count (and its solution), a capped task is split a
// few levels further down into subtasks in search order.  Scanning a
// component's items in order reproduces the sequential search: counts add
// up until the first subtree holding a solution (FEASIBLE, nodes = the sum
// through it) or to the end (INFEASIBLE); a sum passing the budget means the
// sequential search was cut inside, and that component is re-run
// sequentially to get its exact stopping point.

namespace {

constexpr int32_t kHeavyMaxTasks = 16384;   // tasks per round

struct HTask {
  int32_t hc;            // heavy component index
  int32_t depth;
  uint16_t rows[64];
  int32_t status = -2;   // -2 not run yet, -1 capped (being replaced), else final
  uint64_t nodes = 0;
  int8_t sol[64];
};
struct HItem {
  int32_t task;          // -1: a node count
  uint64_t count;
};
struct HComp {
  int32_t item;          // launch-ordered descriptor index
  std::vector<HItem> seq;
  size_t pos = 0;        // seq[0 .. pos) is final and sums to acc
  uint64_t acc = 0;
  bool done = false, rerun = false;
  DevRecord rec{};
  std::vector<int8_t> colors;
};

int split_levels(int k) { return k <= 3 ? 4 : (k == 4 ? 3 : 2); }

// Scans a component's items from its first unresolved one (everything
// before it is final and already summed); true once its sequential result
// is known.
bool resolve(HComp& hc, const DevDesc& d, const std::vector<HTask>& tasks) {
  const uint64_t budget = (uint64_t)d.budget;
  uint64_t& acc = hc.acc;
  for (; hc.pos < hc.seq.size(); ++hc.pos) {
    const HItem& it = hc.seq[hc.pos];
    if (it.task < 0) {
      if (acc + it.count > budget) { hc.rerun = true; return true; }
      acc += it.count;
      continue;
    }
    const HTask& t = tasks[it.task];
    if (t.status < 0) return false;
    if (acc + t.nodes > budget) { hc.rerun = true; return true; }
    acc += t.nodes;
    if (t.status == MPLD_FEASIBLE) {
      hc.rec.status = MPLD_FEASIBLE;
      hc.rec.depth = d.n;
      hc.rec.nodes = acc;
      hc.rec.hash = 0;
      hc.colors.assign(t.sol, t.sol + d.n);
      return true;
    }
  }
  hc.rec.status = MPLD_INFEASIBLE;
  hc.rec.depth = 0;
  hc.rec.nodes = acc;
  hc.rec.hash = 0;
  hc.colors.assign((size_t)d.n, -1);
  return true;
}

}  // namespace

// Device-resident rounds.  Capacities bound the engine's memory; a split
// that does not fit (or a component whose explored nodes pass twice its
// budget) leaves that component to a sequential re-run, which is exact.
constexpr int32_t kEngineTaskCap = 1 << 18;   // tasks (144 B + an 88 B result block each)
constexpr int32_t kEnginePoolCap = 1 << 21;   // split items (16 B each)
constexpr int32_t kEngineMaxRounds = 96;      // depth <= 64: far more than needed
constexpr int32_t kEngineRoundsPerCheck = 3;  // rounds enqueued between looks at the head

static void heavy_engine_device(DeviceBatch& db, bool trace) {
  mpld_context* ctx = db.ctx;
  hipStream_t s = ctx->stream;
  db.sp_rounds = db.sp_tasks_run = db.sp_heavy = db.sp_reruns = 0;
  // which register-tier components stopped at the first cap
  if (!db.sp_host_recs.reserve(sizeof(DevRecord) * (size_t)std::max(1, db.num_comps)))
    fail(MPLD_E_NOMEM, "heavy-component engine: pinned host memory");
  const DevRecord* recs = db.sp_host_recs.as<DevRecord>();
  check_hip(hipMemcpyAsync(db.sp_host_recs.p, db.recs.p, sizeof(DevRecord) * (size_t)db.num_comps,
                           hipMemcpyDeviceToHost, s), "heavy: records");
  check_hip(hipStreamSynchronize(s), "heavy: first pass");
  std::vector<int32_t> heavy;   // launch-order register items
  for (int32_t i = 0; i < db.n_reg; ++i)
    if (recs[db.host_desc[i].comp].status < 0) heavy.push_back(i);
  if (heavy.empty()) return;
  const int32_t H = (int32_t)heavy.size();
  if (H > kEngineTaskCap) fail(MPLD_E_INTERNAL, "heavy-component engine: too many heavy components");
  db.sp_heavy = H;
  int levels = db.tune.heavy_levels > 0 ? db.tune.heavy_levels : split_levels(db.k);
  int64_t kp = 1;
  for (int l = 0; l < levels; ++l) kp *= db.k;
  while (levels > 1 && kp > 512) {
    kp /= db.k;
    --levels;
  }
  // device areas: head + per-component explored nodes and limits; tasks,
  // result blocks, item pool
  const size_t meta_bytes = sizeof(EngineHead) + 16 * (size_t)H;
  if (db.en_meta.bytes < meta_bytes) db.en_meta.alloc(ctx, meta_bytes);
  if (!db.en_tasks.p) {
    db.en_tasks.alloc(ctx, sizeof(EngineTask) * (size_t)kEngineTaskCap);
    db.en_blocks.alloc(ctx, (size_t)kSplitBlockBytes * kEngineTaskCap);
    db.en_pool.alloc(ctx, sizeof(EngineItem) * (size_t)kEnginePoolCap);
  }
  auto* head = db.en_meta.as<EngineHead>();
  auto* hc_nodes = reinterpret_cast<unsigned long long*>(db.en_meta.as<uint8_t>() + sizeof(EngineHead));
  auto* hc_limit = reinterpret_cast<uint64_t*>(db.en_meta.as<uint8_t>() + sizeof(EngineHead) + 8 * (size_t)H);
  // staging: the meta area, then the root tasks
  const size_t roots_at = (meta_bytes + 255) / 256 * 256;
  const size_t stage_bytes = roots_at + sizeof(EngineTask) * (size_t)H;
  if (!db.sp_host_tasks.reserve(stage_bytes)) fail(MPLD_E_NOMEM, "heavy-component engine: pinned host memory");
  uint8_t* st = db.sp_host_tasks.as<uint8_t>();
  std::memset(st, 0, stage_bytes);
  EngineHead* h0 = reinterpret_cast<EngineHead*>(st);
  h0->alloc = H;
  uint64_t* lim = reinterpret_cast<uint64_t*>(st + sizeof(EngineHead) + 8 * (size_t)H);
  EngineTask* roots = reinterpret_cast<EngineTask*>(st + roots_at);
  for (int32_t h = 0; h < H; ++h) {
    const uint64_t budget = (uint64_t)db.host_desc[heavy[h]].budget;
    lim[h] = budget > (UINT64_MAX / 4) ? UINT64_MAX : 2 * budget + (uint64_t)db.tune.heavy_round_cap;
    roots[h].item = heavy[h];
    roots[h].depth = 0;
    roots[h].hc = h;
    roots[h].skip = 0;
  }
  check_hip(hipMemcpyAsync(db.en_meta.p, st, meta_bytes, hipMemcpyHostToDevice, s), "heavy: engine head");
  check_hip(hipMemcpyAsync(db.en_tasks.p, roots, sizeof(EngineTask) * (size_t)H, hipMemcpyHostToDevice, s),
            "heavy: root tasks");
  const int grid = std::max(1, ctx->num_cus * ctx->reg_blocks_per_cu);
  auto* tasks = db.en_tasks.as<EngineTask>();
  auto* blocks = db.en_blocks.as<uint8_t>();
  auto* pool = db.en_pool.as<EngineItem>();
  // head read back into the result staging area
  if (!db.sp_host_out.reserve(sizeof(EngineHead))) fail(MPLD_E_NOMEM, "heavy-component engine: pinned host memory");
  EngineHead hh{};
  for (int32_t r = 0;;) {
    for (int i = 0; i < kEngineRoundsPerCheck; ++i, ++r) {
      check_hip(launch_engine_advance(head, kEngineTaskCap, s), "heavy: advance");
      check_hip(launch_engine_round(db.k, grid, head, tasks, kEngineTaskCap, blocks, pool, kEnginePoolCap,
                                    db.reg_items(), hc_nodes, hc_limit,
                                    (uint64_t)db.tune.heavy_round_cap, (uint32_t)levels, trace, s),
                "heavy: round");
    }
    check_hip(hipMemcpyAsync(db.sp_host_out.p, head, sizeof(EngineHead), hipMemcpyDeviceToHost, s),
              "heavy: engine head");
    check_hip(hipStreamSynchronize(s), "heavy: rounds");
    std::memcpy(&hh, db.sp_host_out.p, sizeof(hh));
    if (std::min(hh.alloc, kEngineTaskCap) == hh.end) break;   // the last round added no task
    if (r >= kEngineMaxRounds) fail(MPLD_E_INTERNAL, "heavy-component engine: too many rounds");
  }
  const int32_t ntasks = std::min(hh.alloc, kEngineTaskCap);
  const int32_t nitems = std::min(hh.pool, kEnginePoolCap);
  db.sp_rounds = hh.rounds;
  db.sp_tasks_run = ntasks;
  const size_t blocks_bytes = (size_t)kSplitBlockBytes * (size_t)ntasks;
  const size_t items_at = (blocks_bytes + 255) / 256 * 256;
  if (!db.sp_host_out.reserve(items_at + sizeof(EngineItem) * (size_t)nitems))
    fail(MPLD_E_NOMEM, "heavy-component engine: pinned host memory");
  check_hip(hipMemcpyAsync(db.sp_host_out.p, blocks, blocks_bytes, hipMemcpyDeviceToHost, s),
            "heavy: result blocks");
  if (nitems > 0)
    check_hip(hipMemcpyAsync(db.sp_host_out.as<uint8_t>() + items_at, pool, sizeof(EngineItem) * (size_t)nitems,
                             hipMemcpyDeviceToHost, s), "heavy: items");
  check_hip(hipStreamSynchronize(s), "heavy: results");
  // one sequential copy out of the page-locked staging area: the walk
  // below reads the blocks and items in tree order, and scattered reads of
  // page-locked memory cost several times more than of ordinary memory
  db.sp_host_copy.resize(items_at + sizeof(EngineItem) * (size_t)nitems);
  std::memcpy(db.sp_host_copy.data(), db.sp_host_out.p, db.sp_host_copy.size());
  const uint8_t* hb = db.sp_host_copy.data();
  const EngineItem* hi = reinterpret_cast<const EngineItem*>(hb + items_at);
  auto result = [&](int32_t t) {
    SplitResult r;
    std::memcpy(&r, hb + (size_t)kSplitBlockBytes * (size_t)t, sizeof(r));
    return r;
  };
  auto solution = [&](int32_t t) { return reinterpret_cast<const int8_t*>(hb + (size_t)kSplitBlockBytes * t + kSplitSolOffset); };
  // each component in search order: a depth-first walk of its task tree;
  // the trace hash appends each finished task's and each item's seg hash
  std::vector<HeavyWrite> wb;
  std::vector<int32_t> rerun;
  struct Walk { int32_t task, next; };
  std::vector<Walk> stack;
  for (int32_t h = 0; h < H; ++h) {
    const DevDesc& d = db.host_desc[heavy[h]];
    const uint64_t budget = (uint64_t)d.budget;
    uint64_t acc = 0, hash = 0;
    bool redo = false, found = false;
    const int8_t* sol = nullptr;
    stack.clear();
    stack.push_back({h, -1});
    while (!stack.empty() && !redo && !found) {
      Walk& w = stack.back();
      const SplitResult r = result(w.task);
      if (w.next < 0) {   // first visit
        if (r.status == MPLD_INFEASIBLE || r.status == MPLD_FEASIBLE) {
          acc += r.nodes;
          if (trace) hash = trace_concat(hash, r.hash, r.nodes);
          if (acc > budget) { redo = true; break; }
          if (r.status == MPLD_FEASIBLE) { found = true; sol = solution(w.task); break; }
          stack.pop_back();
          continue;
        }
        if (r.status != -1) { redo = true; break; }   // not split: budget or space
        if (r.nitems < 1 || (int64_t)r.item_off + r.nitems > nitems)
          fail(MPLD_E_INTERNAL, "heavy-component engine: bad task result");
        w.next = 0;
      }
      if (w.next >= r.nitems) { stack.pop_back(); continue; }
      const EngineItem it = hi[r.item_off + (uint32_t)w.next++];
      acc += it.seg;
      if (trace) hash = trace_concat(hash, it.hash, it.seg);
      if (acc > budget) { redo = true; break; }
      if (it.child == kEngineItemEnd) { stack.pop_back(); continue; }
      if (it.child == kEngineItemSolution) { found = true; sol = solution(w.task); break; }
      if (it.child < 0 || it.child >= ntasks) fail(MPLD_E_INTERNAL, "heavy-component engine: bad subtask");
      const int32_t child = it.child;
      stack.push_back({child, -1});   // invalidates w
    }
    if (redo) { rerun.push_back(heavy[h]); continue; }
    HeavyWrite e{};
    e.comp = d.comp;
    e.out_off = d.out_off;
    e.n = d.n;
    e.rec.status = found ? MPLD_FEASIBLE : MPLD_INFEASIBLE;
    e.rec.depth = found ? d.n : 0;
    e.rec.nodes = acc;
    e.rec.hash = trace ? hash : 0;
    if (found) std::memcpy(e.colors, sol, (size_t)d.n);
    else std::memset(e.colors, -1, (size_t)d.n);
    wb.push_back(e);
  }
  for (int32_t item : rerun) {
    ++db.sp_reruns;
    check_hip(launch_reg_single(trace, db.k, db.reg_items(), item, db.recs.as<DevRecord>(),
                                db.colors.as<int8_t>(), s), "heavy: sequential re-run");
  }
  if (!wb.empty()) {
    if (!db.sp_host_writes.reserve(sizeof(HeavyWrite) * wb.size()))
      fail(MPLD_E_NOMEM, "heavy-component engine: pinned host memory");
    if (db.sp_writes.bytes < sizeof(HeavyWrite) * wb.size())
      db.sp_writes.alloc(ctx, sizeof(HeavyWrite) * wb.size());
    std::memcpy(db.sp_host_writes.p, wb.data(), sizeof(HeavyWrite) * wb.size());
    check_hip(hipMemcpyAsync(db.sp_writes.p, db.sp_host_writes.p, sizeof(HeavyWrite) * wb.size(),
                             hipMemcpyHostToDevice, s), "heavy: write-back upload");
    check_hip(launch_heavy_writeback(db.sp_writes.as<HeavyWrite>(), (int32_t)wb.size(),
                                     db.recs.as<DevRecord>(), db.colors.as<int8_t>(), s),
              "heavy: write-back");
  }
  check_hip(hipStreamSynchronize(s), "heavy: write back");
}

// LDS-tier and big-tier components as subtree tasks.  At the
// root every column has all k rows, so the root column is node 0 and the
// root node's children are its k rows; task (component, c) searches the
// subtree of root row c with budget B - 1 (the root node is counted once,
// here).  The sequential result follows from the tasks in row order: acc
// starts at 1; an exhausted subtree adds its count and the next row
// follows; a subtree holding a solution ends the search (FEASIBLE, acc +
// its count, its depth and colors); the budget reached exactly before a
// row means the next node entry fails its test (BUDGET at depth 1); a
// subtree whose count would cross the budget (or that ran into it) is where
// the sequential search stops: it is searched again with budget B - acc for
// the depth at the stop (row 0's task already ran with exactly that
// budget).  Every row exhausted: INFEASIBLE with acc nodes.  The trace hash
// follows the same order: the root node's, then each counted subtree's
// appended (trace S then T: h(S) B^|T| + h(T)).
static void csr_split(DeviceBatch& db, bool trace) {
  const int32_t first = db.n_reg, count = db.n_lds + db.n_big;
  if (count == 0) return;
  mpld_context* ctx = db.ctx;
  hipStream_t s = ctx->stream;
  struct Comp {
    int32_t pos = 0;      // launch position
    uint64_t acc = 1;
    uint64_t hash = 0;    // trace hash of the nodes counted in acc
    int32_t rerun_row = -1;
    bool done = false;
    LdsResolved res{};
  };
  std::vector<Comp> comps((size_t)count);
  std::vector<LdsTask> tasks;
  std::vector<int32_t> task_of((size_t)count, -1);   // first phase-1 task of each component
  int64_t col = 0;
  for (int32_t i = 0; i < count; ++i) {
    Comp& cp = comps[(size_t)i];
    cp.pos = first + i;
    const DevDesc& d = db.host_desc[(size_t)cp.pos];
    cp.res.comp = d.comp;
    cp.res.out_off = d.out_off;
    cp.res.n = d.n;
    cp.res.src_off = -1;
    if (d.n == 0) {   // no column: the root is a solution
      cp.res.rec.status = MPLD_FEASIBLE;
      cp.res.rec.nodes = 1;
      cp.res.rec.depth = 0;
      cp.res.rec.hash = trace ? trace_node(0, 0u, 0xffffffffu, 0xffffffffu, 0u) : 0;
      cp.done = true;
      continue;
    }
    // the root node: column 0 (every column has all k rows), entering row none
    cp.hash = trace_node(0, 0u, 0xffffffffu, 0u, (uint32_t)d.k);
    cp.res.rec.hash = trace ? cp.hash : 0;
    if (d.budget == 1) {   // the root takes the whole budget
      cp.res.rec.status = MPLD_BUDGET_EXHAUSTED;
      cp.res.rec.nodes = 1;
      cp.res.rec.depth = 1;
      cp.done = true;
      continue;
    }
    task_of[(size_t)i] = (int32_t)tasks.size();
    for (int32_t c = 0; c < d.k; ++c) {
      tasks.push_back(LdsTask{cp.pos, c, d.budget - 1, col});
      col += d.n;
    }
  }
  // Runs a task list (LDS-tier tasks before big-tier ones, as built) and
  // returns their records; task colors land in ct_colors at their col_off.
  auto run = [&](const std::vector<LdsTask>& list, int64_t colors_bytes) {
    std::vector<DevRecord> out(list.size());
    if (list.empty()) return out;
    size_t nsmall = 0, nwide = 0;
    while (nsmall < list.size() && list[nsmall].item < first + db.n_lds) ++nsmall;
    while (nsmall + nwide < list.size() && list[nsmall + nwide].item < first + db.n_lds + db.n_wide)
      ++nwide;
    const size_t tb = sizeof(LdsTask) * list.size(), rb = sizeof(DevRecord) * list.size();
    if (db.ct_tasks.bytes < tb) db.ct_tasks.alloc(ctx, tb);
    if (db.ct_recs.bytes < rb) db.ct_recs.alloc(ctx, rb);
    if (db.ct_colors.bytes < (size_t)std::max<int64_t>(colors_bytes, 1))
      db.ct_colors.alloc(ctx, (size_t)std::max<int64_t>(colors_bytes, 1));
    if (!db.ct_host.reserve(std::max(tb, rb))) fail(MPLD_E_NOMEM, "subtree tasks: pinned host memory");
    std::memcpy(db.ct_host.p, list.data(), tb);
    check_hip(hipMemcpyAsync(db.ct_tasks.p, db.ct_host.p, tb, hipMemcpyHostToDevice, s),
              "subtree tasks: upload");
    const auto* dt = db.ct_tasks.as<LdsTask>();
    auto* drec = db.ct_recs.as<DevRecord>();
    if (nsmall)
      check_hip(launch_lds_tasks(trace, false, db.csr_stitch, 1,
                                 std::max(1, std::min((int)nsmall, blocks_for_lds(ctx, db.lds_small))),
                                 db.lds_small, db.desc.as<DevDesc>(), db.adj32.as<uint32_t>(), dt,
                                 (int32_t)nsmall, nullptr, 0, drec, db.ct_colors.as<int8_t>(), s),
                "subtree tasks (LDS tier)");
    if (nwide)
      check_hip(launch_lds_tasks(trace, true, db.csr_stitch, 0,
                                 std::max(1, std::min({(int)nwide, db.grid_big_tasks,
                                                       blocks_for_lds(ctx, db.lds_wide)})),
                                 db.lds_wide, db.desc.as<DevDesc>(), db.adj32.as<uint32_t>(),
                                 dt + nsmall, (int32_t)nwide, db.gstack.as<uint64_t>(),
                                 db.big_stack_words, drec + nsmall, db.ct_colors.as<int8_t>(), s),
                "subtree tasks (big tier, one wave)");
    const size_t nbig = nsmall + nwide;
    if (nbig < list.size())
      check_hip(launch_lds_tasks(trace, true, db.csr_stitch, db.big_waves,
                                 std::max(1, std::min({(int)(list.size() - nbig), db.grid_big_tasks,
                                                       blocks_for_lds(ctx, db.lds_big)})),
                                 db.lds_big, db.desc.as<DevDesc>(), db.adj32.as<uint32_t>(),
                                 dt + nbig, (int32_t)(list.size() - nbig), db.gstack.as<uint64_t>(),
                                 db.big_stack_words, drec + nbig, db.ct_colors.as<int8_t>(), s),
                "subtree tasks (big tier, workgroup)");
    check_hip(hipMemcpyAsync(db.ct_host.p, drec, rb, hipMemcpyDeviceToHost, s), "subtree tasks: records");
    check_hip(hipStreamSynchronize(s), "subtree tasks");
    std::memcpy(out.data(), db.ct_host.p, rb);
    return out;
  };
  const std::vector<DevRecord> r1 = run(tasks, col);
  db.sp_tasks_run += (int64_t)tasks.size();
  // resolve in row order; collect the re-runs
  std::vector<LdsTask> again;
  std::vector<int32_t> again_comp;
  for (int32_t i = 0; i < count; ++i) {
    Comp& cp = comps[(size_t)i];
    if (cp.done) continue;
    const DevDesc& d = db.host_desc[(size_t)cp.pos];
    const uint64_t B = (uint64_t)d.budget;
    const int32_t t0 = task_of[(size_t)i];
    for (int32_t c = 0; c < d.k; ++c) {
      if (cp.acc == B) {   // the next node entry fails its budget test
        cp.res.rec.status = MPLD_BUDGET_EXHAUSTED;
        cp.res.rec.nodes = B;
        cp.res.rec.depth = 1;
        cp.res.rec.hash = trace ? cp.hash : 0;
        cp.done = true;
        break;
      }
      const DevRecord& r = r1[(size_t)(t0 + c)];
      const bool fits = cp.acc + r.nodes <= B;
      if (r.status == MPLD_INFEASIBLE && fits) {
        cp.acc += r.nodes;
        cp.hash = trace_concat(cp.hash, r.hash, r.nodes);
        continue;
      }
      if ((r.status == MPLD_FEASIBLE && fits) || c == 0) {
        // a solution inside the budget, or row 0, which ran with exactly
        // the budget left (B - 1): the task's result is the search's
        cp.res.rec.status = r.status;
        cp.res.rec.nodes = cp.acc + r.nodes;
        cp.res.rec.hash = trace ? trace_concat(cp.hash, r.hash, r.nodes) : 0;
        cp.res.rec.depth = r.status == MPLD_INFEASIBLE ? 0 : r.depth;
        if (r.status == MPLD_FEASIBLE) cp.res.src_off = tasks[(size_t)(t0 + c)].col_off;
        cp.done = true;
        break;
      }
      // the sequential search stops inside this subtree
      again.push_back(LdsTask{cp.pos, c, (int64_t)(B - cp.acc), 0});
      again_comp.push_back(i);
      cp.rerun_row = c;
      break;
    }
    if (!cp.done && cp.rerun_row < 0) {   // every row exhausted
      cp.res.rec.status = MPLD_INFEASIBLE;
      cp.res.rec.nodes = cp.acc;
      cp.res.rec.hash = trace ? cp.hash : 0;
      cp.res.rec.depth = 0;
      cp.done = true;
    }
  }
  if (!again.empty()) {
    // the re-runs write their colors past the first phase's, which are kept
    int64_t col2 = col;
    for (LdsTask& t : again) {
      t.col_off = col2;
      col2 += db.host_desc[(size_t)t.item].n;
    }
    if (db.ct_colors.bytes < (size_t)col2) {
      DevBuf bigger;
      bigger.alloc(ctx, (size_t)col2);
      if (col > 0)
        check_hip(hipMemcpyAsync(bigger.p, db.ct_colors.p, (size_t)col, hipMemcpyDeviceToDevice, s),
                  "subtree tasks: colors");
      check_hip(hipStreamSynchronize(s), "subtree tasks: colors");
      std::swap(db.ct_colors.p, bigger.p);
      std::swap(db.ct_colors.bytes, bigger.bytes);   // `bigger` frees the old area
    }
    const std::vector<DevRecord> r2 = run(again, col2);
    db.sp_tasks_run += (int64_t)again.size();
    db.sp_reruns += (int64_t)again.size();
    for (size_t j = 0; j < again.size(); ++j) {
      Comp& cp = comps[(size_t)again_comp[j]];
      const DevRecord& r = r2[j];
      cp.res.rec.status = r.status;
      cp.res.rec.nodes = cp.acc + r.nodes;
      cp.res.rec.hash = trace ? trace_concat(cp.hash, r.hash, r.nodes) : 0;
      cp.res.rec.depth = r.status == MPLD_INFEASIBLE ? 0 : r.depth;
      cp.res.src_off = r.status == MPLD_FEASIBLE ? again[j].col_off : -1;
      cp.done = true;
    }
  }
  // write back records and colors
  std::vector<LdsResolved> w;
  w.reserve(comps.size());
  for (const Comp& cp : comps) w.push_back(cp.res);
  const size_t wb = sizeof(LdsResolved) * w.size();
  if (db.ct_resolved.bytes < wb) db.ct_resolved.alloc(ctx, wb);
  if (!db.ct_host.reserve(wb)) fail(MPLD_E_NOMEM, "subtree tasks: pinned host memory");
  std::memcpy(db.ct_host.p, w.data(), wb);
  check_hip(hipMemcpyAsync(db.ct_resolved.p, db.ct_host.p, wb, hipMemcpyHostToDevice, s),
            "subtree tasks: resolved");
  check_hip(launch_csr_writeback(db.ct_resolved.as<LdsResolved>(), (int32_t)w.size(),
                                 db.ct_colors.as<int8_t>(), db.recs.as<DevRecord>(),
                                 db.colors.as<int8_t>(), s),
            "subtree tasks: write-back");
  check_hip(hipStreamSynchronize(s), "subtree tasks: write-back");
}

static void heavy_engine_host(DeviceBatch& db);

// The device-resident engine also follows the stitch-aware order (its
// tasks rebuild each path's row order and tried sets) and carries trace
// hashes; the host-driven one replays rows in ascending order only and
// counts nodes only, so stitch-ordered or traced batches always take the
// device engine.
static void heavy_engine(DeviceBatch& db, bool trace) {
  if (db.tune.heavy_device || db.reg_stitch || trace) heavy_engine_device(db, trace);
  else heavy_engine_host(db);
}

static void heavy_engine_host(DeviceBatch& db) {
  mpld_context* ctx = db.ctx;
  hipStream_t s = ctx->stream;
  db.sp_rounds = db.sp_tasks_run = db.sp_heavy = db.sp_reruns = 0;
  // which register-tier components stopped at the first cap
  if (!db.sp_host_recs.reserve(sizeof(DevRecord) * (size_t)std::max(1, db.num_comps)))
    fail(MPLD_E_NOMEM, "heavy-component engine: pinned host memory");
  DevRecord* recs = db.sp_host_recs.as<DevRecord>();
  check_hip(hipMemcpyAsync(recs, db.recs.p, sizeof(DevRecord) * (size_t)db.num_comps,
                           hipMemcpyDeviceToHost, s), "heavy: records");
  check_hip(hipStreamSynchronize(s), "heavy: first pass");
  std::vector<HComp> hcs;
  std::vector<HTask> tasks;
  std::vector<int32_t> pending;   // tasks not run yet, in creation order
  for (int32_t i = 0; i < db.n_reg; ++i) {
    if (recs[db.host_desc[i].comp].status >= 0) continue;
    HComp hc;
    hc.item = i;
    HTask root;
    root.hc = (int32_t)hcs.size();
    root.depth = 0;
    tasks.push_back(root);
    pending.push_back((int32_t)tasks.size() - 1);
    hc.seq.push_back({(int32_t)tasks.size() - 1, 0});
    hcs.push_back(std::move(hc));
  }
  if (hcs.empty()) return;
  db.sp_heavy = (int64_t)hcs.size();
  int levels = db.tune.heavy_levels > 0 ? db.tune.heavy_levels : split_levels(db.k);
  int64_t kp = 1;   // at most k^levels subtasks per split
  for (int l = 0; l < levels; ++l) kp *= db.k;
  while (levels > 1 && kp > 512) {   // keep the item area bounded
    kp /= db.k;
    --levels;
  }
  const int32_t max_items = (int32_t)kp + 2;   // subtasks, an end item, a solution item
  // task area: the round's item-pool count first (zeroed by the same upload
  // that brings the tasks), the tasks from byte 64 on
  constexpr size_t kTasksAt = 64;
  if (!db.sp_tasks.p) db.sp_tasks.alloc(ctx, kTasksAt + sizeof(SplitTask) * kHeavyMaxTasks);
  if (!db.sp_out.p) db.sp_out.alloc(ctx, (size_t)kSplitBlockBytes * kHeavyMaxTasks);
  // the item pool depends on k and the split depth, which a new schedule
  // may change: grow it when too small
  const size_t pool_bytes = sizeof(SplitItem) * (size_t)max_items * kHeavyMaxTasks;
  if (db.sp_pool.bytes < pool_bytes) db.sp_pool.alloc(ctx, pool_bytes);
  const size_t count_at = (size_t)kSplitBlockBytes * kHeavyMaxTasks;   // pool count copy
  if (!db.sp_host_tasks.reserve(kTasksAt + sizeof(SplitTask) * kHeavyMaxTasks) ||
      !db.sp_host_out.reserve(count_at + 64) || !db.sp_host_pool.reserve(pool_bytes))
    fail(MPLD_E_NOMEM, "heavy-component engine: pinned host memory");
  SplitTask* up = reinterpret_cast<SplitTask*>(db.sp_host_tasks.as<uint8_t>() + kTasksAt);
  const uint8_t* hout = db.sp_host_out.as<uint8_t>();
  const SplitItem* hpool = db.sp_host_pool.as<SplitItem>();
  int32_t* pool_count = db.sp_tasks.as<int32_t>();
  const SplitTask* dtasks = reinterpret_cast<const SplitTask*>(db.sp_tasks.as<uint8_t>() + kTasksAt);
  std::vector<int32_t> run, rest, where;
  for (;;) {
    // this round: pending tasks of unresolved components, oldest first
    run.clear();
    rest.clear();
    for (int32_t id : pending) {
      if (hcs[tasks[id].hc].done) continue;
      if ((int32_t)run.size() < kHeavyMaxTasks) run.push_back(id);
      else rest.push_back(id);
    }
    pending.swap(rest);
    if (run.empty()) break;
    const int32_t nt = (int32_t)run.size();
    for (int32_t i = 0; i < nt; ++i) {
      const HTask& t = tasks[run[i]];
      up[i].item = hcs[t.hc].item;
      up[i].depth = t.depth;
      std::memcpy(up[i].rows, t.rows, sizeof(up[i].rows));
    }
    *db.sp_host_tasks.as<int32_t>() = 0;   // the pool count
    check_hip(hipMemcpyAsync(db.sp_tasks.p, db.sp_host_tasks.p, kTasksAt + sizeof(SplitTask) * nt,
                             hipMemcpyHostToDevice, s), "heavy: tasks");
    const int grid = std::max(1, std::min((nt + 3) / 4, ctx->num_cus * ctx->reg_blocks_per_cu));
    check_hip(launch_reg_split(db.k, grid, dtasks, nt, db.counters.as<int32_t>() + 6,
                               db.reg_items(), (uint64_t)db.tune.heavy_round_cap,
                               (uint32_t)levels, db.sp_out.as<uint8_t>(), db.sp_pool.as<SplitItem>(),
                               pool_count, s),
              "heavy: split launch");
    check_hip(hipMemcpyAsync(db.sp_host_out.p, db.sp_out.p, (size_t)kSplitBlockBytes * nt,
                             hipMemcpyDeviceToHost, s), "heavy: task outputs");
    check_hip(hipMemcpyAsync(db.sp_host_out.as<uint8_t>() + count_at, pool_count, sizeof(int32_t),
                             hipMemcpyDeviceToHost, s), "heavy: pool count");
    check_hip(hipStreamSynchronize(s), "heavy: round");
    int32_t pooled = 0;
    std::memcpy(&pooled, hout + count_at, sizeof(pooled));
    if (pooled < 0 || (size_t)pooled * sizeof(SplitItem) > pool_bytes)
      fail(MPLD_E_INTERNAL, "heavy-component engine: bad item count");
    if (pooled > 0) {
      check_hip(hipMemcpyAsync(db.sp_host_pool.p, db.sp_pool.p, sizeof(SplitItem) * (size_t)pooled,
                               hipMemcpyDeviceToHost, s), "heavy: items");
      check_hip(hipStreamSynchronize(s), "heavy: items");
    }
    ++db.sp_rounds;
    db.sp_tasks_run += nt;
    // finished tasks take their counts; capped ones are replaced by their split
    std::vector<std::vector<HItem>> repl((size_t)nt);
    std::vector<char> touched(hcs.size(), 0);
    for (int32_t i = 0; i < nt; ++i) {
      const uint8_t* blk = hout + (size_t)kSplitBlockBytes * i;
      SplitResult r;
      std::memcpy(&r, blk, sizeof(r));
      const int8_t* sol = reinterpret_cast<const int8_t*>(blk + kSplitSolOffset);
      if (r.status == MPLD_FEASIBLE || r.status == MPLD_INFEASIBLE) {
        HTask& done = tasks[run[i]];
        done.status = r.status;
        done.nodes = r.nodes;
        if (r.status == MPLD_FEASIBLE) std::memcpy(done.sol, sol, 64);
        continue;
      }
      if (r.status != -1 || r.nitems < 1 || r.nitems > max_items ||
          (int64_t)r.item_off + r.nitems > (int64_t)pooled)
        fail(MPLD_E_INTERNAL, "heavy-component engine: bad task result");
      tasks[run[i]].status = -1;
      // a copy: pushing the children below may move `tasks`
      const HTask t = tasks[run[i]];
      touched[t.hc] = 1;
      const SplitItem* its = hpool + r.item_off;
      for (int32_t j = 0; j < r.nitems; ++j) {
        if (its[j].seg) repl[i].push_back({-1, its[j].seg});
        if (its[j].kind == 1) break;
        HTask ch;
        ch.hc = t.hc;
        if (its[j].kind == 0) {
          ch.depth = t.depth + levels;
          if (ch.depth > 64) fail(MPLD_E_INTERNAL, "heavy-component engine: task too deep");
          std::memcpy(ch.rows, t.rows, sizeof(ch.rows));
          for (int l = 0; l < levels; ++l) ch.rows[t.depth + l] = its[j].rows[l];
        } else {   // kind 2: a solution among the split's top levels (already counted)
          ch.depth = t.depth;
          ch.status = MPLD_FEASIBLE;
          ch.nodes = 0;
          std::memcpy(ch.sol, sol, 64);
        }
        tasks.push_back(ch);
        if (ch.status == -2) pending.push_back((int32_t)tasks.size() - 1);
        repl[i].push_back({(int32_t)tasks.size() - 1, 0});
        if (its[j].kind == 2) break;
      }
    }
    // splice replacements into their components' sequences (only past the
    // resolved prefix: a capped task was not final)
    where.assign(tasks.size(), -1);
    for (int32_t i = 0; i < nt; ++i)
      if (tasks[run[i]].status == -1) where[run[i]] = i;
    for (size_t h = 0; h < hcs.size(); ++h) {
      HComp& hc = hcs[h];
      if (hc.done) continue;
      if (touched[h]) {
        std::vector<HItem> tail;
        tail.reserve((hc.seq.size() - hc.pos) * 2);
        for (size_t j = hc.pos; j < hc.seq.size(); ++j) {
          const HItem& it = hc.seq[j];
          const int32_t f = it.task >= 0 ? where[it.task] : -1;
          if (f < 0) {
            tail.push_back(it);
          } else {
            for (const HItem& x : repl[f]) tail.push_back(x);
          }
        }
        hc.seq.resize(hc.pos);
        hc.seq.insert(hc.seq.end(), tail.begin(), tail.end());
      }
      hc.done = resolve(hc, db.host_desc[hc.item], tasks);
    }
  }
  // write the results back where the first pass left its records: one
  // staged copy and one scatter kernel for all resolved components
  std::vector<HeavyWrite> wb;
  for (HComp& hc : hcs) {
    const DevDesc& d = db.host_desc[hc.item];
    if (hc.rerun) {
      ++db.sp_reruns;
      check_hip(launch_reg_single(false, db.k, db.reg_items(),
                                  hc.item, db.recs.as<DevRecord>(), db.colors.as<int8_t>(), s),
                "heavy: sequential re-run");
      continue;
    }
    if (!hc.done) fail(MPLD_E_INTERNAL, "heavy-component engine ended unresolved");
    HeavyWrite w{};
    w.comp = d.comp;
    w.out_off = d.out_off;
    w.n = d.n;
    w.rec = hc.rec;
    std::memcpy(w.colors, hc.colors.data(), (size_t)d.n);
    wb.push_back(w);
  }
  if (!wb.empty()) {
    if (!db.sp_host_writes.reserve(sizeof(HeavyWrite) * wb.size()))
      fail(MPLD_E_NOMEM, "heavy-component engine: pinned host memory");
    if (db.sp_writes.bytes < sizeof(HeavyWrite) * wb.size())
      db.sp_writes.alloc(ctx, sizeof(HeavyWrite) * wb.size());
    std::memcpy(db.sp_host_writes.p, wb.data(), sizeof(HeavyWrite) * wb.size());
    check_hip(hipMemcpyAsync(db.sp_writes.p, db.sp_host_writes.p, sizeof(HeavyWrite) * wb.size(),
                             hipMemcpyHostToDevice, s), "heavy: write-back upload");
    check_hip(launch_heavy_writeback(db.sp_writes.as<HeavyWrite>(), (int32_t)wb.size(),
                                     db.recs.as<DevRecord>(), db.colors.as<int8_t>(), s),
              "heavy: write-back");
  }
  check_hip(hipStreamSynchronize(s), "heavy: write back");
}

// Conflict marking of every component whose record is not FEASIBLE (after
// all search work of the batch, on the same stream).
// Eq. 1 minimisation of the register-tier items (after the marking).
static void enqueue_minimize(DeviceBatch& db, hipStream_t s) {
  if (!db.n_reg) return;
  if (!db.min_out.p) fail(MPLD_E_INTERNAL, "batch was not packed for MPLD_MINIMIZE");
  check_hip(launch_min_reg(db.k, std::min(db.n_reg, 65535), db.reg_items(),
                           db.n_reg, db.partners.as<uint8_t>(), db.colors.as<int8_t>(),
                           db.min_out.as<int32_t>(), db.min_budget, s),
            "Eq. 1 minimisation (register tier)");
}

// reg: also the register-tier items (not when their batched launch marked
// them already).
static void enqueue_mark(DeviceBatch& db, hipStream_t s, bool reg = true) {
  mpld_context* ctx = db.ctx;
  auto* recs = db.recs.as<DevRecord>();
  auto* colors = db.colors.as<int8_t>();
  if (db.n_reg && reg)
    check_hip(launch_mark_reg(db.k, std::min(db.n_reg, ctx->num_cus * 8), db.reg_items(), db.n_reg,
                              recs, colors, s),
              "conflict marking (register tier)");
  const int32_t ncsr = db.n_lds + db.n_big + db.n_dev;
  if (ncsr)
    check_hip(launch_mark_lds(std::min(ncsr, ctx->num_cus * 4), (int)db.mark_lds,
                              db.desc.as<DevDesc>() + db.n_reg, db.adj32.as<uint32_t>(), ncsr, recs,
                              colors, s),
              "conflict marking (CSR components)");
}

void device_solve(DeviceBatch& db, uint32_t flags) {
  mpld_context* ctx = db.ctx;
  hipStream_t s = ctx->stream;
  const bool minimize = flags & MPLD_MINIMIZE;
  const bool mark = flags & (MPLD_MARK_CONFLICTS | MPLD_MINIMIZE);
  if (mark && db.mark_lds > ctx->lds_per_block)
    fail(MPLD_E_UNSUPPORTED, "a component is too large for conflict marking (" +
                                 std::to_string(db.mark_lds) + " bytes of LDS)");
  const bool trace = flags & MPLD_TRACE_HASH;
  const bool split = (flags & MPLD_SPLIT_HEAVY) && !(flags & MPLD_PLAIN);
  const uint64_t cap = split && db.n_reg > 0 ? (uint64_t)db.tune.heavy_first_cap : ~0ull;
  const bool timed = !(flags & MPLD_UNTIMED) || (flags & MPLD_PLAIN);
  db.timed = false;
  if (flags & MPLD_PLAIN) {
    // one launch per component, same search code
    const auto* desc = db.desc.as<DevDesc>();
    const RegItems items = db.reg_items();
    const auto* adj = db.adj32.as<uint32_t>();
    auto* recs = db.recs.as<DevRecord>();
    auto* colors = db.colors.as<int8_t>();
    auto* gstack = db.gstack.as<uint64_t>();
    db.launches = 0;
    check_hip(hipEventRecord(ctx->ev[0], s), "event");
    for (int32_t i = 0; i < (int32_t)db.host_queue.size(); ++i) {
      hipError_t e;
      if (i < db.n_reg)
        e = launch_reg_single(trace, db.k, items, i, recs, colors, s);
      else if (i < db.n_reg + db.n_lds)
        e = launch_lds_single(trace, false, db.csr_stitch, 1, db.lds_small, desc, adj, i, nullptr, recs, colors, s);
      else if (i < db.n_reg + db.n_lds + db.n_wide)
        e = launch_lds_single(trace, true, db.csr_stitch, 0, db.lds_wide, desc, adj, i, gstack, recs, colors, s);
      else if (i < db.n_reg + db.n_lds + db.n_big)
        e = launch_lds_single(trace, true, db.csr_stitch, db.big_waves, db.lds_big, desc, adj, i, gstack, recs, colors, s);
      else
        e = launch_device_tier(trace, db.grid_dev, db.lds_dev, desc + i, adj,
                               db.dev_keys.as<unsigned long long>(), db.dev_stacks.as<uint64_t>(),
                               recs, colors, s);
      check_hip(e, "plain launch");
      ++db.launches;
    }
    if (mark) enqueue_mark(db, s);
    if (minimize) enqueue_minimize(db, s);
    check_hip(hipEventRecord(ctx->ev[1], s), "event");
  } else if ((flags & MPLD_DIRECT) || !db.tune.use_graph || db.n_dev) {
    // direct launches (cooperative launches stay out of graphs)
    if (timed) check_hip(hipEventRecord(ctx->ev[0], s), "event");
    enqueue_batched(db, trace, cap, s, split, mark && !split);
    if (split) {
      db.sp_rounds = db.sp_tasks_run = db.sp_heavy = db.sp_reruns = 0;
      if (db.n_reg) heavy_engine(db, trace);
      csr_split(db, trace);
    }
    if (mark) enqueue_mark(db, s, split);
    if (minimize) enqueue_minimize(db, s);
    if (timed) check_hip(hipEventRecord(ctx->ev[1], s), "event");
  } else {
    // capture the tiered launches once, replay the graph afterwards
    const bool mark_fused = mark && !split;
    const uint32_t key = (trace ? 1u : 0u) | (split ? 2u : 0u) | (mark_fused ? 4u : 0u);
    if (!db.graph || db.graph_flags != key) {
      if (db.graph) {
        check_hip(hipGraphExecDestroy(db.graph), "graph destroy");
        db.graph = nullptr;
      }
      hipGraph_t g = nullptr;
      check_hip(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "begin capture");
      try {
        enqueue_batched(db, trace, cap, s, split, mark_fused);
      } catch (...) {
        (void)hipStreamEndCapture(s, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      check_hip(hipStreamEndCapture(s, &g), "end capture");
      hipError_t e = hipGraphInstantiate(&db.graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      check_hip(e, "graph instantiate");
      db.graph_flags = key;
    }
    if (timed) check_hip(hipEventRecord(ctx->ev[0], s), "event");
    check_hip(hipGraphLaunch(db.graph, s), "graph launch");
    if (split) {
      db.sp_rounds = db.sp_tasks_run = db.sp_heavy = db.sp_reruns = 0;
      if (db.n_reg) heavy_engine(db, trace);
      csr_split(db, trace);
    }
    if (mark) enqueue_mark(db, s, split);
    if (minimize) enqueue_minimize(db, s);
    if (timed) check_hip(hipEventRecord(ctx->ev[1], s), "event");
  }
  db.timed = timed;
}

bool device_time(DeviceBatch& db) {
  if (db.rt_timed) {
    float ms = 0.f;
    const hipError_t e = hipEventElapsedTime(&ms, db.rt_ev[0], db.rt_ev[1]);
    if (e != hipErrorNotReady) {
      check_hip(e, "event time");
      db.last_roundtrip_ms = ms;
      db.rt_timed = false;
    }
  }
  if (!db.timed) return false;
  float ms = 0.f;
  const hipError_t e = hipEventElapsedTime(&ms, db.ctx->ev[0], db.ctx->ev[1]);
  if (e == hipErrorNotReady) return false;
  check_hip(e, "event time");
  db.last_search_ms = ms;
  db.last_total_ms = ms;
  db.timed = false;
  return true;
}

void device_fetch(DeviceBatch& db, std::vector<DevRecord>& recs, std::vector<int8_t>& colors,
                  std::vector<int32_t>* min_nodes) {
  mpld_context* ctx = db.ctx;
  hipStream_t s = ctx->stream;
  (void)ctx;
  check_hip(hipStreamSynchronize(s), "search");
  device_time(db);
  recs.resize((size_t)db.num_comps);
  colors.resize((size_t)db.total_nodes);
  if (db.num_comps)
    check_hip(hipMemcpyAsync(recs.data(), db.recs.p, sizeof(DevRecord) * recs.size(),
                             hipMemcpyDeviceToHost, s), "download records");
  if (db.total_nodes)
    check_hip(hipMemcpyAsync(colors.data(), db.colors.p, colors.size(), hipMemcpyDeviceToHost, s),
              "download colors");
  if (min_nodes) {
    min_nodes->assign((size_t)db.num_comps, 0);
    if (db.min_out.p && db.n_reg) {
      std::vector<int32_t> all((size_t)db.num_comps, 0);
      check_hip(hipMemcpyAsync(all.data(), db.min_out.p, sizeof(int32_t) * all.size(),
                               hipMemcpyDeviceToHost, s), "download minimisation counts");
      check_hip(hipStreamSynchronize(s), "download");
      // only register-tier items write their entry
      for (int32_t i = 0; i < db.n_reg; ++i) {
        const int32_t c = db.host_queue[(size_t)i];
        (*min_nodes)[(size_t)c] = all[(size_t)c];
      }
    }
  }
  check_hip(hipStreamSynchronize(s), "download");
  for (const auto& r : recs)
    if (r.status < 0 || r.status > MPLD_BUDGET_EXHAUSTED)
      fail(MPLD_E_INTERNAL, "search reported a broken state");
}

void assemble_result(const Graph& g, const Split& s, const Image& im, const mpld_options& opt,
                     const std::vector<DevRecord>& recs, const std::vector<int8_t>& lcol,
                     mpld_result* r, const std::vector<int32_t>* min_nodes) {
  const bool trace = opt.flags & MPLD_TRACE_HASH;
  r->colors.assign((size_t)g.n, -1);
  r->comp_of = s.comp_of;
  const int32_t nc = (int32_t)s.comp_ptr.size() - 1;
  r->comps.resize((size_t)nc);
  for (int32_t c = 0; c < nc; ++c) {
    const DevDesc& d = im.desc[c];
    for (int32_t i = 0; i < d.n; ++i) r->colors[s.order[s.comp_ptr[c] + i]] = lcol[d.out_off + i];
  }
  for (int32_t c = 0; c < nc; ++c) {
    const DevDesc& d = im.desc[c];
    mpld_comp_record& rec = r->comps[c];
    rec.size = d.n;
    rec.status = recs[c].status;
    rec.nodes = (int64_t)recs[c].nodes;
    rec.trace_hash = trace ? recs[c].hash : 0;
    rec.depth_at_stop = recs[c].depth;
    rec.first_node = s.order[s.comp_ptr[c]];
    int64_t edges2 = 0, same2 = 0;
    int32_t st = 0;
    for (int32_t p = s.comp_ptr[c]; p < s.comp_ptr[c + 1]; ++p) {
      const int32_t x = s.order[p];
      const int8_t cx = r->colors[x];
      for (int64_t t = g.ptr[x]; t < g.ptr[x + 1]; ++t) {
        const int32_t w = g.adj[t];
        if (s.comp_of[w] != c) continue;
        ++edges2;
        same2 += cx >= 0 && r->colors[w] == cx;
      }
      const int32_t q = g.partner[x];
      if (q > x && s.comp_of[q] == c && r->colors[q] != cx) ++st;
    }
    rec.num_edges = (int32_t)(edges2 / 2);
    const bool colored =
        rec.status == MPLD_FEASIBLE || (opt.flags & (MPLD_MARK_CONFLICTS | MPLD_MINIMIZE));
    rec.stitches = colored ? st : -1;
    rec.conflicts = (int32_t)(same2 / 2);
    rec.min_nodes = min_nodes && !min_nodes->empty() ? (*min_nodes)[(size_t)c] : 0;
  }
  if (opt.flags & MPLD_SIMPLIFY) recover(g, s, opt.k, r->colors);
  tallies(g, r->colors, &r->stitches, &r->conflicts, &r->uncolored);
}

}  // namespace mpld

void* mpld_context::dev_alloc(size_t bytes) {
  void* p = nullptr;
  if (has_alloc) {
    p = alloc.alloc(bytes, alloc.user);
    if (!p) mpld::fail(MPLD_E_NOMEM, "device allocator returned NULL for " + std::to_string(bytes) + " bytes");
  } else {
    mpld::check_hip(hipMalloc(&p, bytes), "hipMalloc");
  }
  return p;
}

void mpld_context::dev_free(void* p) {
  if (!p) return;
  if (has_alloc)
    alloc.free(p, alloc.user);
  else
    (void)hipFree(p);
}
