// abi.cpp - the C ABI of include/mpld.h: argument checks, error mapping,
// and the flow of Sec. 2.2 (front-end -> device search -> recovery).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <exception>
#include <new>

#include "runtime.h"

namespace mpld {
const char* last_error_cstr();
}

using namespace mpld;

namespace {

template <class F>
int32_t guard(F&& f) {
  try {
    f();
    set_last_error("");
    return MPLD_OK;
  } catch (const Error& e) {
    set_last_error(e.what);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return MPLD_E_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return MPLD_E_INTERNAL;
  } catch (...) {
    set_last_error("unknown exception");
    return MPLD_E_INTERNAL;
  }
}

void check_options(const mpld_options* opt) {
  if (!opt) fail(MPLD_E_INVALID, "options are NULL");
  if (opt->struct_size != sizeof(mpld_options))
    fail(MPLD_E_INVALID, "options.struct_size does not match this library's mpld_options");
  if (opt->k < 2 || opt->k > MPLD_MAX_K) fail(MPLD_E_INVALID, "k must be in [2, 8]");
  if (opt->node_budget < 1) fail(MPLD_E_INVALID, "node_budget must be >= 1");
  const uint32_t forced =
      opt->flags & (MPLD_FORCE_WAVE | MPLD_FORCE_LDS | MPLD_FORCE_GLOBAL | MPLD_FORCE_DEVICE);
  if (forced & (forced - 1)) fail(MPLD_E_INVALID, "at most one MPLD_FORCE_* flag");
  if (opt->min_budget < 0) fail(MPLD_E_INVALID, "min_budget must be >= 0 (0 = 10000)");
}

constexpr int32_t kDeviceSplitMinNodes = 32768;

void use_device(mpld_context* ctx) {
  if (!ctx) fail(MPLD_E_INVALID, "context is NULL");
  check_hip(hipSetDevice(ctx->device), "hipSetDevice");
}

// Builds the batch: front-end, then packing and upload with the batch's
// launch parameters (from the tuning cache when one is configured).
void batch_build(mpld_context* ctx, const mpld_graph* g, const mpld_options* opt, mpld_batch* b) {
  if (!g) fail(MPLD_E_INVALID, "graph is NULL");
  check_options(opt);
  b->ctx = ctx;
  b->opt = *opt;
  b->g = make_graph(*g);
  // large sparse graphs are simplified and split on the device (identical
  // result; at 50k nodes about half the host's time, at 5k nodes slower)
  if (device_split_pays(b->g.n, b->g.ptr[(size_t)b->g.n], opt->k) && b->g.n >= kDeviceSplitMinNodes) {
    if (!ctx->graph_builder) ctx->graph_builder = graph_builder_create(ctx, false);
    split_graph_device(*ctx->graph_builder, b->g, opt->k, opt->flags & MPLD_SIMPLIFY, b->s);
  } else {
    b->s = simplify_and_split(b->g, opt->k, opt->flags & MPLD_SIMPLIFY);
  }
  Tune t;
  tune_from_cache(b, nullptr, &t);
  batch_pack(b, t);
}

uint32_t min_budget_of(const mpld_options* opt) {
  return opt->min_budget > 0 ? (uint32_t)opt->min_budget : 10000u;
}

void batch_collect(mpld_batch* b, mpld_result* r) {
  std::vector<DevRecord> recs;
  std::vector<int8_t> lcol;
  std::vector<int32_t> mins;
  const bool minimize = b->opt.flags & MPLD_MINIMIZE;
  device_fetch(b->db, recs, lcol, minimize ? &mins : nullptr);
  assemble_result(b->g, b->s, b->im, b->opt, recs, lcol, r, minimize ? &mins : nullptr);
}

}  // namespace

extern "C" {

uint32_t mpld_abi_version(void) { return MPLD_ABI_VERSION; }

const char* mpld_error_string(int32_t err) {
  switch (err) {
    case MPLD_OK: return "ok";
    case MPLD_E_INVALID: return "invalid argument";
    case MPLD_E_NOMEM: return "out of memory";
    case MPLD_E_DEVICE: return "device error";
    case MPLD_E_NOT_READY: return "not ready";
    case MPLD_E_CANCELLED: return "cancelled";
    case MPLD_E_INTERNAL: return "internal error";
    case MPLD_E_UNSUPPORTED: return "unsupported";
    default: return "unknown error code";
  }
}

const char* mpld_last_error(void) { return last_error_cstr(); }

int32_t mpld_build_graph(const mpld_rect* rects, int32_t n, int32_t dmin_nm, int32_t split_len_nm,
                         mpld_owned_graph** out) {
  return guard([&] {
    if (!out) fail(MPLD_E_INVALID, "out is NULL");
    *out = nullptr;
    auto* g = new mpld_owned_graph();
    try {
      build_layout_graph(rects, n, dmin_nm, split_len_nm, g->g);
    } catch (...) {
      delete g;
      throw;
    }
    *out = g;
  });
}

int32_t mpld_build_graph_device(mpld_context* ctx, const mpld_rect* rects, int32_t n,
                                int32_t dmin_nm, int32_t split_len_nm, mpld_owned_graph** out) {
  return guard([&] {
    if (!out) fail(MPLD_E_INVALID, "out is NULL");
    *out = nullptr;
    use_device(ctx);
    if (!ctx->graph_builder) ctx->graph_builder = graph_builder_create(ctx, false);
    Graph g;
    std::vector<int32_t> se;
    build_layout_graph_device(*ctx->graph_builder, rects, n, dmin_nm, split_len_nm, g, &se);
    auto* og = new mpld_owned_graph();
    og->g.num_nodes = g.n;
    og->g.se.swap(se);
    og->g.ce.reserve((size_t)g.num_ce * 2);
    for (int32_t a = 0; a < g.n; ++a)
      for (int64_t t = g.ptr[a]; t < g.ptr[a + 1]; ++t)
        if (g.adj[t] > a) {
          og->g.ce.push_back(a);
          og->g.ce.push_back(g.adj[t]);
        }
    *out = og;
  });
}

int32_t mpld_split_graph_device(mpld_context* ctx, const mpld_graph* g, int32_t k, uint32_t flags,
                                int32_t* removal_order, int32_t* num_removed, int32_t* comp_of,
                                int32_t* bfs_order, int32_t* comp_ptr, int32_t* num_comps) {
  return guard([&] {
    if (!g || !removal_order || !num_removed || !comp_of || !bfs_order || !comp_ptr || !num_comps)
      fail(MPLD_E_INVALID, "NULL argument");
    if (k < 2 || k > MPLD_MAX_K) fail(MPLD_E_INVALID, "k outside [2, MPLD_MAX_K]");
    use_device(ctx);
    if (!ctx->graph_builder) ctx->graph_builder = graph_builder_create(ctx, false);
    const Graph gr = make_graph(*g);
    Split s;
    split_graph_device(*ctx->graph_builder, gr, k, flags & MPLD_SIMPLIFY, s);
    std::copy(s.removal.begin(), s.removal.end(), removal_order);
    *num_removed = (int32_t)s.removal.size();
    std::copy(s.comp_of.begin(), s.comp_of.end(), comp_of);
    std::copy(s.order.begin(), s.order.end(), bfs_order);
    std::copy(s.comp_ptr.begin(), s.comp_ptr.end(), comp_ptr);
    *num_comps = (int32_t)s.comp_ptr.size() - 1;
  });
}

int32_t mpld_owned_graph_view(const mpld_owned_graph* g, mpld_graph* view) {
  return guard([&] {
    if (!g || !view) fail(MPLD_E_INVALID, "NULL argument");
    view->num_nodes = g->g.num_nodes;
    view->reserved = 0;
    view->num_ce = (int64_t)g->g.ce.size() / 2;
    view->ce = g->g.ce.data();
    view->num_se = (int64_t)g->g.se.size() / 2;
    view->se = g->g.se.data();
  });
}

void mpld_owned_graph_free(mpld_owned_graph* g) { delete g; }

int32_t mpld_context_create(int32_t device, const mpld_allocator* alloc, void* hip_stream,
                            mpld_context** out) {
  return guard([&] {
    if (!out) fail(MPLD_E_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
      fail(MPLD_E_DEVICE, "no HIP device is visible");
    if (device < 0 || device >= count) fail(MPLD_E_DEVICE, "device ordinal out of range");
    check_hip(hipSetDevice(device), "hipSetDevice");
    hipDeviceProp_t prop;
    check_hip(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      fail(MPLD_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    if (alloc && (!alloc->alloc || !alloc->free)) fail(MPLD_E_INVALID, "allocator lacks alloc or free");
    auto* ctx = new mpld_context();
    ctx->device = device;
    ctx->num_cus = prop.multiProcessorCount;
    ctx->lds_per_block = (int)prop.sharedMemPerBlock;
    if (alloc) {
      ctx->alloc = *alloc;
      ctx->has_alloc = true;
    }
    try {
      if (hip_stream) {
        ctx->stream = static_cast<hipStream_t>(hip_stream);
      } else {
        check_hip(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking), "stream");
        ctx->own_stream = true;
      }
      for (auto& e : ctx->ev) check_hip(hipEventCreate(&e), "event");
      ctx->reg_blocks_per_cu = reg_batched_blocks_per_cu(false);
      lds_configure(ctx->lds_per_block);
    } catch (...) {
      mpld_context_destroy(ctx);
      throw;
    }
    *out = ctx;
  });
}

int32_t mpld_context_destroy(mpld_context* ctx) {
  if (!ctx) return MPLD_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->graph_builder) graph_builder_destroy(ctx->graph_builder);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return MPLD_OK;
}

int32_t mpld_batch_create(mpld_context* ctx, const mpld_graph* g, const mpld_options* opt,
                          mpld_batch** out) {
  return guard([&] {
    if (!out) fail(MPLD_E_INVALID, "out is NULL");
    *out = nullptr;
    use_device(ctx);
    auto* b = new mpld_batch();
    try {
      batch_build(ctx, g, opt, b);
    } catch (...) {
      delete b;
      throw;
    }
    *out = b;
  });
}

int32_t mpld_batch_solve(mpld_batch* b, uint32_t flags) {
  return guard([&] {
    if (!b) fail(MPLD_E_INVALID, "batch is NULL");
    use_device(b->ctx);
    const uint32_t how = MPLD_PLAIN | MPLD_DIRECT;
    const uint32_t f = (b->opt.flags & ~how) | (flags & (how | MPLD_SPLIT_HEAVY | MPLD_UNTIMED));
    if (flags & MPLD_ROUNDTRIP)
      device_roundtrip(b->db, b->im, f);
    else
      device_solve(b->db, f);
    b->solved = true;
  });
}

int32_t mpld_batch_result(mpld_batch* b, mpld_result** out) {
  return guard([&] {
    if (!b || !out) fail(MPLD_E_INVALID, "NULL argument");
    *out = nullptr;
    if (!b->solved) fail(MPLD_E_INVALID, "batch was not solved");
    use_device(b->ctx);
    auto* r = new mpld_result();
    try {
      batch_collect(b, r);
    } catch (...) {
      delete r;
      throw;
    }
    *out = r;
  });
}

int32_t mpld_batch_get_info(mpld_batch* b, mpld_batch_info* info) {
  return guard([&] {
    if (!b || !info) fail(MPLD_E_INVALID, "NULL argument");
    use_device(b->ctx);
    device_time(b->db);
    std::memset(info, 0, sizeof(*info));
    info->num_components = b->db.num_comps;
    info->num_wave = b->db.n_reg;
    info->num_lds = b->db.n_lds;
    info->num_global = b->db.n_big;
    info->core_nodes = b->im.total_nodes;
    info->max_size = b->im.max_size;
    info->image_bytes = (int64_t)(b->db.desc.bytes + b->db.regitems.bytes + b->db.adj32.bytes);
    info->core_edges = b->im.core_edges;
    info->last_search_ms = b->db.last_search_ms;
    info->last_total_ms = b->db.last_total_ms;
    info->launches = b->db.launches;
    info->num_device = b->db.n_dev;
    info->heavy_components = (int32_t)b->db.sp_heavy;
    info->split_rounds = (int32_t)b->db.sp_rounds;
    info->split_tasks = (int32_t)b->db.sp_tasks_run;
    info->split_reruns = (int32_t)b->db.sp_reruns;
    info->last_roundtrip_ms = b->db.last_roundtrip_ms;
    info->big_waves = b->db.n_big > b->db.n_wide ? b->db.big_waves : 0;
  });
}

void mpld_batch_free(mpld_batch* b) {
  if (!b) return;
  if (b->ctx) {
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
  }
  delete b;
}

int32_t mpld_decompose(mpld_context* ctx, const mpld_graph* g, const mpld_options* opt,
                       mpld_result** out) {
  return guard([&] {
    if (!out) fail(MPLD_E_INVALID, "out is NULL");
    *out = nullptr;
    use_device(ctx);
    mpld_batch b;
    batch_build(ctx, g, opt, &b);
    // one-shot: no graph to capture; it waits anyway, so heavy components
    // always go to the subtree engine
    device_solve(b.db, opt->flags | MPLD_DIRECT | MPLD_SPLIT_HEAVY);
    b.solved = true;
    auto* r = new mpld_result();
    try {
      batch_collect(&b, r);
    } catch (...) {
      delete r;
      throw;
    }
    *out = r;
  });
}

int32_t mpld_solve_components(mpld_context* ctx, const mpld_component* comps, int32_t count,
                              const mpld_options* opt, mpld_comp_record* out, int8_t* colors_out) {
  return guard([&] {
    use_device(ctx);
    check_options(opt);
    if (count < 0 || (count > 0 && (!comps || !out || !colors_out)))
      fail(MPLD_E_INVALID, "bad component array");
    Image im;
    std::vector<int32_t> pairs;
    for (int32_t c = 0; c < count; ++c) {
      const mpld_component& cp = comps[c];
      if (cp.n < 0 || cp.m < 0 || (cp.m > 0 && !cp.edges))
        fail(MPLD_E_INVALID, "component " + std::to_string(c) + " has a bad size or edge array");
      std::vector<uint64_t> keys((size_t)cp.m);
      for (int64_t e = 0; e < cp.m; ++e) {
        int32_t a = cp.edges[2 * e], b = cp.edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= cp.n || b >= cp.n || a == b)
          fail(MPLD_E_INVALID, "component " + std::to_string(c) + " edge " + std::to_string(e) +
                                   " is out of range or a self loop");
        if (a > b) std::swap(a, b);
        keys[e] = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
      }
      std::sort(keys.begin(), keys.end());
      if (std::adjacent_find(keys.begin(), keys.end()) != keys.end())
        fail(MPLD_E_INVALID, "component " + std::to_string(c) + " has a duplicate edge");
      pairs.resize(2 * keys.size());
      for (size_t e = 0; e < keys.size(); ++e) {
        pairs[2 * e] = (int32_t)(keys[e] >> 32);
        pairs[2 * e + 1] = (int32_t)(keys[e] & 0xffffffffu);
      }
      image_add(im, ctx, cp.n, pairs.data(), cp.m, opt->k, opt->node_budget, opt->flags);
    }
    image_finish(im);
    DeviceBatch db;
    device_upload(ctx, im, db);
    db.min_budget = min_budget_of(opt);
    device_solve(db, opt->flags | MPLD_DIRECT | MPLD_SPLIT_HEAVY);
    std::vector<DevRecord> recs;
    std::vector<int8_t> lcol;
    std::vector<int32_t> mins;
    device_fetch(db, recs, lcol, &mins);
    const bool trace = opt->flags & MPLD_TRACE_HASH;
    for (int32_t c = 0; c < count; ++c) {
      mpld_comp_record& r = out[c];
      r.size = comps[c].n;
      r.status = recs[c].status;
      r.nodes = (int64_t)recs[c].nodes;
      r.trace_hash = trace ? recs[c].hash : 0;
      r.depth_at_stop = recs[c].depth;
      r.stitches = r.status == MPLD_FEASIBLE || (opt->flags & (MPLD_MARK_CONFLICTS | MPLD_MINIMIZE))
                       ? 0 : -1;
      r.first_node = -1;
      r.num_edges = (int32_t)comps[c].m;
      r.conflicts = 0;
      r.min_nodes = (opt->flags & MPLD_MINIMIZE) ? mins[(size_t)c] : 0;
      const int8_t* cc = lcol.data() + im.desc[c].out_off;
      for (int64_t e = 0; e < comps[c].m; ++e) {
        const int8_t a = cc[comps[c].edges[2 * e]];
        r.conflicts += a >= 0 && a == cc[comps[c].edges[2 * e + 1]];
      }
    }
    if (!lcol.empty()) std::memcpy(colors_out, lcol.data(), lcol.size());
  });
}

const int8_t* mpld_result_colors(const mpld_result* r, int32_t* num_nodes) {
  if (!r) return nullptr;
  if (num_nodes) *num_nodes = (int32_t)r->colors.size();
  return r->colors.data();
}

const int32_t* mpld_result_component_of(const mpld_result* r) {
  return r ? r->comp_of.data() : nullptr;
}

int32_t mpld_result_num_components(const mpld_result* r) {
  return r ? (int32_t)r->comps.size() : 0;
}

const mpld_comp_record* mpld_result_components(const mpld_result* r) {
  return r ? r->comps.data() : nullptr;
}

void mpld_result_totals(const mpld_result* r, int64_t* stitches, int64_t* conflicts,
                        int64_t* uncolored) {
  if (!r) return;
  if (stitches) *stitches = r->stitches;
  if (conflicts) *conflicts = r->conflicts;
  if (uncolored) *uncolored = r->uncolored;
}

void mpld_result_timing(const mpld_result* r, double* queue_us, double* total_us) {
  if (!r) return;
  if (queue_us) *queue_us = r->queue_us;
  if (total_us) *total_us = r->total_us;
}

void mpld_result_free(mpld_result* r) { delete r; }

}  // extern "C"
