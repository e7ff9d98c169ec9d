// autotune.cpp - launch-parameter autotuner of a resident batch and its
// cache.  Candidates (register-tier workgroup size and grid cap, queue
// order, graph replay or direct launches, big or device-wide tier for giant
// components) are timed on the batch itself with HIP events; every
// candidate's records and colors must equal the default's (the search is
// deterministic, so any difference is a bug and fails the call).  The best
// is adopted and, with a cache path, appended as one JSON line keyed by the
// device and the batch's shape.
#include <new>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "runtime.h"

namespace mpld {

void batch_pack(mpld_batch* b, const Tune& t) {
  Image im;
  const int32_t nc = (int32_t)b->s.comp_ptr.size() - 1;
  std::vector<int32_t> pairs, part;
  const bool stitch = b->opt.flags & MPLD_STITCH_ORDER;
  const bool partners = stitch || (b->opt.flags & MPLD_MINIMIZE);
  for (int32_t c = 0; c < nc; ++c) {
    local_edges(b->g, b->s, c, pairs);
    const int32_t n = b->s.comp_ptr[c + 1] - b->s.comp_ptr[c];
    uint32_t flags = b->opt.flags;
    if (t.giant_device && n >= t.giant_min_nodes && !stitch &&
        !(flags & (MPLD_FORCE_WAVE | MPLD_FORCE_LDS | MPLD_FORCE_GLOBAL)))
      flags |= MPLD_FORCE_DEVICE;
    if (partners) {   // stitch partners inside the component, in its local numbering
      part.assign((size_t)n, -1);
      for (int32_t i = 0; i < n; ++i) {
        const int32_t q = b->g.partner[b->s.order[b->s.comp_ptr[c] + i]];
        if (q >= 0 && b->s.comp_of[q] == c) part[(size_t)i] = b->s.local[q];
      }
    }
    image_add(im, b->ctx, n, pairs.data(), (int64_t)pairs.size() / 2, b->opt.k,
              b->opt.node_budget, flags, partners ? part.data() : nullptr);
  }
  image_finish(im, t.order);
  b->im = std::move(im);
  device_upload(b->ctx, b->im, b->db, t);   // reallocates every buffer it uses
  b->db.min_budget = b->opt.min_budget > 0 ? (uint32_t)b->opt.min_budget : 10000u;
}

static std::string shape_key(mpld_batch* b) {
  hipDeviceProp_t prop;
  std::string arch = "gfx?";
  if (hipGetDeviceProperties(&prop, b->ctx->device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  int64_t comps = b->db.num_comps, maxn = b->im.max_size;
  int lc = 0, ln = 0;
  while ((1ll << lc) < comps) ++lc;
  while ((1ll << ln) < maxn) ++ln;
  std::ostringstream o;
  o << arch << "|cus=" << b->ctx->num_cus << "|k=" << b->opt.k << "|comps=2^" << lc
    << "|maxn=2^" << ln << "|trace=" << ((b->opt.flags & MPLD_TRACE_HASH) ? 1 : 0);
  return o.str();
}

static const char* cache_path_of(const char* path) {
  if (path && *path) return path;
  const char* e = std::getenv("MPLD_TUNE_CACHE");
  return (e && *e) ? e : nullptr;
}

static bool field(const std::string& line, const char* name, long* out) {
  const std::string pat = std::string("\"") + name + "\": ";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  *out = std::strtol(line.c_str() + p + pat.size(), nullptr, 10);
  return true;
}

bool tune_from_cache(mpld_batch* b, const char* path, Tune* t) {
  const char* p = cache_path_of(path);
  if (!p) return false;
  std::ifstream f(p);
  if (!f) return false;
  // the key uses the batch's shape: component count and largest size
  int64_t comps = (int64_t)b->s.comp_ptr.size() - 1, maxn = 0;
  for (int64_t c = 0; c < comps; ++c) maxn = std::max<int64_t>(maxn, b->s.comp_ptr[c + 1] - b->s.comp_ptr[c]);
  hipDeviceProp_t prop;
  std::string arch = "gfx?";
  if (hipGetDeviceProperties(&prop, b->ctx->device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  int lc = 0, ln = 0;
  while ((1ll << lc) < comps) ++lc;
  while ((1ll << ln) < maxn) ++ln;
  std::ostringstream o;
  o << arch << "|cus=" << b->ctx->num_cus << "|k=" << b->opt.k << "|comps=2^" << lc
    << "|maxn=2^" << ln << "|trace=" << ((b->opt.flags & MPLD_TRACE_HASH) ? 1 : 0);
  const std::string want = "\"key\": \"" + o.str() + "\"";
  std::string line, hit;
  while (std::getline(f, line))
    if (line.find(want) != std::string::npos) hit = line;   // last entry wins
  if (hit.empty()) return false;
  long v;
  if (field(hit, "waves_per_block", &v)) t->waves_per_block = (int32_t)std::max(1L, std::min(4L, v));
  if (field(hit, "max_blocks", &v)) t->max_blocks = (int32_t)std::max(0L, v);
  if (field(hit, "use_graph", &v)) t->use_graph = v ? 1 : 0;
  if (field(hit, "order", &v)) t->order = v ? 1 : 0;
  if (field(hit, "giant_device", &v)) t->giant_device = v ? 1 : 0;
  if (field(hit, "giant_min_nodes", &v)) t->giant_min_nodes = (int32_t)std::max(65L, v);
  if (field(hit, "heavy_first_cap", &v)) t->heavy_first_cap = (int32_t)std::max(64L, v);
  if (field(hit, "heavy_round_cap", &v)) t->heavy_round_cap = (int32_t)std::max(16L, v);
  if (field(hit, "heavy_device", &v)) t->heavy_device = v ? 1 : 0;
  if (field(hit, "root_split", &v)) t->root_split = v ? 1 : 0;
  if (field(hit, "root_split_min_n", &v)) t->root_split_min_n = (int32_t)std::max(2L, v);
  if (field(hit, "root_split_max", &v)) t->root_split_max = (int32_t)std::max(0L, v);
  if (field(hit, "root_split_chunk", &v)) t->root_split_chunk = (int32_t)std::max(1L, v);
  if (field(hit, "big_one_wave", &v)) t->big_one_wave = v ? 1 : 0;
  if (field(hit, "heavy_levels", &v))
    t->heavy_levels = (int32_t)std::max(0L, std::min((long)kSplitMaxLevels, v));
  b->tuned_from_cache = true;
  return true;
}

// Median device time (ms) of `reps` solves; records and colors of the last.
static float time_solves(mpld_batch* b, int reps, std::vector<DevRecord>& recs,
                         std::vector<int8_t>& colors) {
  std::vector<float> ms;
  const uint32_t flags = b->opt.flags & ~(uint32_t)(MPLD_PLAIN | MPLD_DIRECT);
  device_solve(b->db, flags);   // warm-up (and graph capture)
  check_hip(hipStreamSynchronize(b->ctx->stream), "tune warm-up");
  for (int r = 0; r < reps; ++r) {
    device_solve(b->db, flags);
    check_hip(hipStreamSynchronize(b->ctx->stream), "tune");
    device_time(b->db);
    ms.push_back(b->db.last_search_ms);
  }
  device_fetch(b->db, recs, colors);
  std::sort(ms.begin(), ms.end());
  return ms[ms.size() / 2];
}

static bool same_results(const Image& ia, const std::vector<DevRecord>& ra, const std::vector<int8_t>& ca,
                         const Image& ib, const std::vector<DevRecord>& rb, const std::vector<int8_t>& cb) {
  // records by component id; colors by component (out offsets may differ)
  if (ra.size() != rb.size()) return false;
  for (size_t c = 0; c < ra.size(); ++c) {
    if (ra[c].status != rb[c].status || ra[c].nodes != rb[c].nodes || ra[c].depth != rb[c].depth)
      return false;
    const DevDesc& da = ia.desc[c];
    const DevDesc& db = ib.desc[c];
    if (std::memcmp(ca.data() + da.out_off, cb.data() + db.out_off, (size_t)da.n) != 0) return false;
  }
  return true;
}

}  // namespace mpld

using namespace mpld;

static void to_abi(const Tune& t, mpld_tune* o) {
  o->waves_per_block = t.waves_per_block;
  o->max_blocks = t.max_blocks;
  o->use_graph = t.use_graph;
  o->order = t.order;
  o->giant_device = t.giant_device;
  o->giant_min_nodes = t.giant_min_nodes;
  o->heavy_first_cap = t.heavy_first_cap;
  o->heavy_round_cap = t.heavy_round_cap;
  o->heavy_levels = t.heavy_levels;
  o->heavy_device = t.heavy_device;
  o->root_split = t.root_split;
  o->root_split_min_n = t.root_split_min_n;
  o->root_split_max = t.root_split_max;
  o->root_split_chunk = t.root_split_chunk;
  o->big_one_wave = t.big_one_wave;
}

extern "C" {

int32_t mpld_batch_get_tune(mpld_batch* b, mpld_tune* out) {
  if (!b || !out || out->struct_size != sizeof(mpld_tune)) return MPLD_E_INVALID;
  to_abi(b->db.tune, out);
  out->from_cache = b->tuned_from_cache ? 1 : 0;
  return MPLD_OK;
}

int32_t mpld_batch_set_tune(mpld_batch* b, const mpld_tune* in) {
  try {
    if (!b || !in || in->struct_size != sizeof(mpld_tune)) return MPLD_E_INVALID;
    check_hip(hipSetDevice(b->ctx->device), "hipSetDevice");
    Tune t;
    t.waves_per_block = std::max(1, std::min(4, in->waves_per_block));
    t.max_blocks = std::max(0, in->max_blocks);
    t.use_graph = in->use_graph ? 1 : 0;
    t.order = in->order ? 1 : 0;
    t.giant_device = in->giant_device ? 1 : 0;
    t.giant_min_nodes = std::max(65, in->giant_min_nodes);
    t.heavy_first_cap = std::max(64, in->heavy_first_cap);
    t.heavy_round_cap = std::max(16, in->heavy_round_cap);
    t.heavy_levels = std::max(0, std::min(kSplitMaxLevels, in->heavy_levels));
    t.heavy_device = in->heavy_device ? 1 : 0;
    t.root_split = in->root_split ? 1 : 0;
    t.root_split_min_n = std::max(2, in->root_split_min_n);
    t.root_split_max = std::max(0, in->root_split_max);
    t.root_split_chunk = std::max(1, in->root_split_chunk);
    t.big_one_wave = in->big_one_wave ? 1 : 0;
    batch_pack(b, t);
    b->solved = false;
    set_last_error("");
    return MPLD_OK;
  } catch (const Error& e) {
    set_last_error(e.what);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return MPLD_E_NOMEM;
  } catch (...) {
    set_last_error("unexpected exception");
    return MPLD_E_INTERNAL;
  }
}

int32_t mpld_batch_autotune(mpld_batch* b, int32_t reps, const char* cache_path, mpld_tune* out) {
  try {
    if (!b || !out || out->struct_size != sizeof(mpld_tune) || reps < 1) return MPLD_E_INVALID;
    check_hip(hipSetDevice(b->ctx->device), "hipSetDevice");
    mpld_context* ctx = b->ctx;
    // default parameters: the reference result and time
    Tune base;
    batch_pack(b, base);
    std::vector<DevRecord> rec0, rec;
    std::vector<int8_t> col0, col;
    const float base_ms = time_solves(b, reps, rec0, col0);
    const Image im0 = b->im;
    // candidate set; heavy batches (long solves) only try the parameters that
    // change the work schedule, with one repetition each
    const bool heavy = base_ms > 5.0f;
    const int r = heavy ? 1 : reps;
    std::vector<Tune> cands;
    const int n_reg = (int)b->db.n_reg;
    bool has_giant = false;
    for (const DevDesc& d : b->im.desc) has_giant |= d.n >= base.giant_min_nodes;
    for (int wpb : {1, 2, 4})
      for (int capk : {0, 2, 8})
        for (int graph : {1, 0})
          for (int order : {0, 1})
            for (int giant : {0, 1}) {
              if (giant && !has_giant) continue;
              if (heavy && (wpb != 4 || capk != 0 || graph != 1)) continue;
              Tune t;
              t.waves_per_block = wpb;
              t.max_blocks = capk ? ctx->num_cus * capk : 0;
              if (capk && (n_reg + wpb - 1) / wpb <= t.max_blocks) continue;  // same as uncapped
              t.use_graph = graph;
              t.order = order;
              t.giant_device = giant;
              cands.push_back(t);
            }
    // root split of the register-tier items (four-wave workgroups, largest
    // first): off, only for larger items, other helper chunks
    if (!heavy && n_reg > 0) {
      for (const int v : {0, 8, 16, -4, -64}) {
        Tune t;
        if (v == 0) t.root_split = 0;
        else if (v > 0) t.root_split_min_n = v;
        else t.root_split_chunk = -v;
        cands.push_back(t);
      }
    }
    // big tier: a workgroup sharing the column scan instead of one wave
    if (b->db.n_wide > 0) {
      Tune t;
      t.big_one_wave = 0;
      cands.push_back(t);
    }
    Tune best = base;
    float best_ms = base_ms;
    for (const Tune& t : cands) {
      batch_pack(b, t);
      const float ms = time_solves(b, r, rec, col);
      if (!same_results(im0, rec0, col0, b->im, rec, col))
        fail(MPLD_E_INTERNAL, "autotune: a launch configuration changed the search result");
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
    batch_pack(b, best);
    b->solved = false;
    to_abi(best, out);
    out->best_ms = best_ms;
    out->default_ms = base_ms;
    out->candidates = (int32_t)cands.size() + 1;
    out->from_cache = 0;
    if (const char* p = cache_path_of(cache_path)) {
      std::ofstream f(p, std::ios::app);
      if (f) {
        f << "{\"key\": \"" << shape_key(b) << "\", \"waves_per_block\": " << best.waves_per_block
          << ", \"max_blocks\": " << best.max_blocks << ", \"use_graph\": " << best.use_graph
          << ", \"order\": " << best.order << ", \"giant_device\": " << best.giant_device
          << ", \"giant_min_nodes\": " << best.giant_min_nodes
          << ", \"heavy_first_cap\": " << best.heavy_first_cap
          << ", \"heavy_round_cap\": " << best.heavy_round_cap
          << ", \"heavy_levels\": " << best.heavy_levels
          << ", \"heavy_device\": " << best.heavy_device << ", \"root_split\": " << best.root_split
          << ", \"root_split_min_n\": " << best.root_split_min_n
          << ", \"root_split_max\": " << best.root_split_max
          << ", \"root_split_chunk\": " << best.root_split_chunk
          << ", \"big_one_wave\": " << best.big_one_wave << ", \"best_ms\": " << best_ms
          << ", \"default_ms\": " << base_ms << "}\n";
      }
    }
    set_last_error("");
    return MPLD_OK;
  } catch (const Error& e) {
    set_last_error(e.what);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return MPLD_E_NOMEM;
  } catch (...) {
    set_last_error("unexpected exception");
    return MPLD_E_INTERNAL;
  }
}

}  // extern "C"
