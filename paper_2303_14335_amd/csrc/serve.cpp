// serve.cpp - continuous-batching server for whole-layout decomposition
// requests (the serving half of the decomposer library): the device side
// (HipExecutor) of the scheduling core in serve_core.cpp, and the C ABI.
//
// Submit copies a request and hands it to a worker thread for the host
// front-end (layout graph, simplification, sub-graphs, packing).  A single
// scheduler thread owns the context stream and runs ticks:
//   1. admission, in arrival order: a ready request is admitted when its
//      packed image fits the device arena and a range of component slots is
//      free (first fit over bytes and slots);
//   2. upload of the admitted images and their slot descriptors;
//   3. one launch per (trace, count-width) group advancing every resident
//      register-tier component by at most slice_nodes search nodes from the
//      state it keeps in device memory; LDS-tier components of newly
//      admitted requests run to completion in the same tick;
//   4. download of the tick's per-component records; a request whose
//      components are all finished gets its colors downloaded, its device
//      space released, and is finished (recovery, tallies) on a worker.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <deque>
#include <memory>
#include <vector>

#include "runtime.h"
#include "serve_core.h"

namespace mpld {
namespace {

// Layout requests of at least this many rectangles build their graph on the
// device (a fixed cost of about ten launches and two transfers, against
// about 50-90 ns per rectangle for the host's pair search).
constexpr int32_t kDeviceGraphMinRects = 4096;

class HipExecutor : public ServeExecutor {
 public:
  mpld_context* ctx = nullptr;
  mpld_server_options opt{};
  DevBuf arena, slot_desc, slot_rec, slot_state, list, tick_out, counter;
  // stitch partner (local id, 0xff none) of the node whose neighbour mask
  // is arena word w, at byte w: written for stitch-ordered requests
  DevBuf part8;
  // MPLD_MINIMIZE: per slot the minimisation's node budget and its result
  DevBuf slot_minb, slot_min;
  int32_t max_slots = 0;
  // device layout-graph builders for large layout requests (own stream
  // each), taken in turn so that concurrent large requests do not queue on
  // one builder's lock
  std::vector<GraphBuilder*> gbuilders;
  std::atomic<uint32_t> gb_next{0};
  bool device_split = false;   // device-built layouts also split on the device
  // Components above the register tier run to completion on a stream of
  // their own (default priority), one "flight" per tick that admits some,
  // so that a long LDS-tier search does not hold up the register-tier ticks
  // of every other request; flights run in order on that stream, and each
  // tick collects the ones that have finished.
  struct Flight {
    std::vector<std::pair<Request*, int32_t>> items;   // (request, component)
    DevBuf desc, out, gstack, mark_desc;
    PinnedBuf host;             // descriptors up, then the records down
    hipEvent_t start = nullptr, done = nullptr;
    ~Flight() {
      if (start) (void)hipEventDestroy(start);
      if (done) (void)hipEventDestroy(done);
    }
  };
  hipStream_t lds_stream = nullptr;
  hipEvent_t up_ev = nullptr;   // the admitted images are on the device
  std::deque<std::unique_ptr<Flight>> flights;   // in launch order
  std::vector<std::unique_ptr<Flight>> spare;

  ~HipExecutor() override {
    if (ctx) {
      (void)hipSetDevice(ctx->device);
      (void)hipStreamSynchronize(ctx->stream);
      if (lds_stream) (void)hipStreamSynchronize(lds_stream);
    }
    flights.clear();
    spare.clear();
    if (up_ev) (void)hipEventDestroy(up_ev);
    if (lds_stream) (void)hipStreamDestroy(lds_stream);
    for (GraphBuilder* gb : gbuilders) graph_builder_destroy(gb);
  }
  bool busy() override { return !flights.empty(); }
  void front_end(Request* r) override;
  void finish(Request* r) override;
  void upload(Request* r) override;
  void tick(std::vector<Request*>& admitted, std::vector<ServeActive>& active,
            std::vector<Request*>& finished, double* device_ms) override;
  void bind_thread() override { check_hip(hipSetDevice(ctx->device), "serve: hipSetDevice"); }
};

void HipExecutor::front_end(Request* r) {
  try {
    bool built = false, split_done = false;
    if (r->layout) {
      const int32_t nr = (int32_t)r->rects.size();
      if (nr >= kDeviceGraphMinRects && !gbuilders.empty()) {
        // large layouts: pair search on the device, CSR straight back (valid
        // by construction, so no host validation pass)
        GraphBuilder* gb = gbuilders[gb_next.fetch_add(1) % gbuilders.size()];
        if (device_split) {   // simplification and split behind the pair search
          split_done = build_layout_graph_device(*gb, r->rects.data(), nr, r->dmin, r->split, r->g,
                                                 nullptr, &r->s, r->opt.k,
                                                 r->opt.flags & MPLD_SIMPLIFY);
        } else {
          build_layout_graph_device(*gb, r->rects.data(), nr, r->dmin, r->split, r->g, nullptr);
        }
        built = true;
      } else {
        OwnedGraph og;
        build_layout_graph(r->rects.data(), nr, r->dmin, r->split, og, 1);
        r->num_nodes = og.num_nodes;
        r->ce.swap(og.ce);
        r->se.swap(og.se);
      }
      std::vector<mpld_rect>().swap(r->rects);
    }
    if (!built) {
      mpld_graph view{r->num_nodes, 0, (int64_t)r->ce.size() / 2, r->ce.data(),
                      (int64_t)r->se.size() / 2, r->se.data()};
      r->g = make_graph(view);
    }
    if (!split_done) r->s = simplify_and_split(r->g, r->opt.k, r->opt.flags & MPLD_SIMPLIFY);
    const int32_t nc = (int32_t)r->s.comp_ptr.size() - 1;
    const bool stitch = r->opt.flags & MPLD_STITCH_ORDER;
    const bool partners = stitch || (r->opt.flags & MPLD_MINIMIZE);
    std::vector<int32_t> pairs, part;
    for (int32_t c = 0; c < nc; ++c) {
      local_edges(r->g, r->s, c, pairs);
      const int32_t n = r->s.comp_ptr[c + 1] - r->s.comp_ptr[c];
      if (partners) {   // stitch partners inside the component, in its local numbering
        part.assign((size_t)n, -1);
        for (int32_t i = 0; i < n; ++i) {
          const int32_t q = r->g.partner[r->s.order[r->s.comp_ptr[c] + i]];
          if (q >= 0 && r->s.comp_of[q] == c) part[(size_t)i] = r->s.local[q];
        }
      }
      image_add(r->im, ctx, n, pairs.data(), (int64_t)pairs.size() / 2, r->opt.k,
                r->opt.node_budget, r->opt.flags, partners ? part.data() : nullptr);
    }
    r->tier.assign((size_t)nc, 0);
    for (int32_t c : r->im.q_lds) r->tier[c] = 1;
    for (int32_t c : r->im.q_big) r->tier[c] = 2;
    // device footprint: masks, adjacency, colors (each 256-byte aligned)
    auto up = [](int64_t x) { return (x + 255) / 256 * 256; };
    r->off_masks = 0;
    r->off_adj = up((int64_t)r->im.masks.size() * 8);
    r->off_colors = r->off_adj + up((int64_t)r->im.adj32.size() * 4);
    r->bytes = r->off_colors + up(r->im.total_nodes);
    r->recs.assign((size_t)nc, DevRecord{});
    r->remaining = nc;
  } catch (const Error& e) {
    r->error = e.code;
    r->error_text = e.what;
  } catch (const std::bad_alloc&) {
    r->error = MPLD_E_NOMEM;
    r->error_text = "host allocation failed in the front-end";
  }
}

void HipExecutor::finish(Request* r) {
  if (r->error == MPLD_OK) {
    try {
      r->result.reset(new mpld_result());
      const bool minimize = r->opt.flags & MPLD_MINIMIZE;
      if (minimize) {   // only register-tier slots hold a minimisation count
        r->mins.resize(r->recs.size(), 0);
        for (size_t c = 0; c < r->mins.size(); ++c)
          if (r->tier[c] != 0) r->mins[c] = 0;
      }
      assemble_result(r->g, r->s, r->im, r->opt, r->recs, r->lcol, r->result.get(),
                      minimize ? &r->mins : nullptr);
      const auto now = ServeClock::now();
      r->result->queue_us =
          std::chrono::duration<double, std::micro>(r->t_admit - r->t_submit).count();
      r->result->total_us = std::chrono::duration<double, std::micro>(now - r->t_submit).count();
    } catch (const Error& e) {
      r->error = e.code;
      r->error_text = e.what;
      r->result.reset();
    } catch (...) {
      r->error = MPLD_E_NOMEM;
      r->error_text = "host allocation failed while assembling the result";
      r->result.reset();
    }
  }
  // free the bulky parts early; the result and records are all that is kept
  r->g = Graph();
  r->s = Split();
  r->im = Image();
  std::vector<int32_t>().swap(r->ce);
  std::vector<int32_t>().swap(r->se);
  std::vector<int8_t>().swap(r->lcol);
  std::vector<DevDesc>().swap(r->ddesc);
  std::vector<uint32_t>().swap(r->minb);
  std::vector<int32_t>().swap(r->mins);
}

// Enqueues the copy of an admitted request's image to its arena range and
// of its slot descriptors (arena-absolute offsets); the tick's
// synchronisation covers them.
void HipExecutor::upload(Request* r) {
  hipStream_t s = ctx->stream;
  uint8_t* base = arena.as<uint8_t>() + r->arena_off;
  if (!r->im.masks.empty()) {
    check_hip(hipMemcpyAsync(base + r->off_masks, r->im.masks.data(), r->im.masks.size() * 8,
                             hipMemcpyHostToDevice, s), "serve: upload masks");
    if (r->im.stitch || r->im.minimize)   // the partners at the masks' word offsets
      check_hip(hipMemcpyAsync(part8.as<uint8_t>() + (r->arena_off + r->off_masks) / 8,
                               r->im.partner8.data(), r->im.masks.size(), hipMemcpyHostToDevice, s),
                "serve: upload stitch partners");
  }
  if (!r->im.adj32.empty())
    check_hip(hipMemcpyAsync(base + r->off_adj, r->im.adj32.data(), r->im.adj32.size() * 4,
                             hipMemcpyHostToDevice, s), "serve: upload adjacency");
  const int32_t nc = (int32_t)r->recs.size();
  if (nc == 0) return;
  r->ddesc = r->im.desc;
  for (int32_t c = 0; c < nc; ++c) {
    DevDesc& d = r->ddesc[c];
    const int64_t units = r->tier[c] == 0 ? (r->arena_off + r->off_masks) / 8
                                          : (r->arena_off + r->off_adj) / 4;
    d.nbr_off += units;
    d.out_off = (int32_t)(r->arena_off + r->off_colors + d.out_off);
    d.comp = (int32_t)(r->slot_base + c);
  }
  check_hip(hipMemcpyAsync(slot_desc.as<DevDesc>() + r->slot_base, r->ddesc.data(),
                           sizeof(DevDesc) * (size_t)nc, hipMemcpyHostToDevice, s),
            "serve: upload descriptors");
  if (r->opt.flags & MPLD_MINIMIZE) {
    r->minb.assign((size_t)nc, r->opt.min_budget > 0 ? (uint32_t)r->opt.min_budget : 10000u);
    check_hip(hipMemcpyAsync(slot_minb.as<uint32_t>() + r->slot_base, r->minb.data(),
                             sizeof(uint32_t) * (size_t)nc, hipMemcpyHostToDevice, s),
              "serve: upload minimisation budgets");
  }
}

static int count_bits_host(int k) { return k < 4 ? 2 : (k < 8 ? 3 : 4); }
// Launch group of a register-tier component: count width, 8 traced, 16
// stitch-ordered.
static int tick_key(const Request* r) {
  return count_bits_host(r->opt.k) + ((r->opt.flags & MPLD_TRACE_HASH) ? 8 : 0) +
         ((r->opt.flags & MPLD_STITCH_ORDER) ? 16 : 0);
}

void HipExecutor::tick(std::vector<Request*>& admitted, std::vector<ServeActive>& active,
                       std::vector<Request*>& finished, double* device_ms) {
  hipStream_t s = ctx->stream;
  // LDS-tier components of the newly admitted requests, run to completion
  struct LdsItem { Request* r; int32_t comp; };
  // big components: those whose lists fit LDS run on one wave (the
  // one-wave layout), the others on a workgroup; lds_big holds the first
  // group, then the second
  std::vector<LdsItem> lds_small, lds_big, lds_big_wg;
  std::vector<DevDesc> lds_d;
  int lds_small_bytes = 0, lds_big_bytes = 0, lds_wide_bytes_max = 0;
  int64_t big_words = 0;
  int32_t big_max_n = 0;
  for (Request* r : admitted) {
    const int32_t nc = (int32_t)r->recs.size();
    for (int32_t c = 0; c < nc; ++c) {
      if (r->tier[c] == 0) {
        active.push_back({r, c, (int32_t)(r->slot_base + c), true});
        continue;
      }
      const DevDesc& hd = r->im.desc[c];
      const uint32_t* blk = r->im.adj32.data() + hd.nbr_off;
      const int64_t adj_words = (int64_t)blk[hd.n] + hd.n + 1;
      const int32_t maxdeg = (int32_t)blk[adj_words];
      if (r->tier[c] == 1) {
        lds_small.push_back({r, c});
        lds_small_bytes = std::max<int>(lds_small_bytes, (int)lds_bytes_for(hd.n, hd.k, adj_words, maxdeg, false,
                                                                            (r->opt.flags & MPLD_STITCH_ORDER) != 0));
      } else {
        const bool st = (r->opt.flags & MPLD_STITCH_ORDER) != 0;
        const int64_t wb = lds_wide_bytes(hd.n, hd.k, adj_words, maxdeg, st);
        if (wb >= 0 && wb <= ctx->lds_per_block) {
          lds_big.push_back({r, c});
          lds_wide_bytes_max = std::max<int>(lds_wide_bytes_max, (int)wb);
        } else {
          lds_big_wg.push_back({r, c});
          lds_big_bytes = std::max<int>(lds_big_bytes, (int)lds_bytes_for(hd.n, hd.k, adj_words, maxdeg, true, st));
          big_max_n = std::max(big_max_n, hd.n);
        }
        big_words = std::max<int64_t>(big_words, lds_stack_words(hd.n, hd.k, adj_words));
      }
    }
  }
  const size_t n_wide = lds_big.size();
  lds_big.insert(lds_big.end(), lds_big_wg.begin(), lds_big_wg.end());
  auto staged = [&](const LdsItem& it, int32_t out_index) {
    DevDesc d = it.r->im.desc[it.comp];
    d.nbr_off += (it.r->arena_off + it.r->off_adj) / 4;
    d.out_off = (int32_t)(it.r->arena_off + it.r->off_colors + d.out_off);
    d.comp = out_index;   // the record goes to the flight's out[out_index]
    return d;
  };
  for (size_t i = 0; i < lds_small.size(); ++i) lds_d.push_back(staged(lds_small[i], (int32_t)i));
  for (size_t i = 0; i < lds_big.size(); ++i)
    lds_d.push_back(staged(lds_big[i], (int32_t)(lds_small.size() + i)));

  // register tier: group by (trace, stitch order, count width) so each
  // launch has one template
  std::stable_sort(active.begin(), active.end(), [](const ServeActive& a, const ServeActive& b) {
    return tick_key(a.r) < tick_key(b.r);
  });
  std::vector<int32_t> entries(active.size());
  for (size_t i = 0; i < active.size(); ++i)
    entries[i] = active[i].slot | (active[i].fresh ? (int32_t)0x80000000u : 0) |
                 ((active[i].r->opt.flags & (MPLD_MARK_CONFLICTS | MPLD_MINIMIZE)) ? 0x40000000 : 0) |
                 ((active[i].r->opt.flags & MPLD_MINIMIZE) ? 0x20000000 : 0);
  const int32_t len = (int32_t)entries.size();
  const int32_t nl = (int32_t)lds_d.size();
  if (len)
    check_hip(hipMemcpyAsync(list.p, entries.data(), sizeof(int32_t) * len, hipMemcpyHostToDevice, s),
              "serve: upload tick list");
  if (nl) {
    // a flight on the LDS stream, behind this tick's uploads
    std::unique_ptr<Flight> f;
    if (!spare.empty()) {
      f = std::move(spare.back());
      spare.pop_back();
    } else {
      f.reset(new Flight());
      check_hip(hipEventCreate(&f->start), "serve: event");
      check_hip(hipEventCreate(&f->done), "serve: event");
    }
    f->items.clear();
    for (const LdsItem& it : lds_small) f->items.push_back({it.r, it.comp});
    for (const LdsItem& it : lds_big) f->items.push_back({it.r, it.comp});
    const size_t db = sizeof(DevDesc) * (size_t)nl, rb = sizeof(DevRecord) * (size_t)nl;
    if (f->desc.bytes < db) f->desc.alloc(ctx, db);
    if (f->out.bytes < rb) f->out.alloc(ctx, rb);
    const size_t gw = lds_big.empty() ? 0 : (size_t)big_words * lds_big.size();
    if (gw && f->gstack.bytes < sizeof(uint64_t) * gw) f->gstack.alloc(ctx, sizeof(uint64_t) * gw);
    // conflict marking of the components of requests that asked for it
    // (the marking kernel skips the ones whose record is FEASIBLE)
    std::vector<DevDesc> md;
    int64_t mark_bytes = 0;
    for (int32_t i = 0; i < nl; ++i)
      if (f->items[(size_t)i].first->opt.flags & (MPLD_MARK_CONFLICTS | MPLD_MINIMIZE)) {
        md.push_back(lds_d[(size_t)i]);
        mark_bytes = std::max(mark_bytes, mark_lds_bytes(lds_d[(size_t)i].n, lds_d[(size_t)i].k));
      }
    if (mark_bytes > ctx->lds_per_block)
      fail(MPLD_E_UNSUPPORTED, "a component is too large for conflict marking");
    const size_t mb = sizeof(DevDesc) * md.size();
    // staging: descriptors up, records down, marking descriptors up (sized
    // once, before any copy from it is enqueued)
    if (!f->host.reserve(db + rb + mb)) fail(MPLD_E_NOMEM, "serve: pinned host memory");
    std::memcpy(f->host.p, lds_d.data(), db);
    if (mb) std::memcpy(f->host.as<uint8_t>() + db + rb, md.data(), mb);
    check_hip(hipEventRecord(up_ev, s), "serve: event");
    check_hip(hipStreamWaitEvent(lds_stream, up_ev, 0), "serve: stream wait");
    check_hip(hipMemcpyAsync(f->desc.p, f->host.p, db, hipMemcpyHostToDevice, lds_stream),
              "serve: upload LDS descriptors");
    check_hip(hipEventRecord(f->start, lds_stream), "serve: event");
    // per item: 1 traced, 2 stitch-ordered
    std::vector<char> lds_trace(lds_d.size());
    for (size_t i = 0; i < lds_d.size(); ++i) {
      const LdsItem& it = i < lds_small.size() ? lds_small[i] : lds_big[i - lds_small.size()];
      lds_trace[i] = (char)(((it.r->opt.flags & MPLD_TRACE_HASH) ? 1 : 0) |
                            ((it.r->opt.flags & MPLD_STITCH_ORDER) ? 2 : 0));
    }
    auto lds_launch = [&](size_t first, size_t count, bool big, int waves, int bytes) {
      size_t a = first;
      while (a < first + count) {   // one launch per run of equal trace and stitch flags
        size_t b = a;
        while (b < first + count && lds_trace[b] == lds_trace[a]) ++b;
        const int per_cu = std::max(1, std::min(32, (160 * 1024) / std::max(bytes, 1)));
        const int grid = std::max(1, std::min((int)(b - a), ctx->num_cus * per_cu));
        // the big tier's stack areas: one per workgroup, grid <= count
        check_hip(launch_lds_batched((lds_trace[a] & 1) != 0, big, (lds_trace[a] & 2) != 0, waves, grid,
                                     bytes, f->desc.as<DevDesc>() + a, arena.as<uint32_t>(),
                                     (int32_t)(b - a), counter.as<int32_t>() + 1,
                                     big ? f->gstack.as<uint64_t>() : nullptr, (uint64_t)big_words,
                                     f->out.as<DevRecord>(), arena.as<int8_t>(), lds_stream),
                  "serve: LDS launch");
        a = b;
      }
    };
    lds_launch(0, lds_small.size(), false, 1, lds_small_bytes);
    lds_launch(lds_small.size(), n_wide, true, 0, lds_wide_bytes_max);   // one-wave layout
    lds_launch(lds_small.size() + n_wide, lds_big.size() - n_wide, true,
               lds_big_waves(std::max(1, big_max_n)), lds_big_bytes);   // workgroup layout
    if (!md.empty()) {
      if (f->mark_desc.bytes < mb) f->mark_desc.alloc(ctx, mb);
      check_hip(hipMemcpyAsync(f->mark_desc.p, f->host.as<uint8_t>() + db + rb, mb,
                               hipMemcpyHostToDevice, lds_stream), "serve: upload marking descriptors");
      check_hip(launch_mark_lds(std::max(1, std::min((int)md.size(), ctx->num_cus * 4)), (int)mark_bytes,
                                f->mark_desc.as<DevDesc>(), arena.as<uint32_t>(), (int32_t)md.size(),
                                f->out.as<DevRecord>(), arena.as<int8_t>(), lds_stream),
                "serve: conflict marking");
    }
    check_hip(hipMemcpyAsync(f->host.as<uint8_t>() + db, f->out.p, rb, hipMemcpyDeviceToHost,
                             lds_stream), "serve: download LDS records");
    check_hip(hipEventRecord(f->done, lds_stream), "serve: event");
    flights.push_back(std::move(f));
  }
  check_hip(hipEventRecord(ctx->ev[2], s), "serve: event");
  const uint64_t slice = (uint64_t)opt.slice_nodes;
  auto* arena64 = arena.as<uint64_t>();
  auto* arena8 = arena.as<int8_t>();
  for (int32_t a = 0; a < len;) {
    int32_t b = a;
    const Request* ra = active[a].r;
    const int key = tick_key(ra);
    while (b < len && tick_key(active[b].r) == key) ++b;
    const int32_t cnt = b - a;
    const int grid = std::max(1, std::min((cnt + 3) / 4, ctx->num_cus * ctx->reg_blocks_per_cu));
    check_hip(launch_reg_tick((key & 8) != 0, (key & 16) != 0, ra->opt.k, grid,
                              list.as<int32_t>() + a, cnt, counter.as<int32_t>(),
                              slot_desc.as<DevDesc>(), slot_state.as<uint8_t>(),
                              slot_rec.as<DevRecord>(), arena64, arena8, part8.as<uint8_t>(),
                              slot_minb.as<uint32_t>(), slot_min.as<int32_t>(), slice,
                              tick_out.as<DevRecord>() + a, s),
              "serve: tick launch");
    a = b;
  }
  check_hip(hipEventRecord(ctx->ev[3], s), "serve: event");
  std::vector<DevRecord> out((size_t)len);
  if (len)
    check_hip(hipMemcpyAsync(out.data(), tick_out.p, sizeof(DevRecord) * len, hipMemcpyDeviceToHost, s),
              "serve: download tick records");
  check_hip(hipStreamSynchronize(s), "serve: tick");
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]) == hipSuccess) *device_ms += ms;

  // bookkeeping: finished components leave the active set
  std::vector<ServeActive> keep;
  keep.reserve(active.size());
  for (int32_t i = 0; i < len; ++i) {
    ServeActive a = active[i];
    if (out[i].status < 0) {
      a.fresh = false;
      keep.push_back(a);
      continue;
    }
    if (out[i].status > MPLD_BUDGET_EXHAUSTED) fail(MPLD_E_INTERNAL, "serving tick reported a broken state");
    a.r->recs[a.comp] = out[i];
    if (--a.r->remaining == 0) finished.push_back(a.r);
  }
  active.swap(keep);
  // flights that have landed, in launch order
  while (!flights.empty()) {
    Flight& f = *flights.front();
    const hipError_t q = hipEventQuery(f.done);
    if (q == hipErrorNotReady) break;
    check_hip(q, "serve: LDS flight");
    float fms = 0.f;
    if (hipEventElapsedTime(&fms, f.start, f.done) == hipSuccess) *device_ms += fms;
    const DevRecord* lout = reinterpret_cast<const DevRecord*>(
        f.host.as<uint8_t>() + sizeof(DevDesc) * f.items.size());
    for (size_t i = 0; i < f.items.size(); ++i) {
      if (lout[i].status < 0 || lout[i].status > MPLD_BUDGET_EXHAUSTED)
        fail(MPLD_E_INTERNAL, "serving LDS search reported a broken state");
      Request* r = f.items[i].first;
      r->recs[(size_t)f.items[i].second] = lout[i];
      if (--r->remaining == 0) finished.push_back(r);
    }
    spare.push_back(std::move(flights.front()));
    flights.pop_front();
  }
  for (Request* r : admitted)
    if (r->recs.empty()) finished.push_back(r);   // nothing to search
  // colors of finished requests (the core then releases their device space)
  for (Request* r : finished) {
    r->lcol.resize((size_t)r->im.total_nodes);
    if (!r->lcol.empty())
      check_hip(hipMemcpyAsync(r->lcol.data(), arena.as<uint8_t>() + r->arena_off + r->off_colors,
                               r->lcol.size(), hipMemcpyDeviceToHost, s),
                "serve: download colors");
    if ((r->opt.flags & MPLD_MINIMIZE) && !r->recs.empty()) {
      r->mins.assign(r->recs.size(), 0);
      check_hip(hipMemcpyAsync(r->mins.data(), slot_min.as<int32_t>() + r->slot_base,
                               sizeof(int32_t) * r->mins.size(), hipMemcpyDeviceToHost, s),
                "serve: download minimisation counts");
    }
  }
  if (!finished.empty()) check_hip(hipStreamSynchronize(s), "serve: colors");
}

}  // namespace
}  // namespace mpld

using namespace mpld;

struct mpld_server {
  HipExecutor exec;
  std::unique_ptr<ServeCore> core;   // destroyed first: it stops the threads using `exec`
  ~mpld_server() { core.reset(); }
};

namespace {

template <class F>
int32_t guard_s(F&& f) {
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
  }
}

void check_opts(const mpld_options* o) {
  if (!o || o->struct_size != sizeof(mpld_options)) fail(MPLD_E_INVALID, "bad options");
  if (o->k < 2 || o->k > MPLD_MAX_K) fail(MPLD_E_INVALID, "k must be in [2, 8]");
  if (o->node_budget < 1) fail(MPLD_E_INVALID, "node_budget must be >= 1");
  if (o->min_budget < 0) fail(MPLD_E_INVALID, "min_budget must be >= 0 (0 = 10000)");
  if (o->flags & (MPLD_PLAIN | MPLD_FORCE_WAVE | MPLD_FORCE_LDS | MPLD_FORCE_GLOBAL | MPLD_FORCE_DEVICE))
    fail(MPLD_E_INVALID, "serving takes no PLAIN or FORCE_* flags");
}


}  // namespace

extern "C" {

int32_t mpld_server_create(mpld_context* ctx, const mpld_server_options* opt, mpld_server** out) {
  return guard_s([&] {
    if (!ctx || !out) fail(MPLD_E_INVALID, "NULL argument");
    *out = nullptr;
    mpld_server_options o{};
    o.struct_size = sizeof(o);
    if (opt) {
      if (opt->struct_size != sizeof(mpld_server_options)) fail(MPLD_E_INVALID, "server options size");
      o = *opt;
    }
    if (o.max_components <= 0) o.max_components = 65536;
    if (o.max_components > (1 << 28)) fail(MPLD_E_INVALID, "max_components is at most 2^28");
    if (o.arena_bytes <= 0) o.arena_bytes = 256ll << 20;
    if (o.arena_bytes > (2ll << 30) - 256) fail(MPLD_E_INVALID, "arena_bytes is at most 2 GiB");
    if (o.slice_nodes <= 0) o.slice_nodes = 4096;
    if (o.host_threads <= 0) o.host_threads = host_threads();
    check_hip(hipSetDevice(ctx->device), "hipSetDevice");
    auto* s = new mpld_server();
    s->exec.ctx = ctx;
    s->exec.opt = o;
    s->exec.max_slots = o.max_components;
    HipExecutor* x = &s->exec;
    try {
      x->arena.alloc(ctx, (size_t)o.arena_bytes);
      x->part8.alloc(ctx, (size_t)o.arena_bytes / 8 + 8);
      x->slot_minb.alloc(ctx, sizeof(uint32_t) * (size_t)x->max_slots);
      x->slot_min.alloc(ctx, sizeof(int32_t) * (size_t)x->max_slots);
      x->slot_desc.alloc(ctx, sizeof(DevDesc) * (size_t)x->max_slots);
      x->slot_rec.alloc(ctx, sizeof(DevRecord) * (size_t)x->max_slots);
      x->slot_state.alloc(ctx, kRegStateBytes * (size_t)x->max_slots);
      x->list.alloc(ctx, sizeof(int32_t) * (size_t)x->max_slots);
      x->tick_out.alloc(ctx, sizeof(DevRecord) * (size_t)x->max_slots);
      check_hip(hipStreamCreate(&x->lds_stream), "serve: LDS stream");
      check_hip(hipEventCreateWithFlags(&x->up_ev, hipEventDisableTiming), "serve: event");
      x->counter.alloc(ctx, sizeof(int32_t) * 4);
      // one builder by default: with four, the measured p99 latency of a
      // Poisson mix of layout requests rose by about a third
      const int nb = o.graph_builders == 0 ? 1 : std::max(0, o.graph_builders);
      for (int i = 0; i < nb; ++i) {
        x->gbuilders.push_back(graph_builder_create(ctx, true));
        // sized ahead for layouts of up to 64k nodes: growing a builder
        // while requests wait behind it cost several milliseconds each time
        graph_builder_reserve(*x->gbuilders.back(), 1 << 16);
      }
      // device split by default: over three paired runs of 1,000 requests
      // it took p99 latency from 2.9-3.5 ms (host split) to 2.5-2.7 ms
      x->device_split = o.device_split >= 0;
      check_hip(hipMemsetAsync(x->counter.p, 0, sizeof(int32_t) * 4, ctx->stream), "serve: clear");
      check_hip(hipStreamSynchronize(ctx->stream), "serve: clear");
      s->core.reset(new ServeCore(x, o.arena_bytes, x->max_slots, o.host_threads));
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

int32_t mpld_server_submit(mpld_server* s, const mpld_graph* g, const mpld_options* opt,
                           uint64_t* ticket) {
  return guard_s([&] {
    if (!s || !g || !ticket) fail(MPLD_E_INVALID, "NULL argument");
    check_opts(opt);
    if (g->num_nodes < 0 || g->num_ce < 0 || g->num_se < 0 || (g->num_ce && !g->ce) ||
        (g->num_se && !g->se))
      fail(MPLD_E_INVALID, "bad graph");
    auto* r = new Request();
    r->opt = *opt;
    r->num_nodes = g->num_nodes;
    r->ce.assign(g->ce, g->ce + 2 * g->num_ce);
    r->se.assign(g->se, g->se + 2 * g->num_se);
    s->core->submit(r, ticket);
  });
}

int32_t mpld_server_submit_layout(mpld_server* s, const mpld_rect* rects, int32_t n, int32_t dmin_nm,
                                  int32_t split_len_nm, const mpld_options* opt, uint64_t* ticket) {
  return guard_s([&] {
    if (!s || !ticket || n < 0 || (n > 0 && !rects) || dmin_nm < 0 || split_len_nm < 0)
      fail(MPLD_E_INVALID, "bad argument");
    check_opts(opt);
    auto* r = new Request();
    r->opt = *opt;
    r->layout = true;
    r->rects.assign(rects, rects + n);
    r->dmin = dmin_nm;
    r->split = split_len_nm;
    s->core->submit(r, ticket);
  });
}

int32_t mpld_server_poll(mpld_server* s, uint64_t ticket, mpld_result** out) {
  if (!s || !out) return MPLD_E_INVALID;
  return s->core->poll(ticket, out);
}

int32_t mpld_server_wait(mpld_server* s, uint64_t ticket, int64_t timeout_us, mpld_result** out) {
  if (!s || !out) return MPLD_E_INVALID;
  return s->core->wait(ticket, timeout_us, out);
}

int32_t mpld_server_get_stats(mpld_server* s, mpld_server_stats* out) {
  if (!s || !out) return MPLD_E_INVALID;
  *out = s->core->stats();
  return MPLD_OK;
}

int32_t mpld_server_destroy(mpld_server* s) {
  if (!s) return MPLD_OK;
  s->core->shutdown();
  delete s;   // the core's requests, then the executor's device buffers and builders
  return MPLD_OK;
}

}  // extern "C"
