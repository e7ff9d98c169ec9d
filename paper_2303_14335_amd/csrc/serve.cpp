// serve.cpp - continuous-batching server for whole-layout decomposition
// requests (the serving half of the decomposer library).
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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "range_alloc.h"
#include "runtime.h"

namespace mpld {
namespace {

using Clock = std::chrono::steady_clock;

// Layout requests of at least this many rectangles build their graph on the
// device (a fixed cost of about ten launches and two transfers, against
// about 50-90 ns per rectangle for the host's pair search).
constexpr int32_t kDeviceGraphMinRects = 4096;

struct Request {
  uint64_t ticket = 0;
  bool layout = false;
  std::vector<mpld_rect> rects;
  int32_t dmin = 0, split = 0;
  int32_t num_nodes = 0;
  std::vector<int32_t> ce, se;
  mpld_options opt{};
  // front-end
  Graph g;
  Split s;
  Image im;
  std::vector<uint8_t> tier;  // per component: 0 register, 1 LDS, 2 big
  int64_t off_masks = 0, off_adj = 0, off_colors = 0, bytes = 0;
  // residency
  int64_t arena_off = -1;
  int64_t slot_base = -1;
  int32_t remaining = 0;
  std::vector<DevRecord> recs;
  std::vector<int8_t> lcol;
  std::vector<DevDesc> ddesc;  // slot descriptors as uploaded (kept until the tick syncs)
  // completion
  int32_t error = MPLD_OK;
  std::string error_text;
  Clock::time_point t_submit, t_admit;
  std::unique_ptr<mpld_result> result;
};

struct Job {
  int kind;  // 0 front-end, 1 finish
  Request* r;
};

// One resident register-tier component.
struct Active {
  Request* r;
  int32_t comp;
  int32_t slot;
  bool fresh;
};

}  // namespace
}  // namespace mpld

using namespace mpld;

struct mpld_server {
  mpld_context* ctx = nullptr;
  mpld_server_options opt{};
  // device
  DevBuf arena, slot_desc, slot_rec, slot_state, list, tick_out, lds_desc, lds_out, counter, gstack;
  int32_t max_slots = 0;
  RangeAlloc arena_alloc, slot_alloc;
  int64_t gstack_words = 0;
  // host state
  std::mutex mu;
  std::condition_variable cv_work, cv_sched, cv_done;
  std::deque<Job> jobs;
  std::deque<Request*> ready;
  std::vector<Active> active;
  std::unordered_map<uint64_t, Request*> pending;  // submitted, not yet finished
  std::unordered_map<uint64_t, Request*> done;     // finished, not yet fetched
  uint64_t next_ticket = 1;
  bool stop = false;
  mpld_server_stats stats{};
  std::vector<std::thread> workers;
  std::thread scheduler;
  // device layout-graph builders for large layout requests (own stream
  // each), taken in turn so that concurrent large requests do not queue on
  // one builder's lock
  std::vector<GraphBuilder*> gbuilders;
  std::atomic<uint32_t> gb_next{0};
  bool device_split = false;   // device-built layouts also split on the device

  void worker_loop();
  void scheduler_loop();
  void front_end(Request* r);
  void finish(Request* r);
  void complete(Request* r);  // caller holds mu
  bool try_admit(Request* r);
  void upload(Request* r);
  void tick(std::vector<Request*>& admitted);
  void release(Request* r);
};

// ---------------------------------------------------------------------------

void mpld_server::front_end(Request* r) {
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
    std::vector<int32_t> pairs;
    for (int32_t c = 0; c < nc; ++c) {
      local_edges(r->g, r->s, c, pairs);
      const int32_t n = r->s.comp_ptr[c + 1] - r->s.comp_ptr[c];
      image_add(r->im, ctx, n, pairs.data(), (int64_t)pairs.size() / 2, r->opt.k,
                r->opt.node_budget, r->opt.flags);
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

void mpld_server::finish(Request* r) {
  if (r->error == MPLD_OK) {
    try {
      r->result.reset(new mpld_result());
      assemble_result(r->g, r->s, r->im, r->opt, r->recs, r->lcol, r->result.get());
      const auto now = Clock::now();
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
  std::lock_guard<std::mutex> lk(mu);
  complete(r);
}

void mpld_server::complete(Request* r) {
  pending.erase(r->ticket);
  done[r->ticket] = r;
  if (r->error == MPLD_OK) {
    ++stats.completed;
    for (const auto& rec : r->recs) stats.search_nodes += (int64_t)rec.nodes;
  } else {
    ++stats.failed;
  }
  cv_done.notify_all();
}

void mpld_server::worker_loop() {
  for (;;) {
    Job j;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !jobs.empty(); });
      if (jobs.empty()) return;
      j = jobs.front();
      jobs.pop_front();
    }
    if (j.kind == 0) {
      front_end(j.r);
      std::lock_guard<std::mutex> lk(mu);
      ready.push_back(j.r);
      cv_sched.notify_one();
    } else {
      finish(j.r);
    }
  }
}

// Admission by device bytes and slots (caller holds mu).
bool mpld_server::try_admit(Request* r) {
  const int64_t nc = (int64_t)r->recs.size();
  const int64_t off = arena_alloc.alloc(std::max<int64_t>(r->bytes, 256), 256);
  if (off < 0) return false;
  int64_t sb = 0;
  if (nc > 0) {
    sb = slot_alloc.alloc(nc, 1);
    if (sb < 0) {
      arena_alloc.release(off, std::max<int64_t>(r->bytes, 256));
      return false;
    }
  }
  r->arena_off = off;
  r->slot_base = sb;
  r->t_admit = Clock::now();
  stats.resident_bytes = arena_alloc.used();
  stats.resident_components = slot_alloc.used();
  stats.peak_bytes = std::max(stats.peak_bytes, stats.resident_bytes);
  return true;
}

void mpld_server::release(Request* r) {
  std::lock_guard<std::mutex> lk(mu);
  arena_alloc.release(r->arena_off, std::max<int64_t>(r->bytes, 256));
  if (!r->recs.empty()) slot_alloc.release(r->slot_base, (int64_t)r->recs.size());
  stats.resident_bytes = arena_alloc.used();
  stats.resident_components = slot_alloc.used();
}

// Enqueues the copy of an admitted request's image to its arena range and
// of its slot descriptors (arena-absolute offsets); the tick's
// synchronisation covers them.
void mpld_server::upload(Request* r) {
  hipStream_t s = ctx->stream;
  uint8_t* base = arena.as<uint8_t>() + r->arena_off;
  if (!r->im.masks.empty())
    check_hip(hipMemcpyAsync(base + r->off_masks, r->im.masks.data(), r->im.masks.size() * 8,
                             hipMemcpyHostToDevice, s), "serve: upload masks");
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
}

static int count_bits_host(int k) { return k < 4 ? 2 : (k < 8 ? 3 : 4); }

void mpld_server::tick(std::vector<Request*>& admitted) {
  hipStream_t s = ctx->stream;
  // LDS-tier components of the newly admitted requests, run to completion
  struct LdsItem { Request* r; int32_t comp; };
  std::vector<LdsItem> lds_small, lds_big;
  std::vector<DevDesc> lds_d;
  int lds_small_bytes = 0, lds_big_bytes = 0;
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
        lds_small_bytes = std::max<int>(lds_small_bytes, (int)lds_bytes_for(hd.n, hd.k, adj_words, maxdeg, false));
      } else {
        lds_big.push_back({r, c});
        lds_big_bytes = std::max<int>(lds_big_bytes, (int)lds_bytes_for(hd.n, hd.k, adj_words, maxdeg, true));
        big_words = std::max<int64_t>(big_words, lds_stack_words(hd.n, hd.k, adj_words));
        big_max_n = std::max(big_max_n, hd.n);
      }
    }
  }
  auto staged = [&](const LdsItem& it, int32_t out_index) {
    DevDesc d = it.r->im.desc[it.comp];
    d.nbr_off += (it.r->arena_off + it.r->off_adj) / 4;
    d.out_off = (int32_t)(it.r->arena_off + it.r->off_colors + d.out_off);
    d.comp = out_index;   // the record goes to lds_out[out_index]
    return d;
  };
  for (size_t i = 0; i < lds_small.size(); ++i) lds_d.push_back(staged(lds_small[i], (int32_t)i));
  for (size_t i = 0; i < lds_big.size(); ++i)
    lds_d.push_back(staged(lds_big[i], (int32_t)(lds_small.size() + i)));

  // register tier: group by (trace, count width) so each launch has one template
  std::stable_sort(active.begin(), active.end(), [](const Active& a, const Active& b) {
    const int ka = count_bits_host(a.r->opt.k) + ((a.r->opt.flags & MPLD_TRACE_HASH) ? 8 : 0);
    const int kb = count_bits_host(b.r->opt.k) + ((b.r->opt.flags & MPLD_TRACE_HASH) ? 8 : 0);
    return ka < kb;
  });
  std::vector<int32_t> entries(active.size());
  for (size_t i = 0; i < active.size(); ++i)
    entries[i] = active[i].slot | (active[i].fresh ? (int32_t)0x80000000u : 0);
  const int32_t len = (int32_t)entries.size();
  const int32_t nl = (int32_t)lds_d.size();
  if (len)
    check_hip(hipMemcpyAsync(list.p, entries.data(), sizeof(int32_t) * len, hipMemcpyHostToDevice, s),
              "serve: upload tick list");
  if (nl)
    check_hip(hipMemcpyAsync(lds_desc.p, lds_d.data(), sizeof(DevDesc) * nl, hipMemcpyHostToDevice, s),
              "serve: upload LDS descriptors");
  if (!lds_big.empty() && big_words * (int64_t)lds_big.size() > gstack_words) {
    check_hip(hipStreamSynchronize(s), "serve: grow stack");
    gstack_words = big_words * (int64_t)lds_big.size();
    gstack.alloc(ctx, sizeof(uint64_t) * (size_t)gstack_words);
  }
  check_hip(hipEventRecord(ctx->ev[2], s), "serve: event");
  const uint64_t slice = (uint64_t)opt.slice_nodes;
  auto* arena64 = arena.as<uint64_t>();
  auto* arena8 = arena.as<int8_t>();
  for (int32_t a = 0; a < len;) {
    int32_t b = a;
    const Request* ra = active[a].r;
    const int key = count_bits_host(ra->opt.k) + ((ra->opt.flags & MPLD_TRACE_HASH) ? 8 : 0);
    while (b < len && count_bits_host(active[b].r->opt.k) +
                              ((active[b].r->opt.flags & MPLD_TRACE_HASH) ? 8 : 0) == key)
      ++b;
    const int32_t cnt = b - a;
    const int grid = std::max(1, std::min((cnt + 3) / 4, ctx->num_cus * ctx->reg_blocks_per_cu));
    check_hip(launch_reg_tick(key >= 8, ra->opt.k, grid, list.as<int32_t>() + a, cnt,
                              counter.as<int32_t>(), slot_desc.as<DevDesc>(), slot_state.as<uint8_t>(),
                              slot_rec.as<DevRecord>(), arena64, arena8, slice,
                              tick_out.as<DevRecord>() + a, s),
              "serve: tick launch");
    a = b;
  }
  std::vector<char> lds_trace(lds_d.size());
  for (size_t i = 0; i < lds_d.size(); ++i) {
    const LdsItem& it = i < lds_small.size() ? lds_small[i] : lds_big[i - lds_small.size()];
    lds_trace[i] = (it.r->opt.flags & MPLD_TRACE_HASH) ? 1 : 0;
  }
  auto lds_launch = [&](size_t first, size_t count, bool big, int bytes) {
    size_t a = first;
    while (a < first + count) {   // one launch per run of equal trace flag
      size_t b = a;
      while (b < first + count && lds_trace[b] == lds_trace[a]) ++b;
      const int per_cu = std::max(1, std::min(32, (160 * 1024) / std::max(bytes, 1)));
      const int grid = std::max(1, std::min((int)(b - a), ctx->num_cus * per_cu));
      check_hip(launch_lds_batched(lds_trace[a] != 0, big, big ? lds_big_waves(big_max_n) : 1, grid,
                                   bytes, lds_desc.as<DevDesc>() + a,
                                   arena.as<uint32_t>(), (int32_t)(b - a), counter.as<int32_t>() + 1,
                                   big ? gstack.as<uint64_t>() : nullptr, (uint64_t)big_words,
                                   lds_out.as<DevRecord>(), arena8, s),
                "serve: LDS launch");
      a = b;
    }
  };
  lds_launch(0, lds_small.size(), false, lds_small_bytes);
  lds_launch(lds_small.size(), lds_big.size(), true, lds_big_bytes);
  check_hip(hipEventRecord(ctx->ev[3], s), "serve: event");
  std::vector<DevRecord> out((size_t)len), lout((size_t)nl);
  if (len)
    check_hip(hipMemcpyAsync(out.data(), tick_out.p, sizeof(DevRecord) * len, hipMemcpyDeviceToHost, s),
              "serve: download tick records");
  if (nl)
    check_hip(hipMemcpyAsync(lout.data(), lds_out.p, sizeof(DevRecord) * nl, hipMemcpyDeviceToHost, s),
              "serve: download LDS records");
  check_hip(hipStreamSynchronize(s), "serve: tick");
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]) == hipSuccess) stats.device_ms += ms;

  // bookkeeping: finished components leave the active set
  std::vector<Request*> finished;
  std::vector<Active> keep;
  keep.reserve(active.size());
  for (int32_t i = 0; i < len; ++i) {
    Active a = active[i];
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
  for (int32_t i = 0; i < nl; ++i) {
    const LdsItem& it = i < (int32_t)lds_small.size() ? lds_small[i] : lds_big[i - lds_small.size()];
    if (lout[i].status < 0 || lout[i].status > MPLD_BUDGET_EXHAUSTED)
      fail(MPLD_E_INTERNAL, "serving LDS search reported a broken state");
    it.r->recs[it.comp] = lout[i];
    if (--it.r->remaining == 0) finished.push_back(it.r);
  }
  for (Request* r : admitted)
    if (r->recs.empty()) finished.push_back(r);   // nothing to search
  // colors of finished requests, then release their device space
  for (Request* r : finished) {
    r->lcol.resize((size_t)r->im.total_nodes);
    if (!r->lcol.empty())
      check_hip(hipMemcpyAsync(r->lcol.data(), arena.as<uint8_t>() + r->arena_off + r->off_colors,
                               r->lcol.size(), hipMemcpyDeviceToHost, s),
                "serve: download colors");
  }
  if (!finished.empty()) check_hip(hipStreamSynchronize(s), "serve: colors");
  for (Request* r : finished) release(r);
  std::lock_guard<std::mutex> lk(mu);
  ++stats.ticks;
  for (Request* r : finished) jobs.push_back({1, r});
  if (!finished.empty()) cv_work.notify_all();
}

void mpld_server::scheduler_loop() {
  check_hip(hipSetDevice(ctx->device), "serve: hipSetDevice");
  for (;;) {
    std::vector<Request*> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop) break;
      if (ready.empty() && active.empty()) {
        cv_sched.wait_for(lk, std::chrono::milliseconds(2));
        if (stop) break;
      }
      bool waited = false;
      while (!ready.empty()) {
        Request* r = ready.front();
        if (r->error != MPLD_OK) {
          ready.pop_front();
          complete(r);
          continue;
        }
        if (r->bytes > arena_alloc.capacity() || (int64_t)r->recs.size() > max_slots) {
          ready.pop_front();
          r->error = MPLD_E_NOMEM;
          r->error_text = "request needs " + std::to_string(r->bytes) + " device bytes and " +
                          std::to_string(r->recs.size()) + " component slots, more than the server has";
          complete(r);
          continue;
        }
        if (!try_admit(r)) {
          waited = true;
          break;
        }
        ready.pop_front();
        admitted.push_back(r);
      }
      if (waited) ++stats.admission_waits;
    }
    if (admitted.empty() && active.empty()) continue;
    int32_t err = MPLD_OK;
    std::string err_text;
    try {
      for (Request* r : admitted) upload(r);
      tick(admitted);
    } catch (const Error& e) {
      err = e.code;
      err_text = e.what;
    } catch (const std::bad_alloc&) {
      err = MPLD_E_NOMEM;
      err_text = "host allocation failed in the scheduler";
    } catch (...) {
      err = MPLD_E_INTERNAL;
      err_text = "unexpected exception in the scheduler";
    }
    if (err != MPLD_OK) {
      // a device error ends the server: every resident and waiting request fails
      std::lock_guard<std::mutex> lk(mu);
      for (auto& kv : pending) {
        Request* r = kv.second;
        r->error = err;
        r->error_text = err_text;
      }
      stop = true;
      cv_work.notify_all();
      cv_done.notify_all();
      break;
    }
  }
}

// ---------------------------------------------------------------------------

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
  if (o->flags & (MPLD_PLAIN | MPLD_FORCE_WAVE | MPLD_FORCE_LDS | MPLD_FORCE_GLOBAL | MPLD_FORCE_DEVICE))
    fail(MPLD_E_INVALID, "serving takes no PLAIN or FORCE_* flags");
  if (o->flags & MPLD_MARK_CONFLICTS)
    fail(MPLD_E_UNSUPPORTED, "serving does not mark conflicts (MPLD_MARK_CONFLICTS)");
  if (o->flags & MPLD_STITCH_ORDER)
    fail(MPLD_E_UNSUPPORTED, "serving keeps the ascending row order (MPLD_STITCH_ORDER)");
  if (o->flags & MPLD_MINIMIZE)
    fail(MPLD_E_UNSUPPORTED, "serving does not run the Eq. 1 minimisation (MPLD_MINIMIZE)");
}

int32_t submit_request(mpld_server* s, Request* r, uint64_t* ticket) {
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    delete r;
    fail(MPLD_E_CANCELLED, "server is stopping");
  }
  r->ticket = s->next_ticket++;
  s->pending[r->ticket] = r;
  ++s->stats.submitted;
  s->jobs.push_back({0, r});
  s->cv_work.notify_one();
  *ticket = r->ticket;
  return MPLD_OK;
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
    if (o.arena_bytes <= 0) o.arena_bytes = 256ll << 20;
    if (o.arena_bytes > (2ll << 30) - 256) fail(MPLD_E_INVALID, "arena_bytes is at most 2 GiB");
    if (o.slice_nodes <= 0) o.slice_nodes = 4096;
    if (o.host_threads <= 0) o.host_threads = host_threads();
    check_hip(hipSetDevice(ctx->device), "hipSetDevice");
    auto* s = new mpld_server();
    s->ctx = ctx;
    s->opt = o;
    s->max_slots = o.max_components;
    try {
      s->arena.alloc(ctx, (size_t)o.arena_bytes);
      s->slot_desc.alloc(ctx, sizeof(DevDesc) * (size_t)s->max_slots);
      s->slot_rec.alloc(ctx, sizeof(DevRecord) * (size_t)s->max_slots);
      s->slot_state.alloc(ctx, kRegStateBytes * (size_t)s->max_slots);
      s->list.alloc(ctx, sizeof(int32_t) * (size_t)s->max_slots);
      s->tick_out.alloc(ctx, sizeof(DevRecord) * (size_t)s->max_slots);
      s->lds_desc.alloc(ctx, sizeof(DevDesc) * (size_t)s->max_slots);
      s->lds_out.alloc(ctx, sizeof(DevRecord) * (size_t)s->max_slots);
      s->counter.alloc(ctx, sizeof(int32_t) * 4);
      // one builder by default: with four, the measured p99 latency of a
      // Poisson mix of layout requests rose by about a third
      const int nb = o.graph_builders == 0 ? 1 : std::max(0, o.graph_builders);
      for (int i = 0; i < nb; ++i) {
        s->gbuilders.push_back(graph_builder_create(ctx, true));
        // sized ahead for layouts of up to 64k nodes: growing a builder
        // while requests wait behind it cost several milliseconds each time
        graph_builder_reserve(*s->gbuilders.back(), 1 << 16);
      }
      // device split by default: over three paired runs of 1,000 requests
      // it took p99 latency from 2.9-3.5 ms (host split) to 2.5-2.7 ms
      s->device_split = o.device_split >= 0;
      check_hip(hipMemsetAsync(s->counter.p, 0, sizeof(int32_t) * 4, ctx->stream), "serve: clear");
      check_hip(hipStreamSynchronize(ctx->stream), "serve: clear");
    } catch (...) {
      for (GraphBuilder* gb : s->gbuilders) graph_builder_destroy(gb);
      delete s;
      throw;
    }
    s->arena_alloc.reset(o.arena_bytes);
    s->slot_alloc.reset(s->max_slots);
    for (int t = 0; t < o.host_threads; ++t) s->workers.emplace_back([s] { s->worker_loop(); });
    s->scheduler = std::thread([s] { s->scheduler_loop(); });
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
    submit_request(s, r, ticket);
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
    submit_request(s, r, ticket);
  });
}

static int32_t take_done(mpld_server* s, uint64_t ticket, mpld_result** out) {
  // caller holds mu; the ticket is finished
  Request* r = s->done[ticket];
  s->done.erase(ticket);
  const int32_t code = r->error;
  set_last_error(r->error_text);
  if (code == MPLD_OK) *out = r->result.release();
  delete r;
  return code;
}

int32_t mpld_server_poll(mpld_server* s, uint64_t ticket, mpld_result** out) {
  if (!s || !out) return MPLD_E_INVALID;
  *out = nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->done.count(ticket)) return take_done(s, ticket, out);
  if (s->pending.count(ticket)) return MPLD_E_NOT_READY;
  set_last_error("unknown ticket");
  return MPLD_E_INVALID;
}

int32_t mpld_server_wait(mpld_server* s, uint64_t ticket, int64_t timeout_us, mpld_result** out) {
  if (!s || !out) return MPLD_E_INVALID;
  *out = nullptr;
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] { return s->done.count(ticket) || !s->pending.count(ticket) || s->stop; };
  if (timeout_us < 0)
    s->cv_done.wait(lk, ready);
  else
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
  if (s->done.count(ticket)) return take_done(s, ticket, out);
  if (s->pending.count(ticket)) return s->stop ? MPLD_E_CANCELLED : MPLD_E_NOT_READY;
  set_last_error("unknown ticket");
  return MPLD_E_INVALID;
}

int32_t mpld_server_get_stats(mpld_server* s, mpld_server_stats* out) {
  if (!s || !out) return MPLD_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return MPLD_OK;
}

int32_t mpld_server_destroy(mpld_server* s) {
  if (!s) return MPLD_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_sched.notify_all();
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  if (s->scheduler.joinable()) s->scheduler.join();
  for (auto& t : s->workers)
    if (t.joinable()) t.join();
  (void)hipSetDevice(s->ctx->device);
  (void)hipStreamSynchronize(s->ctx->stream);
  // every request is either pending (not finished) or done (not fetched)
  for (auto& kv : s->pending) delete kv.second;
  for (auto& kv : s->done) delete kv.second;
  for (GraphBuilder* gb : s->gbuilders) graph_builder_destroy(gb);
  delete s;
  return MPLD_OK;
}

}  // extern "C"
