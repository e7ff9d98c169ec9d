// serve_double.cpp - the server's scheduling core (csrc/serve_core.cpp)
// against a host-only double of its device executor, for a
// ThreadSanitizer build: several submitting threads, waiting and polling
// threads, the worker pool and the scheduler run concurrently; admission
// waits for arena bytes and slots; some requests fail in the front-end,
// some are too large for the arena; a second core is shut down with
// requests still in flight.  Every result is checked against what its
// request determines, and the statistics against the counts.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "serve_core.h"

using namespace mpld;

namespace {

int g_fail = 0;
std::mutex g_fail_mu;
#define CHECK(cond, ...)                                               \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::lock_guard<std::mutex> lk_(g_fail_mu);                      \
      std::fprintf(stderr, "FAILED %s:%d: ", __FILE__, __LINE__);        \
      std::fprintf(stderr, __VA_ARGS__);                               \
      std::fprintf(stderr, "\n");                                      \
      g_fail = 1;                                                      \
    }                                                                  \
  } while (0)

// Request i (num_nodes = i): i % 5 + 1 components, each needing
// 1 + (i + c) % 4 ticks and reporting i * 10 + c search nodes; 700 bytes per
// component; i % 17 == 3 fails in the front-end; i % 29 == 7 asks for more
// bytes than any arena here.
int comps_of(int i) { return i % 5 + 1; }

class FakeExecutor : public ServeExecutor {
 public:
  void front_end(Request* r) override {
    jitter(r->num_nodes);
    const int i = r->num_nodes;
    if (i % 17 == 3) {
      r->error = MPLD_E_INVALID;
      r->error_text = "front-end rejects this request";
      return;
    }
    const int nc = comps_of(i);
    r->recs.assign((size_t)nc, DevRecord{});
    r->remaining = nc;
    r->bytes = i % 29 == 7 ? (int64_t)1 << 40 : 700 * nc;
    r->im.total_nodes = nc;
  }
  void finish(Request* r) override {
    jitter(r->num_nodes + 1);
    r->result.reset(new mpld_result());
    r->result->colors.assign(r->lcol.begin(), r->lcol.end());
  }
  void upload(Request* r) override {
    // the scheduler's own state: no lock needed, only its thread is here
    uploaded_.push_back(r->ticket);
  }
  void tick(std::vector<Request*>& admitted, std::vector<ServeActive>& active,
            std::vector<Request*>& finished, double* device_ms) override {
    for (Request* r : admitted) {
      for (int32_t c = 0; c < (int32_t)r->recs.size(); ++c) {
        active.push_back({r, c, (int32_t)(r->slot_base + c), true});
        left_[{r, c}] = 1 + (r->num_nodes + c) % 4;
      }
      if (r->recs.empty()) finished.push_back(r);
    }
    std::vector<ServeActive> keep;
    for (ServeActive a : active) {
      if (--left_[{a.r, a.comp}] > 0) {
        a.fresh = false;
        keep.push_back(a);
        continue;
      }
      left_.erase({a.r, a.comp});
      a.r->recs[(size_t)a.comp].status = MPLD_FEASIBLE;
      a.r->recs[(size_t)a.comp].nodes = (uint64_t)(a.r->num_nodes * 10 + a.comp);
      if (--a.r->remaining == 0) {
        a.r->lcol.assign((size_t)a.r->im.total_nodes, (int8_t)(a.r->num_nodes % 3));
        finished.push_back(a.r);
      }
    }
    active.swap(keep);
    *device_ms += 0.001;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }

 private:
  static void jitter(int seed) {
    std::this_thread::sleep_for(std::chrono::microseconds((seed * 37) % 200));
  }
  std::vector<uint64_t> uploaded_;
  std::map<std::pair<Request*, int32_t>, int> left_;
};

void run_mix() {
  FakeExecutor ex;
  const int64_t arena = 6000;     // room for a few requests at a time
  ServeCore core(&ex, arena, 12, 4);
  constexpr int kSubmitters = 4, kPer = 120;
  std::vector<std::vector<std::pair<int, uint64_t>>> tickets(kSubmitters);
  std::vector<std::thread> th;
  for (int t = 0; t < kSubmitters; ++t)
    th.emplace_back([&, t] {
      for (int j = 0; j < kPer; ++j) {
        const int i = t * kPer + j + 1;
        auto* r = new Request();
        r->num_nodes = i;
        uint64_t tk = 0;
        core.submit(r, &tk);
        tickets[(size_t)t].push_back({i, tk});
      }
    });
  for (auto& x : th) x.join();
  th.clear();
  std::atomic<int> ok{0}, invalid{0}, nomem{0};
  std::atomic<bool> watching{true};
  std::thread watcher([&] {   // statistics read while the scheduler ticks
    int64_t last = 0;
    while (watching.load()) {
      const mpld_server_stats st = core.stats();
      CHECK(st.completed + st.failed >= last, "counts went back");
      last = st.completed + st.failed;
      std::this_thread::yield();
    }
  });
  for (int t = 0; t < kSubmitters; ++t)
    th.emplace_back([&, t] {
      for (auto [i, tk] : tickets[(size_t)t]) {
        mpld_result* res = nullptr;
        int32_t code = MPLD_E_NOT_READY;
        if (i % 2) {
          while ((code = core.poll(tk, &res)) == MPLD_E_NOT_READY) std::this_thread::yield();
        } else {
          code = core.wait(tk, -1, &res);
        }
        if (i % 17 == 3) {
          CHECK(code == MPLD_E_INVALID, "request %d: %d", i, code);
          ++invalid;
        } else if (i % 29 == 7) {
          CHECK(code == MPLD_E_NOMEM, "request %d: %d", i, code);
          ++nomem;
        } else {
          CHECK(code == MPLD_OK && res, "request %d: %d", i, code);
          if (res) {
            CHECK((int)res->colors.size() == comps_of(i), "request %d colors", i);
            for (int8_t c : res->colors) CHECK(c == i % 3, "request %d color", i);
          }
          ++ok;
        }
        delete res;
        mpld_result* again = nullptr;
        CHECK(core.poll(tk, &again) == MPLD_E_INVALID, "ticket %llu fetched twice",
              (unsigned long long)tk);
      }
    });
  for (auto& x : th) x.join();
  watching = false;
  watcher.join();
  const mpld_server_stats st = core.stats();
  const int n = kSubmitters * kPer;
  CHECK(st.submitted == n, "submitted %lld", (long long)st.submitted);
  CHECK(st.completed == ok.load(), "completed %lld vs %d", (long long)st.completed, ok.load());
  CHECK(st.failed == invalid.load() + nomem.load(), "failed %lld", (long long)st.failed);
  CHECK(st.peak_bytes <= arena, "peak %lld", (long long)st.peak_bytes);
  CHECK(st.admission_waits > 0, "no admission waits");
  CHECK(st.resident_bytes == 0 && st.resident_components == 0, "space not released");
  int64_t nodes = 0;
  for (int t = 0; t < kSubmitters; ++t)
    for (auto [i, tk] : tickets[(size_t)t]) {
      (void)tk;
      if (i % 17 == 3 || i % 29 == 7) continue;
      for (int c = 0; c < comps_of(i); ++c) nodes += i * 10 + c;
    }
  CHECK(st.search_nodes == nodes, "search nodes %lld vs %lld", (long long)st.search_nodes,
        (long long)nodes);
  std::printf("mix: %d ok, %d invalid, %d nomem, %lld ticks, %lld admission waits\n", ok.load(),
              invalid.load(), nomem.load(), (long long)st.ticks, (long long)st.admission_waits);
}

void run_shutdown_in_flight() {
  FakeExecutor ex;
  auto* core = new ServeCore(&ex, 3000, 8, 3);
  std::vector<uint64_t> tks;
  for (int i = 1; i <= 200; ++i) {
    auto* r = new Request();
    r->num_nodes = i;
    uint64_t tk = 0;
    core->submit(r, &tk);
    tks.push_back(tk);
  }
  std::thread waiter([&] {
    for (uint64_t tk : tks) {
      mpld_result* res = nullptr;
      const int32_t code = core->wait(tk, -1, &res);
      CHECK(code == MPLD_OK || code == MPLD_E_CANCELLED || code == MPLD_E_INVALID ||
                code == MPLD_E_NOMEM,
            "wait during shutdown: %d", code);
      delete res;
    }
  });
  std::this_thread::sleep_for(std::chrono::milliseconds(3));
  core->shutdown();
  waiter.join();
  bool refused = false;
  try {
    auto* r = new Request();
    uint64_t tk = 0;
    core->submit(r, &tk);
  } catch (const Error& e) {
    refused = e.code == MPLD_E_CANCELLED;
  }
  CHECK(refused, "submit after shutdown accepted");
  delete core;
  std::printf("shutdown with requests in flight: ok\n");
}

}  // namespace

int main() {
  run_mix();
  run_shutdown_in_flight();
  if (g_fail) return 1;
  std::printf("serve double passed\n");
  return 0;
}
