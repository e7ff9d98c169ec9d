// serve_core.h - the scheduling core of the continuous-batching server:
// tickets, the worker pool for host front-ends and result assembly,
// admission by device bytes and component slots, and the tick loop.  The
// device side (uploads, the tick kernels, result downloads) is behind
// ServeExecutor, so that the core can also run against a host-only double
// (the thread-sanitizer test of the scheduling logic).
//
// Threads: submit/poll/wait/get_stats come from callers; `host_threads`
// workers run front-ends and finishes; one scheduler thread runs
// admission and ticks.  Every field of the core is guarded by `mu` except
// `active`, which only the scheduler thread touches.  A request belongs to
// exactly one thread at a time: the worker running its front-end, the
// scheduler from `ready` until it is finished, then the worker assembling
// its result, then whoever fetches it.
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "range_alloc.h"
#include "runtime.h"

namespace mpld {

using ServeClock = std::chrono::steady_clock;

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
  std::vector<DevRecord> recs;   // one per component
  std::vector<int8_t> lcol;
  std::vector<DevDesc> ddesc;    // slot descriptors as uploaded (kept until the tick syncs)
  std::vector<uint32_t> minb;    // MPLD_MINIMIZE: per slot node budget (kept as ddesc)
  std::vector<int32_t> mins;     // MPLD_MINIMIZE: per component minimisation nodes
  // completion
  int32_t error = MPLD_OK;
  std::string error_text;
  ServeClock::time_point t_submit, t_admit;
  std::unique_ptr<mpld_result> result;
};

// One resident register-tier component.
struct ServeActive {
  Request* r;
  int32_t comp;
  int32_t slot;
  bool fresh;
};

class ServeExecutor {
 public:
  virtual ~ServeExecutor() = default;
  // Worker threads, several requests at once: the host front-end of one
  // request; sets r->bytes, r->recs (one entry per component) and
  // r->remaining, or r->error and r->error_text.
  virtual void front_end(Request* r) = 0;
  // Worker threads: the result of a finished request (r->result), or
  // r->error; frees what the request no longer needs.
  virtual void finish(Request* r) = 0;
  // Scheduler thread: copies of an admitted request (r->arena_off and
  // r->slot_base are set).
  virtual void upload(Request* r) = 0;
  // Scheduler thread: one tick.  Appends the register-tier components of
  // `admitted` to `active` and advances every active component; starts the
  // other components of `admitted`, which may run past this tick (busy()
  // is true until a later tick has collected them); drops finished
  // components from `active` (their records go to r->recs), and appends to
  // `finished` every request whose components are all done, with its
  // colors in r->lcol.  Adds its device time to *device_ms.  Throws Error on
  // a device error.
  virtual void tick(std::vector<Request*>& admitted, std::vector<ServeActive>& active,
                    std::vector<Request*>& finished, double* device_ms) = 0;
  // Scheduler thread, once at its start.
  virtual void bind_thread() {}
  // Scheduler thread: work is still running that a tick will collect
  // (then the scheduler ticks even with nothing else to do).
  virtual bool busy() { return false; }
};

class ServeCore {
 public:
  // arena_bytes / max_slots: the admission limits; the executor outlives
  // the core.
  ServeCore(ServeExecutor* exec, int64_t arena_bytes, int32_t max_slots, int host_threads);
  ~ServeCore();
  ServeCore(const ServeCore&) = delete;
  ServeCore& operator=(const ServeCore&) = delete;

  // Takes the request; MPLD_E_CANCELLED (thrown) once the core is stopping.
  void submit(Request* r, uint64_t* ticket);
  int32_t poll(uint64_t ticket, mpld_result** out);
  int32_t wait(uint64_t ticket, int64_t timeout_us, mpld_result** out);
  mpld_server_stats stats();
  // Stops the scheduler after its current tick and the workers; requests
  // not finished by then stay pending (waits on them return
  // MPLD_E_CANCELLED).  Idempotent; the destructor calls it.
  void shutdown();

 private:
  void worker_loop();
  void scheduler_loop();
  void complete(Request* r);        // caller holds mu
  bool try_admit(Request* r);       // caller holds mu
  void release(Request* r);         // caller holds mu
  int32_t take_done(uint64_t ticket, mpld_result** out);   // caller holds mu

  struct Job {
    int kind;  // 0 front-end, 1 finish
    Request* r;
  };

  ServeExecutor* exec_;
  int32_t max_slots_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_sched_, cv_done_;
  std::deque<Job> jobs_;
  std::deque<Request*> ready_;
  std::vector<ServeActive> active_;                   // scheduler thread only
  std::unordered_map<uint64_t, Request*> pending_;   // submitted, not yet finished
  std::unordered_map<uint64_t, Request*> done_;      // finished, not yet fetched
  uint64_t next_ticket_ = 1;
  bool stop_ = false;
  mpld_server_stats stats_{};
  RangeAlloc arena_alloc_, slot_alloc_;
  std::vector<std::thread> workers_;
  std::thread scheduler_;
};

}  // namespace mpld
