// serve_core.cpp - the scheduling core of the continuous-batching server
// (see serve_core.h).  Host code only: the device work is the executor's.
#include "serve_core.h"

#include <algorithm>
#include <new>

namespace mpld {

ServeCore::ServeCore(ServeExecutor* exec, int64_t arena_bytes, int32_t max_slots, int host_threads)
    : exec_(exec), max_slots_(max_slots) {
  arena_alloc_.reset(arena_bytes);
  slot_alloc_.reset(max_slots);
  for (int t = 0; t < host_threads; ++t) workers_.emplace_back([this] { worker_loop(); });
  scheduler_ = std::thread([this] { scheduler_loop(); });
}

ServeCore::~ServeCore() {
  shutdown();
  // every request is either pending (not finished) or done (not fetched)
  for (auto& kv : pending_) delete kv.second;
  for (auto& kv : done_) delete kv.second;
}

void ServeCore::shutdown() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
    cv_sched_.notify_all();
    cv_work_.notify_all();
    cv_done_.notify_all();
  }
  if (scheduler_.joinable()) scheduler_.join();
  for (auto& t : workers_)
    if (t.joinable()) t.join();
}

void ServeCore::submit(Request* r, uint64_t* ticket) {
  r->t_submit = ServeClock::now();
  std::lock_guard<std::mutex> lk(mu_);
  if (stop_) {
    delete r;
    fail(MPLD_E_CANCELLED, "server is stopping");
  }
  r->ticket = next_ticket_++;
  pending_[r->ticket] = r;
  ++stats_.submitted;
  jobs_.push_back({0, r});
  cv_work_.notify_one();
  *ticket = r->ticket;
}

int32_t ServeCore::take_done(uint64_t ticket, mpld_result** out) {
  Request* r = done_[ticket];
  done_.erase(ticket);
  const int32_t code = r->error;
  set_last_error(r->error_text);
  if (code == MPLD_OK) *out = r->result.release();
  delete r;
  return code;
}

int32_t ServeCore::poll(uint64_t ticket, mpld_result** out) {
  *out = nullptr;
  std::lock_guard<std::mutex> lk(mu_);
  if (done_.count(ticket)) return take_done(ticket, out);
  if (pending_.count(ticket)) return MPLD_E_NOT_READY;
  set_last_error("unknown ticket");
  return MPLD_E_INVALID;
}

int32_t ServeCore::wait(uint64_t ticket, int64_t timeout_us, mpld_result** out) {
  *out = nullptr;
  std::unique_lock<std::mutex> lk(mu_);
  auto is_ready = [&] { return done_.count(ticket) || !pending_.count(ticket) || stop_; };
  if (timeout_us < 0)
    cv_done_.wait(lk, is_ready);
  else
    cv_done_.wait_for(lk, std::chrono::microseconds(timeout_us), is_ready);
  if (done_.count(ticket)) return take_done(ticket, out);
  if (pending_.count(ticket)) return stop_ ? MPLD_E_CANCELLED : MPLD_E_NOT_READY;
  set_last_error("unknown ticket");
  return MPLD_E_INVALID;
}

mpld_server_stats ServeCore::stats() {
  std::lock_guard<std::mutex> lk(mu_);
  return stats_;
}

void ServeCore::complete(Request* r) {
  pending_.erase(r->ticket);
  done_[r->ticket] = r;
  if (r->error == MPLD_OK) {
    ++stats_.completed;
    for (const auto& rec : r->recs) stats_.search_nodes += (int64_t)rec.nodes;
  } else {
    ++stats_.failed;
  }
  cv_done_.notify_all();
}

void ServeCore::worker_loop() {
  for (;;) {
    Job j;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_work_.wait(lk, [&] { return stop_ || !jobs_.empty(); });
      if (jobs_.empty()) return;
      j = jobs_.front();
      jobs_.pop_front();
    }
    if (j.kind == 0) {
      exec_->front_end(j.r);
      std::lock_guard<std::mutex> lk(mu_);
      ready_.push_back(j.r);
      cv_sched_.notify_one();
    } else {
      exec_->finish(j.r);
      std::lock_guard<std::mutex> lk(mu_);
      complete(j.r);
    }
  }
}

bool ServeCore::try_admit(Request* r) {
  const int64_t nc = (int64_t)r->recs.size();
  const int64_t off = arena_alloc_.alloc(std::max<int64_t>(r->bytes, 256), 256);
  if (off < 0) return false;
  int64_t sb = 0;
  if (nc > 0) {
    sb = slot_alloc_.alloc(nc, 1);
    if (sb < 0) {
      arena_alloc_.release(off, std::max<int64_t>(r->bytes, 256));
      return false;
    }
  }
  r->arena_off = off;
  r->slot_base = sb;
  r->t_admit = ServeClock::now();
  stats_.resident_bytes = arena_alloc_.used();
  stats_.resident_components = slot_alloc_.used();
  stats_.peak_bytes = std::max(stats_.peak_bytes, stats_.resident_bytes);
  return true;
}

void ServeCore::release(Request* r) {
  arena_alloc_.release(r->arena_off, std::max<int64_t>(r->bytes, 256));
  if (!r->recs.empty()) slot_alloc_.release(r->slot_base, (int64_t)r->recs.size());
  stats_.resident_bytes = arena_alloc_.used();
  stats_.resident_components = slot_alloc_.used();
}

void ServeCore::scheduler_loop() {
  exec_->bind_thread();
  std::vector<Request*> resident;   // admitted and not finished (scheduler thread only)
  for (;;) {
    std::vector<Request*> admitted;
    {
      std::unique_lock<std::mutex> lk(mu_);
      if (stop_) break;
      if (ready_.empty() && active_.empty()) {
        cv_sched_.wait_for(lk, exec_->busy() ? std::chrono::microseconds(50)
                                             : std::chrono::microseconds(2000));
        if (stop_) break;
      }
      bool waited = false;
      while (!ready_.empty()) {
        Request* r = ready_.front();
        if (r->error != MPLD_OK) {
          ready_.pop_front();
          complete(r);
          continue;
        }
        if (r->bytes > arena_alloc_.capacity() || (int64_t)r->recs.size() > max_slots_) {
          ready_.pop_front();
          r->error = MPLD_E_NOMEM;
          r->error_text = "request needs " + std::to_string(r->bytes) + " device bytes and " +
                          std::to_string(r->recs.size()) +
                          " component slots, more than the server has";
          complete(r);
          continue;
        }
        if (!try_admit(r)) {
          waited = true;
          break;
        }
        ready_.pop_front();
        admitted.push_back(r);
      }
      if (waited) ++stats_.admission_waits;
    }
    if (admitted.empty() && active_.empty() && !exec_->busy()) continue;
    int32_t err = MPLD_OK;
    std::string err_text;
    std::vector<Request*> finished;
    double device_ms = 0.0;
    resident.insert(resident.end(), admitted.begin(), admitted.end());
    try {
      for (Request* r : admitted) exec_->upload(r);
      exec_->tick(admitted, active_, finished, &device_ms);
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
    std::lock_guard<std::mutex> lk(mu_);
    if (err != MPLD_OK) {
      // a device error ends the server: the requests on the device fail
      // with it; the others stay pending (their waits return CANCELLED)
      for (Request* r : resident) {
        r->error = err;
        r->error_text = err_text;
        complete(r);
      }
      active_.clear();
      stop_ = true;
      cv_work_.notify_all();
      cv_done_.notify_all();
      break;
    }
    stats_.device_ms += device_ms;
    ++stats_.ticks;
    for (Request* r : finished) {
      release(r);
      resident.erase(std::find(resident.begin(), resident.end(), r));
      jobs_.push_back({1, r});
    }
    if (!finished.empty()) cv_work_.notify_all();
  }
}

}  // namespace mpld
