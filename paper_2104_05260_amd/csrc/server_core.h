// Scheduling core of the continuous-batching server (see
// include/hsma_server.h): request queue, tickets, slot admission with
// system affinity, completion, cancellation and shutdown.  It holds no
// device code: a Backend launches a request's work on a slot and reports
// its completion through notify_complete(), from any thread.  The library
// uses the HIP backend in server.cpp; a CPU test drives the same core with
// a fake backend under ThreadSanitizer and AddressSanitizer.
//
// Backend interface (all calls except notify_complete's caller come from
// the core's scheduler thread, never under the core's lock):
//   int slots() const;
//   hsma_status launch(int slot, Request<Payload>& r, std::string& err);
//       enqueue r on the slot; on success the backend later calls
//       core.notify_complete(slot) exactly once
//   void complete(int slot, Request<Payload>& r);
//       the slot's work is done: fill r.res (status, energy, outputs)
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hsma_server.h"

namespace hsma {
namespace serve {

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class Payload>
struct Request {
  uint64_t id = 0;
  uint64_t system = 0;  // affinity key (0: none)
  int cls = 0;          // plan class
  int64_t n = 0;
  Payload payload;
  hsma_result res{};
  bool done = false;
};

template <class Backend, class Payload>
class Core {
 public:
  typedef Request<Payload> Req;

  // affinity_depth: how many of a slot's most recent (system, class) pairs
  // count as still held by it (the backend's per-slot step cache)
  Core(Backend& be, int queue_capacity, int affinity_depth = 8)
      : be_(be), queue_capacity_(queue_capacity), affinity_depth_(affinity_depth < 1 ? 1 : affinity_depth) {
    const int ns = be_.slots();
    slot_req_.resize(ns);
    slot_done_.assign(ns, 0);
    slot_hist_.resize(ns);
    slot_used_.assign(ns, 0);
  }
  Core(const Core&) = delete;
  Core& operator=(const Core&) = delete;
  ~Core() { shutdown(); }

  void start() { th_ = std::thread([this] { loop(); }); }

  // Queues r; returns its ticket in *ticket.  BUSY when the queue is full,
  // CANCELLED after shutdown.
  hsma_status submit(const std::shared_ptr<Req>& r, uint64_t* ticket, std::string& err) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_) {
        err = "server is shutting down";
        return HSMA_ERR_CANCELLED;
      }
      if (queue_capacity_ > 0 && (int)pending_.size() >= queue_capacity_) {
        err = "request queue is full";
        return HSMA_ERR_BUSY;
      }
      r->id = next_id_++;
      r->res.slot = -1;
      r->res.t_submit = now_s();
      tickets_[r->id] = r;
      pending_.push_back(r);
      *ticket = r->id;
    }
    cv_.notify_all();
    return HSMA_OK;
  }

  // Blocks until the request is done; fills *out and forgets the ticket.
  hsma_status wait(uint64_t ticket, hsma_result* out, std::string& err) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end()) {
      err = "unknown ticket";
      return HSMA_ERR_INVALID_ARG;
    }
    std::shared_ptr<Req> r = it->second;
    ++waiters_;
    cv_done_.wait(lk, [&] { return r->done; });
    *out = r->res;
    tickets_.erase(ticket);
    if (--waiters_ == 0) cv_idle_.notify_all();
    if (out->status != HSMA_OK) err = "request failed";
    return out->status;
  }

  // Called by the backend (any thread) when a launched request's work ended.
  // The notification happens under the lock: once the scheduler can see the
  // completion, this thread no longer touches the core, which may then be
  // shut down and destroyed.
  void notify_complete(int slot) {
    std::lock_guard<std::mutex> lk(mu_);
    slot_done_[slot] = 1;
    cv_.notify_all();
  }

  // Stops admitting: queued requests complete as CANCELLED, running ones
  // finish, then the scheduler thread exits.  Idempotent.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      for (auto& r : pending_) {
        r->res.status = HSMA_ERR_CANCELLED;
        r->res.t_done = now_s();
        r->done = true;
      }
      pending_.clear();
    }
    cv_done_.notify_all();
    cv_.notify_all();
    if (th_.joinable()) th_.join();
  }

  // After shutdown: waits until threads blocked in wait() have left.
  void wait_idle() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_idle_.wait(lk, [&] { return waiters_ == 0; });
  }

  int64_t completed() const {
    std::lock_guard<std::mutex> lk(mu_);
    return completed_;
  }
  int64_t affinity_hits() const {
    std::lock_guard<std::mutex> lk(mu_);
    return affinity_hits_;
  }

 private:
  // Free slot for r: a free slot among whose affinity_depth most recent
  // requests the same system and class ran (its captured step can be
  // replayed), else the least recently used free slot; -1 when none is
  // free.  Under mu_.
  int pick_slot(const Req& r) {
    int best = -1;
    for (int i = 0; i < (int)slot_req_.size(); ++i) {
      if (slot_req_[i]) continue;
      if (r.system != 0)
        for (const auto& h : slot_hist_[i])
          if (h.first == r.system && h.second == r.cls) {
            ++affinity_hits_;
            return i;
          }
      if (best < 0 || slot_used_[i] < slot_used_[best]) best = i;
    }
    return best;
  }

  // Records that slot s runs (system, class), most recent first.  Under mu_.
  void remember(int s, uint64_t system, int cls) {
    if (system == 0) return;
    auto& h = slot_hist_[s];
    for (size_t k = 0; k < h.size(); ++k)
      if (h[k].first == system && h[k].second == cls) {
        h.erase(h.begin() + (long)k);
        break;
      }
    h.emplace_front(system, cls);
    if ((int)h.size() > affinity_depth_) h.pop_back();
  }

  void loop() {
    std::vector<std::pair<int, std::shared_ptr<Req>>> admit, finished;
    for (;;) {
      admit.clear();
      finished.clear();
      {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
          for (int i = 0; i < (int)slot_req_.size(); ++i)
            if (slot_req_[i] && slot_done_[i]) {
              finished.emplace_back(i, slot_req_[i]);
              slot_done_[i] = 0;
            }
          // admission in arrival order; a request waits for a free slot
          while (!pending_.empty()) {
            const int s = pick_slot(*pending_.front());
            if (s < 0) break;
            slot_req_[s] = pending_.front();
            remember(s, pending_.front()->system, pending_.front()->cls);
            slot_used_[s] = ++use_clock_;
            admit.emplace_back(s, pending_.front());
            pending_.pop_front();
          }
          if (!admit.empty() || !finished.empty()) break;
          bool running = false;
          for (const auto& q : slot_req_) running |= (bool)q;
          if (stop_ && !running) return;
          cv_.wait(lk);
        }
      }
      for (auto& f : finished) {
        be_.complete(f.first, *f.second);
        f.second->res.t_done = now_s();
        finish(f.first, f.second);
      }
      for (auto& a : admit) {
        a.second->res.t_start = now_s();
        a.second->res.slot = a.first;
        std::string err;
        const hsma_status st = be_.launch(a.first, *a.second, err);
        if (st != HSMA_OK) {
          a.second->res.status = st;
          a.second->res.t_done = now_s();
          finish(a.first, a.second);
        }
      }
    }
  }

  void finish(int slot, const std::shared_ptr<Req>& r) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      slot_req_[slot].reset();
      slot_done_[slot] = 0;
      r->done = true;
      ++completed_;
    }
    cv_done_.notify_all();
  }

  Backend& be_;
  const int queue_capacity_;
  const int affinity_depth_;
  mutable std::mutex mu_;
  std::condition_variable cv_, cv_done_, cv_idle_;
  std::deque<std::shared_ptr<Req>> pending_;
  std::unordered_map<uint64_t, std::shared_ptr<Req>> tickets_;
  std::vector<std::shared_ptr<Req>> slot_req_;
  std::vector<int> slot_done_;
  std::vector<std::deque<std::pair<uint64_t, int>>> slot_hist_;  // (system, class), most recent first
  std::vector<uint64_t> slot_used_;
  uint64_t next_id_ = 1, use_clock_ = 0;
  int64_t completed_ = 0, affinity_hits_ = 0;
  int waiters_ = 0;
  bool stop_ = false;
  std::thread th_;
};

}  // namespace serve
}  // namespace hsma
