// The serving core (server_core.h) on the CPU with a fake backend, for the
// thread and address sanitizers: many submitting and waiting threads,
// completions signalled from another thread after a random delay, launch
// failures, a full queue, shutdown with queued and running requests,
// destruction while threads still block in wait().
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <queue>
#include <random>
#include <thread>
#include <vector>

#include "server_core.h"

namespace {

struct Payload {
  double a = 0, b = 0;
};

struct FakeBackend;
typedef hsma::serve::Core<FakeBackend, Payload> CoreT;
typedef hsma::serve::Request<Payload> Req;

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::abort();                                                     \
    }                                                                   \
  } while (0)

// Completes launched work from its own thread after a delay; the result of
// a request is a function of its payload so that waiters can check it.
struct FakeBackend {
  int nslots;
  int delay_us;
  CoreT* core = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::vector<std::pair<std::chrono::steady_clock::time_point, int>> due;
  std::vector<double> slot_value;
  std::atomic<int> launched{0};
  bool stop = false;
  std::thread th;

  FakeBackend(int ns, int d) : nslots(ns), delay_us(d), slot_value(ns, 0.0) {
    th = std::thread([this] { run(); });
  }
  ~FakeBackend() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    th.join();
  }
  int slots() const { return nslots; }
  hsma_status launch(int slot, Req& r, std::string& err) {
    if (r.n == 13) {
      err = "fake launch failure";
      return HSMA_ERR_DEVICE;
    }
    slot_value[slot] = r.payload.a * 2.0 + r.payload.b;  // the "device work"
    launched.fetch_add(1);
    std::lock_guard<std::mutex> lk(mu);
    due.emplace_back(std::chrono::steady_clock::now() + std::chrono::microseconds(delay_us * (1 + slot % 3)), slot);
    cv.notify_all();
    return HSMA_OK;
  }
  void complete(int slot, Req& r) {
    r.res.energy = slot_value[slot];
    r.res.status = HSMA_OK;
  }
  // (no timed condition-variable waits: this libtsan does not intercept the
  // clock-based wait they compile to, so the delay is a sleep outside the lock)
  void run() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      if (stop) return;
      if (due.empty()) {
        cv.wait(lk);
        continue;
      }
      auto it = std::min_element(due.begin(), due.end());
      const auto when = it->first;
      if (std::chrono::steady_clock::now() < when) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        lk.lock();
        continue;
      }
      const int slot = it->second;
      due.erase(it);
      lk.unlock();
      core->notify_complete(slot);
      lk.lock();
    }
  }
};

std::shared_ptr<Req> make(double a, double b, int64_t n, uint64_t system) {
  auto r = std::make_shared<Req>();
  r->payload.a = a;
  r->payload.b = b;
  r->n = n;
  r->system = system;
  r->res.status = HSMA_OK;
  return r;
}

void many_threads() {
  FakeBackend be(6, 30);
  CoreT core(be, 0);
  be.core = &core;
  core.start();
  std::vector<std::thread> ths;
  std::atomic<int> ok{0}, failed{0};
  for (int t = 0; t < 8; ++t)
    ths.emplace_back([&, t] {
      std::mt19937 rng(t);
      std::vector<std::pair<uint64_t, double>> mine;
      for (int i = 0; i < 150; ++i) {
        const double a = t * 1000 + i, b = rng() % 7;
        const int64_t n = (i % 37 == 5) ? 13 : 100 + i;
        uint64_t ticket = 0;
        std::string err;
        CHECK(core.submit(make(a, b, n, 1 + (uint64_t)(i % 4)), &ticket, err) == HSMA_OK);
        mine.emplace_back(ticket, n == 13 ? -1.0 : a * 2.0 + b);
        if (i % 5 == 4) {
          for (auto& m : mine) {
            hsma_result res{};
            std::string e2;
            const hsma_status st = core.wait(m.first, &res, e2);
            if (m.second < 0) {
              CHECK(st == HSMA_ERR_DEVICE);
              failed.fetch_add(1);
            } else {
              CHECK(st == HSMA_OK && res.energy == m.second && res.slot >= 0 && res.slot < 6);
              CHECK(res.t_submit <= res.t_start && res.t_start <= res.t_done);
              ok.fetch_add(1);
            }
          }
          mine.clear();
        }
      }
      for (auto& m : mine) {
        hsma_result res{};
        std::string e2;
        const hsma_status st = core.wait(m.first, &res, e2);
        CHECK(m.second < 0 ? st == HSMA_ERR_DEVICE : (st == HSMA_OK && res.energy == m.second));
        (m.second < 0 ? failed : ok).fetch_add(1);
      }
    });
  for (auto& th : ths) th.join();
  CHECK(ok.load() + failed.load() == 8 * 150);
  CHECK(core.completed() == 8 * 150);
  CHECK(core.affinity_hits() > 0);
  hsma_result res{};
  std::string err;
  CHECK(core.wait(987654321ull, &res, err) == HSMA_ERR_INVALID_ARG);
  core.shutdown();
  uint64_t ticket = 0;
  CHECK(core.submit(make(1, 1, 10, 0), &ticket, err) == HSMA_ERR_CANCELLED);
}

void full_queue_and_shutdown() {
  FakeBackend be(2, 300000);  // slow: 0.3-0.9 s per request (queued ones stay queued under load)
  CoreT core(be, 4);
  be.core = &core;
  core.start();
  std::vector<uint64_t> tickets;
  std::string err;
  int busy = 0;
  for (int i = 0; i < 12; ++i) {
    uint64_t t = 0;
    const hsma_status st = core.submit(make(i, 0, 10, 0), &t, err);
    if (st == HSMA_ERR_BUSY) ++busy;
    else {
      CHECK(st == HSMA_OK);
      tickets.push_back(t);
    }
  }
  CHECK(busy > 0);
  // waiters block on every ticket while shutdown cancels the queued ones
  std::vector<std::thread> ths;
  std::atomic<int> cancelled{0}, done{0};
  for (uint64_t t : tickets)
    ths.emplace_back([&, t] {
      hsma_result res{};
      std::string e;
      const hsma_status st = core.wait(t, &res, e);
      if (st == HSMA_ERR_CANCELLED) cancelled.fetch_add(1);
      else {
        CHECK(st == HSMA_OK);
        done.fetch_add(1);
      }
    });
  // shut down once a request runs (the others, 0.3 s or more behind it,
  // are still queued)
  for (int k = 0; k < 5000 && be.launched.load() == 0; ++k) std::this_thread::sleep_for(std::chrono::milliseconds(1));
  core.shutdown();
  for (auto& th : ths) th.join();
  CHECK(cancelled.load() + done.load() == (int)tickets.size());
  CHECK(cancelled.load() > 0 && done.load() > 0);
  core.wait_idle();
}

void destroy_with_blocked_waiters() {
  FakeBackend be(1, 5000);
  auto* core = new CoreT(be, 0);
  be.core = core;
  core->start();
  std::string err;
  std::vector<uint64_t> tickets(5);
  for (auto& t : tickets) CHECK(core->submit(make(3, 4, 10, 0), &t, err) == HSMA_OK);
  std::vector<std::thread> ths;
  for (uint64_t t : tickets)
    ths.emplace_back([core, t] {
      hsma_result res{};
      std::string e;
      const hsma_status st = core->wait(t, &res, e);
      CHECK(st == HSMA_OK || st == HSMA_ERR_CANCELLED);
    });
  std::this_thread::sleep_for(std::chrono::milliseconds(2));
  core->shutdown();
  core->wait_idle();  // every waiter has returned before the core goes
  for (auto& th : ths) th.join();
  delete core;
}

}  // namespace

int main() {
  many_threads();
  full_queue_and_shutdown();
  destroy_with_blocked_waiters();
  std::printf("server core checks passed\n");
  return 0;
}
