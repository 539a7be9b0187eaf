// A CPU stand-in for the part of the HIP runtime API that the request
// server's host code uses, for running that code under ThreadSanitizer and
// AddressSanitizer without a GPU (tests/test_host_sanitizers.py).  "Device"
// memory is host memory; a stream is a worker thread that runs its queued
// operations in order (copies, event records and waits, host functions,
// and the work a fake plan enqueues); hipEventSynchronize blocks until the
// event's last record has run on its stream.
#pragma once

#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 };
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipEventBlockingSync = 1 };
typedef void (*hipHostFn_t)(void* user);

namespace fakehip {

struct Event {
  std::mutex mu;
  std::condition_variable cv;
  uint64_t recorded = 0;  // records enqueued
  uint64_t done = 0;      // records executed
};

struct Stream {
  std::mutex mu;
  std::condition_variable cv, idle_cv;
  std::deque<std::function<void()>> q;
  bool stop = false, busy = false;
  std::thread th;
  Stream() {
    th = std::thread([this] {
      for (;;) {
        std::function<void()> f;
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return stop || !q.empty(); });
          if (q.empty()) return;
          f = std::move(q.front());
          q.pop_front();
          busy = true;
        }
        f();
        {
          std::lock_guard<std::mutex> lk(mu);
          busy = false;
          if (q.empty()) idle_cv.notify_all();
        }
      }
    });
  }
  ~Stream() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    th.join();
  }
  void push(std::function<void()> f) {
    {
      std::lock_guard<std::mutex> lk(mu);
      q.push_back(std::move(f));
    }
    cv.notify_all();
  }
  void drain() {
    std::unique_lock<std::mutex> lk(mu);
    idle_cv.wait(lk, [&] { return q.empty() && !busy; });
  }
};

inline std::mutex& alloc_mu() {
  static std::mutex m;
  return m;
}
inline int64_t& live_bytes() {
  static int64_t b = 0;
  return b;
}

}  // namespace fakehip

typedef fakehip::Stream* hipStream_t;
typedef fakehip::Event* hipEvent_t;

inline const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake HIP error"; }
inline hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
inline hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipMemGetInfo(size_t* freeb, size_t* totalb) {
  *freeb = (size_t)64 << 30;
  *totalb = (size_t)128 << 30;
  return hipSuccess;
}
inline hipError_t hipMalloc(void** p, size_t bytes) {
  *p = std::malloc(bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
template <class T>
inline hipError_t hipMalloc(T** p, size_t bytes) {
  return hipMalloc(reinterpret_cast<void**>(p), bytes);
}
inline hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t bytes) { return hipMalloc(p, bytes); }
inline hipError_t hipHostFree(void* p) { return hipFree(p); }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new fakehip::Stream();
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t s) {
  s->drain();
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  s->push([dst, src, bytes] { std::memcpy(dst, src, bytes); });
  return hipSuccess;
}
inline hipError_t hipLaunchHostFunc(hipStream_t s, hipHostFn_t fn, void* user) {
  s->push([fn, user] { fn(user); });
  return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new fakehip::Event();
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    gen = ++e->recorded;
  }
  s->push([e, gen] {
    std::lock_guard<std::mutex> lk(e->mu);
    if (gen > e->done) e->done = gen;
    e->cv.notify_all();
  });
  return hipSuccess;
}
inline hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    gen = e->recorded;
  }
  s->push([e, gen] {
    std::unique_lock<std::mutex> lk(e->mu);
    e->cv.wait(lk, [&] { return e->done >= gen; });
  });
  return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t e) {
  std::unique_lock<std::mutex> lk(e->mu);
  const uint64_t gen = e->recorded;
  e->cv.wait(lk, [&] { return e->done >= gen; });
  return hipSuccess;
}
