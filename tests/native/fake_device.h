// Stand-in for the library's device.h when the request server's host code
// (server.cpp) is compiled on the CPU against the fake HIP runtime
// (fake_hip/hip/hip_runtime.h) under the sanitizers.  It provides the types
// and calls server.cpp uses, with a plan whose "step" is a stream task
// writing a closed-form result into the request's buffers:
//   potential_i = scale * q_i,  force_i = q_i * (x_i - lo),  energy = scale * sum q_i^2,
// and that touches every byte of the arena its particle count needs, so a
// slot arena smaller than a class needs shows up under AddressSanitizer.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/hsma.h"

struct double4 {
  double x, y, z, w;
};

namespace hsma {

struct Desc {
  double sx, sy, sz, sigma, scale;
};

struct HostPlan {
  hsma_params prm{};
  double lo[3]{}, L[3]{};
  double cond = 0;
  std::vector<Desc> desc_particles, desc_check;
  std::vector<int> check_axis;
  std::vector<double> Praw, SQ, ysurf;
};

typedef std::function<bool(const std::vector<double>& M, int rows, int cols, std::vector<double>& P, double& cond)>
    PinvFn;

struct LsqJob {
  const std::vector<double>* M = nullptr;
  int rows = 0, cols = 0;
  std::vector<double>* P = nullptr;
  std::vector<double> Rdiag;
  double cond = 0;
  bool ok = false;
};

inline int64_t max_particles(int near_rule) { return near_rule == 0 ? ((int64_t)1 << 30) - 1 : (int64_t)64 << 20; }

inline hsma_status set_last_error(hsma_status s, const std::string&) { return s; }

// The fitting matrix of a class: rows x cols with rows > cols, full rank.
inline void fake_matrix(const hsma_params& prm, const double L[3], std::vector<double>& M, int& rows, int& cols) {
  cols = 4 + prm.p % 5;
  rows = 2 * cols + 3;
  M.assign((size_t)rows * cols, 0.0);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) M[(size_t)r * cols + c] = (r == c ? 2.0 : 0.0) + 0.01 * (r + 1) * (c + 1) * L[1];
}

inline hsma_status device_pinv_batch(std::vector<LsqJob>& jobs, std::string&) {
  for (LsqJob& j : jobs) {
    j.P->assign((size_t)j.rows * j.cols, 0.0);
    for (int r = 0; r < j.rows; ++r)
      for (int c = 0; c < j.cols; ++c) (*j.P)[(size_t)c * j.rows + r] = (*j.M)[(size_t)r * j.cols + c];
    j.Rdiag.assign(j.cols, 1.0);
    j.cond = 1.0;
    j.ok = true;
  }
  return HSMA_OK;
}

inline hsma_status build_host_plan(const hsma_params& prm, const double lo[3], const double L[3], HostPlan& out,
                                   std::string& msg, const PinvFn* pinv = nullptr) {
  if (prm.p < 2) {
    msg = "p must be >= 2";
    return HSMA_ERR_INVALID_ARG;
  }
  out = HostPlan{};
  out.prm = prm;
  for (int k = 0; k < 3; ++k) {
    out.lo[k] = lo[k];
    out.L[k] = L[k];
  }
  std::vector<double> M, P;
  int rows = 0, cols = 0;
  fake_matrix(prm, L, M, rows, cols);
  double cond = 1.0;
  if (pinv && !(*pinv)(M, rows, cols, P, cond)) {
    msg = "rank deficient";
    return HSMA_ERR_RANK;
  }
  out.cond = cond;
  out.Praw.assign((size_t)cols * 2 * prm.K, 0.5);
  out.SQ.assign((size_t)prm.F * cols, 0.25);
  out.ysurf.assign((size_t)prm.F * 3, 1.0);
  out.desc_particles.assign(27, Desc{0, 0, 0, 1, 1});
  out.desc_check.assign(18, Desc{0, 0, 0, 1, 1});
  out.check_axis.assign((size_t)2 * prm.K, 0);
  return HSMA_OK;
}

inline hsma_status validate_host_input(const hsma_params&, const double lo[3], const double L[3], int64_t n,
                                       const double* xyz, const double* q, std::string& msg) {
  double s = 0, a = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(xyz[3 * i + k]) || !(L[k] > 0) || !std::isfinite(lo[k])) {
        msg = "non-finite input";
        return HSMA_ERR_OUT_OF_DOMAIN;
      }
    s += q[i];
    a += std::fabs(q[i]);
  }
  if (std::fabs(s) > 1e-12 * a) {
    msg = "not neutral";
    return HSMA_ERR_NOT_NEUTRAL;
  }
  return HSMA_OK;
}

struct DevicePlan {
  static constexpr int kGraphCache = 8;
  HostPlan host;
  bool use_graph = false;
  long long graph_replays = 0;
  int* d_status = nullptr;
  void* arena = nullptr;
  int64_t cap_n = 0, cur_n = -1;
  double lo[3] = {0, 0, 0}, scale = 1;
  hipEvent_t ev_done = nullptr;
  bool done_recorded = false;
  struct Key {
    int64_t n;
    const void *x, *q, *f;
  };
  std::vector<Key> keys;

  DevicePlan() = default;
  DevicePlan(const DevicePlan&) = delete;
  DevicePlan& operator=(const DevicePlan&) = delete;
  ~DevicePlan() {
    if (done_recorded) (void)hipEventSynchronize(ev_done);
    if (ev_done) (void)hipEventDestroy(ev_done);
    if (d_status) (void)hipFree(d_status);
  }
  hsma_status init(std::string&) {
    if (hipMalloc((void**)&d_status, sizeof(int)) != hipSuccess) return HSMA_ERR_OOM;
    *d_status = 0;
    if (hipEventCreateWithFlags(&ev_done, hipEventDisableTiming) != hipSuccess) return HSMA_ERR_DEVICE;
    return HSMA_OK;
  }
  hsma_status init_scalable(std::string&) { return HSMA_OK; }
  // arena bytes for n particles: grows with the class's order, so classes
  // of one slot need different sizes
  size_t carve(int64_t nmax, char*) const {
    const int64_t cn = nmax > 64 ? nmax : 64;
    return (size_t)(4096 + cn * (48 + 8 * host.prm.p));
  }
  void attach_arena(void* base, int64_t nmax) {
    if (done_recorded) (void)hipEventSynchronize(ev_done);
    arena = base;
    cap_n = nmax > 64 ? nmax : 64;
    cur_n = -1;
  }
  void arena_reused() { cur_n = -1; }
  hsma_status set_box(const double l[3], double s, hipStream_t, std::string&) {
    for (int k = 0; k < 3; ++k) lo[k] = l[k];
    scale = s;
    return HSMA_OK;
  }
  hsma_status run(hipStream_t st, int64_t n, const double* x, const double* q, double* d_e, double* pot,
                  double* force, std::string& err) {
    if (n < 1 || n > cap_n || !arena) {
      err = "fake plan: particle count above the attached arena";
      return HSMA_ERR_INVALID_ARG;
    }
    // a step whose key (size, buffers) this plan has run before counts as
    // a replay (the library captures such steps in graphs)
    const Key key{n, x, q, force};
    bool seen = false;
    for (const Key& k : keys) seen |= k.n == key.n && k.x == key.x && k.q == key.q && k.f == key.f;
    if (use_graph && seen) ++graph_replays;
    if (!seen) keys.push_back(key);
    cur_n = n;
    const size_t bytes = carve(n, nullptr);
    unsigned char* ar = static_cast<unsigned char*>(arena);
    const double s = scale, l0 = lo[0], l1 = lo[1], l2 = lo[2];
    int* status = d_status;
    st->push([=] {
      std::memset(ar, 0x5a, bytes);  // the step's use of its arena
      double e = 0;
      for (int64_t i = 0; i < n; ++i) {
        e += s * q[i] * q[i];
        if (pot) pot[i] = s * q[i];
        if (force) {
          force[3 * i] = q[i] * (x[3 * i] - l0);
          force[3 * i + 1] = q[i] * (x[3 * i + 1] - l1);
          force[3 * i + 2] = q[i] * (x[3 * i + 2] - l2);
        }
      }
      if (d_e) *d_e = e;
      *status = 0;
    });
    if (hipEventRecord(ev_done, st) != hipSuccess) return HSMA_ERR_DEVICE;
    done_recorded = true;
    return HSMA_OK;
  }
  hsma_status wait_done(std::string&) {
    if (done_recorded) (void)hipEventSynchronize(ev_done);
    return HSMA_OK;
  }
};

}  // namespace hsma
