// The request server's host code (server.cpp: slots, plan classes, shared
// slot arenas, host and device requests, completion by per-slot waiters,
// creation and destruction) run end to end on the CPU against the fake HIP
// runtime and the fake plan of fake_device.h, under ThreadSanitizer or
// AddressSanitizer + UBSan, with request patterns of the serving benchmark
// at reduced sizes: one slot and eight, all requests at once and spread
// arrivals, several submitting threads, declared and new plan classes
// (whose arenas differ), device-resident replicas with system ids and
// ready events, shutdown with queued requests.  Every result is checked
// against the fake plan's closed form.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../../include/hsma_server.h"

namespace {

std::atomic<int> g_fail{0};
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                   \
    }                                                             \
  } while (0)

struct Sys {
  int n = 0;
  double L[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0};
  std::vector<double> x, q;
};

Sys make_sys(unsigned seed, int n, double L0, const double shape[3]) {
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  Sys s;
  s.n = n;
  for (int k = 0; k < 3; ++k) {
    s.L[k] = L0 * shape[k];
    s.lo[k] = 0.25 * (k + 1);
  }
  s.x.resize(3 * (size_t)n);
  s.q.resize(n);
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) s.x[3 * i + k] = s.lo[k] + s.L[k] * u(rng);
    s.q[i] = (i % 2 == 0) ? 1.0 : -1.0;
  }
  return s;
}

hsma_params params(int p, int K, int F) {
  hsma_params prm{};
  prm.geometry = HSMA_GEOM_3D;
  prm.precision = HSMA_FP32C;
  prm.lambda = 1.5;
  prm.p = p;
  prm.K = K;
  prm.F = F;
  prm.M = 10;
  prm.nz = 80;
  prm.coulomb_k = 1.0;
  prm.tree_order = 12;
  prm.tree_theta = 0.5;
  return prm;
}

// The fake plan's result for system s run at box scale `scale`.
void check(const Sys& s, double scale, const hsma_result& r, const double* pot, const double* force) {
  CHECK(r.status == HSMA_OK);
  double e = 0;
  for (int i = 0; i < s.n; ++i) e += scale * s.q[i] * s.q[i];
  CHECK(r.energy == e);
  for (int i = 0; i < s.n; ++i) {
    if (pot) CHECK(pot[i] == scale * s.q[i]);
    if (force)
      for (int k = 0; k < 3; ++k) CHECK(force[3 * i + k] == s.q[i] * (s.x[3 * i + k] - s.lo[k]));
    if (g_fail) return;
  }
}

hsma_server* make_server(const hsma_params& prm, int max_n, int slots, int n_classes = 0,
                         const hsma_class* classes = nullptr) {
  hsma_server_cfg cfg{};
  cfg.params = prm;
  for (int k = 0; k < 3; ++k) cfg.box_len[k] = 1.0;
  cfg.max_n = max_n;
  cfg.max_slots = slots;
  cfg.n_classes = n_classes;
  cfg.classes = classes;
  hsma_server* sv = nullptr;
  CHECK(hsma_server_create(&cfg, &sv) == HSMA_OK);
  return sv;
}

uint64_t submit_host(hsma_server* sv, const Sys& s, double* pot, double* force, const hsma_params* prm = nullptr,
                     bool by_box = false) {
  hsma_request r{};
  r.n = s.n;
  r.xyz = s.x.data();
  r.q = s.q.data();
  for (int k = 0; k < 3; ++k) {
    r.box_lo[k] = s.lo[k];
    r.box_len[k] = by_box ? s.L[k] : 0.0;
  }
  r.scale = s.L[0];
  r.params = prm;
  r.potential = pot;
  r.force = force;
  uint64_t t = 0;
  CHECK(hsma_server_submit(sv, &r, &t) == HSMA_OK);
  return t;
}

// A mix of host requests: all at once (twice), then spread arrivals.
void host_mix(int slots, int count, unsigned seed) {
  const double cube[3] = {1, 1, 1};
  std::mt19937 rng(seed);
  std::vector<Sys> sys;
  int nmax = 0;
  for (int i = 0; i < count; ++i) {
    const int n = 2 * (25 + (int)(rng() % 600));
    sys.push_back(make_sys(seed * 1000 + i, n, std::cbrt(n / 0.05), cube));
    nmax = std::max(nmax, n);
  }
  hsma_server* sv = make_server(params(8, 162, 512), nmax, slots);
  std::vector<std::vector<double>> pot(count), force(count);
  for (int i = 0; i < count; ++i) {
    pot[i].assign(sys[i].n, 0.0);
    force[i].assign(3 * (size_t)sys[i].n, 0.0);
  }
  for (int pass = 0; pass < 3; ++pass) {
    std::vector<uint64_t> tk;
    for (int i = 0; i < count; ++i) {
      if (pass == 2) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
      tk.push_back(submit_host(sv, sys[i], i % 3 ? pot[i].data() : nullptr, force[i].data()));
    }
    for (int i = 0; i < count; ++i) {
      hsma_result r{};
      CHECK(hsma_server_wait(sv, tk[i], &r) == HSMA_OK);
      check(sys[i], sys[i].L[0], r, i % 3 ? pot[i].data() : nullptr, force[i].data());
    }
  }
  // several submitting threads, each waiting for its own requests
  std::vector<std::thread> th;
  for (int w = 0; w < 4; ++w)
    th.emplace_back([&, w] {
      for (int i = w; i < count; i += 4) {
        std::vector<double> f(3 * (size_t)sys[i].n);
        const uint64_t t = submit_host(sv, sys[i], nullptr, f.data());
        hsma_result r{};
        CHECK(hsma_server_wait(sv, t, &r) == HSMA_OK);
        check(sys[i], sys[i].L[0], r, nullptr, f.data());
      }
    });
  for (auto& t : th) t.join();
  hsma_server_stats st{};
  CHECK(hsma_server_get_stats(sv, &st) == HSMA_OK);
  CHECK(st.completed == 4 * count && st.classes == 1);
  hsma_server_destroy(sv);
}

// Declared and new plan classes in one server: requests alternate between
// them, and a class created by a request needs a larger arena.
void class_mix() {
  const double cube[3] = {1, 1, 1}, shapeB[3] = {1.0, 1.2, 0.9}, shapeC[3] = {1.0, 1.1, 1.0};
  hsma_params pa = params(8, 162, 512), pb = params(10, 242, 800), pc = params(12, 300, 900);
  hsma_class decl[1];
  decl[0].params = pb;
  for (int k = 0; k < 3; ++k) decl[0].box_len[k] = shapeB[k];
  std::vector<Sys> sys;
  std::vector<int> kind;
  for (int i = 0; i < 48; ++i) {
    const int n = 2 * (40 + 7 * i);
    const int c = i % 3;
    const double* sh = c == 0 ? cube : (c == 1 ? shapeB : shapeC);
    sys.push_back(make_sys(7000 + i, n, std::cbrt(n / 0.05), sh));
    kind.push_back(c);
  }
  hsma_server* sv = make_server(pa, 800, 3, 1, decl);
  for (int round = 0; round < 2; ++round) {
    std::vector<uint64_t> tk;
    std::vector<std::vector<double>> f(sys.size());
    for (size_t i = 0; i < sys.size(); ++i) {
      f[i].assign(3 * (size_t)sys[i].n, 0.0);
      const hsma_params* prm = kind[i] == 0 ? nullptr : (kind[i] == 1 ? &pb : &pc);
      tk.push_back(submit_host(sv, sys[i], nullptr, f[i].data(), prm, kind[i] != 0));
    }
    for (size_t i = 0; i < sys.size(); ++i) {
      hsma_result r{};
      CHECK(hsma_server_wait(sv, tk[i], &r) == HSMA_OK);
      check(sys[i], sys[i].L[0], r, nullptr, f[i].data());
      CHECK(r.plan_class == kind[i]);
    }
  }
  hsma_server_stats st{};
  CHECK(hsma_server_get_stats(sv, &st) == HSMA_OK);
  CHECK(st.classes == 3);
  hsma_server_destroy(sv);
}

// Device-resident replicas: buffers stay put, requests carry system ids and
// a ready event recorded on the caller's stream after it moved the
// positions; repeated keys on a slot count as replays.
void replicas() {
  const double cube[3] = {1, 1, 1};
  const int R = 12;
  std::vector<Sys> sys;
  std::vector<double*> dx(R), dq(R), df(R), de(R);
  for (int i = 0; i < R; ++i) {
    const int n = 2 * (100 + 13 * i);
    sys.push_back(make_sys(9000 + i, n, std::cbrt(n / 0.05), cube));
    CHECK(hipMalloc((void**)&dx[i], sizeof(double) * 3 * n) == hipSuccess);
    CHECK(hipMalloc((void**)&dq[i], sizeof(double) * n) == hipSuccess);
    CHECK(hipMalloc((void**)&df[i], sizeof(double) * 3 * n) == hipSuccess);
    CHECK(hipMalloc((void**)&de[i], sizeof(double)) == hipSuccess);
    std::memcpy(dq[i], sys[i].q.data(), sizeof(double) * n);
  }
  hipStream_t user = nullptr;
  hipEvent_t ready = nullptr;
  CHECK(hipStreamCreateWithFlags(&user, hipStreamNonBlocking) == hipSuccess);
  CHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming) == hipSuccess);
  hsma_server* sv = make_server(params(8, 162, 512), 2 * (100 + 13 * (R - 1)), 4);
  for (int round = 0; round < 5; ++round) {
    std::vector<uint64_t> tk;
    for (int i = 0; i < R; ++i) {
      // the caller's own stream writes the positions, then the request waits for it
      CHECK(hipMemcpyAsync(dx[i], sys[i].x.data(), sizeof(double) * 3 * sys[i].n, hipMemcpyHostToDevice, user) ==
            hipSuccess);
      CHECK(hipEventRecord(ready, user) == hipSuccess);
      hsma_request r{};
      r.n = sys[i].n;
      r.xyz = dx[i];
      r.q = dq[i];
      for (int k = 0; k < 3; ++k) r.box_lo[k] = sys[i].lo[k];
      r.scale = sys[i].L[0];
      r.force = df[i];
      r.energy = de[i];
      r.flags = HSMA_REQ_DEVICE;
      r.system_id = (uint64_t)i + 1;
      r.ready_event = ready;
      uint64_t t = 0;
      CHECK(hsma_server_submit(sv, &r, &t) == HSMA_OK);
      tk.push_back(t);
    }
    for (int i = 0; i < R; ++i) {
      hsma_result r{};
      CHECK(hsma_server_wait(sv, tk[i], &r) == HSMA_OK);
      check(sys[i], sys[i].L[0], r, nullptr, df[i]);
      CHECK(*de[i] == r.energy);
    }
  }
  hsma_server_stats st{};
  CHECK(hsma_server_get_stats(sv, &st) == HSMA_OK);
  std::printf("replicas: completed %lld graph replays %lld affinity hits %lld\n", (long long)st.completed,
              (long long)st.graph_replays, (long long)st.affinity_hits);
  CHECK(st.completed == 5 * R && st.graph_replays > 0 && st.affinity_hits > 0);
  hsma_server_destroy(sv);
  CHECK(hipStreamSynchronize(user) == hipSuccess);
  (void)hipEventDestroy(ready);
  (void)hipStreamDestroy(user);
  for (int i = 0; i < R; ++i) {
    (void)hipFree(dx[i]);
    (void)hipFree(dq[i]);
    (void)hipFree(df[i]);
    (void)hipFree(de[i]);
  }
}

// Shutdown with requests queued behind a busy slot: queued ones come back
// cancelled, admitted ones complete, wait() answers for every ticket.
void shutdown_queued() {
  const double cube[3] = {1, 1, 1};
  std::vector<Sys> sys;
  for (int i = 0; i < 24; ++i) sys.push_back(make_sys(500 + i, 1200, std::cbrt(1200 / 0.05), cube));
  hsma_server* sv = make_server(params(8, 162, 512), 1200, 1);
  std::vector<uint64_t> tk;
  std::vector<std::vector<double>> f(sys.size());
  for (size_t i = 0; i < sys.size(); ++i) {
    f[i].assign(3 * 1200, 0.0);
    tk.push_back(submit_host(sv, sys[i], nullptr, f[i].data()));
  }
  hsma_server_shutdown(sv);
  int done = 0, cancelled = 0;
  for (size_t i = 0; i < sys.size(); ++i) {
    hsma_result r{};
    const hsma_status s = hsma_server_wait(sv, tk[i], &r);
    if (s == HSMA_OK) {
      ++done;
      check(sys[i], sys[i].L[0], r, nullptr, f[i].data());
    } else {
      CHECK(s == HSMA_ERR_CANCELLED);
      ++cancelled;
    }
  }
  CHECK(done + cancelled == (int)sys.size());
  hsma_request r{};
  uint64_t t = 0;
  r.n = sys[0].n;
  r.xyz = sys[0].x.data();
  r.q = sys[0].q.data();
  r.scale = 1.0;
  CHECK(hsma_server_submit(sv, &r, &t) == HSMA_ERR_CANCELLED);
  hsma_server_destroy(sv);
}

}  // namespace

int main() {
  host_mix(1, 40, 1);
  host_mix(8, 96, 2);
  class_mix();
  replicas();
  shutdown_queued();
  if (g_fail) {
    std::printf("%d checks failed\n", g_fail.load());
    return 1;
  }
  std::printf("server flow checks passed\n");
  return 0;
}
