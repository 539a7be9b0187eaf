// Continuous-batching request server (see include/hsma_server.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hsma_server.h"
#include "device.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t id = 0;
  int64_t n = 0;
  std::vector<double> xyz, q;
  double lo[3] = {0, 0, 0};
  double scale = 1;
  double* pot = nullptr;
  double* force = nullptr;
  hsma_result res{};
  bool done = false;
};

// One device slot: a plan (constants + arena) re-targeted per request, its
// own stream, device input/output buffers and pinned host staging.
struct Slot {
  std::unique_ptr<hsma::DevicePlan> plan;
  hipStream_t stream = nullptr;
  hipEvent_t done_ev = nullptr;
  double* d_io = nullptr;   // xyz (3 cap) | q (cap) | pot (cap) | force (3 cap) | energy
  double* h_io = nullptr;   // pinned mirror, plus one int status at the end
  int64_t cap = 0;
  std::shared_ptr<Req> req;  // running request
  hsma_status enqueue_status = HSMA_OK;
};

}  // namespace

struct hsma_server {
  hsma_server_cfg cfg{};
  int device = 0;
  std::vector<Slot> slots;
  int64_t bytes_per_slot = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Req>> pending;
  std::unordered_map<uint64_t, std::shared_ptr<Req>> tickets;
  uint64_t next_id = 1;
  bool stop = false;
  int waiters = 0;
  std::condition_variable cv_idle;
  std::thread th;

  void loop();
  hsma_status dispatch(Slot& s, const std::shared_ptr<Req>& r, std::string& err);
  void complete(Slot& s);
};

hsma_status hsma_server::dispatch(Slot& s, const std::shared_ptr<Req>& r, std::string& err) {
  const int64_t n = r->n, cap = s.cap;
  double* h = s.h_io;
  std::memcpy(h, r->xyz.data(), sizeof(double) * 3 * n);
  std::memcpy(h + 3 * cap, r->q.data(), sizeof(double) * n);
  double* d_xyz = s.d_io;
  double* d_q = s.d_io + 3 * cap;
  double* d_pot = s.d_io + 4 * cap;
  double* d_force = s.d_io + 5 * cap;
  double* d_e = s.d_io + 8 * cap;
  hipError_t e;
  if ((e = hipMemcpyAsync(d_xyz, h, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s.stream)) != hipSuccess ||
      (e = hipMemcpyAsync(d_q, h + 3 * cap, sizeof(double) * n, hipMemcpyHostToDevice, s.stream)) != hipSuccess) {
    err = std::string("copy in: ") + hipGetErrorString(e);
    return HSMA_ERR_DEVICE;
  }
  hsma_status st = s.plan->set_box(r->lo, r->scale, s.stream, err);
  if (st != HSMA_OK) return st;
  st = s.plan->run(s.stream, n, d_xyz, d_q, d_e, r->pot ? d_pot : nullptr, r->force ? d_force : nullptr, err);
  if (st != HSMA_OK) return st;
  int* h_status = (int*)(h + 8 * cap + 1);
  if ((e = hipMemcpyAsync(h + 8 * cap, d_e, sizeof(double), hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
      (e = hipMemcpyAsync(h_status, s.plan->d_status, sizeof(int), hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
      (r->pot && (e = hipMemcpyAsync(h + 4 * cap, d_pot, sizeof(double) * n, hipMemcpyDeviceToHost, s.stream)) != hipSuccess) ||
      (r->force && (e = hipMemcpyAsync(h + 5 * cap, d_force, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s.stream)) != hipSuccess) ||
      (e = hipEventRecord(s.done_ev, s.stream)) != hipSuccess) {
    err = std::string("copy out: ") + hipGetErrorString(e);
    return HSMA_ERR_DEVICE;
  }
  return HSMA_OK;
}

void hsma_server::complete(Slot& s) {
  std::shared_ptr<Req> r = s.req;
  const int64_t cap = s.cap;
  const double* h = s.h_io;
  if (r->pot) std::memcpy(r->pot, h + 4 * cap, sizeof(double) * r->n);
  if (r->force) std::memcpy(r->force, h + 5 * cap, sizeof(double) * 3 * r->n);
  r->res.energy = h[8 * cap];
  r->res.status = (hsma_status) * (const int*)(h + 8 * cap + 1);
  r->res.t_done = now_s();
  s.req.reset();
  std::lock_guard<std::mutex> lk(mu);
  r->done = true;
  cv_done.notify_all();
}

void hsma_server::loop() {
  (void)hipSetDevice(device);
  for (;;) {
    // admit queued requests into free slots, in arrival order
    std::vector<std::pair<size_t, std::shared_ptr<Req>>> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      bool running = false;
      for (const Slot& s : slots) running |= (bool)s.req;
      if (!running && pending.empty()) {
        if (stop) break;
        cv_work.wait_for(lk, std::chrono::milliseconds(20));
        continue;
      }
      for (size_t i = 0; i < slots.size() && !pending.empty(); ++i) {
        if (slots[i].req) continue;
        admit.emplace_back(i, pending.front());
        slots[i].req = pending.front();
        pending.pop_front();
      }
    }
    for (auto& a : admit) {
      Slot& s = slots[a.first];
      a.second->res.t_start = now_s();
      a.second->res.slot = (int)a.first;
      std::string err;
      hsma_status st = dispatch(s, a.second, err);
      if (st != HSMA_OK) {
        (void)hipStreamSynchronize(s.stream);
        a.second->res.status = st;
        a.second->res.t_done = now_s();
        s.req.reset();
        std::lock_guard<std::mutex> lk(mu);
        a.second->done = true;
        cv_done.notify_all();
      }
    }
    // retire finished requests
    bool any = false;
    for (Slot& s : slots) {
      if (!s.req) continue;
      if (hipEventQuery(s.done_ev) == hipSuccess) {
        complete(s);
        any = true;
      }
    }
    if (!any && admit.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

extern "C" {

hsma_status hsma_server_create(const hsma_server_cfg* cfg, hsma_server** out) {
  if (!cfg || !out) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (cfg->max_n < 1 || cfg->max_slots < 1)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "max_n and max_slots must be positive");
  if (cfg->max_n > hsma::max_particles(cfg->params.near_rule))
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "max_n is above the particles one call can take");
  std::unique_ptr<hsma_server> sv(new hsma_server());
  sv->cfg = *cfg;
  std::string msg;
  hsma::HostPlan hp;
  const double lo0[3] = {0, 0, 0};
  hsma_status st = hsma::build_host_plan(cfg->params, lo0, cfg->box_len, hp, msg);
  if (st != HSMA_OK) return hsma::set_last_error(st, msg);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return hsma::set_last_error(HSMA_ERR_NO_DEVICE, "no HIP device");
  (void)hipGetDevice(&sv->device);
  size_t freeb = 0, totalb = 0;
  (void)hipMemGetInfo(&freeb, &totalb);
  const int64_t budget = cfg->hbm_budget > 0 ? cfg->hbm_budget : (int64_t)(freeb / 2);
  for (int i = 0; i < cfg->max_slots; ++i) {
    Slot s;
    s.plan.reset(new hsma::DevicePlan());
    s.plan->host = hp;
    if ((st = s.plan->init(msg)) != HSMA_OK) return hsma::set_last_error(st, msg);
    if ((st = s.plan->init_scalable(msg)) != HSMA_OK) return hsma::set_last_error(st, msg);
    if ((st = s.plan->reserve(cfg->max_n, msg)) != HSMA_OK) return hsma::set_last_error(st, msg);
    s.plan->use_graph = true;  // repeated sizes in a slot replay a captured step
    s.cap = cfg->max_n;
    const int64_t io_bytes = (int64_t)sizeof(double) * (8 * s.cap + 2);
    const int64_t plan_bytes = (int64_t)(sizeof(double) * 2 * (hp.Praw.size() + hp.SQ.size() * 2 + hp.ysurf.size() * 2) +
                                         sizeof(hsma::Desc) * 2 * (hp.desc_particles.size() + hp.desc_check.size()) +
                                         sizeof(double4) * 2 * hp.check_axis.size());
    const int64_t per = (int64_t)s.plan->arena_bytes + io_bytes + plan_bytes;
    if (i == 0) sv->bytes_per_slot = per;
    if ((int64_t)(i + 1) * per > budget) {
      if (i == 0) return hsma::set_last_error(HSMA_ERR_OOM, "HBM budget smaller than one slot");
      break;
    }
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done_ev, hipEventDisableTiming) != hipSuccess ||
        hipMalloc((void**)&s.d_io, sizeof(double) * (8 * s.cap + 2)) != hipSuccess ||
        hipHostMalloc((void**)&s.h_io, sizeof(double) * (8 * s.cap + 2)) != hipSuccess)
      return hsma::set_last_error(HSMA_ERR_OOM, "slot allocation failed");
    sv->slots.push_back(std::move(s));
  }
  hsma_server* raw = sv.get();
  raw->th = std::thread([raw] { raw->loop(); });
  *out = sv.release();
  return HSMA_OK;
}

hsma_status hsma_server_get_slots(const hsma_server* s, int* nslots, int64_t* bytes_per_slot) {
  if (!s) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL server");
  if (nslots) *nslots = (int)s->slots.size();
  if (bytes_per_slot) *bytes_per_slot = s->bytes_per_slot;
  return HSMA_OK;
}

hsma_status hsma_server_submit(hsma_server* s, const hsma_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket || !req->xyz || !req->q) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (req->n < 1) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "n must be >= 1");
  if (req->n > s->cfg.max_n) return hsma::set_last_error(HSMA_ERR_OOM, "request larger than a slot (max_n)");
  if (!(req->scale > 0) || !std::isfinite(req->scale)) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "scale must be > 0");
  double L[3];
  for (int k = 0; k < 3; ++k) L[k] = s->cfg.box_len[k] * req->scale;
  std::string msg;
  hsma_status st = hsma::validate_host_input(s->cfg.params, req->box_lo, L, req->n, req->xyz, req->q, msg);
  if (st != HSMA_OK) return hsma::set_last_error(st, msg);
  auto r = std::make_shared<Req>();
  r->n = req->n;
  r->xyz.assign(req->xyz, req->xyz + 3 * req->n);
  r->q.assign(req->q, req->q + req->n);
  for (int k = 0; k < 3; ++k) r->lo[k] = req->box_lo[k];
  r->scale = req->scale;
  r->pot = req->potential;
  r->force = req->force;
  r->res.status = HSMA_OK;
  r->res.slot = -1;
  r->res.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return hsma::set_last_error(HSMA_ERR_CANCELLED, "server is shutting down");
    if (s->cfg.queue_capacity > 0 && (int)s->pending.size() >= s->cfg.queue_capacity)
      return hsma::set_last_error(HSMA_ERR_BUSY, "request queue is full");
    r->id = s->next_id++;
    s->tickets[r->id] = r;
    s->pending.push_back(r);
    *ticket = r->id;
  }
  s->cv_work.notify_one();
  return HSMA_OK;
}

hsma_status hsma_server_wait(hsma_server* s, uint64_t ticket, hsma_result* out) {
  if (!s || !out) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  std::shared_ptr<Req> r;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "unknown ticket");
  r = it->second;
  ++s->waiters;
  s->cv_done.wait(lk, [&] { return r->done; });
  *out = r->res;
  s->tickets.erase(ticket);
  if (--s->waiters == 0) s->cv_idle.notify_all();
  if (out->status != HSMA_OK) hsma::set_last_error(out->status, "request failed");
  return out->status;
}

void hsma_server_shutdown(hsma_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto& r : s->pending) {
      r->res.status = HSMA_ERR_CANCELLED;
      r->res.t_done = now_s();
      r->done = true;
    }
    s->pending.clear();
    s->cv_done.notify_all();
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
}

void hsma_server_destroy(hsma_server* s) {
  if (!s) return;
  hsma_server_shutdown(s);
  {
    // threads already blocked in hsma_server_wait leave before the memory goes
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_idle.wait(lk, [&] { return s->waiters == 0; });
  }
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    sl.plan.reset();
    if (sl.d_io) (void)hipFree(sl.d_io);
    if (sl.h_io) (void)hipHostFree(sl.h_io);
    if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete s;
}

}  // extern "C"
