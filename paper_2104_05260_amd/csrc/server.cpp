// Continuous-batching request server (see include/hsma_server.h): the HIP
// backend of the scheduling core in server_core.h, plan classes, and the C
// interface.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hsma_server.h"
#include "device.h"
#include "server_core.h"

namespace {

using hsma::serve::now_s;

// A plan class: parameters and a unit box (box_len / box_len[0]); the host
// plan is built for the unit box and re-targeted per request.
struct PlanClass {
  hsma_params prm{};
  double unit[3] = {1, 1, 1};
  hsma::HostPlan host;
};

bool same_params(const hsma_params& a, const hsma_params& b) {
  return a.geometry == b.geometry && a.precision == b.precision && a.lambda == b.lambda && a.p == b.p &&
         a.K == b.K && a.F == b.F && a.Fw == b.Fw && a.surface_rule == b.surface_rule &&
         a.near_rule == b.near_rule && a.M == b.M && a.gamma_up == b.gamma_up && a.gamma_low == b.gamma_low &&
         a.nz == b.nz && a.coulomb_k == b.coulomb_k && a.tree_order == b.tree_order &&
         a.tree_theta == b.tree_theta && a.lsq_solver == b.lsq_solver;
}

// What a request carries besides the core's fields.
struct Payload {
  bool device = false;
  std::vector<double> xyz, q;        // host requests: copies of the inputs
  const double* d_xyz = nullptr;     // device requests: the caller's buffers
  const double* d_q = nullptr;
  double* pot = nullptr;             // outputs (host or device)
  double* force = nullptr;
  double* energy = nullptr;          // device requests: device energy or NULL
  hipEvent_t ready = nullptr;
  double lo[3] = {0, 0, 0};
  double scale = 1;
};

typedef hsma::serve::Request<Payload> Req;

// One device slot: a stream, one arena shared by the slot's plans (one per
// plan class it has run; only one runs at a time), device input/output
// buffers for host requests and pinned staging.
struct Slot {
  hipStream_t stream = nullptr;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  std::vector<std::unique_ptr<hsma::DevicePlan>> plans;  // by class index
  double* d_io = nullptr;  // xyz (3 cap) | q (cap) | pot (cap) | force (3 cap) | energy
  double* h_io = nullptr;  // pinned mirror, then energy and one int status
  int64_t cap = 0;
  int last_class = -1;  // class of the slot's previous request
  bool replayed = false;
  hipEvent_t done_ev = nullptr;  // recorded after each step's outputs
  bool device_error = false;     // the wait for done_ev failed (set by the slot's waiter)
};

struct GpuBackend;
typedef hsma::serve::Core<GpuBackend, Payload> CoreT;

// Completion: one thread per slot blocks on the slot's end-of-step event
// and tells the core; `launched` counts steps enqueued, `handled` those
// reported.
struct SlotWaiter {
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  uint64_t launched = 0, handled = 0;
  bool stop = false;
  void post() {
    {
      std::lock_guard<std::mutex> lk(mu);
      ++launched;
    }
    cv.notify_one();
  }
};

}  // namespace

struct hsma_server {
  hsma_server_cfg cfg{};
  int device = 0;
  int64_t bytes_per_slot = 0;
  std::vector<Slot> slots;
  std::vector<std::unique_ptr<SlotWaiter>> waiters;  // by slot, started after the core
  std::mutex class_mu;  // guards classes (submit threads add, the scheduler reads)
  std::vector<std::unique_ptr<PlanClass>> classes;
  std::unique_ptr<GpuBackend> backend;
  std::unique_ptr<CoreT> core;
  std::atomic<int64_t> graph_replays{0};  // written by the scheduler thread

  const PlanClass* cls(int i) {
    std::lock_guard<std::mutex> lk(class_mu);
    return classes[(size_t)i].get();
  }
  hsma_status find_or_create_class(const hsma_params& prm, double box_len[3], int* idx, double* scale,
                                   std::string& err);
};

namespace {

// Unit box of a box: box / box[0] (box[0] is the scale).
void unit_box(const double L[3], double u[3]) {
  for (int k = 0; k < 3; ++k) u[k] = L[k] / L[0];
}

// The slot's plan for class c, created on first use: the class's host plan,
// its constants on the device, the slot's arena carved for max_n particles
// (grown, and the other plans re-carved, when this class needs more).
hsma_status slot_plan(hsma_server* sv, Slot& s, int c, hsma::DevicePlan** out, std::string& err) {
  if ((int)s.plans.size() <= c) s.plans.resize((size_t)c + 1);
  if (!s.plans[c]) {
    std::unique_ptr<hsma::DevicePlan> p(new hsma::DevicePlan());
    p->host = sv->cls(c)->host;
    hsma_status st = p->init(err);
    if (st != HSMA_OK) return st;
    if ((st = p->init_scalable(err)) != HSMA_OK) return st;
    p->use_graph = true;
    const size_t need = p->carve(s.cap, nullptr);
    if (need > s.arena_bytes) {
      if (s.arena) (void)hipFree(s.arena);
      s.arena = nullptr;
      s.arena_bytes = 0;
      if (hipMalloc(&s.arena, need) != hipSuccess) {
        err = "slot arena allocation failed";
        return HSMA_ERR_OOM;
      }
      s.arena_bytes = need;
      for (auto& q : s.plans)
        if (q) q->attach_arena(s.arena, s.cap);
    }
    p->attach_arena(s.arena, s.cap);
    s.plans[c] = std::move(p);
  }
  *out = s.plans[c].get();
  return HSMA_OK;
}

// The slot waiter's loop: for each step enqueued on the slot, wait for its
// end-of-step event (a blocking wait, no polling), then report the slot
// done.  Exits once stopped with nothing pending.
void slot_waiter(hsma_server* sv, int si) {
  SlotWaiter& w = *sv->waiters[(size_t)si];
  Slot& s = sv->slots[(size_t)si];
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(w.mu);
      w.cv.wait(lk, [&] { return w.stop || w.launched > w.handled; });
      if (w.launched == w.handled) return;
    }
    if (hipEventSynchronize(s.done_ev) != hipSuccess) s.device_error = true;
    {
      std::lock_guard<std::mutex> lk(w.mu);
      ++w.handled;
    }
    sv->core->notify_complete(si);
  }
}

struct GpuBackend {
  hsma_server* sv;
  explicit GpuBackend(hsma_server* s) : sv(s) {}
  int slots() const { return (int)sv->slots.size(); }

  hsma_status launch(int si, Req& r, std::string& err) {
    Slot& s = sv->slots[si];
    hsma::DevicePlan* plan = nullptr;
    hsma_status st = slot_plan(sv, s, r.cls, &plan, err);
    if (st != HSMA_OK) return st;
    // the slot's plans share its arena: after another class's step this
    // plan's check schedule there is gone
    if (s.last_class != r.cls) plan->arena_reused();
    s.last_class = r.cls;
    const int64_t n = r.n, cap = s.cap;
    Payload& p = r.payload;
    double* h = s.h_io;
    const double* x = p.d_xyz;
    const double* q = p.d_q;
    double* pot = p.pot;
    double* force = p.force;
    double* d_e = s.d_io + 8 * cap;
    hipError_t e;
#define SVCHK(call, what)                                         \
  do {                                                            \
    if ((e = (call)) != hipSuccess) {                             \
      err = std::string(what) + ": " + hipGetErrorString(e);      \
      return e == hipErrorOutOfMemory ? HSMA_ERR_OOM : HSMA_ERR_DEVICE; \
    }                                                             \
  } while (0)
    if (!p.device) {
      std::memcpy(h, p.xyz.data(), sizeof(double) * 3 * n);
      std::memcpy(h + 3 * cap, p.q.data(), sizeof(double) * n);
      x = s.d_io;
      q = s.d_io + 3 * cap;
      pot = p.pot ? s.d_io + 4 * cap : nullptr;
      force = p.force ? s.d_io + 5 * cap : nullptr;
      SVCHK(hipMemcpyAsync(s.d_io, h, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s.stream), "copy in");
      SVCHK(hipMemcpyAsync(s.d_io + 3 * cap, h + 3 * cap, sizeof(double) * n, hipMemcpyHostToDevice, s.stream),
            "copy in");
    } else if (p.ready) {
      SVCHK(hipStreamWaitEvent(s.stream, p.ready, 0), "wait for the inputs' event");
    }
    if ((st = plan->set_box(p.lo, p.scale, s.stream, err)) != HSMA_OK) return st;
    const long long replays0 = plan->graph_replays;
    if ((st = plan->run(s.stream, n, x, q, d_e, pot, force, err)) != HSMA_OK) return st;
    s.replayed = plan->graph_replays != replays0;
    // energy and device status to the pinned staging; host outputs too
    SVCHK(hipMemcpyAsync(h + 8 * cap, d_e, sizeof(double), hipMemcpyDeviceToHost, s.stream), "copy out");
    SVCHK(hipMemcpyAsync(h + 8 * cap + 1, plan->d_status, sizeof(int), hipMemcpyDeviceToHost, s.stream), "copy out");
    if (!p.device) {
      if (p.pot) SVCHK(hipMemcpyAsync(h + 4 * cap, pot, sizeof(double) * n, hipMemcpyDeviceToHost, s.stream), "copy out");
      if (p.force)
        SVCHK(hipMemcpyAsync(h + 5 * cap, force, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s.stream), "copy out");
    } else if (p.energy) {
      SVCHK(hipMemcpyAsync(p.energy, d_e, sizeof(double), hipMemcpyDeviceToDevice, s.stream), "copy out");
    }
    SVCHK(hipEventRecord(s.done_ev, s.stream), "completion event");
    sv->waiters[(size_t)si]->post();
#undef SVCHK
    return HSMA_OK;
  }

  void complete(int si, Req& r) {
    Slot& s = sv->slots[si];
    const int64_t cap = s.cap;
    const double* h = s.h_io;
    Payload& p = r.payload;
    if (!p.device) {
      if (p.pot) std::memcpy(p.pot, h + 4 * cap, sizeof(double) * r.n);
      if (p.force) std::memcpy(p.force, h + 5 * cap, sizeof(double) * 3 * r.n);
    }
    int status = 0;
    std::memcpy(&status, h + 8 * cap + 1, sizeof(int));
    r.res.energy = h[8 * cap];
    r.res.status = s.device_error ? HSMA_ERR_DEVICE : (hsma_status)status;
    s.device_error = false;
    r.res.replayed = s.replayed ? 1 : 0;
    r.res.plan_class = r.cls;
    if (s.replayed) ++sv->graph_replays;
  }
};

}  // namespace

// The class of (prm, box shape); box_len returns the box the device uses,
// the class's unit box times box_len[0].  Unit boxes that agree to 1e-14
// relative are one shape (L * 1.2 / L need not round to 1.2).
hsma_status hsma_server::find_or_create_class(const hsma_params& prm, double box_len[3], int* idx,
                                              double* scale, std::string& err) {
  for (int k = 0; k < 3; ++k)
    if (!(box_len[k] > 0) || !std::isfinite(box_len[k])) {
      err = "box lengths must be finite and positive";
      return HSMA_ERR_INVALID_ARG;
    }
  double u[3];
  unit_box(box_len, u);
  *scale = box_len[0];
  auto same_shape = [&](const double* cu) {
    for (int k = 0; k < 3; ++k)
      if (!(std::fabs(cu[k] - u[k]) <= 1e-14 * cu[k])) return false;
    return true;
  };
  std::lock_guard<std::mutex> lk(class_mu);
  for (size_t i = 0; i < classes.size(); ++i) {
    const PlanClass& c = *classes[i];
    if (same_params(c.prm, prm) && same_shape(c.unit)) {
      *idx = (int)i;
      for (int k = 0; k < 3; ++k) box_len[k] = c.unit[k] * *scale;
      return HSMA_OK;
    }
  }
  if (prm.near_rule < 0 || prm.near_rule > 2 || cfg.max_n > hsma::max_particles(prm.near_rule)) {
    err = "the server's max_n is above the particles one call can take with this near rule";
    return HSMA_ERR_INVALID_ARG;
  }
  std::unique_ptr<PlanClass> c(new PlanClass());
  c->prm = prm;
  for (int k = 0; k < 3; ++k) c->unit[k] = u[k];
  const double lo0[3] = {0, 0, 0};
  const hsma_status st = hsma::build_host_plan(prm, lo0, c->unit, c->host, err);
  if (st != HSMA_OK) return st;
  for (int k = 0; k < 3; ++k) box_len[k] = c->unit[k] * *scale;
  classes.push_back(std::move(c));
  *idx = (int)classes.size() - 1;
  return HSMA_OK;
}

namespace {

// Host plans of several classes; the least-squares factorisations of those
// with lsq_solver 1 run together on the device (one grouped launch sequence):
// a first pass records each class's fitting matrix, the grouped device
// CholeskyQR2 factors them all, a second pass builds each plan with its
// pseudo-inverse.
hsma_status build_classes(const std::vector<hsma_class>& in, std::vector<std::unique_ptr<PlanClass>>& out,
                          std::string& err) {
  const size_t nc = in.size();
  std::vector<std::vector<double>> Ms(nc), Ps(nc);
  std::vector<hsma::LsqJob> jobs;
  std::vector<int> job_of(nc, -1);
  const double lo0[3] = {0, 0, 0};
  for (size_t i = 0; i < nc; ++i) {
    if (in[i].params.lsq_solver != 1) continue;
    double u[3];
    if (!(in[i].box_len[0] > 0)) {
      err = "box lengths must be finite and positive";
      return HSMA_ERR_INVALID_ARG;
    }
    unit_box(in[i].box_len, u);
    int rows = 0, cols = 0;
    const hsma::PinvFn record = [&](const std::vector<double>& M, int r, int c, std::vector<double>& P, double& cond) {
      Ms[i] = M;
      rows = r;
      cols = c;
      P.assign((size_t)r * c, 0.0);
      cond = 1.0;
      return true;
    };
    hsma::HostPlan tmp;
    const hsma_status st = hsma::build_host_plan(in[i].params, lo0, u, tmp, err, &record);
    if (st != HSMA_OK) return st;
    job_of[i] = (int)jobs.size();
    hsma::LsqJob j;
    j.rows = rows;
    j.cols = cols;
    jobs.push_back(j);
  }
  for (size_t i = 0; i < nc; ++i)
    if (job_of[i] >= 0) {
      jobs[job_of[i]].M = &Ms[i];
      jobs[job_of[i]].P = &Ps[i];
    }
  hsma_status st = hsma::device_pinv_batch(jobs, err);
  if (st != HSMA_OK) return st;
  for (size_t i = 0; i < nc; ++i) {
    std::unique_ptr<PlanClass> c(new PlanClass());
    c->prm = in[i].params;
    unit_box(in[i].box_len, c->unit);
    const int jb = job_of[i];
    const hsma::PinvFn provide = [&](const std::vector<double>& M, int r, int cc, std::vector<double>& P, double& cond) {
      if (M.size() != Ms[i].size() || (size_t)r * cc != Ps[i].size()) return false;
      P = Ps[i];
      cond = jobs[jb].cond;
      return jobs[jb].ok;
    };
    st = hsma::build_host_plan(in[i].params, lo0, c->unit, c->host, err, jb >= 0 ? &provide : nullptr);
    if (st != HSMA_OK) return st;
    out.push_back(std::move(c));
  }
  return HSMA_OK;
}

}  // namespace

extern "C" {

hsma_status hsma_server_create(const hsma_server_cfg* cfg, hsma_server** out) {
  if (!cfg || !out) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (cfg->max_n < 1 || cfg->max_slots < 1)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "max_n and max_slots must be positive");
  if (cfg->max_n > hsma::max_particles(cfg->params.near_rule))
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "max_n is above the particles one call can take");
  if (cfg->n_classes < 0 || (cfg->n_classes > 0 && !cfg->classes))
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "classes: NULL list or negative count");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return hsma::set_last_error(HSMA_ERR_NO_DEVICE, "no HIP device");
  std::unique_ptr<hsma_server> sv(new hsma_server());
  sv->cfg = *cfg;
  sv->cfg.classes = nullptr;  // not kept
  (void)hipGetDevice(&sv->device);
  std::string msg;
  // the default class and the declared ones (grouped factorisation)
  std::vector<hsma_class> decl(1);
  decl[0].params = cfg->params;
  for (int k = 0; k < 3; ++k) decl[0].box_len[k] = cfg->box_len[k];
  for (int i = 0; i < cfg->n_classes; ++i) {
    if (cfg->max_n > hsma::max_particles(cfg->classes[i].params.near_rule))
      return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "max_n is above the particles one call can take");
    decl.push_back(cfg->classes[i]);
  }
  hsma_status st;
  try {
    st = build_classes(decl, sv->classes, msg);
  } catch (const std::bad_alloc&) {
    return hsma::set_last_error(HSMA_ERR_OOM, "host allocation failed");
  }
  if (st != HSMA_OK) return hsma::set_last_error(st, msg);
  // slot size: the per-class arenas share one buffer (the largest), the
  // plan constants add up
  size_t arena = 0, consts = 0;
  for (const auto& c : sv->classes) {
    hsma::DevicePlan probe;
    probe.host = c->host;
    arena = std::max(arena, probe.carve(cfg->max_n, nullptr));
    const hsma::HostPlan& hp = c->host;
    consts += sizeof(double) * 2 * (hp.Praw.size() + hp.SQ.size() * 2 + hp.ysurf.size() * 2) +
              sizeof(hsma::Desc) * 2 * (hp.desc_particles.size() + hp.desc_check.size()) +
              sizeof(double4) * 2 * hp.check_axis.size();
  }
  const int64_t io_bytes = (int64_t)sizeof(double) * (8 * cfg->max_n + 2);
  sv->bytes_per_slot = (int64_t)arena + (int64_t)consts + io_bytes;
  size_t freeb = 0, totalb = 0;
  (void)hipMemGetInfo(&freeb, &totalb);
  const int64_t budget = cfg->hbm_budget > 0 ? cfg->hbm_budget : (int64_t)(freeb / 2);
  const int nslots = (int)std::min<int64_t>(cfg->max_slots, budget / std::max<int64_t>(1, sv->bytes_per_slot));
  if (nslots < 1) return hsma::set_last_error(HSMA_ERR_OOM, "HBM budget smaller than one slot");
  sv->slots.resize(nslots);
  for (int i = 0; i < nslots; ++i) {
    Slot& s = sv->slots[i];
    s.cap = cfg->max_n;
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done_ev, hipEventDisableTiming | hipEventBlockingSync) != hipSuccess ||
        hipMalloc((void**)&s.d_io, sizeof(double) * (8 * s.cap + 2)) != hipSuccess ||
        hipHostMalloc((void**)&s.h_io, sizeof(double) * (8 * s.cap + 2)) != hipSuccess ||
        hipMalloc(&s.arena, arena) != hipSuccess) {
      hsma_server* raw = sv.release();
      hsma_server_destroy(raw);
      return hsma::set_last_error(HSMA_ERR_OOM, "slot allocation failed");
    }
    s.arena_bytes = arena;
    // the default class's plan in every slot up front (first requests do
    // not pay for its upload)
    hsma::DevicePlan* p = nullptr;
    if ((st = slot_plan(sv.get(), s, 0, &p, msg)) != HSMA_OK) {
      hsma_server* raw = sv.release();
      hsma_server_destroy(raw);
      return hsma::set_last_error(st, msg);
    }
  }
  sv->backend.reset(new GpuBackend(sv.get()));
  // affinity over as many recent systems per slot as a slot plan keeps
  // captured steps
  sv->core.reset(new CoreT(*sv->backend, cfg->queue_capacity, hsma::DevicePlan::kGraphCache));
  for (int i = 0; i < nslots; ++i) sv->waiters.emplace_back(new SlotWaiter());
  for (int i = 0; i < nslots; ++i) sv->waiters[(size_t)i]->th = std::thread(slot_waiter, sv.get(), i);
  sv->core->start();
  *out = sv.release();
  return HSMA_OK;
}

hsma_status hsma_server_get_slots(const hsma_server* s, int* nslots, int64_t* bytes_per_slot) {
  if (!s) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL server");
  if (nslots) *nslots = (int)s->slots.size();
  if (bytes_per_slot) *bytes_per_slot = s->bytes_per_slot;
  return HSMA_OK;
}

hsma_status hsma_server_get_stats(const hsma_server* s, hsma_server_stats* out) {
  if (!s || !out || !s->core) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  hsma_server* m = const_cast<hsma_server*>(s);
  out->completed = s->core->completed();
  out->affinity_hits = s->core->affinity_hits();
  out->slots = (int)s->slots.size();
  {
    std::lock_guard<std::mutex> lk(m->class_mu);
    out->classes = (int)s->classes.size();
  }
  out->graph_replays = m->graph_replays.load();
  return HSMA_OK;
}

hsma_status hsma_server_submit(hsma_server* s, const hsma_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket || !req->xyz || !req->q) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (req->n < 1) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "n must be >= 1");
  if (req->n > s->cfg.max_n) return hsma::set_last_error(HSMA_ERR_OOM, "request larger than a slot (max_n)");
  if (req->flags & ~HSMA_REQ_DEVICE) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "unknown request flags");
  const hsma_params& prm = req->params ? *req->params : s->cfg.params;
  double L[3];
  const bool given = req->box_len[0] != 0 || req->box_len[1] != 0 || req->box_len[2] != 0;
  if (given) {
    for (int k = 0; k < 3; ++k) L[k] = req->box_len[k];
  } else {
    if (!(req->scale > 0) || !std::isfinite(req->scale))
      return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "scale must be > 0");
    for (int k = 0; k < 3; ++k) L[k] = s->cfg.box_len[k] * req->scale;
  }
  std::string msg;
  auto r = std::make_shared<Req>();
  hsma_status st;
  try {
    st = s->find_or_create_class(prm, L, &r->cls, &r->payload.scale, msg);
    if (st != HSMA_OK) return hsma::set_last_error(st, msg);
    Payload& p = r->payload;
    p.device = (req->flags & HSMA_REQ_DEVICE) != 0;
    for (int k = 0; k < 3; ++k) p.lo[k] = req->box_lo[k];
    p.pot = req->potential;
    p.force = req->force;
    if (p.device) {
      p.d_xyz = req->xyz;
      p.d_q = req->q;
      p.energy = req->energy;
      p.ready = (hipEvent_t)req->ready_event;
    } else {
      st = hsma::validate_host_input(prm, req->box_lo, L, req->n, req->xyz, req->q, msg);
      if (st != HSMA_OK) return hsma::set_last_error(st, msg);
      p.xyz.assign(req->xyz, req->xyz + 3 * req->n);
      p.q.assign(req->q, req->q + req->n);
    }
  } catch (const std::bad_alloc&) {
    return hsma::set_last_error(HSMA_ERR_OOM, "host allocation failed");
  }
  r->n = req->n;
  r->system = req->system_id;
  r->res.status = HSMA_OK;
  st = s->core->submit(r, ticket, msg);
  if (st != HSMA_OK) return hsma::set_last_error(st, msg);
  return HSMA_OK;
}

hsma_status hsma_server_wait(hsma_server* s, uint64_t ticket, hsma_result* out) {
  if (!s || !out) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  std::string msg;
  const hsma_status st = s->core->wait(ticket, out, msg);
  if (st != HSMA_OK) hsma::set_last_error(st, msg);
  return st;
}

void hsma_server_shutdown(hsma_server* s) {
  if (!s || !s->core) return;
  s->core->shutdown();
}

void hsma_server_destroy(hsma_server* s) {
  if (!s) return;
  if (s->core) {
    s->core->shutdown();   // running steps finish (their waiters report them)
    s->core->wait_idle();  // threads blocked in hsma_server_wait leave first
  }
  for (auto& w : s->waiters) {
    {
      std::lock_guard<std::mutex> lk(w->mu);
      w->stop = true;
    }
    w->cv.notify_one();
    if (w->th.joinable()) w->th.join();
  }
  s->waiters.clear();
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    std::string err;
    for (auto& p : sl.plans)
      if (p) (void)p->wait_done(err);
    sl.plans.clear();
    if (sl.arena) (void)hipFree(sl.arena);
    if (sl.d_io) (void)hipFree(sl.d_io);
    if (sl.h_io) (void)hipHostFree(sl.h_io);
    if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  s->core.reset();
  delete s;
}

}  // extern "C"
