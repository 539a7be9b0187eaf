// C interface of the HSMA library (see include/hsma.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "device.h"


namespace {
thread_local std::string g_err;

hsma_status fail(hsma_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

std::string size_message(const hsma_plan* plan) {
  const int rule = plan->dev.host.prm.near_rule;
  return "too many particles for one call (at most " + std::to_string(hsma::max_particles(rule)) +
         (rule == 0 ? ")" : rule == 1 ? " with the sphere near set)" : " with the treecode)");
}
}  // namespace

namespace hsma {
hsma_status set_last_error(hsma_status s, const std::string& msg) { return fail(s, msg); }

}  // namespace hsma

namespace {

hsma_status check_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(HSMA_ERR_NO_DEVICE, "no HIP device available");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(HSMA_ERR_NO_DEVICE, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(HSMA_ERR_NO_DEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(HSMA_ERR_NO_DEVICE, std::string("device is ") + prop.gcnArchName + ", library built for gfx950");
  return HSMA_OK;
}
}  // namespace

extern "C" {

void hsma_params_default(hsma_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->geometry = HSMA_GEOM_3D;
  p->precision = HSMA_FP32C;
  p->lambda = 1.5;
  p->p = 10;
  p->K = 2 * 11 * 11;
  p->F = 800;
  p->Fw = 0;
  p->surface_rule = 0;
  p->near_rule = 0;
  p->M = 10;
  p->gamma_up = 0.0;
  p->gamma_low = 0.0;
  p->nz = 80;
  p->coulomb_k = 1.0;
  p->tree_order = 12;
  p->tree_theta = 0.5;
}

const char* hsma_last_error(void) { return g_err.c_str(); }

hsma_status hsma_plan_create(const hsma_params* params, const double box_lo[3], const double box_len[3],
                             hsma_plan** out) {
  if (!params || !box_lo || !box_len || !out) return fail(HSMA_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (!std::isfinite(params->coulomb_k)) return fail(HSMA_ERR_INVALID_ARG, "coulomb_k must be finite");
  std::unique_ptr<hsma_plan> plan;
  try {
    plan.reset(new hsma_plan());
    std::string msg;
    hsma_status s = hsma::build_host_plan(*params, box_lo, box_len, plan->dev.host, msg);
    if (s != HSMA_OK) return fail(s, msg);
    s = check_device();
    if (s != HSMA_OK) return s;
    s = plan->dev.init(msg);
    if (s != HSMA_OK) return fail(s, msg);
  } catch (const std::bad_alloc&) {
    return fail(HSMA_ERR_OOM, "host allocation failed");
  } catch (...) {
    return fail(HSMA_ERR_DEVICE, "unexpected exception during plan creation");
  }
  *out = plan.release();
  return HSMA_OK;
}

void hsma_plan_destroy(hsma_plan* plan) {
  if (!plan) return;
  // the plan's own work only: every call records ev_done at its end, and a
  // call on another stream first waits for the previous call's ev_done, so
  // ev_done completes after all of the plan's work (other streams and other
  // plans on the device are not waited for)
  std::string err;
  (void)plan->dev.wait_done(err);
  delete plan;
}

hsma_status hsma_compute_device(hsma_plan* plan, void* stream, int64_t n, const double* d_xyz, const double* d_q,
                                double* d_energy, double* d_potential, double* d_force) {
  if (!plan || !d_xyz || !d_q) return fail(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (n < 1) return fail(HSMA_ERR_INVALID_ARG, "n must be >= 1");
  if (n > hsma::max_particles(plan->dev.host.prm.near_rule)) return fail(HSMA_ERR_INVALID_ARG, size_message(plan));
  std::string msg;
  hsma_status s;
  try {
    s = plan->dev.run((hipStream_t)stream, n, d_xyz, d_q, d_energy, d_potential, d_force, msg);
  } catch (const std::bad_alloc&) {
    return fail(HSMA_ERR_OOM, "host allocation failed");
  } catch (...) {
    return fail(HSMA_ERR_DEVICE, "unexpected exception");
  }
  if (s != HSMA_OK) return fail(s, msg);
  return HSMA_OK;
}

hsma_status hsma_compute_device_noalloc(hsma_plan* plan, void* stream, int64_t n, const double* d_xyz,
                                        const double* d_q, double* d_energy, double* d_potential, double* d_force) {
  if (!plan || !d_xyz || !d_q) return fail(HSMA_ERR_INVALID_ARG, "NULL argument");
  std::string msg;
  hsma_status s;
  try {
    s = plan->dev.run_noalloc((hipStream_t)stream, n, d_xyz, d_q, d_energy, d_potential, d_force, msg);
  } catch (...) {
    return fail(HSMA_ERR_DEVICE, "unexpected exception");
  }
  if (s != HSMA_OK) return fail(s, msg);
  return HSMA_OK;
}

hsma_status hsma_plan_device_status(hsma_plan* plan) {
  if (!plan) return fail(HSMA_ERR_INVALID_ARG, "NULL plan");
  {
    std::string err;
    if (plan->dev.wait_done(err) != HSMA_OK) return fail(HSMA_ERR_DEVICE, "waiting for the plan's last call: " + err);
  }
  int st = 0;
  if (hipMemcpy(&st, plan->dev.d_status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(HSMA_ERR_DEVICE, "status read failed");
  if (st == HSMA_ERR_NOT_NEUTRAL) return fail(HSMA_ERR_NOT_NEUTRAL, "system is not charge neutral");
  if (st == HSMA_ERR_OUT_OF_DOMAIN) return fail(HSMA_ERR_OUT_OF_DOMAIN, "a particle is outside the domain or not finite");
  return (hsma_status)st;
}

hsma_status hsma_compute(hsma_plan* plan, int64_t n, const double* xyz, const double* q, double* energy,
                         double* potential, double* force) {
  if (!plan || !xyz || !q) return fail(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (n < 1) return fail(HSMA_ERR_INVALID_ARG, "n must be >= 1");
  if (n > hsma::max_particles(plan->dev.host.prm.near_rule)) return fail(HSMA_ERR_INVALID_ARG, size_message(plan));
  const hsma::HostPlan& hp = plan->dev.host;
  {
    std::string msg;
    hsma_status vs = hsma::validate_host_input(hp.prm, hp.lo, hp.L, n, xyz, q, msg);
    if (vs != HSMA_OK) return fail(vs, msg);
  }
  hsma::DevicePlan& d = plan->dev;
  auto hipfail = [](hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? HSMA_ERR_OOM : HSMA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  if (!d.own_stream) {
    if ((e = hipStreamCreate(&d.own_stream)) != hipSuccess) return hipfail(e, "hipStreamCreate");
  }
  if (n > d.stage_cap) {
    void* ps[] = {d.d_in_xyz, d.d_in_q, d.d_out_pot, d.d_out_force, d.d_out_energy};
    for (void* p : ps)
      if (p) (void)hipFree(p);
    d.d_in_xyz = d.d_in_q = d.d_out_pot = d.d_out_force = d.d_out_energy = nullptr;
    d.stage_cap = 0;
    if ((e = hipMalloc((void**)&d.d_in_xyz, sizeof(double) * 3 * n)) != hipSuccess) return hipfail(e, "hipMalloc");
    if ((e = hipMalloc((void**)&d.d_in_q, sizeof(double) * n)) != hipSuccess) return hipfail(e, "hipMalloc");
    if ((e = hipMalloc((void**)&d.d_out_pot, sizeof(double) * n)) != hipSuccess) return hipfail(e, "hipMalloc");
    if ((e = hipMalloc((void**)&d.d_out_force, sizeof(double) * 3 * n)) != hipSuccess) return hipfail(e, "hipMalloc");
    if ((e = hipMalloc((void**)&d.d_out_energy, sizeof(double))) != hipSuccess) return hipfail(e, "hipMalloc");
    d.stage_cap = n;
  }
  hipStream_t st = d.own_stream;
  if ((e = hipMemcpyAsync(d.d_in_xyz, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, st)) != hipSuccess)
    return hipfail(e, "copy in");
  if ((e = hipMemcpyAsync(d.d_in_q, q, sizeof(double) * n, hipMemcpyHostToDevice, st)) != hipSuccess)
    return hipfail(e, "copy in");
  hsma_status s = hsma_compute_device(plan, st, n, d.d_in_xyz, d.d_in_q, d.d_out_energy,
                                      potential ? d.d_out_pot : nullptr, force ? d.d_out_force : nullptr);
  if (s != HSMA_OK) return s;
  if (energy && (e = hipMemcpyAsync(energy, d.d_out_energy, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hipfail(e, "copy out");
  if (potential &&
      (e = hipMemcpyAsync(potential, d.d_out_pot, sizeof(double) * n, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hipfail(e, "copy out");
  if (force && (e = hipMemcpyAsync(force, d.d_out_force, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hipfail(e, "copy out");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hipfail(e, "hipStreamSynchronize");
  return HSMA_OK;
}

hsma_status hsma_plan_set_timing(hsma_plan* plan, int enable) {
  if (!plan) return fail(HSMA_ERR_INVALID_ARG, "NULL plan");
  plan->dev.timing = enable != 0;
  plan->dev.timed_calls = 0;
  return HSMA_OK;
}

hsma_status hsma_plan_get_timing(hsma_plan* plan, hsma_timing* out) {
  if (!plan || !out) return fail(HSMA_ERR_INVALID_ARG, "NULL argument");
  hsma::DevicePlan& d = plan->dev;
  std::memset(out, 0, sizeof(*out));
  out->calls = d.timed_calls;
  double* acc[] = {&out->step_ms, &out->check_ms, &out->near_ms, &out->sphere_ms};
  for (int c = 0; c < d.timed_calls; ++c)
    for (int stg = 0; stg < hsma::DevicePlan::kStages; ++stg) {
      const size_t i = ((size_t)c * hsma::DevicePlan::kStages + stg) * 2;
      if (i + 1 >= d.events.size()) continue;
      if (hipEventSynchronize(d.events[i + 1]) != hipSuccess) return fail(HSMA_ERR_DEVICE, "event sync failed");
      float ms = 0;
      if (hipEventElapsedTime(&ms, d.events[i], d.events[i + 1]) != hipSuccess)
        return fail(HSMA_ERR_DEVICE, "hipEventElapsedTime failed");
      *acc[stg] += ms;
    }
  return HSMA_OK;
}

hsma_status hsma_plan_set_graph(hsma_plan* plan, int enable) {
  if (!plan) return fail(HSMA_ERR_INVALID_ARG, "NULL plan");
  plan->dev.use_graph = enable != 0;
  return HSMA_OK;
}

hsma_status hsma_plan_get_info(const hsma_plan* plan, hsma_plan_info* info) {
  if (!plan || !info) return fail(HSMA_ERR_INVALID_ARG, "NULL argument");
  const hsma::HostPlan& h = plan->dev.host;
  info->nb = h.nb;
  info->n_rows = h.nrows;
  info->n_check = (int)h.check_axis.size();
  info->n_desc = (int)h.desc_particles.size();
  info->radius = h.R;
  info->cond = h.cond;
  info->near_pairs = plan->dev.near_pairs;
  info->check_pairs = plan->dev.check_pairs;
  info->surface_pairs = plan->dev.sphere_pairs;
  if (h.prm.near_rule == 1 && plan->dev.cur_n > 0) {
    // sphere near set: the pairs actually summed, from the last step's masks
    std::string err;
    long long inside = 0;
    const hsma_status st = plan->dev.sphere_sources(inside, err);
    if (st != HSMA_OK) return fail(st, err);
    const long long n = plan->dev.cur_n;
    info->near_pairs = n * inside - n;
    info->check_pairs = (long long)h.check_axis.size() * inside;
  }
  return HSMA_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ test hooks
// Host-only views of the plan (no device needed), used by the CPU tests to
// check the host FP64 plan against the oracle.
struct hsma_host_plan {
  hsma::HostPlan h;
};

namespace hsma {
uint32_t hilbert_key_host(uint32_t x, uint32_t y, uint32_t z);
}

extern "C" {

uint32_t hsma_debug_hilbert_key(uint32_t x, uint32_t y, uint32_t z) { return hsma::hilbert_key_host(x, y, z); }

hsma_status hsma_debug_solid_harmonics(int p, const double xi[3], double* val, double* grad) {
  if (p < 1 || p > 24 || !xi || !val) return fail(HSMA_ERR_INVALID_ARG, "bad argument");
  hsma::solid_harmonics(p, xi, val, grad);
  return HSMA_OK;
}

hsma_status hsma_debug_host_plan_create(const hsma_params* params, const double box_lo[3], const double box_len[3],
                                        hsma_host_plan** out) {
  if (!params || !box_lo || !box_len || !out) return fail(HSMA_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  try {
    std::unique_ptr<hsma_host_plan> hp(new hsma_host_plan());
    std::string msg;
    hsma_status s = hsma::build_host_plan(*params, box_lo, box_len, hp->h, msg);
    if (s != HSMA_OK) return fail(s, msg);
    *out = hp.release();
  } catch (...) {
    return fail(HSMA_ERR_OOM, "host allocation failed");
  }
  return HSMA_OK;
}

void hsma_debug_host_plan_destroy(hsma_host_plan* hp) { delete hp; }

// Copies the named array (as doubles) into out[0..cap) and returns its
// length, or -1 for an unknown name.
int64_t hsma_debug_host_plan_get(const hsma_host_plan* hp, const char* name, double* out, int64_t cap) {
  if (!hp || !name) return -1;
  const hsma::HostPlan& h = hp->h;
  std::vector<double> tmp;
  const std::string n(name);
  if (n == "Praw") tmp = h.Praw;
  else if (n == "check_pos") tmp = h.check_pos;
  else if (n == "check_axis") tmp.assign(h.check_axis.begin(), h.check_axis.end());
  else if (n == "ysurf") tmp = h.ysurf;
  else if (n == "nsurf") tmp = h.nsurf;
  else if (n == "SQ") tmp = h.SQ;
  else if (n == "SD") tmp = h.SD;
  else if (n == "scalars") tmp = {h.R, (double)h.nb, (double)h.nrows, h.cond};
  else if (n == "desc_particles" || n == "desc_check") {
    const auto& v = n == "desc_particles" ? h.desc_particles : h.desc_check;
    for (const auto& d : v) {
      tmp.push_back(d.sx); tmp.push_back(d.sy); tmp.push_back(d.sz);
      tmp.push_back(d.sigma); tmp.push_back(d.scale);
    }
  } else if (n == "check_groups") {
    for (const auto& g : h.check_groups) {
      tmp.push_back(g.first); tmp.push_back(g.count); tmp.push_back(g.desc_off); tmp.push_back(g.ndesc);
    }
  } else return -1;
  if (out) std::memcpy(out, tmp.data(), sizeof(double) * (size_t)std::min<int64_t>(cap, (int64_t)tmp.size()));
  return (int64_t)tmp.size();
}

}  // extern "C"
