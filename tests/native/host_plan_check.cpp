// Host-only driver for the sanitizer test: builds host plans for a spread of
// parameter sets (both geometries, both near sets, both surface rules,
// invalid inputs), checks the plans' structural invariants, runs the host
// input validation, and exits non-zero on any mismatch.  Built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_2104_05260_amd/csrc/hsma_internal.h"

// The device least-squares solver lives in the HIP library; this host-only
// build has no device, as hsma_plan_create would report without one.
namespace hsma {
hsma_status device_pinv_batch(std::vector<LsqJob>&, std::string& err) {
  err = "no device in the host-only build";
  return HSMA_ERR_NO_DEVICE;
}
}  // namespace hsma

namespace {

int failures = 0;

void expect(bool ok, const char* what, int cs) {
  if (!ok) {
    std::fprintf(stderr, "case %d: %s\n", cs, what);
    ++failures;
  }
}

hsma_params base_params() {
  hsma_params p{};
  p.geometry = HSMA_GEOM_3D;
  p.precision = HSMA_FP32C;
  p.lambda = 1.5;
  p.p = 6;
  p.K = 100;
  p.F = 200;
  p.Fw = 0;
  p.surface_rule = 0;
  p.near_rule = 0;
  p.M = 4;
  p.gamma_up = 0.0;
  p.gamma_low = 0.0;
  p.nz = 16;
  p.coulomb_k = 1.0;
  return p;
}

// invariants of a successfully built plan
void check_plan(const hsma::HostPlan& P, int cs) {
  const size_t nt = P.check_axis.size();
  expect(P.check_pos.size() == 3 * nt, "check_pos size", cs);
  expect(P.Praw.size() == (size_t)P.nb * 2 * nt, "Praw size", cs);
  expect(P.SQ.size() == (size_t)P.prm.F * P.nb && P.SD.size() == P.SQ.size(), "SQ/SD size", cs);
  expect(P.ysurf.size() == 3 * (size_t)P.prm.F && P.nsurf.size() == P.ysurf.size(), "sphere points", cs);
  expect(P.face_groups >= 0 && P.face_groups <= (int)P.check_groups.size(), "face_groups", cs);
  size_t covered = 0;
  for (const hsma::Group& g : P.check_groups) {
    expect(g.count >= 1 && g.count <= hsma::kGroup, "group count", cs);
    expect(g.first == (int)covered, "groups tile the targets in order", cs);
    expect(g.desc_off >= 0 && (size_t)(g.desc_off + g.ndesc) <= P.desc_check.size(), "desc range", cs);
    for (int t = g.first; t < g.first + g.count; ++t)
      expect(P.check_axis[t] == P.check_axis[g.first] || P.check_axis[g.first] == 2, "one axis per face group", cs);
    covered += g.count;
  }
  expect(covered == nt, "groups cover every target", cs);
  for (double v : P.Praw) expect(std::isfinite(v), "Praw finite", cs);
  for (double v : P.SQ) expect(std::isfinite(v), "SQ finite", cs);
  expect(!P.desc_particles.empty(), "image table", cs);
}

}  // namespace

int main() {
  const double lo[3] = {0.0, 0.0, 0.0};
  struct Case {
    hsma_params p;
    double L[3];
    hsma_status want;
  };
  std::vector<Case> cases;
  hsma_params p = base_params();
  cases.push_back({p, {10, 10, 10}, HSMA_OK});
  p.near_rule = 1;
  cases.push_back({p, {10, 11, 9}, HSMA_OK});
  p = base_params();
  p.surface_rule = 1;
  p.F = 200;  // 2 x 10^2
  cases.push_back({p, {8, 8, 8}, HSMA_OK});
  p = base_params();
  p.geometry = HSMA_GEOM_2D;
  p.lambda = 1.6;
  p.gamma_up = -0.6;
  p.gamma_low = 0.3;
  cases.push_back({p, {20, 20, 10}, HSMA_OK});
  p.near_rule = 1;
  cases.push_back({p, {20, 20, 10}, HSMA_OK});
  p = base_params();
  p.lambda = 2.0;  // sphere beyond the 27 cells
  cases.push_back({p, {10, 10, 10}, HSMA_ERR_GEOMETRY});
  p = base_params();
  p.K = 10;  // 20 rows < 48 unknowns
  cases.push_back({p, {10, 10, 10}, HSMA_ERR_RANK});
  p = base_params();
  p.near_rule = 3;
  cases.push_back({p, {10, 10, 10}, HSMA_ERR_INVALID_ARG});
  p = base_params();
  p.p = 0;
  cases.push_back({p, {10, 10, 10}, HSMA_ERR_INVALID_ARG});
  for (size_t i = 0; i < cases.size(); ++i) {
    hsma::HostPlan P;
    std::string msg;
    const hsma_status s = hsma::build_host_plan(cases[i].p, lo, cases[i].L, P, msg);
    expect(s == cases[i].want, "status", (int)i);
    if (s == HSMA_OK) check_plan(P, (int)i);
  }
  // host input validation
  hsma_params v = base_params();
  const double L[3] = {10, 10, 10};
  std::vector<double> xyz = {1, 1, 1, 2, 2, 2, 3, 3, 3, 4, 4, 4};
  std::vector<double> q = {1, -1, 2, -2};
  std::string msg;
  expect(hsma::validate_host_input(v, lo, L, 4, xyz.data(), q.data(), msg) == HSMA_OK, "valid input", 100);
  q[0] = 1.5;
  expect(hsma::validate_host_input(v, lo, L, 4, xyz.data(), q.data(), msg) == HSMA_ERR_NOT_NEUTRAL, "non-neutral",
         101);
  q[0] = 1;
  xyz[4] = std::nan("");
  expect(hsma::validate_host_input(v, lo, L, 4, xyz.data(), q.data(), msg) == HSMA_ERR_OUT_OF_DOMAIN, "NaN", 102);
  xyz[4] = 2;
  v.geometry = HSMA_GEOM_2D;
  xyz[11] = 10.0;  // on the upper interface
  expect(hsma::validate_host_input(v, lo, L, 4, xyz.data(), q.data(), msg) == HSMA_ERR_OUT_OF_DOMAIN, "slab", 103);
  // basis at many degrees and points: finite values and gradients
  for (int deg = 1; deg <= 24; ++deg) {
    const int nb = (deg + 1) * (deg + 1) - 1;
    std::vector<double> val(nb), grad(3 * (size_t)nb);
    const double x[3] = {0.3, -0.7, 0.55};
    hsma::solid_harmonics(deg, x, val.data(), grad.data());
    for (double w : val) expect(std::isfinite(w), "basis finite", 200 + deg);
    for (double w : grad) expect(std::isfinite(w), "gradient finite", 200 + deg);
  }
  if (failures) std::fprintf(stderr, "%d failures\n", failures);
  else std::printf("host plan checks passed\n");
  return failures ? 1 : 0;
}
