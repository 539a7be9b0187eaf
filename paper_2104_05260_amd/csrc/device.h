// Device-resident plan and per-step buffers of the HSMA library.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hsma_internal.h"

namespace hsma {

constexpr int kMaxTimedCalls = 4096;

// What a captured step graph depends on.
struct GraphKey {
  int64_t n = -1;
  const void *xyz = nullptr, *q = nullptr, *energy = nullptr, *pot = nullptr, *force = nullptr;
  hipStream_t stream = nullptr;
  bool operator==(const GraphKey& o) const {
    return n == o.n && xyz == o.xyz && q == o.q && energy == o.energy && pot == o.pot && force == o.force &&
           stream == o.stream;
  }
};

struct DevicePlan {
  HostPlan host;
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t side = nullptr;       // check chain of a step, forked from the call's stream
  hipStream_t side_near = nullptr;  // near pass of a step, forked from the call's stream
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join_near = nullptr;

  // tuning of the work decomposition (the no-allocation entry point runs
  // with smaller targets so that its partial sums fit the static scratch)
  int part_target = 4194304;   // waves per particle pair launch (about; at most kMaxFarChunks per group)
  int check_target = 2048;     // minimum waves per check pair launch (about)
  int check_target_max = 65536;
  int near_target = kNearWaves;  // near-pass waves per launch (about)
  int tree_target = kTreeWaves;  // treecode waves per launch (about)
  long long check_pairs_per_item = 100000;
  double close_factor = 0.1;   // close-pair radius / typical tile extent (FP32 path)

  // plan constants on the device
  Desc* d_desc_part = nullptr;
  Desc* d_desc_check = nullptr;
  double4* d_check_pos = nullptr;
  int* d_check_axis = nullptr;
  Group* d_check_groups = nullptr;
  int* d_check_tgroup = nullptr;
  double* d_Praw = nullptr;
  double* d_SQ = nullptr;
  double* d_SD = nullptr;
  double* d_ysurf = nullptr;
  double* d_nsurf = nullptr;
  double* d_v = nullptr;
  double* d_A = nullptr;
  float4* d_surf32 = nullptr;
  double4* d_surf64 = nullptr;
  double* d_qd = nullptr;
  int* d_status = nullptr;
  double* d_energy_scratch = nullptr;

  // per-size arena: one device allocation (d_arena) carved into the
  // buffers below; the no-allocation entry point carves the same layout
  // from the library's static scratch instead
  void* d_arena = nullptr;
  int64_t cap_n = 0, cur_n = -1;
  size_t part_cap = 0, cpart_cap = 0, work_cap = 0, cwork_cap = 0;
  uint32_t* d_key[2] = {nullptr, nullptr};
  int* d_val[2] = {nullptr, nullptr};
  uint32_t* d_hist = nullptr;
  double4* d_pos_w = nullptr;
  double4* d_pos64 = nullptr;
  float4* d_src32 = nullptr;
  double4* d_src64 = nullptr;
  double4* d_tile_c = nullptr;
  float4* d_tile_h = nullptr;
  int* d_perm = nullptr;
  double* d_red = nullptr;
  double* d_epart = nullptr;
  void* d_part = nullptr;
  void* d_cpart = nullptr;
  CheckSched* d_csched = nullptr;
  unsigned long long* d_cull = nullptr;  // sphere near set: ndesc x ntiles source masks
  unsigned* d_clist = nullptr;           // sphere near set: non-empty (entry, tile) pairs
  int* d_ccount = nullptr;
  // treecode (near rule 2): node centres + radii, boxes (lo, hi), moments
  double4* d_tnode = nullptr;
  double4* d_tbox = nullptr;
  double* d_tmom64 = nullptr;
  float* d_tmom32 = nullptr;
  TreeLevels tree_{};
  hipEvent_t stage_ev = nullptr;
  PartSched psched_{};
  int ntiles_ = 0, ngroups_ = 0, ncwork_ = 0, cwork_face_ = 0, nchunks_ = 0, nsphere_ = 0, sph_chunk_ = 0,
      nrsblk_ = 0;

  // host-call staging
  int64_t stage_cap = 0;
  double* d_in_xyz = nullptr;
  double* d_in_q = nullptr;
  double* d_out_pot = nullptr;
  double* d_out_force = nullptr;
  double* d_out_energy = nullptr;

  // last-step facts
  long long near_pairs = 0, check_pairs = 0, sphere_pairs = 0;

  // optional per-stage event timing (hsma_plan_set_timing)
  enum { kStStep = 0, kStCheck, kStNear, kStSphere, kStages };
  bool timing = false;
  int timed_calls = 0;
  std::vector<hipEvent_t> events;   // kStages * 2 events per timed call
  hsma_status record(hipStream_t st, int stage, int edge, std::string& err);
  void build_tree(hipStream_t st, int n);
  template <bool CHECKS>
  hsma_status launch_tree(hipStream_t st, long comp, long slot, std::string& err);
  int tree_cwaves_ = 0, tree_csplit_ = 1;  // treecode at the check targets (0: direct check sums)
  int tree_cgroup0_ = 0;                    // first check group summed by the treecode
  int tree_cbase_ = 0;                      // direct check waves before the treecode's

  void* h_stage = nullptr;       // pinned staging of the check schedule
  size_t stage_bytes = 0;
  size_t arena_bytes = 0;        // device bytes of the per-size arena

  // box re-targeting (serving: many boxes of one shape share one plan class)
  bool scalable = false;
  double unit_L[3] = {0, 0, 0}, unit_R = 0, cur_scale = 1.0;
  Desc* d_unit_desc_part = nullptr;
  Desc* d_unit_desc_check = nullptr;
  double4* d_unit_check_pos = nullptr;
  double* d_unit_Praw = nullptr;
  double* d_unit_SQ = nullptr;
  double* d_unit_SD = nullptr;
  double* d_unit_ysurf = nullptr;
  // sphere near set: number of source images inside the sphere in the last
  // step (waits for that step)
  hsma_status sphere_sources(long long& inside, std::string& err) const;
  hsma_status init_scalable(std::string& err);
  hsma_status set_box(const double lo[3], double scale, hipStream_t st, std::string& err);

  // step-parameter block and graph replay
  void* d_sp = nullptr;
  double sp_host[12] = {0};     // last values written to d_sp
  bool sp_valid = false;
  bool use_graph = false;
  // captured steps, most recently used first, and the keys of recent eager
  // calls (a key seen again is captured)
  static constexpr int kGraphCache = 8, kGraphSeen = 16;
  std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
  std::vector<GraphKey> seen_keys;
  void drop_graphs();
  long long graph_replays = 0;
  hsma_status enqueue_step(hipStream_t st, int n, const double* d_xyz, const double* d_q, double* d_energy,
                           double* d_pot, double* d_force, std::string& err);

  hsma_status init(std::string& err);
  // Allocates the per-size arena for any particle count up to nmax.
  hsma_status reserve(int64_t nmax, std::string& err);
  // Bytes of the per-size arena for particle counts up to nmax under the
  // current decomposition targets; with base != nullptr also points the
  // arena buffers into [base, base + result).
  size_t carve(int64_t nmax, char* base);
  // Uses [base, base + carve(nmax)) as the arena (owned by the caller, e.g.
  // a server slot shared by several plans that never run at once).
  void attach_arena(void* base, int64_t nmax);
  // Another plan has written the shared arena since this plan's last call:
  // the next call uploads its check schedule again (the only arena content
  // that outlives a call).
  void arena_reused() { cur_n = -1; }
  // Ordering of the plan's calls: each call waits for the previous call's
  // work (ev_done, recorded at its end on its stream) when it runs on
  // another stream, so calls on different streams never share the arena
  // at the same time, and ev_done covers all of the plan's work.
  hipEvent_t ev_done = nullptr;
  bool done_recorded = false;
  hipStream_t done_stream = nullptr;
  hsma_status order_after_previous(hipStream_t st, std::string& err);
  hsma_status mark_done(hipStream_t st, std::string& err);
  // Waits for all work enqueued by the plan.
  hsma_status wait_done(std::string& err);
  // The device's static scratch (address from hipGetSymbolAddress at
  // plan creation) and the step run on it without any allocation.
  void* scratch = nullptr;
  hsma_status run_noalloc(hipStream_t st, int64_t n, const double* d_xyz, const double* d_q, double* d_energy,
                          double* d_pot, double* d_force, std::string& err);
  void capacity_bounds(int64_t n, size_t& part_bytes, size_t& cpart_bytes, size_t& nwork, size_t& ncwork) const;
  // element size of the check-partial buffer: 8 bytes when any check sum
  // runs in FP64 (FP64 path; face rows of the sphere near set), else 4.
  // Reservation, the capacity check and the launches' slot stride all use it.
  size_t cpart_elem() const {
    return (host.prm.precision == HSMA_FP64 || host.prm.near_rule == 1) ? sizeof(double) : sizeof(float);
  }
  hsma_status prepare(int64_t n, hipStream_t st, std::string& err);
  hsma_status set_step_params(hipStream_t st, std::string& err);
  hsma_status run(hipStream_t st, int64_t n, const double* d_xyz, const double* d_q, double* d_energy,
                  double* d_pot, double* d_force, std::string& err);
  void free_arena();
  ~DevicePlan();
};

}  // namespace hsma

// The C interface's plan handle (include/hsma.h).
struct hsma_plan {
  hsma::DevicePlan dev;
};
