// Internal declarations shared by the plan builder, the device runtime and
// the C interface of the HSMA library.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/hsma.h"

namespace hsma {

// Work decomposition of the pair kernels.
constexpr int kWave = 64;               // wavefront width on CDNA
#ifndef HSMA_TPL
#define HSMA_TPL 1
#endif
constexpr int kTPL = HSMA_TPL;          // targets per lane
constexpr int kGroup = kWave * kTPL;    // targets per wave (one "target group")
constexpr int kTile = 64;               // sources per tile
// Waves per block of the far particle sums: consecutive target groups on
// the same chunk of sources, kept in step by a barrier per source tile so
// that the tile's scalar loads are served once from the CU's scalar cache.
#ifndef HSMA_FAR_WAVES
#define HSMA_FAR_WAVES 4
#endif
constexpr int kFarWaves = HSMA_FAR_WAVES;

// Particles per call: 32-bit particle indices with headroom; the sphere
// near set and the treecode pack a tile index into 20 bits (2^20 tiles).
constexpr int64_t kMaxParticles = ((int64_t)1 << 30) - 1;
constexpr int64_t kMaxParticlesTiled = (int64_t)kTile << 20;
inline int64_t max_particles(int near_rule) {
  return near_rule == 0 ? kMaxParticles : kMaxParticlesTiled;
}

// One entry of an image table: the source set is every particle mapped by
//   (x, y, z) -> (x + sx, y + sy, sigma * z + sz)  with charge scaled by `scale`
// (sigma = +-1).  40 bytes, read by scalar loads on the device.
struct Desc {
  double sx, sy, sz, sigma, scale;
};
static_assert(sizeof(Desc) == 40, "Desc layout");

// A target group: `count` targets starting at `first`, summed over the image
// table entries [desc_off, desc_off + ndesc).
struct Group {
  int first, count, desc_off, ndesc;
};

// One wave's work: group `group`, flattened (image, tile) range [f0, f1),
// partial results written to slot `slot`.
struct Work {
  int group, f0, f1, slot;
};

// Particle work schedule (computed from the wave index, not stored): group
// g = 0..ngroups-1 of kGroup sorted particles; its range [0, F) of (image,
// tile) pairs cut into nch chunks of `chunk`; far wave b takes chunk
// b / ngroups of group b % ngroups and writes slot = chunk index.  The
// near pass deals the group's near (image entry, tile) pairs, in scan
// order, round-robin to nnear waves per group, which write slots
// nch .. nch + nnear - 1.
constexpr int kMaxNearSplit = 64;
constexpr int kMaxFarChunks = 256;  // far chunks per group at most (partial slots per target)
constexpr int kNearWaves = 8192;  // near-pass waves per launch (about, when there are enough candidates)
struct PartSched {
  int n, ngroups, ndesc, F, nch, chunk, nnear;
  int split;  // treecode: waves per (image entry, group)
};
constexpr int kTreeWaves = 65536;  // treecode waves per launch (about, at least one per (image entry, group))
constexpr int kTreeMaxSplit = 8;

// No-allocation entry point: a static device array of kScratchBytes per
// GPU holds the per-size arena of one call of at most kNoAllocMaxN
// particles, with these decomposition targets (fewer, longer waves and
// fewer partial slots than the allocating path).
constexpr size_t kScratchBytes = (size_t)48 << 20;
constexpr int64_t kNoAllocMaxN = 16384;
constexpr int kNoAllocPartTarget = 2048;
constexpr int kNoAllocCheckTarget = 1024;
constexpr int kNoAllocCheckTargetMax = 2048;
constexpr int kNoAllocNearTarget = 1024;
constexpr int kNoAllocTreeTarget = 4096;

// Treecode over the tiles (near rule 2): level 0 holds the tiles in sorted
// (Hilbert) order; node i of level l >= 1 groups nodes 8i .. 8i + 7 of
// level l - 1, so it covers tiles [8^l i, 8^l (i + 1)).  Nodes of levels
// >= 1 are stored level after level from index off[l].
constexpr int kTreeMaxLev = 12;
constexpr int kTreeMaxOrder = 12;
constexpr int kTreeMom = (kTreeMaxOrder + 1) * (kTreeMaxOrder + 2) / 2;  // complex moments, m <= n <= order
constexpr int kTreeMomStride = 192;  // reals per node (re, im of each moment), >= 2 kTreeMom
struct TreeLevels {
  int nlev;                // levels, 1 (tiles only) .. kTreeMaxLev
  int cnt[kTreeMaxLev];    // nodes per level; cnt[0] = tiles
  int off[kTreeMaxLev];    // first index of level l >= 1 in the node arrays
  int nodes;               // nodes of levels >= 1
};
inline TreeLevels tree_levels(int ntiles) {
  TreeLevels t{};
  t.cnt[0] = ntiles;
  t.nlev = 1;
  while (t.cnt[t.nlev - 1] > 1 && t.nlev < kTreeMaxLev) {
    t.off[t.nlev] = t.nodes;
    t.cnt[t.nlev] = (t.cnt[t.nlev - 1] + 7) / 8;
    t.nodes += t.cnt[t.nlev];
    ++t.nlev;
  }
  return t;
}

// Check-target schedule of one check group: far waves first_work ..
// first_work + nch - 1 take chunks of `chunk` and write slots slot0 + c;
// the group's near wave writes slot0 + nch.
struct CheckSched {
  int first_work, nch, chunk, slot0;
};

// Host-side FP64 plan: everything that depends on the box and the method
// parameters but not on the particles.
struct HostPlan {
  hsma_params prm{};
  double lo[3]{}, L[3]{};
  double R = 0;
  int nb = 0;                       // unknowns (p+1)^2 - 1
  int nrows = 0;                    // least-squares rows
  double cond = 0;

  std::vector<Desc> desc_particles; // near set for particle targets
  std::vector<Desc> desc_check;     // concatenated tables of the check groups

  // Check targets (box-centred FP64), grouped; each group uses its own
  // image table.  Outputs per target: value and one field component.
  std::vector<double> check_pos;    // ncheck * 3
  std::vector<int> check_axis;      // field component reported per target
  std::vector<Group> check_groups;
  int face_groups = 0;              // check groups [0, face_groups) hold face-pair targets

  // A = Praw * v,  v[2t] = value at check target t, v[2t+1] = field
  // component check_axis[t] at t.  Row-major nb x (2*ncheck).
  std::vector<double> Praw;

  // Sphere: points, normals, and the maps A -> Q (charges), A -> D
  // (double-layer strengths), row-major F x nb.
  std::vector<double> ysurf, nsurf;
  std::vector<double> SQ, SD;
};

// Pseudo-inverse of the fitting matrix M (rows x cols, row-major): P = R^-1
// Q^T (cols x rows) and a condition estimate (max / min |R_ii|); false when
// M is rank deficient.
typedef std::function<bool(const std::vector<double>& M, int rows, int cols, std::vector<double>& P, double& cond)>
    PinvFn;

// One matrix of a grouped device factorisation (device_pinv_batch).
struct LsqJob {
  const std::vector<double>* M = nullptr;  // rows x cols, row-major
  int rows = 0, cols = 0;
  std::vector<double>* P = nullptr;        // out: cols x rows
  std::vector<double> Rdiag;                // out: diagonal of R
  double cond = 0;                          // out
  bool ok = false;                          // out: full column rank
};

// CholeskyQR2 of every job's M on the current device (FP64; Gram matrices
// on the matrix cores, all jobs in the same launches); synchronous.
hsma_status device_pinv_batch(std::vector<LsqJob>& jobs, std::string& err);

// Builds the plan; returns HSMA_OK or an error with *msg set.  pinv: the
// pseudo-inverse to use (nullptr: by prm.lsq_solver, host Householder QR or
// device CholeskyQR2).
hsma_status build_host_plan(const hsma_params& prm, const double lo[3], const double L[3],
                            HostPlan& out, std::string& msg, const PinvFn* pinv = nullptr);

// Real solid harmonics (scaled coordinates xi = r / R): values (nb) and,
// if grad != nullptr, gradients w.r.t. xi (nb x 3).  Ordering: degree
// n = 1..p, within a degree m = 0, then (cos, sin) parts for m = 1..n.
void solid_harmonics(int p, const double xi[3], double* val, double* grad);

// Lattice generator of the surface rule (Fibonacci or best Zaremba index).
int lattice_generator(int F, int Fw);

// Records msg as the calling thread's hsma_last_error() and returns s.
hsma_status set_last_error(hsma_status s, const std::string& msg);

// Host-side input validation of hsma_compute (finite values, neutrality,
// slab domain) for a box with lower corner lo and lengths L.
hsma_status validate_host_input(const hsma_params& prm, const double lo[3], const double L[3], int64_t n,
                                const double* xyz, const double* q, std::string& msg);

}  // namespace hsma
