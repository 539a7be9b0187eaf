// gfx950 kernels of the HSMA hot path and the per-step launch sequence.
//
// Per step (Sec. 2.2 of the paper, in this order):
//   ingest   wrap into the centred box, validate, Hilbert-curve keys
//   sort     stable LSD radix sort of the keys (spatially compact tiles)
//   tiles    64-particle source tiles: centre, half extent, offsets
//   check    near sums at the check targets (telescoped face-pair sets,
//            full near set on the slab interfaces)            -> v
//   lsq      A = Praw v  (FP64)
//   surface  Q_k, D_k of the sphere sources from A            (FP64)
//   near     near-set sums at the particles (dominant kernel)
//   sphere   sphere charge + dipole sums at the particles
//   final    sum partials, F = q E, energy partials; scatter to input order
//   energy   FP64 reduction in fixed order
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "device.h"

namespace hsma {

// ----------------------------------------------------------------- helpers
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64 1/sqrt: the hardware estimate (measured relative error below
// 2^-24 on gfx950) refined by one third-order step of the expansion
// (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - x y^2: the relative
// error goes from d to about (5/2) d^3, so the result is within a few units
// of rounding (measured max 1.4e-16 relative, as with two Newton steps), in
// five FP64 operations instead of eight.
__device__ __forceinline__ double rsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __fma_rn(-(x * y), y, 1.0);
  const double p = __fma_rn(0.375, e, 0.5);
  return __fma_rn(y * e, p, y);
}

// Waves per block of the partial-sum reductions (at most, for finalize;
// always, for the check rows): wave w of P sums every P-th slot from slot
// w, and the waves' sums are combined in wave order.
constexpr int kFinParts = 16;
// Waves per block of the check-row reduction: it runs on the side stream
// beside the particle sums, and a 16-wave block waited for a CU to drain
// (the treecode step on 50,000 ions: 2.4 ms for 0.55 ms of check sums).
constexpr int kCheckParts = 4;
constexpr int kFinBatch = 4;  // slots whose loads a wave issues together

// Knuth's error-free sum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

template <typename Real> struct SrcT;
template <> struct SrcT<float> { typedef float4 T; };
template <> struct SrcT<double> { typedef double4 T; };

// Lane l's value of v (l wave-uniform), as a VALU read, no memory access.
__device__ __forceinline__ double readlane_d(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Position of cell (x, y, z) (10 bits each) along a 3D Hilbert curve,
// following Skilling's transpose formulation (AIP Conf. Proc. 707, 2004):
// undo the excess rotations and reflections level by level, Gray-encode,
// then interleave the three transposed words.  Consecutive keys are
// face-adjacent cells, so runs of sorted particles stay spatially compact.
__host__ __device__ inline uint32_t hilbert_key3(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t X[3] = {x & 1023u, y & 1023u, z & 1023u};
  const uint32_t M = 1u << 9;
  for (uint32_t Q = M; Q > 1; Q >>= 1) {
    const uint32_t P = Q - 1;
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0;
  for (uint32_t Q = M; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  X[0] ^= t;
  X[1] ^= t;
  X[2] ^= t;
  uint32_t key = 0;
  for (int b = 9; b >= 0; --b)
    key = (key << 3) | (((X[0] >> b) & 1u) << 2) | (((X[1] >> b) & 1u) << 1) | ((X[2] >> b) & 1u);
  return key;
}

uint32_t hilbert_key_host(uint32_t x, uint32_t y, uint32_t z) { return hilbert_key3(x, y, z); }

// Box-dependent scalars of one step, read from device memory by the
// kernels so that a captured step graph does not depend on the box.
struct StepParams {
  double3 lo, L, hbox;
  double rc2;   // close-pair radius^2 of the particle sums
  double rc2c;  // the same for the FP32 check sums
  double R2;    // squared sphere radius (sphere near set)
};

__global__ void k_set_params(StepParams* sp, double3 lo, double3 L, double3 hbox, double rc2, double rc2c,
                             double R2) {
  sp->lo = lo;
  sp->L = L;
  sp->hbox = hbox;
  sp->rc2 = rc2;
  sp->rc2c = rc2c;
  sp->R2 = R2;
}

// ----------------------------------------------------------------- ingest
// Centred, wrapped FP64 positions + charge; 30-bit Hilbert key of a 1024^3
// cell grid; per-block partial sums (sum q, sum |q|, invalid count).
__global__ __launch_bounds__(256) void k_ingest(int n, const double* __restrict__ xyz, const double* __restrict__ q,
                                                const StepParams* __restrict__ sp, int slab, double4* __restrict__ pos,
                                                uint32_t* __restrict__ key, int* __restrict__ val,
                                                double* __restrict__ red) {
  __shared__ double s0[256], s1[256], s2[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const double3 lo = sp->lo, L = sp->L;
  double sq = 0, sa = 0, bad = 0;
  if (i < n) {
    double x = xyz[3 * (size_t)i] - (lo.x + 0.5 * L.x);
    double y = xyz[3 * (size_t)i + 1] - (lo.y + 0.5 * L.y);
    double z = xyz[3 * (size_t)i + 2] - (lo.z + 0.5 * L.z);
    const double qi = q[i];
    x -= L.x * floor(x / L.x + 0.5);
    y -= L.y * floor(y / L.y + 0.5);
    if (!slab) z -= L.z * floor(z / L.z + 0.5);
    const bool fin = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(qi);
    const bool out = slab && !(fabs(z) < 0.5 * L.z);
    bad = (!fin || out) ? 1.0 : 0.0;
    sq = qi;
    sa = fabs(qi);
    // NaN-safe clamped cell indices
    const double fx = fmin(fmax((x / L.x + 0.5) * 1024.0, 0.0), 1023.0);
    const double fy = fmin(fmax((y / L.y + 0.5) * 1024.0, 0.0), 1023.0);
    const double fz = fmin(fmax((z / L.z + 0.5) * 1024.0, 0.0), 1023.0);
    const uint32_t cx = (uint32_t)fx, cy = (uint32_t)fy, cz = (uint32_t)fz;
    key[i] = hilbert_key3(cx, cy, cz);
    val[i] = i;
    pos[i] = make_double4(fin ? x : 0.0, fin ? y : 0.0, fin ? z : 0.0, fin ? qi : 0.0);
  }
  s0[threadIdx.x] = sq;
  s1[threadIdx.x] = sa;
  s2[threadIdx.x] = bad;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s0[threadIdx.x] += s0[threadIdx.x + o];
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red[3 * blockIdx.x] = s0[0];
    red[3 * blockIdx.x + 1] = s1[0];
    red[3 * blockIdx.x + 2] = s2[0];
  }
}

// Fixed-order reduction of the ingest partials into the device status word.
// Called by every thread of a block of at least 256 threads; threads from
// 256 on only take part in the barriers.
__device__ void validate_block(int nblk, const double* __restrict__ red, int* __restrict__ status, double* s0,
                               double* s1, double* s2) {
  const int t = threadIdx.x;
  if (t < 256) {
    double a = 0, b = 0, c = 0;
    for (int i = t; i < nblk; i += 256) {
      a += red[3 * i];
      b += red[3 * i + 1];
      c += red[3 * i + 2];
    }
    s0[t] = a;
    s1[t] = b;
    s2[t] = c;
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      s0[t] += s0[t + o];
      s1[t] += s1[t + o];
      s2[t] += s2[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    int st = HSMA_OK;
    if (s2[0] > 0) st = HSMA_ERR_OUT_OF_DOMAIN;
    else if (!(fabs(s0[0]) <= 1e-12 * s1[0])) st = HSMA_ERR_NOT_NEUTRAL;
    status[0] = st;
  }
}

__global__ __launch_bounds__(256) void k_validate(int nblk, const double* __restrict__ red, int* __restrict__ status) {
  __shared__ double s0[256], s1[256], s2[256];
  validate_block(nblk, red, status, s0, s1, s2);
}

// ----------------------------------------------------------------- radix sort
// Stable LSD radix sort, 8-bit digits, 1024 keys per block.
constexpr int kRsBlock = 1024;

__global__ __launch_bounds__(256) void k_rs_hist(const uint32_t* __restrict__ keys, int n, int shift,
                                                 uint32_t* __restrict__ hist, int nblk) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  for (int k = 0; k < 4; ++k) {
    const int i = blockIdx.x * kRsBlock + k * 256 + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// In-place exclusive scan of len entries with one 1024-thread block.
__global__ __launch_bounds__(1024) void k_rs_scan(uint32_t* __restrict__ a, int len) {
  // exclusive prefix sum in place, one block walking the array in
  // coalesced tiles of 4096 counters (4 per thread) with a running carry
  __shared__ uint32_t ws[16];
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  uint32_t carry = 0;
  for (int base = 0; base < len; base += 4096) {
    const int i0 = base + 4 * tid;
    const uint32_t v0 = i0 < len ? a[i0] : 0u, v1 = i0 + 1 < len ? a[i0 + 1] : 0u;
    const uint32_t v2 = i0 + 2 < len ? a[i0 + 2] : 0u, v3 = i0 + 3 < len ? a[i0 + 3] : 0u;
    const uint32_t t1 = v0 + v1, t2 = t1 + v2, t3 = t2 + v3;
    uint32_t x = t3;  // inclusive scan of the thread totals across the wave
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) ws[wv] = x;
    __syncthreads();
    uint32_t wpre = 0, total = 0;
    for (int k = 0; k < 16; ++k) {
      const uint32_t w = ws[k];
      wpre += k < wv ? w : 0u;
      total += w;
    }
    const uint32_t ex = carry + wpre + (x - t3);
    if (i0 < len) a[i0] = ex;
    if (i0 + 1 < len) a[i0 + 1] = ex + v0;
    if (i0 + 2 < len) a[i0 + 2] = ex + t1;
    if (i0 + 3 < len) a[i0 + 3] = ex + t2;
    carry += total;
    __syncthreads();  // ws is rewritten by the next tile
  }
}

__global__ __launch_bounds__(256) void k_rs_scatter(const uint32_t* __restrict__ kin, const int* __restrict__ vin,
                                                    uint32_t* __restrict__ kout, int* __restrict__ vout, int n,
                                                    int shift, const uint32_t* __restrict__ off, int nblk) {
  __shared__ uint32_t cnt[16][256];
  __shared__ uint32_t base[256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = tid; i < 16 * 256; i += 256) cnt[i >> 8][i & 255] = 0;
  base[tid] = off[(size_t)tid * nblk + blockIdx.x];
  __syncthreads();
  uint32_t keyv[4], dig[4];
  int valv[4], rank[4];
  bool ok[4];
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int k = 0; k < 4; ++k) {
    const int i = blockIdx.x * kRsBlock + k * 256 + tid;
    ok[k] = i < n;
    keyv[k] = ok[k] ? kin[i] : 0u;
    valv[k] = ok[k] ? vin[i] : 0;
    dig[k] = (keyv[k] >> shift) & 255u;
    unsigned long long m = __ballot(ok[k]);
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (dig[k] >> bit) & 1u;
      const unsigned long long bb = __ballot(on);
      m &= on ? bb : ~bb;
    }
    rank[k] = __popcll(m & below);
    if (ok[k] && rank[k] == 0) cnt[k * 4 + wave][dig[k]] = __popcll(m);
  }
  __syncthreads();
  uint32_t run = 0;
  for (int s = 0; s < 16; ++s) {
    const uint32_t c = cnt[s][tid];
    cnt[s][tid] = run;
    run += c;
  }
  __syncthreads();
  for (int k = 0; k < 4; ++k) {
    if (!ok[k]) continue;
    const uint32_t d = dig[k];
    const uint32_t pos = base[d] + cnt[k * 4 + wave][d] + (uint32_t)rank[k];
    kout[pos] = keyv[k];
    vout[pos] = valv[k];
  }
}

// ----------------------------------------------------------------- tiles
// One wave per tile of 64 sorted particles: FP64 sorted copy, centre and
// half extent of the bounding box, offsets from the centre.  Padding slots
// carry zero charge and a far-away offset so they contribute exactly 0.
constexpr float kFar = 1.0e15f;

// Tile t built by one wave; o is the input index of sorted slot t*64+lane
// (ignored past n).
__device__ __forceinline__ void build_tile(int t, int n, int o, const double4* __restrict__ pos,
                                           double4* __restrict__ pos64, float4* __restrict__ src32,
                                           double4* __restrict__ src64, double4* __restrict__ tile_c,
                                           float4* __restrict__ tile_h, int* __restrict__ perm) {
  const int lane = threadIdx.x & (kWave - 1);
  const int s = t * kTile + lane;
  const bool ok = s < n;
  const double4 p = ok ? pos[o] : make_double4(0, 0, 0, 0);
  const double mnx = wave_min(ok ? p.x : INFINITY), mxx = wave_max(ok ? p.x : -INFINITY);
  const double mny = wave_min(ok ? p.y : INFINITY), mxy = wave_max(ok ? p.y : -INFINITY);
  const double mnz = wave_min(ok ? p.z : INFINITY), mxz = wave_max(ok ? p.z : -INFINITY);
  const double cx = 0.5 * (mnx + mxx), cy = 0.5 * (mny + mxy), cz = 0.5 * (mnz + mxz);
  if (lane == 0) {
    tile_c[t] = make_double4(cx, cy, cz, 0.0);
    // half extents rounded up so that the bound stays conservative
    tile_h[t] = make_float4((float)(0.5 * (mxx - mnx)) * 1.0001f + 1e-30f, (float)(0.5 * (mxy - mny)) * 1.0001f + 1e-30f,
                            (float)(0.5 * (mxz - mnz)) * 1.0001f + 1e-30f, 0.f);
  }
  pos64[s] = p;
  if (ok) {
    src32[s] = make_float4((float)(p.x - cx), (float)(p.y - cy), (float)(p.z - cz), (float)p.w);
    src64[s] = make_double4(p.x - cx, p.y - cy, p.z - cz, p.w);
    perm[s] = o;
  } else {
    src32[s] = make_float4(kFar, kFar, kFar, 0.f);
    src64[s] = make_double4(kFar, kFar, kFar, 0.0);
    perm[s] = -1;
  }
}

__global__ __launch_bounds__(64) void k_tiles(int n, const int* __restrict__ order, const double4* __restrict__ pos,
                                              double4* __restrict__ pos64, float4* __restrict__ src32,
                                              double4* __restrict__ src64, double4* __restrict__ tile_c,
                                              float4* __restrict__ tile_h, int* __restrict__ perm) {
  const int s = blockIdx.x * kTile + threadIdx.x;
  build_tile(blockIdx.x, n, s < n ? order[s] : 0, pos, pos64, src32, src64, tile_c, tile_h, perm);
}

// Small systems (n <= kSmallSort): validation and the key sort in one
// launch of ceil(n / kWave) blocks.  Word i = (key_i, i) is unique, and its
// rank (the number of smaller words) is its place in the sorted order, which
// is therefore the stable radix sort's.  Every block stages the n keys in
// LDS; its kRankWaves waves count the smaller words of its kWave targets
// over contiguous shares of the key range, and the counts are added.  The
// tiles are then built from the order by k_tiles.
constexpr int kSmallSort = 4096;
constexpr int kRankWaves = 16;

__global__ __launch_bounds__(kWave * kRankWaves) void k_rank(int n, int nblk, const double* __restrict__ red,
                                                            int* __restrict__ status,
                                                            const uint32_t* __restrict__ key,
                                                            int* __restrict__ order) {
  __shared__ uint32_t sk[kSmallSort];
  __shared__ int cnt[kRankWaves][kWave];
  __shared__ double s0[256], s1[256], s2[256];
  if (blockIdx.x == 0) validate_block(nblk, red, status, s0, s1, s2);  // block-uniform branch
  for (int t = threadIdx.x; t < n; t += blockDim.x) sk[t] = key[t];
  __syncthreads();
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = blockIdx.x * kWave + lane;
  const uint32_t ki = i < n ? sk[i] : 0u;
  // word j < word i  <=>  k_j < k_i, or k_j == k_i and j < i
  const int per = (n + kRankWaves - 1) / kRankWaves;
  const int j0 = min(n, w * per), j1 = min(n, j0 + per);
  int c = 0;
#pragma unroll 8
  for (int j = j0; j < j1; ++j) {
    const uint32_t kj = sk[j];  // the same address in every lane: one broadcast read
    c += (kj < ki) | ((kj == ki) & (j < i));
  }
  cnt[w][lane] = c;
  __syncthreads();
  if (w == 0 && i < n) {
    int r = 0;
    for (int q = 0; q < kRankWaves; ++q) r += cnt[q][lane];
    order[r] = i;
  }
}

// Sphere near set: bit l of cull[d * ntiles + t] says whether the image of
// sorted source t*64+l under image entry d lies strictly inside the sphere,
// |y|^2 = (y_x^2 + y_y^2) + y_z^2 < R^2 in FP64 with explicitly rounded
// operations (image position: x + s_x, y + s_y, sigma z + s_z).  Padding
// slots read as inside (they carry no charge).  One wave per (tile, entry).
__global__ __launch_bounds__(64) void k_cull(int n, int ntiles, const double4* __restrict__ pos64,
                                             const Desc* __restrict__ desc, const StepParams* __restrict__ sp,
                                             unsigned long long* __restrict__ cull) {
  const int t = blockIdx.x, d = blockIdx.y;
  const int s = t * kTile + threadIdx.x;
  bool in = true;
  if (s < n) {
    const double4 p = pos64[s];
    const Desc ds = desc[d];
    const double yx = __dadd_rn(p.x, ds.sx), yy = __dadd_rn(p.y, ds.sy);
    const double yz = __dadd_rn(__dmul_rn(ds.sigma, p.z), ds.sz);
    const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(yx, yx), __dmul_rn(yy, yy)), __dmul_rn(yz, yz));
    in = r2 < sp->R2;
  }
  const unsigned long long m = __ballot(in);
  if (threadIdx.x == 0) cull[(long)d * ntiles + t] = m;
}

// The (image entry, tile) pairs with at least one source inside the sphere,
// in entry-major order, packed as d << kTileBits | t; count in *count.  One
// block: each thread counts a contiguous run of entries, a block scan gives
// the offsets, the runs are written in order.
constexpr int kTileBits = 20;
constexpr int kCompactThreads = 1024;

__global__ __launch_bounds__(kCompactThreads) void k_compact(int nent, int ntiles,
                                                             const unsigned long long* __restrict__ cull,
                                                             unsigned* __restrict__ list, int* __restrict__ count) {
  __shared__ int sc[kCompactThreads];
  const int per = (nent + kCompactThreads - 1) / kCompactThreads;
  const int b = threadIdx.x * per, e = min(nent, b + per);
  int c = 0;
  for (int i = b; i < e; ++i) c += cull[i] != 0ull;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int o = 1; o < kCompactThreads; o <<= 1) {
    const int v = threadIdx.x >= o ? sc[threadIdx.x - o] : 0;
    __syncthreads();
    sc[threadIdx.x] += v;
    __syncthreads();
  }
  int w = sc[threadIdx.x] - c;
  for (int i = b; i < e; ++i)
    if (cull[i] != 0ull) list[w++] = ((unsigned)(i / ntiles) << kTileBits) | (unsigned)(i % ntiles);
  if (threadIdx.x == kCompactThreads - 1) *count = sc[threadIdx.x];
}

// Sphere near set view passed to the pair kernels (all null for the cell
// stencil): source masks per (entry, tile), the compacted non-empty pairs
// and their number.
struct CullView {
  const unsigned long long* mask;
  const unsigned* list;
  const int* count;
};

// ----------------------------------------------------------------- pair sums
// One wave per work item: a group of up to 64*kTPL targets against a
// contiguous range of (image entry, source tile) pairs.  Sources are read
// with wave-uniform (scalar) loads, so a source costs no VGPRs and no LDS.
// Coordinates: targets are kept as offsets from their group's box centre;
// each tile contributes the FP32-rounded FP64 shift between its image
// centre and the group centre, so close pairs subtract small numbers.
// Accumulation: the potential terms q / r (FP32 pair arithmetic) are
// summed in FP64, one conversion and one FP64 add per pair.  Without it the
// rounding of the FP32 running sum inside a tile, whose partial sums grow
// like a random walk of +-q/r terms, was the largest error of the energy
// (about 3.5x the pair terms' own rounding in an emulation of this loop on
// the 20,000-ion slab); measured against the FP64 path the relative energy
// error went from 7.0e-7 / 2.45e-6 / 5.5e-8 to 4.1e-7 / 6.3e-7 / 2.7e-7
// on the 50,000-ion, slab and 999,999-ion systems, for 8 % of the loop's
// throughput.  The field (bar 1e-5) keeps FP32 sums.
//
// The work is split by distance.  A (tile, image) whose bounding box stays
// at least rc from the group's ("far") goes through the FAR kernel, a plain
// FP32 loop.  The few others ("near": the group's own tile and its
// neighbours) go through the NEAR kernel, which recomputes the difference
// vector of any pair closer than rc from the FP64 positions and drops the
// self pair.  Both kernels classify tiles with the same FP64 arithmetic, so
// every pair is summed exactly once.
//
// Sphere near set: the wave walks its share of the compacted list of
// (image entry, tile) pairs that hold at least one source inside the
// sphere, and the sources of a tile the sphere cuts enter with zero charge
// (bit k of the tile's mask), so the loop is the same as for the stencil.
//
// Tile classification shared by the far and near kernels.  Explicitly
// rounded operations (no FMA contraction) so that both kernels reach the
// same decision for every (group, image, tile) and each pair is summed once.
__device__ __forceinline__ double shifted_dz(const Desc& ds, double cz, double cgz) {
  return __dsub_rn(__dadd_rn(__dmul_rn(ds.sigma, cz), ds.sz), cgz);
}
__device__ __forceinline__ double gap2_of(double dlx, double dly, double dlz, double hx, double hy, double hz) {
  const double gx = fmax(0.0, __dsub_rn(fabs(dlx), hx));
  const double gy = fmax(0.0, __dsub_rn(fabs(dly), hy));
  const double gz = fmax(0.0, __dsub_rn(fabs(dlz), hz));
  return __dadd_rn(__dadd_rn(__dmul_rn(gx, gx), __dmul_rn(gy, gy)), __dmul_rn(gz, gz));
}

#ifndef HSMA_FAR_UNROLL
#define HSMA_FAR_UNROLL 16
#endif
// Register budget of the pair kernels: 8 waves per SIMD (<= 64 VGPRs).  The
// loop is bound by VALU + transcendental issue, and without this bound the
// compiler spends registers on interleaving and drops to 4 waves (-25 %).
// The FP64 variant keeps 4 waves so that its doubles do not spill; the FP32
// near pass, a few per cent of the pairs, gets 6 for its FP64 close-pair
// registers.
#ifndef HSMA_WAVES_PER_EU
#define HSMA_WAVES_PER_EU 8
#endif
#define HSMA_PAIR_ATTR \
  __attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? (NEAR ? 6 : HSMA_WAVES_PER_EU) : 4)))

template <typename Real, bool NEAR, bool PARTICLES>
__global__ __launch_bounds__(kWave * kFarWaves) HSMA_PAIR_ATTR void k_pair(const double4* __restrict__ tgt, const Group* __restrict__ cgroups,
                                             const CheckSched* __restrict__ csched, int ncg, int cbase,
                                             PartSched ps,
                                             const Desc* __restrict__ desc,
                                             int ntiles, const double4* __restrict__ tile_c,
                                             const float4* __restrict__ tile_h,
                                             const typename SrcT<Real>::T* __restrict__ src,
                                             const double4* __restrict__ pos64, const StepParams* __restrict__ sp,
                                             CullView cv,
                                             Real* __restrict__ part, long comp_stride, long slot_stride) {
  typedef typename SrcT<Real>::T S;
  Work w;
  Group g;
  int part_i = 0, nparts = 1;  // this wave's share of the group's range
  if constexpr (PARTICLES) {
    int gi;
    if constexpr (NEAR) {
      // near work split over ps.nnear waves per group (blocks of kWave
      // tiles dealt round-robin, see below); slots nch .. nch + nnear - 1
      const int c = blockIdx.x / ps.ngroups;
      gi = blockIdx.x - c * ps.ngroups;
      w = Work{gi, 0, ps.F, ps.nch + c};
      part_i = c;
      nparts = ps.nnear;
    } else {
      // kFarWaves waves per block: consecutive groups, the same chunk (see
      // the far loop)
      const int ngb = (ps.ngroups + kFarWaves - 1) / kFarWaves;
      const int c = blockIdx.x / ngb;
      gi = (blockIdx.x - c * ngb) * kFarWaves + (int)(threadIdx.x / kWave);
      const int f0 = c * ps.chunk;
      w = Work{gi, f0, min(ps.F, f0 + ps.chunk), c};
      part_i = c;
      nparts = ps.nch;
    }
    g = Group{gi * kGroup, max(0, min(kGroup, ps.n - gi * kGroup)), 0, ps.ndesc};
  } else {
    // checks: cbase offsets the launch index (a launch may cover a subset
    // of the groups: its far waves, or its groups for the near pass)
    const int bid = (int)blockIdx.x + cbase;
    int gi;
    if constexpr (NEAR) {
      gi = bid;
    } else {
      // the check group whose far waves include this one (binary search)
      int lo = 0, hi = ncg - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (csched[mid].first_work <= bid) lo = mid;
        else hi = mid - 1;
      }
      gi = lo;
    }
    const CheckSched cs = csched[gi];
    g = cgroups[gi];
    const int F = g.ndesc * ntiles;
    if constexpr (NEAR) {
      w = Work{gi, 0, F, cs.slot0 + cs.nch};
    } else {
      const int c = bid - cs.first_work;
      const int f0 = c * cs.chunk;
      w = Work{gi, f0, min(F, f0 + cs.chunk), cs.slot0 + c};
      part_i = c;
      nparts = cs.nch;
    }
  }
  const double3 hbox = sp->hbox;
  // FP64 check sums need neither close-pair corrections nor self exclusion:
  // every tile goes through the far kernel (a face check group spans a whole
  // face, so its box overlaps many tiles)
  const double rc2 = PARTICLES ? sp->rc2 : (sizeof(Real) == 8 ? -1.0 : sp->rc2c);
  const int lane = threadIdx.x % kWave;
  // the far particle kernel runs kFarWaves waves per block in step (a block
  // barrier per source tile), so that the block's waves read each tile from
  // the scalar cache together; a wave past the last group only keeps step
  constexpr bool kStep = PARTICLES && !NEAR;
  const bool active = g.count > 0;
  bool valid[kTPL];
  Real ox[kTPL], oy[kTPL], oz[kTPL];
  double mnx = INFINITY, mny = INFINITY, mnz = INFINITY, mxx = -INFINITY, mxy = -INFINITY, mxz = -INFINITY;
  double4 tp[kTPL];
#pragma unroll
  for (int j = 0; j < kTPL; ++j) {
    const int l = j * kWave + lane;
    valid[j] = l < g.count;
    tp[j] = tgt[valid[j] ? g.first + l : 0];
    if (valid[j]) {
      mnx = fmin(mnx, tp[j].x); mxx = fmax(mxx, tp[j].x);
      mny = fmin(mny, tp[j].y); mxy = fmax(mxy, tp[j].y);
      mnz = fmin(mnz, tp[j].z); mxz = fmax(mxz, tp[j].z);
    }
  }
  mnx = wave_min(mnx); mxx = wave_max(mxx);
  mny = wave_min(mny); mxy = wave_max(mxy);
  mnz = wave_min(mnz); mxz = wave_max(mxz);
  const double cgx = active ? 0.5 * (mnx + mxx) : 0.0, cgy = active ? 0.5 * (mny + mxy) : 0.0,
               cgz = active ? 0.5 * (mnz + mxz) : 0.0;
  const double hgx = active ? 0.5 * (mxx - mnx) : 0.0, hgy = active ? 0.5 * (mxy - mny) : 0.0,
               hgz = active ? 0.5 * (mxz - mnz) : 0.0;
  // potential: FP64 accumulator per target (the pair terms are summed into
  // it in FP64, so the sum adds no rounding of its own); field: Real
  double ph[kTPL];
  Real ex[kTPL], ey[kTPL], ez[kTPL];
#pragma unroll
  for (int j = 0; j < kTPL; ++j) {
    ox[j] = (Real)(tp[j].x - cgx);
    oy[j] = (Real)(tp[j].y - cgy);
    oz[j] = (Real)(tp[j].z - cgz);
    ph[j] = 0.0;
    ex[j] = ey[j] = ez[j] = (Real)0;
  }
  const int tbase = g.first + lane;  // sorted index of this lane's first target

  // One (image, tile) pair: sum its 64 sources into the accumulators.
  // m: sphere near set mask of the tile's sources (all ones for the cell
  // stencil); cleared bits contribute nothing.
  auto do_tile = [&](const Desc& ds, const bool own, const int tile, const double dlx, const double dly,
                     const double dlz, const unsigned long long m) {
    const Real sg = (Real)ds.sigma;
    const Real sc = (Real)ds.scale;
    Real ux[kTPL], uy[kTPL], uz[kTPL];
    Real qx[kTPL], qy[kTPL], qz[kTPL];
    double pp[kTPL];
#pragma unroll
    for (int j = 0; j < kTPL; ++j) {
      ux[j] = ox[j] - (Real)dlx;
      uy[j] = oy[j] - (Real)dly;
      uz[j] = sg * (oz[j] - (Real)dlz);
      pp[j] = 0.0;
      qx[j] = qy[j] = qz[j] = (Real)0;
    }
    const S* __restrict__ s = src + (long)tile * kTile;
    if (!NEAR && PARTICLES && own) {
      // a far tile that holds the group's own particles under a shifted
      // image: drop each target's own image (summed in FP64 by finalize)
      for (int k = 0; k < kTile; ++k) {
        const S v = s[k];
        const long si = (long)tile * kTile + k;
#pragma unroll
        for (int j = 0; j < kTPL; ++j) {
          const bool self = si == (long)(tbase + j * kWave);
          const bool drop = self || !((m >> k) & 1ull);
          const Real dx = ux[j] - (Real)v.x;
          const Real dy = uy[j] - (Real)v.y;
          const Real dz = uz[j] - (Real)v.z;
          const Real r2 = self ? (Real)1 : dx * dx + dy * dy + dz * dz;
          const Real ri = rsq(r2);
          const Real a = (drop ? (Real)0 : (Real)v.w) * ri;
          pp[j] += (double)a;
          const Real b = a * (ri * ri);
          qx[j] += b * dx;
          qy[j] += b * dy;
          qz[j] += b * dz;
        }
      }
    } else if constexpr (!NEAR) {
      // the plain loop; a tile cut by the sphere runs the same loop with
      // the charges of the sources outside it set to zero, over the
      // blocks of HSMA_FAR_UNROLL sources between its first and last
      // source inside (m != 0 here: empty tiles never reach this point)
      auto far_loop = [&](auto masked) {
        int k0 = 0, k1 = kTile;
        if constexpr (decltype(masked)::value) {
          k0 = __builtin_ctzll(m) / HSMA_FAR_UNROLL * HSMA_FAR_UNROLL;
          k1 = (kTile - __builtin_clzll(m) + HSMA_FAR_UNROLL - 1) / HSMA_FAR_UNROLL * HSMA_FAR_UNROLL;
        }
#pragma unroll HSMA_FAR_UNROLL
        for (int k = k0; k < k1; ++k) {
          const S v = s[k];
          Real qv = (Real)v.w;
          if constexpr (decltype(masked)::value) qv = ((m >> k) & 1ull) ? qv : (Real)0;
#pragma unroll
          for (int j = 0; j < kTPL; ++j) {
            const Real dx = ux[j] - (Real)v.x;
            const Real dy = uy[j] - (Real)v.y;
            const Real dz = uz[j] - (Real)v.z;
            const Real r2 = dx * dx + dy * dy + dz * dz;
            const Real ri = rsq(r2);
            const Real a = qv * ri;
            pp[j] += (double)a;
            const Real b = a * (ri * ri);
            qx[j] += b * dx;
            qy[j] += b * dy;
            qz[j] += b * dz;
          }
        }
      };
      if (m == ~0ull) far_loop(std::false_type{});
      else far_loop(std::true_type{});
    } else {
      // the tile's FP64 positions, one per lane: a close pair reads its
      // source's from lane k (no memory access inside the loop)
      const double4 p64 = pos64[(long)tile * kTile + lane];
#pragma unroll 2
      for (int k = 0; k < kTile; ++k) {
        const S v = s[k];
#pragma unroll
        for (int j = 0; j < kTPL; ++j) {
          Real dx = ux[j] - (Real)v.x;
          Real dy = uy[j] - (Real)v.y;
          Real dz = uz[j] - (Real)v.z;
          Real r2 = dx * dx + dy * dy + dz * dz;
          Real qq = ((m >> k) & 1ull) ? (Real)v.w : (Real)0;
          const long si = (long)tile * kTile + k;
          if (PARTICLES && own && si == (long)(tbase + j * kWave)) {
            // the target itself or one of its own images: summed in FP64 by
            // the finalize kernel (self pair excluded there)
            qq = (Real)0;
            r2 = (Real)1;
          } else if ((double)r2 < rc2) {
            // close pair: difference vector from the FP64 positions
            const double psx = readlane_d(p64.x, k), psy = readlane_d(p64.y, k), psz = readlane_d(p64.z, k);
            dx = (Real)(tp[j].x - (psx + ds.sx));
            dy = (Real)(tp[j].y - (psy + ds.sy));
            dz = sg * (Real)(tp[j].z - (ds.sigma * psz + ds.sz));
            r2 = dx * dx + dy * dy + dz * dz;
          }
          const Real ri = rsq(r2);
          const Real a = qq * ri;
          pp[j] += (double)a;
          const Real b = a * (ri * ri);
          qx[j] += b * dx;
          qy[j] += b * dy;
          qz[j] += b * dz;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kTPL; ++j) {
      ph[j] += ds.scale * pp[j];
      ex[j] += sc * qx[j];
      ey[j] += sc * qy[j];
      ez[j] += (sc * sg) * qz[j];
    }
  };

  // The group's own tiles hold the targets themselves: under every image a
  // target must not meet itself or its own image in the FP32 sums (those
  // terms share one distance for all particles, so their rounding would not
  // average out; finalize sums them in FP64).  Near kernel and far kernel
  // both drop source index == target index inside own tiles.
  const int own0 = PARTICLES ? g.first / kTile : 0;
  const int own1 = PARTICLES ? (g.first + g.count - 1) / kTile : -1;

  const unsigned long long* __restrict__ cull = cv.mask;
  if (cv.list) {
    // sphere near set: the wave takes its share of the compacted non-empty
    // (entry, tile) pairs (the same share of the same list for every group)
    const int C = *cv.count;
    const int per = (C + nparts - 1) / nparts;
    const int f0 = min(C, part_i * per), f1 = min(C, f0 + per);
    const unsigned tmask = (1u << kTileBits) - 1u;
    if constexpr (NEAR) {
      // every wave scans the list in blocks of kWave entries; the near
      // entries, in list order, are dealt round-robin to the group's waves
      int skip = part_i;  // near entries to pass over before this wave's next one
      for (int fb = 0; fb < C; fb += kWave) {
        const int fl = fb + lane;
        bool near = false;
        if (fl < C) {
          const unsigned e = cv.list[fl];
          const int tile = (int)(e & tmask);
          const Desc dsl = desc[g.desc_off + (int)(e >> kTileBits)];
          const double4 cs = tile_c[tile];
          const float4 hs = tile_h[tile];
          const double dlx = __dsub_rn(__dadd_rn(cs.x, dsl.sx), cgx);
          const double dly = __dsub_rn(__dadd_rn(cs.y, dsl.sy), cgy);
          const double dlz = shifted_dz(dsl, cs.z, cgz);
          near = gap2_of(dlx, dly, dlz, __dadd_rn(hgx, (double)hs.x), __dadd_rn(hgy, (double)hs.y),
                         __dadd_rn(hgz, (double)hs.z)) < rc2;
        }
        unsigned long long m = __ballot(near);
        const int cnt = __popcll(m);
        if (cnt <= skip) {
          skip -= cnt;
          continue;
        }
        while (m) {
          const int l = __ffsll((long long)m) - 1;
          m &= m - 1;
          if (skip > 0) {
            --skip;
            continue;
          }
          skip = nparts - 1;
          const unsigned e = cv.list[fb + l];
          const int di = (int)(e >> kTileBits), nt = (int)(e & tmask);
          const Desc ds = desc[g.desc_off + di];
          const double4 cs = tile_c[nt];
          const double dlx = __dsub_rn(__dadd_rn(cs.x, ds.sx), cgx);
          const double dly = __dsub_rn(__dadd_rn(cs.y, ds.sy), cgy);
          const double dlz = shifted_dz(ds, cs.z, cgz);
          do_tile(ds, nt >= own0 && nt <= own1, nt, dlx, dly, dlz, cull[(long)di * ntiles + nt]);
        }
      }
    } else {
      int cur = -1;
      Desc ds{};
      bool img_far = false;
      for (int f = f0; f < f1; ++f) {
        if constexpr (kStep) __syncthreads();
        if (!active) continue;
        const unsigned e = cv.list[f];
        const int di = (int)(e >> kTileBits), tile = (int)(e & tmask);
        if (di != cur) {
          cur = di;
          ds = desc[g.desc_off + di];
          img_far = gap2_of(__dsub_rn(ds.sx, cgx), __dsub_rn(ds.sy, cgy), __dsub_rn(ds.sz, cgz),
                            __dadd_rn(hgx, hbox.x), __dadd_rn(hgy, hbox.y), __dadd_rn(hgz, hbox.z)) >= rc2;
        }
        const double4 cs = tile_c[tile];
        const double dlx = __dsub_rn(__dadd_rn(cs.x, ds.sx), cgx);
        const double dly = __dsub_rn(__dadd_rn(cs.y, ds.sy), cgy);
        const double dlz = shifted_dz(ds, cs.z, cgz);
        if (!img_far) {
          const float4 hs = tile_h[tile];
          if (gap2_of(dlx, dly, dlz, __dadd_rn(hgx, (double)hs.x), __dadd_rn(hgy, (double)hs.y),
                      __dadd_rn(hgz, (double)hs.z)) < rc2)
            continue;  // summed by the near pass
        }
        do_tile(ds, tile >= own0 && tile <= own1, tile, dlx, dly, dlz, cull[(long)di * ntiles + tile]);
      }
    }
  }
  if constexpr (NEAR) {
    if (!cv.list) {
      // near pass over the cell stencil: every wave of the group scans the
      // (image entry, block of kWave tiles) pairs, and the near tiles, in
      // scan order, are dealt round-robin to its nparts waves.  The near
      // tiles cluster in a few blocks of the central image, so dealing
      // whole blocks (or contiguous ranges) would leave most of them to one
      // wave.
      const int nblk = (ntiles + kWave - 1) / kWave;
      const int nb = g.ndesc * nblk;
      int skip = part_i;  // near tiles to pass over before this wave's next one
      for (int b = 0; b < nb; ++b) {
        const int di = b / nblk;
        const int tb = (b - di * nblk) * kWave;
        const int t1 = min(ntiles, tb + kWave);
        const Desc ds = desc[g.desc_off + di];
        // every tile of this image lies inside the shifted box: if the box
        // is far from the group, so is each of its tiles
        if (gap2_of(__dsub_rn(ds.sx, cgx), __dsub_rn(ds.sy, cgy), __dsub_rn(ds.sz, cgz), __dadd_rn(hgx, hbox.x),
                    __dadd_rn(hgy, hbox.y), __dadd_rn(hgz, hbox.z)) >= rc2)
          continue;
        // lane-parallel scan: lane l classifies tile tb + l, then the wave
        // walks the near ones in increasing tile order
        const int tile = tb + lane;
        bool near = false;
        if (tile < t1) {
          const double4 cs = tile_c[tile];
          const float4 hs = tile_h[tile];
          const double dlx = __dsub_rn(__dadd_rn(cs.x, ds.sx), cgx);
          const double dly = __dsub_rn(__dadd_rn(cs.y, ds.sy), cgy);
          const double dlz = shifted_dz(ds, cs.z, cgz);
          near = gap2_of(dlx, dly, dlz, __dadd_rn(hgx, (double)hs.x), __dadd_rn(hgy, (double)hs.y),
                         __dadd_rn(hgz, (double)hs.z)) < rc2;
          if (cull && near) near = cull[(long)di * ntiles + tile] != 0ull;
        }
        unsigned long long m = __ballot(near);
        const int cnt = __popcll(m);
        if (cnt <= skip) {
          skip -= cnt;
          continue;
        }
        while (m) {
          const int l = __ffsll((long long)m) - 1;
          m &= m - 1;
          if (skip > 0) {
            --skip;
            continue;
          }
          skip = nparts - 1;
          const int nt = tb + l;
          const double4 cs = tile_c[nt];
          const double dlx = __dsub_rn(__dadd_rn(cs.x, ds.sx), cgx);
          const double dly = __dsub_rn(__dadd_rn(cs.y, ds.sy), cgy);
          const double dlz = shifted_dz(ds, cs.z, cgz);
          do_tile(ds, nt >= own0 && nt <= own1, nt, dlx, dly, dlz, cull ? cull[(long)di * ntiles + nt] : ~0ull);
        }
      }
    }
  }
  // far kernel over the cell stencil: [f0, f1) of the entry-major range
  int f = (NEAR || cv.list) ? w.f1 : w.f0;
  while (f < w.f1) {
    const int di = f / ntiles;
    const int t0 = f - di * ntiles;
    const int t1 = min(ntiles, t0 + (w.f1 - f));
    f += t1 - t0;
    const Desc ds = desc[g.desc_off + di];
    // every tile of this image lies inside the shifted box: if the box is
    // far from the group, so is each of its tiles
    const bool img_far = gap2_of(__dsub_rn(ds.sx, cgx), __dsub_rn(ds.sy, cgy), __dsub_rn(ds.sz, cgz),
                                 __dadd_rn(hgx, hbox.x), __dadd_rn(hgy, hbox.y), __dadd_rn(hgz, hbox.z)) >= rc2;
    if constexpr (!NEAR) {
      for (int tile = t0; tile < t1; ++tile) {
        if constexpr (kStep) __syncthreads();
        if (!active) continue;
        unsigned long long cm = ~0ull;
        if (cull) {
          cm = cull[(long)di * ntiles + tile];
          if (cm == 0ull) continue;  // every source of this image outside the sphere
        }
        const double4 cs = tile_c[tile];
        const double dlx = __dsub_rn(__dadd_rn(cs.x, ds.sx), cgx);
        const double dly = __dsub_rn(__dadd_rn(cs.y, ds.sy), cgy);
        const double dlz = shifted_dz(ds, cs.z, cgz);
        if (!img_far) {
          const float4 hs = tile_h[tile];
          if (gap2_of(dlx, dly, dlz, __dadd_rn(hgx, (double)hs.x), __dadd_rn(hgy, (double)hs.y),
                      __dadd_rn(hgz, (double)hs.z)) < rc2)
            continue;  // summed by the near pass
        }
        do_tile(ds, tile >= own0 && tile <= own1, tile, dlx, dly, dlz, cm);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kTPL; ++j) {
    if (!valid[j]) continue;
    const long o = (long)w.slot * slot_stride + (PARTICLES ? (long)g.first : 0L) + j * kWave + lane;
    // potential as an unevaluated (hi, lo) pair of Real
    const Real hi = (Real)ph[j];
    part[o] = hi;
    part[o + comp_stride] = (Real)(ph[j] - (double)hi);
    part[o + 2 * comp_stride] = ex[j];
    part[o + 3 * comp_stride] = ey[j];
    part[o + 4 * comp_stride] = ez[j];
  }
}

// Sphere sources: charge Q_k and double-layer strength D_k at y_k, normal
// n_k.  phi += Q/|d| - D (n.d)/|d|^3,  E += Q d/|d|^3 + D (n/|d|^3 - 3 (n.d) d/|d|^5).
// Records: surf[2k] = (y, Q), surf[2k+1] = (n, D), box-centred coordinates.
// Grid: (target group, chunk of `chunk` sources); slot = slot0 + chunk index.
// Always FP64: the Green representation of the harmonic part cancels
// strongly inside the sphere (u on the sphere exceeds u in the box by about
// lambda^p), so FP32 rounding of Q_k, D_k and y_k would be amplified into a
// smooth error field; these sums are N x F pairs, a few per mille of the
// near-set work.  FP32 partials store the potential as a (hi, lo) pair.
constexpr int kSphereChunkMin = 16, kSphereChunkMax = 256;

// Sphere sources per wave: enough waves (about 1024) to keep small systems
// from running on a handful of long waves, at most kSphereChunkMax.
static int sphere_chunk(int F, int ngroups) {
  const long long want = ((long long)F * ngroups + 1023) / 1024;
  const long long c = (want + kSphereChunkMin - 1) / kSphereChunkMin * kSphereChunkMin;
  return (int)std::min<long long>(kSphereChunkMax, std::max<long long>(kSphereChunkMin, c));
}

template <typename Real>
__global__ __launch_bounds__(64) void k_pair_sphere(const double4* __restrict__ tgt, int n,
                                                    const double4* __restrict__ surf, int F, int chunk,
                                                    Real* __restrict__ part, long comp_stride, int slot0) {
  const int lane = threadIdx.x;
  const int first = blockIdx.x * kGroup;
  const int kb = blockIdx.y * chunk, ke = min(F, kb + chunk);
  double tx[kTPL], ty[kTPL], tz[kTPL];
  double ph[kTPL], ex[kTPL], ey[kTPL], ez[kTPL];
#pragma unroll
  for (int j = 0; j < kTPL; ++j) {
    const int t = min(first + j * kWave + lane, n - 1);
    const double4 p = tgt[t];
    tx[j] = p.x;
    ty[j] = p.y;
    tz[j] = p.z;
    ph[j] = ex[j] = ey[j] = ez[j] = 0.0;
  }
  for (int k = kb; k < ke; ++k) {
    const double4 a0 = surf[2 * k], a1 = surf[2 * k + 1];
#pragma unroll
    for (int j = 0; j < kTPL; ++j) {
      const double dx = tx[j] - a0.x, dy = ty[j] - a0.y, dz = tz[j] - a0.z;
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double ri = rsq(r2);
      const double ri2 = ri * ri;
      const double ri3 = ri * ri2;
      const double a = a0.w * ri;
      const double nd = a1.x * dx + a1.y * dy + a1.z * dz;
      const double t = a1.w * nd * ri3;
      ph[j] += a - t;
      const double c1 = ri2 * (a - 3.0 * t);
      const double c2 = a1.w * ri3;
      ex[j] += c1 * dx + c2 * a1.x;
      ey[j] += c1 * dy + c2 * a1.y;
      ez[j] += c1 * dz + c2 * a1.z;
    }
  }
#pragma unroll
  for (int j = 0; j < kTPL; ++j) {
    const int t = first + j * kWave + lane;
    if (t >= n) continue;
    const long o = (long)(slot0 + blockIdx.y) * 5 * comp_stride + t;
    const Real hi = (Real)ph[j];
    part[o] = hi;
    part[o + comp_stride] = (Real)(ph[j] - (double)hi);
    part[o + 2 * comp_stride] = (Real)ex[j];
    part[o + 3 * comp_stride] = (Real)ey[j];
    part[o + 4 * comp_stride] = (Real)ez[j];
  }
}

// ----------------------------------------------------------------- check / LSQ / sphere
// Sum the work-item partials of every check target in a fixed order:
// v[2t] = potential, v[2t+1] = field component axis[t].  One block per
// check group; the two halves of the block take alternate slots and are
// combined at the end (error-free for the FP32 potential).
// ------------------------------------------------------------ treecode
// Near rule 2: the far part of the cell-stencil sums at the particles by a
// treecode.  A source node (levels >= 1 of the tile hierarchy) far enough
// from a target group, (r_node + r_group) < theta * distance, acts through
// its multipole expansion about its centre; other nodes are opened; tiles
// reached that way are summed directly (the near pass keeps the tile
// pairs within the close-pair radius, as for rule 0).  The expansion is
// the addition theorem of the solid harmonics,
//   1 / |x - y| = sum_{n >= 0} sum_{|m| <= n} conj(U_n^m(y)) T_n^m(x),
// |y| < |x|, with the regular U and irregular T harmonics fixed by
//   U_0^0 = 1, U_m^m = (x + iy) / (2m) U_{m-1}^{m-1},
//   U_n^m = ((2n - 1) z U_{n-1}^m - r^2 U_{n-2}^m) / ((n + m)(n - m)),
//   T_0^0 = 1 / r, T_m^m = (2m - 1) (x + iy) / r^2 T_{m-1}^{m-1},
//   T_n^m = ((2n - 1) z T_{n-1}^m - ((n - 1)^2 - m^2) T_{n-2}^m) / r^2,
// and X_n^{-m} = (-1)^m conj(X_n^m).  The moments of a node about its
// centre c are M_n^m = sum_j q_j U_n^m(y_j - c); its potential is
// sum conj(M_n^m) T_n^m(x - c), and the field follows from
//   d/dz T_n^m = -T_{n+1}^m,  (d/dx + i d/dy) T_n^m = -T_{n+1}^{m+1}.
// Moments are built in FP64 (tiles of level-1 nodes directly, higher
// levels by shifting the children's moments, U_n^m(a + b) =
// sum_k sum_l U_k^l(a) U_{n-k}^{m-l}(b)) and evaluated in FP32.

__device__ __forceinline__ int tree_idx(int n, int m) { return n * (n + 1) / 2 + m; }

// A value equal in every lane, marked as such for the compiler (so that
// what depends on it stays in scalar registers and branches).
__device__ __forceinline__ double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// X_n^m of a table of m >= 0 entries (re, im interleaved), any |m| <= n
__device__ __forceinline__ void tree_get(const double* t, int n, int m, double& re, double& im) {
  const int am = m < 0 ? -m : m;
  re = t[2 * tree_idx(n, am)];
  im = t[2 * tree_idx(n, am) + 1];
  if (m < 0) {
    const double s = (am & 1) ? -1.0 : 1.0;
    re *= s;
    im *= -s;
  }
}

// Level-1 nodes: bounding box of their (up to 8) tiles, centre, radius,
// and moments from their particles.  One block of 8 waves per node, wave
// w on tile 8 * node + w; each moment is a wave sum per tile, then a sum
// over the tiles in tile order.
__global__ __launch_bounds__(512) void k_tree_p2m(int n, int ntiles, int order, TreeLevels tl,
                                                 const double4* __restrict__ pos64,
                                                 const double4* __restrict__ tile_c,
                                                 const float4* __restrict__ tile_h, double4* __restrict__ node_c,
                                                 double4* __restrict__ node_box, double* __restrict__ mom64,
                                                 float* __restrict__ mom32) {
  __shared__ double sbox[8][6];
  __shared__ double sc[3];
  __shared__ double srad[8];
  __shared__ double sm[8][2 * kTreeMom];
  const int node = blockIdx.x;
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int t = 8 * node + w;
  const bool has = t < ntiles;
  if (lane == 0) {
    if (has) {
      const double4 c = tile_c[t];
      const float4 h = tile_h[t];
      sbox[w][0] = c.x - (double)h.x; sbox[w][1] = c.y - (double)h.y; sbox[w][2] = c.z - (double)h.z;
      sbox[w][3] = c.x + (double)h.x; sbox[w][4] = c.y + (double)h.y; sbox[w][5] = c.z + (double)h.z;
    } else {
      sbox[w][0] = sbox[w][1] = sbox[w][2] = INFINITY;
      sbox[w][3] = sbox[w][4] = sbox[w][5] = -INFINITY;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = sbox[0][d];
      hi[d] = sbox[0][3 + d];
      for (int k = 1; k < 8; ++k) {
        lo[d] = fmin(lo[d], sbox[k][d]);
        hi[d] = fmax(hi[d], sbox[k][3 + d]);
      }
      sc[d] = 0.5 * (lo[d] + hi[d]);
    }
    const double hx = 0.5 * (hi[0] - lo[0]), hy = 0.5 * (hi[1] - lo[1]), hz = 0.5 * (hi[2] - lo[2]);
    const int g = tl.off[1] + node;
    node_box[2 * g] = make_double4(lo[0], lo[1], lo[2], sqrt(hx * hx + hy * hy + hz * hz));
    node_box[2 * g + 1] = make_double4(hi[0], hi[1], hi[2], 0.0);
  }
  __syncthreads();
  const int s = t * kTile + lane;
  double q = 0, yx = 0, yy = 0, yz = 0;
  if (has && s < n) {
    const double4 p = pos64[s];
    q = p.w;
    yx = p.x - sc[0];
    yy = p.y - sc[1];
    yz = p.z - sc[2];
  }
  const double r2 = yx * yx + yy * yy + yz * yz;
  // radius of the node's particles about its centre (the opening test's r)
  const double rw = wave_max(has && s < n ? sqrt(r2) : 0.0);
  if (lane == 0) srad[w] = rw;
  double ur = 1.0, ui = 0.0;  // sectoral U_m^m
  for (int m = 0; m <= order; ++m) {
    if (m > 0) {
      const double f = 1.0 / (2 * m);
      const double nr = f * (yx * ur - yy * ui), ni = f * (yx * ui + yy * ur);
      ur = nr;
      ui = ni;
    }
    double pr = 0.0, pi = 0.0, cr = ur, ci = ui;  // U_{n-1}^m, U_n^m
    for (int nn = m; nn <= order; ++nn) {
      if (nn > m) {
        const double inv = 1.0 / ((double)(nn + m) * (double)(nn - m));
        const double a = (2 * nn - 1) * yz;
        const double nr = (a * cr - r2 * pr) * inv, ni = (a * ci - r2 * pi) * inv;
        pr = cr;
        pi = ci;
        cr = nr;
        ci = ni;
      }
      const double vr = wave_sum_d(q * cr), vi = wave_sum_d(q * ci);
      if (lane == 0) {
        sm[w][2 * tree_idx(nn, m)] = vr;
        sm[w][2 * tree_idx(nn, m) + 1] = vi;
      }
    }
  }
  __syncthreads();
  const int nr2 = (order + 1) * (order + 2);
  const long g = (long)tl.off[1] + node;
  if (threadIdx.x == 0) {
    double r = srad[0];
    for (int k = 1; k < 8; ++k) r = fmax(r, srad[k]);
    node_c[g] = make_double4(sc[0], sc[1], sc[2], r);
  }
  for (int k = threadIdx.x; k < nr2; k += blockDim.x) {
    double acc = 0.0;
    for (int ww = 0; ww < 8; ++ww) acc += sm[ww][k];
    mom64[g * kTreeMomStride + k] = acc;
    mom32[g * kTreeMomStride + k] = (float)acc;
  }
}

// Nodes of level l >= 2: box from the children's boxes, moments by
// shifting the children's moments to the node centre.  One block of 8
// waves per node: wave w shifts child 8 * node + w (lane k on moments k and
// k + 64), and the 8 shifted sets are added in child order.
__global__ __launch_bounds__(512) void k_tree_m2m(int level, int order, TreeLevels tl, double4* __restrict__ node_c,
                                                 double4* __restrict__ node_box, double* __restrict__ mom64,
                                                 float* __restrict__ mom32) {
  __shared__ double su[8][2 * kTreeMom];
  __shared__ double smc[8][2 * kTreeMom];
  __shared__ double sc[3];
  const int node = blockIdx.x;
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int c0 = 8 * node, c1 = min(c0 + 8, tl.cnt[level - 1]);
  const int coff = tl.off[level - 1];
  const int g = tl.off[level] + node;
  if (w == 0) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double4 cc4 = make_double4(0, 0, 0, 0);
    const bool hasc = lane < c1 - c0;
    if (hasc) {
      const double4 a = node_box[2 * (coff + c0 + lane)], b = node_box[2 * (coff + c0 + lane) + 1];
      lo[0] = a.x; lo[1] = a.y; lo[2] = a.z;
      hi[0] = b.x; hi[1] = b.y; hi[2] = b.z;
      cc4 = node_c[coff + c0 + lane];
    }
    double c[3], h[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = wave_min(lo[d]);
      hi[d] = wave_max(hi[d]);
      c[d] = 0.5 * (lo[d] + hi[d]);
      h[d] = 0.5 * (hi[d] - lo[d]);
    }
    // particle radius: within the box's half diagonal, and within each
    // child's centre distance plus its radius; the smaller bound is kept
    const double ex = cc4.x - c[0], ey = cc4.y - c[1], ez = cc4.z - c[2];
    const double hd = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    const double rad = fmin(hd, wave_max(hasc ? sqrt(ex * ex + ey * ey + ez * ez) + cc4.w : 0.0));
    if (lane == 0) {
      sc[0] = c[0];
      sc[1] = c[1];
      sc[2] = c[2];
      node_c[g] = make_double4(c[0], c[1], c[2], rad);
      node_box[2 * g] = make_double4(lo[0], lo[1], lo[2], hd);
      node_box[2 * g + 1] = make_double4(hi[0], hi[1], hi[2], 0.0);
    }
  }
  __syncthreads();
  const int nm = (order + 1) * (order + 2) / 2;
  const int ch = c0 + w;
  const bool has = ch < c1;
  if (has) {
    const double4 cc = node_c[coff + ch];
    const double tx = cc.x - sc[0], ty = cc.y - sc[1], tz = cc.z - sc[2];
    for (int k = lane; k < 2 * nm; k += kWave) smc[w][k] = mom64[(long)(coff + ch) * kTreeMomStride + k];
    if (lane <= order) {
      // column m = lane of U(t)
      const int m = lane;
      double ur = 1.0, ui = 0.0;
      for (int k = 1; k <= m; ++k) {
        const double f = 1.0 / (2 * k);
        const double nr = f * (tx * ur - ty * ui), ni = f * (tx * ui + ty * ur);
        ur = nr;
        ui = ni;
      }
      const double r2 = tx * tx + ty * ty + tz * tz;
      double pr = 0.0, pi = 0.0, cr = ur, ci = ui;
      for (int nn = m; nn <= order; ++nn) {
        if (nn > m) {
          const double inv = 1.0 / ((double)(nn + m) * (double)(nn - m));
          const double a = (2 * nn - 1) * tz;
          const double nr = (a * cr - r2 * pr) * inv, ni = (a * ci - r2 * pi) * inv;
          pr = cr;
          pi = ci;
          cr = nr;
          ci = ni;
        }
        su[w][2 * tree_idx(nn, m)] = cr;
        su[w][2 * tree_idx(nn, m) + 1] = ci;
      }
    }
  }
  __syncthreads();
  // this wave's child, shifted: lane k on moments k and k + 64
  double accr[2] = {0.0, 0.0}, acci[2] = {0.0, 0.0};
  if (has) {
    for (int hh = 0; hh < 2; ++hh) {
      const int kk = lane + hh * kWave;
      if (kk >= nm) continue;
      int tn = 0;
      while (tree_idx(tn + 1, 0) <= kk) ++tn;
      const int tm = kk - tree_idx(tn, 0);
      for (int k = 0; k <= tn; ++k) {
        for (int l = -k; l <= k; ++l) {
          const int nn = tn - k, mm = tm - l;
          if (mm > nn || mm < -nn) continue;
          double ar, ai, br, bi;
          tree_get(su[w], k, l, ar, ai);
          tree_get(smc[w], nn, mm, br, bi);
          accr[hh] += ar * br - ai * bi;
          acci[hh] += ar * bi + ai * br;
        }
      }
    }
  }
  __syncthreads();  // the tables are read; reuse su as the per-child results
  for (int hh = 0; hh < 2; ++hh) {
    const int kk = lane + hh * kWave;
    if (kk < nm) {
      su[w][2 * kk] = accr[hh];
      su[w][2 * kk + 1] = acci[hh];
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 2 * nm; k += blockDim.x) {
    double acc = 0.0;
    for (int ww = 0; ww < c1 - c0; ++ww) acc += su[ww][k];
    mom64[(long)g * kTreeMomStride + k] = acc;
    mom32[(long)g * kTreeMomStride + k] = (float)acc;
  }
}

// Potential and field (-grad) at X (relative to the node centre) of the
// moments M (re, im of (n, m), m <= n <= P; P may be below the order the
// moments were built to), FP32.  The irregular harmonics T_n^m, n <= P + 1,
// are generated column by column and used at once: T_n^m feeds the
// potential through M_n^m, d/dz through M_{n-1}^m, and (d/dx + i d/dy)
// through M_{n-1}^{m-1} and M_{n-1}^{m+1}; the terms of m >= 1 count twice
// in the potential and in d/dz (the conjugate columns -m), so column 0 runs
// on its own.  Which terms a step (n, m) has depends only on where n sits
// in its column, so the first steps and the last (n = P + 1: no potential
// term) are peeled off and the steps in between run without branches: a
// rolled loop with a branch per term spent more scalar instructions (loop
// control, address arithmetic) than vector ones and waited on each
// moment's load.  The loops stay rolled otherwise, so the moments come in
// a few at a time through scalar loads (fully unrolled, the compiler would
// hold all of them at once).  Every accumulator sees the same operations in
// the same order as the plain definition.
__device__ __forceinline__ void tree_eval(const float* __restrict__ M, int P, float X, float Y, float Z, double& phi,
                                          float& fx, float& fy, float& fz) {
  const float r2 = X * X + Y * Y + Z * Z;
  const float ri = rsq(r2);
  const float ri2 = ri * ri;
  const float wr = X * ri2, wi = Y * ri2;
  const float zr = Z * ri2;
  // the potential's terms are summed in FP64 (on the 50,000-ion system the
  // energy error at order 12 went from 1.2e-6 to 4.5e-7 for 1 % of the time)
  double phi0 = 0.0, phi1 = 0.0;
  float dz0 = 0.f, dz1 = 0.f, Wr = 0.f, Wi = 0.f;
  // column m = 0: T_n^0 is real.  Step n: recursion (n >= 1), potential
  // (n <= P), d/dz (n >= 1), and + M_{n-1}^1 conj(T_n^0) (n >= 2).  The
  // factors 2n - 1 and (n - 1)^2 and the place in M are carried from step
  // to step: pv points at M_{n-1}^0, and M_n^0 is 2n reals further.
  {
    float p = 0.f, t = ri;
    auto step0 = [&](const float af, const float bf, const float* __restrict__ row, const float* __restrict__ pv,
                     auto pot, auto wplus) {
      const float a = af * zr;
      const float b = bf * ri2;
      const float nt = a * t - b * p;
      p = t;
      t = nt;
      if constexpr (decltype(pot)::value) phi0 = fma((double)row[0], (double)t, phi0);  // M_n^0
      dz0 = fmaf(pv[0], t, dz0);
      if constexpr (decltype(wplus)::value) {
        Wr = fmaf(pv[2], t, Wr);
        Wi = fmaf(pv[3], t, Wi);
      }
    };
    phi0 = fma((double)M[0], (double)t, phi0);  // n = 0
    step0(1.f, 0.f, M + 2, M, std::true_type{}, std::false_type{});
    float af = 3.f, bf = 1.f;
    const float* __restrict__ pv = M + 2;  // M_1^0
#pragma unroll 1
    for (int n = 2; n <= P; ++n) {
      const float* __restrict__ nx = pv + 2 * n;  // M_n^0
      step0(af, bf, nx, pv, std::true_type{}, std::true_type{});
      pv = nx;
      bf += af;
      af += 2.f;
    }
    step0(af, bf, pv, pv, std::false_type{}, std::true_type{});  // n = P + 1
  }
  // columns m >= 1.  Step n of column m: recursion (n > m), potential
  // (n <= P), d/dz (n - 1 >= m), - conj(M_{n-1}^{m-1}) T_n^m (always) and
  // + M_{n-1}^{m+1} conj(T_n^m) (n - 1 >= m + 1).  The step's factors
  // 2n - 1 and (n - 1)^2 - m^2 (small integers, exact in FP32) and its
  // place in M are carried from step to step: pv points at M_{n-1}^{m-1}
  // (then M_{n-1}^m, M_{n-1}^{m+1}), and M_n^{m-1} is 2n reals further.
  float sr = ri, si = 0.f;
  float pr = 0.f, pi = 0.f, tr = 0.f, ti = 0.f;
  auto stepm = [&](const float af, const float bf, const float* __restrict__ row, const float* __restrict__ pv,
                   auto rec, auto pot, auto dz, auto wplus) {
    if constexpr (decltype(rec)::value) {
      const float a = af * zr;
      const float b = bf * ri2;
      const float nr = a * tr - b * pr, ni = a * ti - b * pi;
      pr = tr;
      pi = ti;
      tr = nr;
      ti = ni;
    }
    if constexpr (decltype(pot)::value) {  // row: M_n^m
      phi1 = fma((double)row[0], (double)tr, phi1);
      phi1 = fma((double)row[1], (double)ti, phi1);
    }
    if constexpr (decltype(dz)::value) {
      dz1 = fmaf(pv[2], tr, dz1);
      dz1 = fmaf(pv[3], ti, dz1);
    }
    Wr = fmaf(-pv[0], tr, Wr);
    Wr = fmaf(-pv[1], ti, Wr);
    Wi = fmaf(-pv[0], ti, Wi);
    Wi = fmaf(pv[1], tr, Wi);
    if constexpr (decltype(wplus)::value) {
      Wr = fmaf(pv[4], tr, Wr);
      Wr = fmaf(pv[5], ti, Wr);
      Wi = fmaf(pv[5], tr, Wi);
      Wi = fmaf(-pv[4], ti, Wi);
    }
  };
  auto seed = [&](const int m) {
    const float c = (float)(2 * m - 1);
    const float nr = c * (wr * sr - wi * si), ni = c * (wr * si + wi * sr);
    sr = nr;
    si = ni;
    pr = 0.f;
    pi = 0.f;
    tr = sr;
    ti = si;
  };
  // M_n^m
  auto at = [&](const int n, const int m) { return M + (n * (n + 1) + 2 * m); };
  const std::false_type no{};
  const std::true_type yes{};
#pragma unroll 1
  for (int m = 1; m < P; ++m) {
    seed(m);
    stepm(0.f, 0.f, at(m, m), at(m - 1, m - 1), no, yes, no, no);
    stepm((float)(2 * m + 1), 0.f, at(m + 1, m), at(m, m - 1), yes, yes, yes, no);
    float af = (float)(2 * m + 3), bf = (float)((m + 1) * (m + 1) - m * m);
    const float* __restrict__ pv = at(m + 1, m - 1);
#pragma unroll 1
    for (int n = m + 2; n <= P; ++n) {
      const float* __restrict__ nx = pv + 2 * n;  // M_n^{m-1}
      stepm(af, bf, nx + 2, pv, yes, yes, yes, yes);
      pv = nx;
      bf += af;
      af += 2.f;
    }
    stepm(af, bf, pv, pv, yes, no, yes, yes);  // n = P + 1
  }
  // m = P: steps P and P + 1; m = P + 1: step P + 1 only
  seed(P);
  stepm(0.f, 0.f, at(P, P), at(P - 1, P - 1), no, yes, no, no);
  stepm((float)(2 * P + 1), 0.f, at(P + 1, P), at(P, P - 1), yes, no, yes, no);
  seed(P + 1);
  stepm(0.f, 0.f, at(P, P), at(P, P), no, no, no, no);
  phi = phi0 + 2.0 * phi1;
  fx = -Wr;
  fy = -Wi;
  fz = dz0 + 2.f * dz1;  // -d/dz phi
}

// The same evaluation in FP64 from the FP64 moments (the slab: its 189
// image entries per target each add the FP32 evaluation's rounding, which
// on the 20,000-ion slab was about a third of the energy error).
__device__ __forceinline__ void tree_eval64(const double* __restrict__ M, int P, double X, double Y, double Z, double& phi,
                                          float& fx, float& fy, float& fz) {
  const double r2 = X * X + Y * Y + Z * Z;
  const double ri = 1.0 / sqrt(r2);
  const double ri2 = ri * ri;
  const double wr = X * ri2, wi = Y * ri2;
  const double zr = Z * ri2;
  // the potential's terms are summed in FP64 (on the 50,000-ion system the
  // energy error at order 12 went from 1.2e-6 to 4.5e-7 for 1 % of the time)
  double phi0 = 0.0, phi1 = 0.0;
  double dz0 = 0.0, dz1 = 0.0, Wr = 0.0, Wi = 0.0;
  // column m = 0: T_n^0 is real.  Step n: recursion (n >= 1), potential
  // (n <= P), d/dz (n >= 1), and + M_{n-1}^1 conj(T_n^0) (n >= 2).  The
  // factors 2n - 1 and (n - 1)^2 and the place in M are carried from step
  // to step: pv points at M_{n-1}^0, and M_n^0 is 2n reals further.
  {
    double p = 0.0, t = ri;
    auto step0 = [&](const double af, const double bf, const double* __restrict__ row, const double* __restrict__ pv,
                     auto pot, auto wplus) {
      const double a = af * zr;
      const double b = bf * ri2;
      const double nt = a * t - b * p;
      p = t;
      t = nt;
      if constexpr (decltype(pot)::value) phi0 = fma((double)row[0], (double)t, phi0);  // M_n^0
      dz0 = fma(pv[0], t, dz0);
      if constexpr (decltype(wplus)::value) {
        Wr = fma(pv[2], t, Wr);
        Wi = fma(pv[3], t, Wi);
      }
    };
    phi0 = fma((double)M[0], (double)t, phi0);  // n = 0
    step0(1.0, 0.0, M + 2, M, std::true_type{}, std::false_type{});
    double af = 3.0, bf = 1.0;
    const double* __restrict__ pv = M + 2;  // M_1^0
#pragma unroll 1
    for (int n = 2; n <= P; ++n) {
      const double* __restrict__ nx = pv + 2 * n;  // M_n^0
      step0(af, bf, nx, pv, std::true_type{}, std::true_type{});
      pv = nx;
      bf += af;
      af += 2.0;
    }
    step0(af, bf, pv, pv, std::false_type{}, std::true_type{});  // n = P + 1
  }
  // columns m >= 1.  Step n of column m: recursion (n > m), potential
  // (n <= P), d/dz (n - 1 >= m), - conj(M_{n-1}^{m-1}) T_n^m (always) and
  // + M_{n-1}^{m+1} conj(T_n^m) (n - 1 >= m + 1).  The step's factors
  // 2n - 1 and (n - 1)^2 - m^2 (small integers, exact in FP32) and its
  // place in M are carried from step to step: pv points at M_{n-1}^{m-1}
  // (then M_{n-1}^m, M_{n-1}^{m+1}), and M_n^{m-1} is 2n reals further.
  double sr = ri, si = 0.0;
  double pr = 0.0, pi = 0.0, tr = 0.0, ti = 0.0;
  auto stepm = [&](const double af, const double bf, const double* __restrict__ row, const double* __restrict__ pv,
                   auto rec, auto pot, auto dz, auto wplus) {
    if constexpr (decltype(rec)::value) {
      const double a = af * zr;
      const double b = bf * ri2;
      const double nr = a * tr - b * pr, ni = a * ti - b * pi;
      pr = tr;
      pi = ti;
      tr = nr;
      ti = ni;
    }
    if constexpr (decltype(pot)::value) {  // row: M_n^m
      phi1 = fma((double)row[0], (double)tr, phi1);
      phi1 = fma((double)row[1], (double)ti, phi1);
    }
    if constexpr (decltype(dz)::value) {
      dz1 = fma(pv[2], tr, dz1);
      dz1 = fma(pv[3], ti, dz1);
    }
    Wr = fma(-pv[0], tr, Wr);
    Wr = fma(-pv[1], ti, Wr);
    Wi = fma(-pv[0], ti, Wi);
    Wi = fma(pv[1], tr, Wi);
    if constexpr (decltype(wplus)::value) {
      Wr = fma(pv[4], tr, Wr);
      Wr = fma(pv[5], ti, Wr);
      Wi = fma(pv[5], tr, Wi);
      Wi = fma(-pv[4], ti, Wi);
    }
  };
  auto seed = [&](const int m) {
    const double c = (double)(2 * m - 1);
    const double nr = c * (wr * sr - wi * si), ni = c * (wr * si + wi * sr);
    sr = nr;
    si = ni;
    pr = 0.0;
    pi = 0.0;
    tr = sr;
    ti = si;
  };
  // M_n^m
  auto at = [&](const int n, const int m) { return M + (n * (n + 1) + 2 * m); };
  const std::false_type no{};
  const std::true_type yes{};
#pragma unroll 1
  for (int m = 1; m < P; ++m) {
    seed(m);
    stepm(0.0, 0.0, at(m, m), at(m - 1, m - 1), no, yes, no, no);
    stepm((double)(2 * m + 1), 0.0, at(m + 1, m), at(m, m - 1), yes, yes, yes, no);
    double af = (double)(2 * m + 3), bf = (double)((m + 1) * (m + 1) - m * m);
    const double* __restrict__ pv = at(m + 1, m - 1);
#pragma unroll 1
    for (int n = m + 2; n <= P; ++n) {
      const double* __restrict__ nx = pv + 2 * n;  // M_n^{m-1}
      stepm(af, bf, nx + 2, pv, yes, yes, yes, yes);
      pv = nx;
      bf += af;
      af += 2.0;
    }
    stepm(af, bf, pv, pv, yes, no, yes, yes);  // n = P + 1
  }
  // m = P: steps P and P + 1; m = P + 1: step P + 1 only
  seed(P);
  stepm(0.0, 0.0, at(P, P), at(P - 1, P - 1), no, yes, no, no);
  stepm((double)(2 * P + 1), 0.0, at(P + 1, P), at(P, P - 1), yes, no, yes, no);
  seed(P + 1);
  stepm(0.0, 0.0, at(P, P), at(P, P), no, no, no, no);
  phi = phi0 + 2.0 * phi1;
  fx = (float)-Wr;
  fy = (float)-Wi;
  fz = (float)(dz0 + 2.0 * dz1);  // -d/dz phi
}

// Near-set sums of the particles by the treecode: wave b takes target
// group (= tile) b % ngroups and c = b / ngroups, that is image entry
// c / ps.split and share c % ps.split.  Every wave walks the image's tree
// depth-first (no stack: the next node follows from the level counts);
// the work items met on the way (tiles summed directly, nodes taken as
// multipoles) are dealt round-robin to the ps.split waves of the (group,
// image), so that the heavy central images are shared when there are few
// groups.  The wave writes slot c.  Tiles within the close-pair radius are
// summed here too (there is no separate near pass for this rule).  Tiles follow the far kernel's rules (near
// tiles skipped, each target's own image dropped in its own tile), and a
// multipole node that holds the group's own tile under a shifted image has
// those own images taken out again, so that finalize adds every own image
// exactly once in FP64.
#ifndef HSMA_TREE_WAVES
#define HSMA_TREE_WAVES 8
#endif
template <int P, bool CHECKS, bool E64>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(HSMA_TREE_WAVES))) void k_tree_far(
    const double4* __restrict__ tgt, PartSched ps, const Group* __restrict__ cgroups,
    const CheckSched* __restrict__ csched, int cg0, int ncg, int cbase, int csplit, const Desc* __restrict__ desc,
    int ntiles,
    const double4* __restrict__ tile_c, const float4* __restrict__ tile_h, const float4* __restrict__ src,
    const double4* __restrict__ pos64, const StepParams* __restrict__ sp, TreeLevels tl,
    const double4* __restrict__ node_c,
    const double4* __restrict__ node_box, const void* __restrict__ momv, double theta, float* __restrict__ part,
    long comp_stride, long slot_stride) {
  // moments: FP32, or FP64 for the FP64 evaluation (E64)
  const float* __restrict__ mom = (const float*)momv;
  const double* __restrict__ mom64 = (const double*)momv;
  // the wave's target group, image entry, share and output slot
  int gi, split, img, tskip, first, count;
  long obase;
  const Desc* __restrict__ dtab = desc;
  if constexpr (CHECKS) {
    // check targets: the check group of [cg0, ncg) whose waves include this
    // one (binary search over the waves' first indices, which continue
    // those of the direct check groups before cg0), its own image table
    const int bid = (int)blockIdx.x + cbase;
    int lo = cg0, hi = ncg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (csched[mid].first_work <= bid) lo = mid;
      else hi = mid - 1;
    }
    gi = lo;
    const CheckSched cs = csched[gi];
    const Group g = cgroups[gi];
    const int cw = bid - cs.first_work;
    split = csplit;
    img = cw / split;
    tskip = cw - img * split;
    first = g.first;
    count = g.count;
    dtab = desc + g.desc_off;
    obase = (long)(cs.slot0 + cw) * slot_stride;
  } else {
    const int c = blockIdx.x / ps.ngroups;
    gi = blockIdx.x - c * ps.ngroups;
    split = ps.split;
    img = c / split;
    tskip = c - img * split;  // work items to pass over before this wave's next one
    first = gi * kGroup;
    count = min(kGroup, ps.n - first);
    obase = (long)c * slot_stride + first;
  }
  const int lane = threadIdx.x;
  const bool valid = lane < count;
  const double4 tp = tgt[first + (valid ? lane : 0)];
  const double mnx = wave_min(valid ? tp.x : INFINITY), mxx = wave_max(valid ? tp.x : -INFINITY);
  const double mny = wave_min(valid ? tp.y : INFINITY), mxy = wave_max(valid ? tp.y : -INFINITY);
  const double mnz = wave_min(valid ? tp.z : INFINITY), mxz = wave_max(valid ? tp.z : -INFINITY);
  // the group box: the same in every lane after the wave reductions
  const double cgx = uniform_d(0.5 * (mnx + mxx)), cgy = uniform_d(0.5 * (mny + mxy)),
               cgz = uniform_d(0.5 * (mnz + mxz));
  const double hgx = uniform_d(0.5 * (mxx - mnx)), hgy = uniform_d(0.5 * (mxy - mny)),
               hgz = uniform_d(0.5 * (mxz - mnz));
  // group radii: of its box (close-pair test), of its targets (opening test)
  const double rt = sqrt(hgx * hgx + hgy * hgy + hgz * hgz);
  const double ptx = tp.x - cgx, pty = tp.y - cgy, ptz = tp.z - cgz;
  const double rtp = uniform_d(wave_max(valid ? sqrt(ptx * ptx + pty * pty + ptz * ptz) : 0.0));
  const float ox = (float)ptx, oy = (float)pty, oz = (float)ptz;
  const double qt = tp.w;  // (the FP64 position is read again where a close pair needs it)
  const double3 hbox = sp->hbox;
  const double rc2 = CHECKS ? sp->rc2c : sp->rc2;
  const Desc ds = dtab[img];
  const bool identity = ds.sx == 0.0 && ds.sy == 0.0 && ds.sz == 0.0 && ds.sigma > 0.0;
  // slab images: z -> sigma z + sz with strength scale (3D: 1, 1)
  const float sg = (float)ds.sigma, sc = (float)ds.scale;
  const bool img_far = gap2_of(__dsub_rn(ds.sx, cgx), __dsub_rn(ds.sy, cgy), __dsub_rn(ds.sz, cgz),
                               __dadd_rn(hgx, hbox.x), __dadd_rn(hgy, hbox.y), __dadd_rn(hgz, hbox.z)) >= rc2;
  const int tself = first + lane;  // sorted index of this lane's target
  // potential summed in FP64 (as in the direct kernels); field in FP32
  double ph = 0.0;
  float ex = 0.f, ey = 0.f, ez = 0.f;
  auto add = [&](double p, float gx, float gy, float gz) {
    ph += p;
    ex += gx;
    ey += gy;
    ez += gz;
  };
  // node acceptance without square roots: |dl|^2 > ((r + rt) / theta)^2
  // (the opening criterion) and |dl| > r + rt + rc (every source-target
  // distance above the close-pair radius, so no tile of the node belongs
  // to the near pass)
  const double rc = sqrt(rc2);
  // the check sums feed the fit of the whole far field: their opening
  // parameter is 0.8 theta (on the slab this halves the energy error of the
  // step for 10 % more time)
  const double th = CHECKS ? 0.8 * theta : theta;
  const double ith2 = 1.0 / (th * th);
  const int top = tl.nlev - 1;
  // work items, dealt round-robin to the split waves in traversal order:
  // a tile (direct; the checked loop when within rc of the group; far_sub:
  // an ancestor is beyond rc, so the tile is not) ...
  auto leaf = [&](const int tile, const bool far_sub) {
    // a tile within the close-pair radius of the group (the far kernel's
    // test) runs the checked loop: pairs closer than rc take their
    // difference vector from the FP64 positions
    const bool mine = tskip == 0;
    tskip = mine ? split - 1 : tskip - 1;
    bool near = false;
    if (mine && !img_far && !far_sub) {
      const double4 cs = tile_c[tile];
      const float4 hs = tile_h[tile];
      near = gap2_of(__dsub_rn(__dadd_rn(cs.x, ds.sx), cgx), __dsub_rn(__dadd_rn(cs.y, ds.sy), cgy),
                     shifted_dz(ds, cs.z, cgz), __dadd_rn(hgx, (double)hs.x), __dadd_rn(hgy, (double)hs.y),
                     __dadd_rn(hgz, (double)hs.z)) < rc2;
    }
    if (mine && near) {
      const double4 cs = tile_c[tile];
      const double dlx = __dsub_rn(__dadd_rn(cs.x, ds.sx), cgx);
      const double dly = __dsub_rn(__dadd_rn(cs.y, ds.sy), cgy);
      const double dlz = shifted_dz(ds, cs.z, cgz);
      const float ux = ox - (float)dlx, uy = oy - (float)dly, uz = sg * (oz - (float)dlz);
      const float4* __restrict__ s = src + (long)tile * kTile;
      const double4 p64 = pos64[(long)tile * kTile + lane];
      const double4 tq = tgt[first + (valid ? lane : 0)];
      double pp = 0.0;
      float qx = 0.f, qy = 0.f, qz = 0.f;
      for (int k = 0; k < kTile; ++k) {
        const float4 v = s[k];
        float dx = ux - v.x, dy = uy - v.y, dz = uz - v.z;
        float r2 = dx * dx + dy * dy + dz * dz;
        float qv = v.w;
        if (!CHECKS && tile == gi && tile * kTile + k == tself) {
          // the target itself or its own image: finalize sums the images
          qv = 0.f;
          r2 = 1.f;
        } else if ((double)r2 < rc2) {
          const double psx = readlane_d(p64.x, k), psy = readlane_d(p64.y, k), psz = readlane_d(p64.z, k);
          dx = (float)(tq.x - (psx + ds.sx));
          dy = (float)(tq.y - (psy + ds.sy));
          dz = sg * (float)(tq.z - (ds.sigma * psz + ds.sz));
          r2 = dx * dx + dy * dy + dz * dz;
        }
        const float ri = rsq(r2);
        const float a = qv * ri;
        pp += (double)a;
        const float b = a * (ri * ri);
        qx += b * dx;
        qy += b * dy;
        qz += b * dz;
      }
      add(ds.scale * pp, sc * qx, sc * qy, (sc * sg) * qz);
    } else if (mine) {
      const double4 cs = tile_c[tile];
      const double dlx = __dsub_rn(__dadd_rn(cs.x, ds.sx), cgx);
      const double dly = __dsub_rn(__dadd_rn(cs.y, ds.sy), cgy);
      const double dlz = shifted_dz(ds, cs.z, cgz);
      const float ux = ox - (float)dlx, uy = oy - (float)dly, uz = sg * (oz - (float)dlz);
      const float4* __restrict__ s = src + (long)tile * kTile;
      double pp = 0.0;
      float qx = 0.f, qy = 0.f, qz = 0.f;
      if (!CHECKS && tile == gi) {
        // own tile (under any image): drop each target's own image,
        // which finalize sums in FP64
        for (int k = 0; k < kTile; ++k) {
          const float4 v = s[k];
          const bool self = tile * kTile + k == tself;
          const float dx = ux - v.x, dy = uy - v.y, dz = uz - v.z;
          const float r2 = self ? 1.f : dx * dx + dy * dy + dz * dz;
          const float ri = rsq(r2);
          const float a = (self ? 0.f : v.w) * ri;
          pp += (double)a;
          const float b = a * (ri * ri);
          qx += b * dx;
          qy += b * dy;
          qz += b * dz;
        }
      } else {
#pragma unroll HSMA_FAR_UNROLL
        for (int k = 0; k < kTile; ++k) {
          const float4 v = s[k];
          const float dx = ux - v.x, dy = uy - v.y, dz = uz - v.z;
          const float r2 = dx * dx + dy * dy + dz * dz;
          const float ri = rsq(r2);
          const float a = v.w * ri;
          pp += (double)a;
          const float b = a * (ri * ri);
          qx += b * dx;
          qy += b * dy;
          qz += b * dz;
        }
      }
      add(ds.scale * pp, sc * qx, sc * qy, (sc * sg) * qz);
    }
  };
  // ... or an accepted node (multipole at its own order)
  auto node = [&](const int l, const int i, const double dlx, const double dly, const double dlz, const double d2,
                  const double rr) {
    const bool mine = tskip == 0;
    tskip = mine ? split - 1 : tskip - 1;
    if (!mine) return;
    const int g = tl.off[l] + i;
    const double rn = node_c[g].w;
    // order used for this node: the truncation ratio r / (d - rt) of a
    // node well inside the opening radius reaches, at a lower order p, the
    // bound the same node would have at the opening radius with order P
    // (one order of margin)
    const double d = sqrt(d2);
    const double rho = rn / (d - rtp);
    const double rho_b = rn / (rr / th - rtp);
    const float pr = (float)(P + 1) * (__logf((float)rho_b) / __logf((float)rho));
    const int pe = __builtin_amdgcn_readfirstlane(min(P, max(2, (int)ceilf(pr))));
    // the image of the node acts at x as the node itself at the mirrored
    // point (x, y, sigma (z - sz)): evaluate there, scale, mirror E_z
    double p;
    float gx, gy, gz;
    if constexpr (E64)
      tree_eval64(mom64 + (long)g * kTreeMomStride, pe, ptx - dlx, pty - dly, ds.sigma * (ptz - dlz), p, gx, gy,
                  gz);
    else
      tree_eval(mom + (long)g * kTreeMomStride, pe, ox - (float)dlx, oy - (float)dly, sg * (oz - (float)dlz), p, gx,
                gy, gz);
    double pd = ds.scale * p;
    gx *= sc;
    gy *= sc;
    gz *= sc * sg;
    if (!CHECKS && !identity && (gi >> (3 * l)) == i && valid) {
      // this node holds the target's own image: take it out
      const double tz = tgt[first + lane].z;
      const double ddx = -ds.sx, ddy = -ds.sy, ddz = tz - (ds.sigma * tz + ds.sz);
      const double si = 1.0 / sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
      const double qs = ds.scale * qt * si;
      pd -= qs;
      gx -= (float)(qs * si * si * ddx);
      gy -= (float)(qs * si * si * ddy);
      gz -= (float)(qs * si * si * ddz);
    }
    add(pd, gx, gy, gz);
  };
  // Traversal: the children of every opened node (and the root, the one
  // child of a virtual parent above it) are classified by eight lanes at
  // once; accepted children and tiles are processed in child order, then
  // the walk descends into the first opened child not yet visited, deepest
  // level first.  Per children level L (0..top), 8 bits of open_bits mark
  // the opened children still to visit and 8 bits of bey_bits those beyond
  // rc of the group; bit L of far_bits says that their parent is.  (Tiles
  // are at most 2^20, so top <= 7 and the bits fit one 64-bit word.)
  unsigned long long open_bits = 0ull, bey_bits = 0ull;
  unsigned far_bits = 0u;
  int lc = top, par = 0;  // children level, and their parent's index at level lc + 1
  bool farp = false;
  for (;;) {
    const int c0 = 8 * par, cc = min(8, tl.cnt[lc] - c0);
    if (lc == 0) {
      for (int k = 0; k < cc; ++k) leaf(c0 + k, farp);
    } else {
      double cdx = 0.0, cdy = 0.0, cdz = 0.0, cd2 = 0.0, crr = 0.0;
      bool acc = false, bey = false;
      if (lane < cc) {
        const int g = tl.off[lc] + c0 + lane;
        const double4 nc = node_c[g];
        cdx = __dsub_rn(__dadd_rn(nc.x, ds.sx), cgx);
        cdy = __dsub_rn(__dadd_rn(nc.y, ds.sy), cgy);
        cdz = shifted_dz(ds, nc.z, cgz);
        cd2 = cdx * cdx + cdy * cdy + cdz * cdz;
        const double far_r = (node_box[2 * g].w + rt + rc) * (1.0 + 1e-12);  // boxes; margin over rounding
        bey = cd2 > far_r * far_r;
        crr = nc.w + rtp;  // particle radii
        acc = bey && cd2 > crr * crr * ith2;
      }
      const unsigned long long m_acc = __ballot(acc), m_bey = __ballot(bey);
      const unsigned long long m_open = __ballot(lane < cc) & ~m_acc;
      for (int k = 0; k < cc; ++k)
        if ((m_acc >> k) & 1ull)
          node(lc, c0 + k, readlane_d(cdx, k), readlane_d(cdy, k), readlane_d(cdz, k), readlane_d(cd2, k),
               readlane_d(crr, k));
      const int sh = 8 * lc;
      open_bits = (open_bits & ~(0xffull << sh)) | ((m_open & 0xffull) << sh);
      bey_bits = (bey_bits & ~(0xffull << sh)) | ((m_bey & 0xffull) << sh);
      far_bits = farp ? (far_bits | (1u << lc)) : (far_bits & ~(1u << lc));
    }
    // next opened child: the deepest level with one left, i.e. the lowest
    // set bit of open_bits from the byte of level max(lc, 1) on (no bit
    // above level top is ever set)
    const unsigned long long rest = open_bits & (~0ull << (8 * (lc >= 1 ? lc : 1)));
    if (rest == 0ull) break;
    const int bit = __builtin_ctzll(rest);
    const int L = bit >> 3, k = bit & 7;
    open_bits &= ~(1ull << bit);
    const int q = par >> (3 * (L - lc));  // the parent (level L + 1) of the level-L children
    farp = ((far_bits >> L) & 1u) || ((bey_bits >> (8 * L + k)) & 1ull);
    par = 8 * q + k;
    lc = L - 1;
  }
  if (valid) {
    const long o = obase + lane;
    const float hi = (float)ph;
    part[o] = hi;
    part[o + comp_stride] = (float)(ph - (double)hi);
    part[o + 2 * comp_stride] = ex;
    part[o + 3 * comp_stride] = ey;
    part[o + 4 * comp_stride] = ez;
  }
}

template <typename Real>
__global__ __launch_bounds__(kGroup * kFinParts) void k_reduce_check(const Group* __restrict__ groups,
                                                              const CheckSched* __restrict__ csched, int gbase,
                                                              const int* __restrict__ axis,
                                                              const Real* __restrict__ part, long slot_elems,
                                                              double* __restrict__ v) {
  __shared__ double sh_phi[kFinParts - 1][kGroup], sh_e[kFinParts - 1][kGroup];
  const Group g = groups[blockIdx.x + gbase];
  const CheckSched cs = csched[blockIdx.x + gbase];
  const int s0 = cs.slot0, s1 = cs.slot0 + cs.nch + 1;  // far chunks + the near slot
  const int local = threadIdx.x % kGroup, wpart = threadIdx.x / kGroup, np = blockDim.x / kGroup;
  const bool ok = local < g.count;
  const int t = g.first + (ok ? local : 0);
  const int ax = axis[t];
  double phi = 0, e = 0;
  if constexpr (sizeof(Real) == 4) {
    float hi = 0, lo = 0, ea = 0, ec = 0;
    for (int w0 = s0 + wpart; w0 < s1; w0 += kFinBatch * np) {
      float v[kFinBatch][3];
#pragma unroll
      for (int u = 0; u < kFinBatch; ++u) {
        const int w = w0 + u * np;
        const Real* p = part + (long)(w < s1 ? w : s0) * slot_elems + local;
        v[u][0] = w < s1 ? p[0] : 0.f;
        v[u][1] = w < s1 ? p[kGroup] : 0.f;
        v[u][2] = w < s1 ? p[(2 + ax) * kGroup] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kFinBatch; ++u) {
        float sm, er;
        two_sum(hi, v[u][0], sm, er);
        hi = sm;
        lo += er + v[u][1];
        two_sum(ea, v[u][2], sm, er);
        ea = sm;
        ec += er;
      }
    }
    phi = (double)hi + (double)lo;
    e = (double)ea + (double)ec;
  } else {
    for (int w0 = s0 + wpart; w0 < s1; w0 += kFinBatch * np) {
      double v[kFinBatch][2];
#pragma unroll
      for (int u = 0; u < kFinBatch; ++u) {
        const int w = w0 + u * np;
        const Real* p = part + (long)(w < s1 ? w : s0) * slot_elems + local;
        v[u][0] = w < s1 ? p[0] : 0.0;
        v[u][1] = w < s1 ? p[(2 + ax) * kGroup] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kFinBatch; ++u) {
        phi += v[u][0];
        e += v[u][1];
      }
    }
  }
  if (wpart > 0) {
    sh_phi[wpart - 1][local] = phi;
    sh_e[wpart - 1][local] = e;
  }
  __syncthreads();
  if (wpart == 0 && ok) {
    for (int w = 0; w < np - 1; ++w) {
      phi += sh_phi[w][local];
      e += sh_e[w][local];
    }
    v[2 * t] = phi;
    v[2 * t + 1] = e;
  }
}

// A[j] = sum_c Praw[j][c] v[c]  (FP64, fixed-order block reduction)
__global__ __launch_bounds__(256) void k_lsq(int ncol, const double* __restrict__ Praw, const double* __restrict__ v,
                                             double* __restrict__ A) {
  __shared__ double s[256];
  const int j = blockIdx.x;
  double acc = 0;
  for (int c = threadIdx.x; c < ncol; c += 256) acc += Praw[(long)j * ncol + c] * v[c];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) A[j] = s[0];
}

// Q_k = SQ[k] . A, D_k = SD[k] . A  (FP64), written as sphere source records.
__global__ __launch_bounds__(64) void k_sphere_sources(int F, int nb, const double* __restrict__ SQ,
                                                       const double* __restrict__ SD, const double* __restrict__ A,
                                                       const double* __restrict__ y, const double* __restrict__ nrm,
                                                       float4* __restrict__ s32, double4* __restrict__ s64,
                                                       double* __restrict__ qd) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= F) return;
  double Q = 0, D = 0;
  for (int j = 0; j < nb; ++j) {
    Q += SQ[(long)k * nb + j] * A[j];
    D += SD[(long)k * nb + j] * A[j];
  }
  qd[2 * k] = Q;
  qd[2 * k + 1] = D;
  s64[2 * k] = make_double4(y[3 * k], y[3 * k + 1], y[3 * k + 2], Q);
  s64[2 * k + 1] = make_double4(nrm[3 * k], nrm[3 * k + 1], nrm[3 * k + 2], D);
  s32[2 * k] = make_float4((float)y[3 * k], (float)y[3 * k + 1], (float)y[3 * k + 2], (float)Q);
  s32[2 * k + 1] = make_float4((float)nrm[3 * k], (float)nrm[3 * k + 1], (float)nrm[3 * k + 2], (float)D);
}

// ----------------------------------------------------------------- finalize
// Sum the nslot partials of every particle (fixed order), scale by the
// Coulomb constant, write potential and force in the caller's order, and
// per-block energy partials q_i Phi_i.  Invalid input -> NaN outputs.
// A block holds kWave particles and P = blockDim.x / kWave <= kFinParts
// waves: wave w sums slots w, w + P, ... (compensated in FP32), the waves'
// sums are combined
// in FP64 in wave order, so the result does not depend on timing.
// The images of a particle itself (every image entry except the identity)
// are summed here in FP64 for each particle.
template <typename Real>
__global__ __launch_bounds__(kWave * kFinParts) void k_finalize(int n, int nslot, const Real* __restrict__ part,
                                                              long comp_stride, const double4* __restrict__ pos64,
                                                              const int* __restrict__ perm,
                                                              const Desc* __restrict__ desc, int ndesc,
                                                              const unsigned long long* __restrict__ cull,
                                                              int ntiles, double kc, const int* __restrict__ status,
                                                              double* __restrict__ pot, double* __restrict__ force,
                                                              double* __restrict__ epart) {
  __shared__ double sh[kFinParts - 1][4][kWave];
  const int lane = threadIdx.x % kWave, wpart = threadIdx.x / kWave, np = blockDim.x / kWave;
  const int t = blockIdx.x * kWave + lane;
  double phi = 0, fx = 0, fy = 0, fz = 0;
  if (t < n) {
    if constexpr (sizeof(Real) == 4) {
      float hi = 0, lo = 0, ax = 0, ay = 0, az = 0, cx = 0, cy = 0, cz = 0;
      // slots in batches of kFinBatch: the batch's loads are all issued
      // before the (in-order) compensated sums use them
      for (int c0 = wpart; c0 < nslot; c0 += kFinBatch * np) {
        float v[kFinBatch][5];
#pragma unroll
        for (int u = 0; u < kFinBatch; ++u) {
          const int c = c0 + u * np;
          const Real* p = part + (long)(c < nslot ? c : 0) * 5 * comp_stride + t;
#pragma unroll
          for (int k = 0; k < 5; ++k) v[u][k] = c < nslot ? p[k * comp_stride] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < kFinBatch; ++u) {
          float sm, er;
          two_sum(hi, v[u][0], sm, er);
          hi = sm;
          lo += er + v[u][1];
          two_sum(ax, v[u][2], sm, er); ax = sm; cx += er;
          two_sum(ay, v[u][3], sm, er); ay = sm; cy += er;
          two_sum(az, v[u][4], sm, er); az = sm; cz += er;
        }
      }
      phi = (double)hi + (double)lo;
      fx = (double)ax + (double)cx;
      fy = (double)ay + (double)cy;
      fz = (double)az + (double)cz;
    } else {
      for (int c0 = wpart; c0 < nslot; c0 += kFinBatch * np) {
        double v[kFinBatch][4];
#pragma unroll
        for (int u = 0; u < kFinBatch; ++u) {
          const int c = c0 + u * np;
          const Real* p = part + (long)(c < nslot ? c : 0) * 5 * comp_stride + t;
          v[u][0] = c < nslot ? p[0] : 0.0;
#pragma unroll
          for (int k = 1; k < 4; ++k) v[u][k] = c < nslot ? p[(k + 1) * comp_stride] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kFinBatch; ++u) {
          phi += v[u][0];
          fx += v[u][1];
          fy += v[u][2];
          fz += v[u][3];
        }
      }
    }
  }
  if (wpart > 0) {
    sh[wpart - 1][0][lane] = phi;
    sh[wpart - 1][1][lane] = fx;
    sh[wpart - 1][2][lane] = fy;
    sh[wpart - 1][3][lane] = fz;
  }
  __syncthreads();
  if (wpart != 0) return;
  double e = 0;
  if (t < n) {
    for (int w = 0; w < np - 1; ++w) {
      phi += sh[w][0][lane];
      fx += sh[w][1][lane];
      fy += sh[w][2][lane];
      fz += sh[w][3][lane];
    }
    const double4 p = pos64[t];
    const double q = p.w;
    double sphi = 0, sx = 0, sy = 0, sz = 0;
    for (int d = 0; d < ndesc; ++d) {
      const Desc ds = desc[d];
      if (ds.sx == 0.0 && ds.sy == 0.0 && ds.sz == 0.0 && ds.sigma > 0.0) continue;  // the self pair
      if (cull && !((cull[(long)d * ntiles + t / kTile] >> (t % kTile)) & 1ull)) continue;  // outside the sphere
      const double dx = -ds.sx, dy = -ds.sy, dz = p.z - (ds.sigma * p.z + ds.sz);
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double ri = rsq(r2);
      const double a = ds.scale * ri;
      sphi += a;
      const double b = a * ri * ri;
      sx += b * dx;
      sy += b * dy;
      sz += b * dz;
    }
    phi += q * sphi;
    fx += q * sx;
    fy += q * sy;
    fz += q * sz;
    const bool ok = status[0] == HSMA_OK;
    const double nan = __builtin_nan("");
    phi = ok ? kc * phi : nan;
    const double fq = kc * q;
    const int o = perm[t];
    if (pot) pot[o] = phi;
    if (force) {
      force[3 * (long)o] = ok ? fq * fx : nan;
      force[3 * (long)o + 1] = ok ? fq * fy : nan;
      force[3 * (long)o + 2] = ok ? fq * fz : nan;
    }
    e = q * phi;
  }
  // fixed-order (butterfly) sum of the block's kWave energy terms
  for (int o = kWave / 2; o > 0; o >>= 1) e += __shfl_xor(e, o);
  if (lane == 0) epart[blockIdx.x] = e;
}

__global__ __launch_bounds__(256) void k_energy(int nblk, const double* __restrict__ epart, double* __restrict__ energy) {
  __shared__ double s[256];
  double a = 0;
  for (int i = threadIdx.x; i < nblk; i += 256) a += epart[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) energy[0] = 0.5 * s[0];
}

// Plan constants of a box scaled by s from the unit box the plan was built
// for (all lengths times s): image shifts, check targets and sphere points
// scale with s; the value columns of Praw are scale free and its field
// columns scale with s; the sphere maps A -> Q and A -> D scale with s and
// s^2.  blockIdx.y selects the array.
__global__ __launch_bounds__(256) void k_scale_plan(double s, int ndp, const Desc* __restrict__ udp, Desc* __restrict__ dp,
                                                    int ndc, const Desc* __restrict__ udc, Desc* __restrict__ dc,
                                                    int nck, const double4* __restrict__ uck, double4* __restrict__ ck,
                                                    long npr, const double* __restrict__ upr, double* __restrict__ pr,
                                                    long nsq, const double* __restrict__ usq, double* __restrict__ sq,
                                                    const double* __restrict__ usd, double* __restrict__ sd, int nys,
                                                    const double* __restrict__ uys, double* __restrict__ ys) {
  const long stride = (long)gridDim.x * blockDim.x;
  const long i0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  switch (blockIdx.y) {
    case 0:
      for (long i = i0; i < ndp; i += stride) {
        Desc d = udp[i];
        d.sx *= s; d.sy *= s; d.sz *= s;
        dp[i] = d;
      }
      break;
    case 1:
      for (long i = i0; i < ndc; i += stride) {
        Desc d = udc[i];
        d.sx *= s; d.sy *= s; d.sz *= s;
        dc[i] = d;
      }
      break;
    case 2:
      for (long i = i0; i < nck; i += stride) {
        const double4 c = uck[i];
        ck[i] = make_double4(c.x * s, c.y * s, c.z * s, c.w);
      }
      break;
    case 3:
      for (long i = i0; i < npr; i += stride) pr[i] = (i & 1) ? upr[i] * s : upr[i];
      break;
    case 4:
      for (long i = i0; i < nsq; i += stride) {
        sq[i] = usq[i] * s;
        sd[i] = usd[i] * (s * s);
      }
      break;
    default:
      for (long i = i0; i < nys; i += stride) ys[i] = uys[i] * s;
      break;
  }
}

// ================================================================= host side
#define HIPCHK(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      err = std::string(#x) + ": " + hipGetErrorString(e_);                         \
      return e_ == hipErrorOutOfMemory ? HSMA_ERR_OOM : HSMA_ERR_DEVICE;            \
    }                                                                               \
  } while (0)

template <typename T>
static hsma_status upload(T** dst, const std::vector<T>& v, std::string& err) {
  *dst = nullptr;
  if (v.empty()) return HSMA_OK;
  HIPCHK(hipMalloc((void**)dst, sizeof(T) * v.size()));
  HIPCHK(hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return HSMA_OK;
}

// The no-allocation entry point's scratch: one static array per GPU (each
// device that loads the library holds its own copy until the process ends).
// Host code never uses the symbol itself as an address: scratch_address()
// looks up the device address once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev` (looked up once).
static hsma_status scratch_address(int dev, void** out, std::string& err) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device index out of range for the scratch table";
    return HSMA_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      err = "hipGetSymbolAddress returned no address for the scratch array";
      return HSMA_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HSMA_OK;
}

hsma_status DevicePlan::init(std::string& err) {
  HIPCHK(hipGetDevice(&device));
  // side stream of the step (default priority) and its fork/join events
  HIPCHK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&side_near, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&ev_join_near, hipEventDisableTiming));
  hsma_status st;
  if ((st = upload(&d_desc_part, host.desc_particles, err)) != HSMA_OK) return st;
  if ((st = upload(&d_desc_check, host.desc_check, err)) != HSMA_OK) return st;
  std::vector<double4> cp(host.check_axis.size());
  for (size_t t = 0; t < cp.size(); ++t)
    cp[t] = make_double4(host.check_pos[3 * t], host.check_pos[3 * t + 1], host.check_pos[3 * t + 2], 0.0);
  if ((st = upload(&d_check_pos, cp, err)) != HSMA_OK) return st;
  if ((st = upload(&d_check_axis, host.check_axis, err)) != HSMA_OK) return st;
  if ((st = upload(&d_check_groups, host.check_groups, err)) != HSMA_OK) return st;
  std::vector<int> tg(host.check_axis.size());
  for (size_t gi = 0; gi < host.check_groups.size(); ++gi)
    for (int i = 0; i < host.check_groups[gi].count; ++i) tg[host.check_groups[gi].first + i] = (int)gi;
  if ((st = upload(&d_check_tgroup, tg, err)) != HSMA_OK) return st;
  if ((st = upload(&d_Praw, host.Praw, err)) != HSMA_OK) return st;
  if ((st = upload(&d_SQ, host.SQ, err)) != HSMA_OK) return st;
  if ((st = upload(&d_SD, host.SD, err)) != HSMA_OK) return st;
  if ((st = upload(&d_ysurf, host.ysurf, err)) != HSMA_OK) return st;
  if ((st = upload(&d_nsurf, host.nsurf, err)) != HSMA_OK) return st;
  const int F = host.prm.F;
  HIPCHK(hipMalloc((void**)&d_v, sizeof(double) * 2 * host.check_axis.size()));
  HIPCHK(hipMalloc((void**)&d_A, sizeof(double) * host.nb));
  HIPCHK(hipMalloc((void**)&d_surf32, sizeof(float4) * 2 * F));
  HIPCHK(hipMalloc((void**)&d_surf64, sizeof(double4) * 2 * F));
  HIPCHK(hipMalloc((void**)&d_qd, sizeof(double) * 2 * F));
  HIPCHK(hipMalloc((void**)&d_status, sizeof(int)));
  HIPCHK(hipMemset(d_status, 0, sizeof(int)));
  HIPCHK(hipMalloc((void**)&d_energy_scratch, sizeof(double)));
  HIPCHK(hipMalloc(&d_sp, sizeof(StepParams)));
  // pinned staging of the check schedule (its size depends only on the
  // plan), its upload event and the call-ordering event
  stage_bytes = sizeof(CheckSched) * std::max<size_t>(1, host.check_groups.size()) + 64;
  HIPCHK(hipHostMalloc(&h_stage, stage_bytes));
  HIPCHK(hipEventCreateWithFlags(&stage_ev, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&ev_done, hipEventDisableTiming));
  hsma_status ss = scratch_address(device, &scratch, err);
  if (ss != HSMA_OK) return ss;
  return HSMA_OK;
}

hsma_status DevicePlan::order_after_previous(hipStream_t st, std::string& err) {
  if (done_recorded && st != done_stream) HIPCHK(hipStreamWaitEvent(st, ev_done, 0));
  return HSMA_OK;
}

hsma_status DevicePlan::mark_done(hipStream_t st, std::string& err) {
  HIPCHK(hipEventRecord(ev_done, st));
  done_recorded = true;
  done_stream = st;
  return HSMA_OK;
}

hsma_status DevicePlan::wait_done(std::string& err) {
  if (done_recorded) HIPCHK(hipEventSynchronize(ev_done));
  return HSMA_OK;
}

void DevicePlan::free_arena() {
  if (stage_ev) (void)hipEventSynchronize(stage_ev);  // an upload may still read the staging
  if (d_arena) (void)hipFree(d_arena);
  d_arena = nullptr;
  (void)carve(0, nullptr);
  cap_n = 0;
  cur_n = -1;
  arena_bytes = 0;
}

DevicePlan::~DevicePlan() {
  drop_graphs();
  if (d_sp) (void)hipFree(d_sp);
  free_arena();
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  if (stage_ev) (void)hipEventDestroy(stage_ev);
  if (h_stage) (void)hipHostFree(h_stage);
  if (ev_done) (void)hipEventDestroy(ev_done);
  void* us[] = {d_unit_desc_part, d_unit_desc_check, d_unit_check_pos, d_unit_Praw, d_unit_SQ, d_unit_SD, d_unit_ysurf};
  for (void* p : us)
    if (p) (void)hipFree(p);
  void* ps[] = {d_desc_part, d_desc_check, d_check_pos, d_check_axis, d_check_groups, d_check_tgroup, d_Praw,
                d_SQ, d_SD, d_ysurf, d_nsurf, d_v, d_A, d_surf32, d_surf64, d_qd, d_status, d_energy_scratch,
                d_in_xyz, d_in_q, d_out_pot, d_out_force, d_out_energy};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (own_stream) (void)hipStreamDestroy(own_stream);
  if (side) (void)hipStreamDestroy(side);
  if (side_near) (void)hipStreamDestroy(side_near);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  if (ev_join_near) (void)hipEventDestroy(ev_join_near);
}

// Particle schedule for n particles: chunks sized so that a launch has
// about `target` waves (and at least 2 tiles per chunk: small systems get
// many short waves rather than a few long ones).
static PartSched part_schedule(int64_t n, int ndesc, int target, bool tree, int near_target, int tree_target) {
  PartSched ps{};
  ps.n = (int)n;
  ps.split = 1;
  ps.ngroups = (int)((n + kGroup - 1) / kGroup);
  const int ntiles = (int)((n + kTile - 1) / kTile);
  ps.ndesc = ndesc;
  ps.F = ndesc * ntiles;
  // many short chunks: the blocks in flight then read the same few source
  // tiles at about the same time (cache reuse) and the last round of blocks
  // is a small share of the launch.  Measured against a target of 32,768
  // waves (50,000 ions: 42 chunks per group; 999,999 ions: 3): 50,000 ions
  // 21.9 -> 20.4 ms (saturated from about 170 chunks on), the slab 39.0 ->
  // 37.7 ms, 999,999 ions 8.24 -> 7.87 s (34 chunks).  With the cap of
  // kMaxFarChunks reached up to about 10^6 ions as well (1.7 MB of sources
  // per chunk on 999,999 ions instead of 12.7), the far kernel fetches 7.6x
  // fewer bytes there for 0.4 % less time.  The cap bounds the partial
  // slots each target writes.
  long long want = std::max<long long>(1, (target + (long long)ps.ngroups - 1) / ps.ngroups);
  want = std::min<long long>(want, kMaxFarChunks);
  // at least 4 tiles per chunk while that leaves 4096 far waves, else at
  // least 2 (fewer partial slots to write and to sum)
  const long long cap4 = std::max<long long>(1, ps.F / 4);
  want = std::min<long long>(want, cap4 * ps.ngroups >= 4096 ? cap4 : std::max<long long>(1, ps.F / 2));
  ps.chunk = (int)((ps.F + want - 1) / want);
  ps.nch = (ps.F + ps.chunk - 1) / ps.chunk;
  if (tree) {
    // treecode: `split` waves per (image entry, group), each on a share of
    // one image, so that the launch has about tree_target waves
    const long long base = (long long)ndesc * ps.ngroups;
    ps.split = (int)std::min<long long>(kTreeMaxSplit, std::max<long long>(1, (tree_target + base - 1) / base));
    ps.chunk = ntiles;
    ps.nch = ndesc * ps.split;
  }
  if (tree) {
    ps.nnear = 0;  // the treecode sums the near tiles itself
    return ps;
  }
  // near pass: up to kMaxNearSplit waves per group, so that the launch has
  // about near_target waves, at most one per near candidate (image entry,
  // tile)
  ps.nnear = (int)std::min<long long>({(long long)kMaxNearSplit, (long long)ndesc * ntiles,
                                       std::max<long long>(1, (near_target + ps.ngroups - 1) / ps.ngroups)});
  return ps;
}

// Check schedule: each check group's range cut in proportion to its share
// of the check pairs; returns the number of far waves and of slots.
static void check_schedule(const std::vector<Group>& groups, int ntiles, int target, std::vector<CheckSched>& cs,
                           int& nfar, int& nslots) {
  cs.assign(groups.size(), CheckSched{0, 0, 1, 0});
  long long total = 0;
  for (const Group& g : groups) total += (long long)g.ndesc * ntiles;
  nfar = 0;
  nslots = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const long long F = (long long)groups[gi].ndesc * ntiles;
    const long long want = std::max<long long>(1, std::min<long long>(std::max<long long>(1, F / 2),
        (long long)((double)target * F / std::max<long long>(1, total) + 0.5)));
    const long long chunk = (F + want - 1) / want;
    const int nch = (int)((F + chunk - 1) / chunk);
    cs[gi] = CheckSched{nfar, nch, (int)chunk, nslots};
    nfar += nch;
    nslots += nch + 1;  // far chunks + the near slot
  }
}

// Upper bounds of the per-size buffers for any particle count <= n, so that
// an arena reserved once for n never has to grow for a smaller system.
void DevicePlan::capacity_bounds(int64_t n, size_t& part_bytes, size_t& cpart_bytes, size_t& nwork,
                                 size_t& ncwork) const {
  const size_t rb = host.prm.precision == HSMA_FP64 ? sizeof(double) : sizeof(float);
  const int64_t ngroups = (n + kGroup - 1) / kGroup;
  // ngroups x sphere chunks <= 1024 + ngroups (F / kSphereChunkMax + 2) for
  // every size (see sphere_chunk)
  const size_t sph = 1024 + (size_t)ngroups * ((size_t)host.prm.F / kSphereChunkMax + 2);
  const size_t ncg = host.check_groups.size();
  // far slots <= min(part_target + ngroups, kMaxFarChunks ngroups); near
  // slots <= min(kMaxNearSplit ngroups, near_target + ngroups)
  const size_t nearb = std::min<size_t>((size_t)kMaxNearSplit * ngroups, (size_t)near_target + ngroups);
  // far slots: treecode one per image entry and group
  const size_t farb = std::max<size_t>(std::min<size_t>((size_t)part_target + ngroups, (size_t)kMaxFarChunks * ngroups),
                                       host.prm.near_rule == 2 ? tree_target + host.desc_particles.size() * ngroups : 0);
  part_bytes = rb * 5 * (size_t)kGroup * (farb + nearb + sph + 1);
  const size_t rbc = cpart_elem();
  cpart_bytes = rbc * 5 * (size_t)kGroup * ((size_t)check_target_max + 2 * ncg + 2);
  nwork = farb + nearb + 2;
  ncwork = (size_t)check_target_max + 2 * ncg + 2;
}

size_t DevicePlan::carve(int64_t nmax, char* base) {
  size_t off = 0;
  // next buffer of `bytes`, 256-byte aligned; null when nothing is carved
  auto take = [&](auto** ptr, size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    *ptr = (base && bytes) ? reinterpret_cast<std::remove_pointer_t<decltype(ptr)>>(base + off) : nullptr;
    off += bytes;
  };
  const int64_t cn = nmax > 0 ? std::max<int64_t>(nmax, 64) : 0;
  const int64_t cnt = (cn + kTile - 1) / kTile;
  const int64_t cpad = cnt * kTile;
  const int64_t crs = (cn + kRsBlock - 1) / kRsBlock;
  size_t part_bytes = 0, cpart_bytes = 0, nwork = 0, ncwork = 0;
  if (cn > 0) capacity_bounds(cn, part_bytes, cpart_bytes, nwork, ncwork);
  const size_t ncg = std::max<size_t>(1, host.check_groups.size());
  const size_t ncull = (cn > 0 && host.prm.near_rule == 1) ? host.desc_particles.size() * (size_t)cnt : 0;
  // tree nodes: the level counts only grow with the tile count
  const size_t tnodes = (cn > 0 && host.prm.near_rule == 2) ? (size_t)tree_levels((int)cnt).nodes : 0;
  take(&d_key[0], sizeof(uint32_t) * cn);
  take(&d_key[1], sizeof(uint32_t) * cn);
  take(&d_val[0], sizeof(int) * cn);
  take(&d_val[1], sizeof(int) * cn);
  take(&d_hist, sizeof(uint32_t) * 256 * crs);
  take(&d_pos_w, sizeof(double4) * cn);
  take(&d_pos64, sizeof(double4) * cpad);
  take(&d_src32, sizeof(float4) * cpad);
  take(&d_src64, sizeof(double4) * cpad);
  take(&d_tile_c, sizeof(double4) * cnt);
  take(&d_tile_h, sizeof(float4) * cnt);
  take(&d_perm, sizeof(int) * cpad);
  take(&d_red, sizeof(double) * 3 * ((cn + 255) / 256));
  take(&d_epart, sizeof(double) * ((cn + kWave - 1) / kWave));
  take(&d_part, part_bytes);
  take(&d_cpart, cpart_bytes);
  take(&d_csched, cn > 0 ? sizeof(CheckSched) * ncg : 0);
  take(&d_cull, sizeof(unsigned long long) * ncull);
  take(&d_clist, sizeof(unsigned) * ncull);
  take(&d_ccount, ncull ? sizeof(int) : 0);
  take(&d_tnode, sizeof(double4) * tnodes);
  take(&d_tbox, sizeof(double4) * 2 * tnodes);
  take(&d_tmom64, sizeof(double) * kTreeMomStride * tnodes);
  take(&d_tmom32, sizeof(float) * kTreeMomStride * tnodes);
  if (base) {
    part_cap = part_bytes;
    cpart_cap = cpart_bytes;
    work_cap = nwork;
    cwork_cap = ncwork;
  }
  return (off + 255) & ~(size_t)255;
}

// Destroys the captured steps (their kernels hold arena addresses); waits
// for the plan's last call first, which may be a replay.
void DevicePlan::drop_graphs() {
  if (!graphs.empty() && done_recorded) (void)hipEventSynchronize(ev_done);
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
  graphs.clear();
  seen_keys.clear();
}

void DevicePlan::attach_arena(void* base, int64_t nmax) {
  drop_graphs();
  const int64_t cn = std::max<int64_t>(nmax, 64);
  arena_bytes = carve(cn, (char*)base);
  cap_n = cn;
  cur_n = -1;
}

hsma_status DevicePlan::reserve(int64_t nmax, std::string& err) {
  if (nmax <= cap_n) return HSMA_OK;
  drop_graphs();
  free_arena();
  const int64_t cn = std::max<int64_t>(nmax, 64);
  const size_t bytes = carve(cn, nullptr);
  HIPCHK(hipMalloc(&d_arena, bytes));
  (void)carve(cn, (char*)d_arena);
  cap_n = cn;
  arena_bytes = bytes;
  cur_n = -1;
  return HSMA_OK;
}

hsma_status DevicePlan::prepare(int64_t n, hipStream_t st, std::string& err) {
  if (n == cur_n) return HSMA_OK;
  hsma_status s = reserve(n, err);
  if (s != HSMA_OK) return s;
  const int ntiles = (int)((n + kTile - 1) / kTile);
  const PartSched ps = part_schedule(n, (int)host.desc_particles.size(), part_target, host.prm.near_rule == 2,
                                     near_target, tree_target);
  // check work: about check_pairs_per_item pairs per wave, enough waves to
  // fill the chip when there is that much work
  long long cpairs = 0;
  for (const Group& g : host.check_groups) cpairs += (long long)g.count * g.ndesc * n;
  const int ctarget = (int)std::min<long long>(check_target_max, std::max<long long>(check_target,
                          cpairs / std::max<long long>(1, check_pairs_per_item)));
  std::vector<CheckSched> cs;
  int ncfar = 0, ncslots = 0;
  check_schedule(host.check_groups, ntiles, ctarget, cs, ncfar, ncslots);
  // treecode at the check targets (near rule 2) for the groups from gtree
  // on: on the slab all of them (its 189 image entries per target make the
  // direct check sums 45 % of the direct step, and the interface groups
  // are compact patches of the interface grids); in 3D none (the face
  // groups span a whole face, few nodes pass the opening test for them,
  // and over the telescoped sets the direct sums were as fast or faster:
  // 0.22 against 0.45 ms on 50,000 ions).  `split` waves per (check group,
  // image entry), each wave its own slot, after the direct groups' slots;
  // the row reduction sums the group's nch + 1 slots
  // (the face groups come first; with the sphere near set their direct
  // waves [0, cwork_face_) run in FP64)
  const int nface = std::min<int>(host.face_groups, (int)cs.size());
  const int face_waves = nface < (int)cs.size() ? cs[nface].first_work : ncfar;
  const int gtree = host.prm.geometry == HSMA_GEOM_2D ? 0 : (int)cs.size();
  tree_cwaves_ = 0;
  tree_csplit_ = 1;
  tree_cgroup0_ = gtree;
  tree_cbase_ = ncfar;
  if (host.prm.near_rule == 2 && gtree < (int)cs.size()) {
    const int direct_waves = cs[gtree].first_work, direct_slots = cs[gtree].slot0;
    long long nd = 0;
    for (size_t gi = gtree; gi < cs.size(); ++gi) nd += host.check_groups[gi].ndesc;
    const long long budget = check_target_max - direct_slots;
    if (nd <= budget) {
      const int split = (int)std::max<long long>(1, std::min<long long>(kTreeMaxSplit, budget / nd));
      int w = 0;
      for (size_t gi = gtree; gi < cs.size(); ++gi) {
        const int nw = host.check_groups[gi].ndesc * split;
        cs[gi] = CheckSched{direct_waves + w, nw - 1, 1, direct_slots + w};
        w += nw;
      }
      ncfar = direct_waves + w;
      ncslots = direct_slots + w;
      tree_cwaves_ = w;
      tree_csplit_ = split;
      tree_cbase_ = direct_waves;
    }
  }
  const int sch = sphere_chunk(host.prm.F, ps.ngroups);
  const int nsc = (host.prm.F + sch - 1) / sch;
  const size_t rb = host.prm.precision == HSMA_FP64 ? sizeof(double) : sizeof(float);
  const long comp = (long)ps.ngroups * kGroup;
  const size_t rbc = cpart_elem();
  if (rb * 5 * (size_t)comp * (ps.nch + ps.nnear + nsc) > part_cap || rbc * 5 * (size_t)kGroup * ncslots > cpart_cap ||
      (size_t)(ps.nch + ps.nnear) * ps.ngroups > work_cap || (size_t)ncfar + cs.size() > cwork_cap) {
    err = "internal error: work decomposition exceeds the reserved arena";
    return HSMA_ERR_DEVICE;
  }
  // the check schedule goes through pinned staging on the call's stream;
  // the previous upload from the staging buffer must have completed
  if (!cs.empty()) {
    HIPCHK(hipEventSynchronize(stage_ev));
    std::memcpy(h_stage, cs.data(), sizeof(CheckSched) * cs.size());
    HIPCHK(hipMemcpyAsync(d_csched, h_stage, sizeof(CheckSched) * cs.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(stage_ev, st));
  }
  cur_n = n;
  ntiles_ = ntiles;
  tree_ = tree_levels(ntiles);
  ngroups_ = ps.ngroups;
  psched_ = ps;
  ncwork_ = ncfar;
  cwork_face_ = face_waves;
  nchunks_ = ps.nch;
  nsphere_ = nsc;
  sph_chunk_ = sch;
  nrsblk_ = (int)((n + kRsBlock - 1) / kRsBlock);
  return HSMA_OK;
}

// Event pair (stage, edge) of the current timed call, created on demand.
// Treecode (near rule 2, FP32): the node boxes and moments level by level
// (after the tiles, before the check and particle branches fork).
void DevicePlan::build_tree(hipStream_t st, int n) {
  const int P = host.prm.tree_order;
  const TreeLevels tl = tree_;
  if (tl.nlev >= 2)
    hipLaunchKernelGGL(k_tree_p2m, dim3(tl.cnt[1]), dim3(512), 0, st, n, ntiles_, P, tl, (const double4*)d_pos64,
                       (const double4*)d_tile_c, (const float4*)d_tile_h, d_tnode, d_tbox, d_tmom64, d_tmom32);
  for (int l = 2; l < tl.nlev; ++l)
    hipLaunchKernelGGL(k_tree_m2m, dim3(tl.cnt[l]), dim3(512), 0, st, l, P, tl, d_tnode, d_tbox, d_tmom64, d_tmom32);
}

// Treecode sums at the particles (CHECKS false: one wave per (image entry,
// share, group), slots of the particle buffer) or at the check targets
// (CHECKS true: tree_cwaves_ waves in check-group order, the check
// schedule's slots).
template <bool CHECKS>
hsma_status DevicePlan::launch_tree(hipStream_t st, long comp, long slot, std::string& err) {
  const int P = host.prm.tree_order;
  const TreeLevels tl = tree_;
  const int grid = CHECKS ? tree_cwaves_ : psched_.nch * psched_.ngroups;
  if (grid <= 0) return HSMA_OK;
  // the slab evaluates the multipoles in FP64 (from the FP64 moments)
  const bool e64 = host.prm.geometry == HSMA_GEOM_2D;
  const void* momp = e64 ? (const void*)d_tmom64 : (const void*)d_tmom32;
#define HSMA_TREE_FAR1(PP, EE)                                                                                     \
  hipLaunchKernelGGL((k_tree_far<PP, CHECKS, EE>), dim3(grid), dim3(64), 0, st,                                    \
                     CHECKS ? (const double4*)d_check_pos : (const double4*)d_pos64, psched_,                     \
                     (const Group*)d_check_groups, (const CheckSched*)d_csched, tree_cgroup0_,                   \
                     (int)host.check_groups.size(), tree_cbase_,                                                 \
                     tree_csplit_, CHECKS ? (const Desc*)d_desc_check : (const Desc*)d_desc_part, ntiles_,         \
                     (const double4*)d_tile_c, (const float4*)d_tile_h, (const float4*)d_src32,                   \
                     (const double4*)d_pos64, (const StepParams*)d_sp, tl, (const double4*)d_tnode,               \
                     (const double4*)d_tbox, momp, host.prm.tree_theta,                                           \
                     CHECKS ? (float*)d_cpart : (float*)d_part, comp, slot)
#define HSMA_TREE_FAR(PP)                                                                                          \
  do {                                                                                                             \
    if (e64) HSMA_TREE_FAR1(PP, true);                                                                             \
    else HSMA_TREE_FAR1(PP, false);                                                                                \
  } while (0)
  switch (P) {
    case 4: HSMA_TREE_FAR(4); break;
    case 6: HSMA_TREE_FAR(6); break;
    case 8: HSMA_TREE_FAR(8); break;
    case 10: HSMA_TREE_FAR(10); break;
    case 12: HSMA_TREE_FAR(12); break;
    default:
      err = "tree order must be 4, 6, 8, 10 or 12";
      return HSMA_ERR_INVALID_ARG;
  }
#undef HSMA_TREE_FAR
#undef HSMA_TREE_FAR1
  HIPCHK(hipGetLastError());
  return HSMA_OK;
}

hsma_status DevicePlan::record(hipStream_t st, int stage, int edge, std::string& err) {
  if (!timing || timed_calls >= kMaxTimedCalls) return HSMA_OK;
  const size_t idx = ((size_t)timed_calls * kStages + stage) * 2 + edge;
  while (events.size() <= idx) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    events.push_back(e);
  }
  HIPCHK(hipEventRecord(events[idx], st));
  return HSMA_OK;
}

// The kernels of one step, in order, on stream st (no host synchronisation:
// this sequence is what a step graph captures).
hsma_status DevicePlan::enqueue_step(hipStream_t st, int n, const double* d_xyz, const double* d_q,
                                     double* d_energy, double* d_pot, double* d_force, std::string& err) {
  hsma_status s = HSMA_OK;
  const hipStream_t stream_arg = st;
  const bool fp64 = host.prm.precision == HSMA_FP64;
  const int slab = host.prm.geometry == HSMA_GEOM_2D;
  const int nblk = (n + 255) / 256;
  const int nfin = (n + kWave - 1) / kWave;  // finalize blocks (energy partials)
  // finalize waves per block: about 8 slots for each
  const int fparts = std::min(kFinParts, std::max(1, (nchunks_ + psched_.nnear + nsphere_) / 8));
  if ((s = record(st, kStStep, 0, err)) != HSMA_OK) return s;
  hipLaunchKernelGGL(k_ingest, dim3(nblk), dim3(256), 0, st, n, d_xyz, d_q, (const StepParams*)d_sp, slab, d_pos_w, d_key[0],
                     d_val[0], d_red);
  if (n <= kSmallSort) {
    hipLaunchKernelGGL(k_rank, dim3((n + kWave - 1) / kWave), dim3(kWave * kRankWaves), 0, st, n, nblk,
                       (const double*)d_red, d_status, (const uint32_t*)d_key[0], d_val[0]);
  } else {
    hipLaunchKernelGGL(k_validate, dim3(1), dim3(256), 0, st, nblk, (const double*)d_red, d_status);
    // radix sort: 4 passes of 8 bits over the 30-bit keys (result back in buffer 0)
    for (int pass = 0; pass < 4; ++pass) {
      const int sh = 8 * pass;
      const int a = pass & 1, b = a ^ 1;
      hipLaunchKernelGGL(k_rs_hist, dim3(nrsblk_), dim3(256), 0, st, (const uint32_t*)d_key[a], n, sh, d_hist,
                         nrsblk_);
      hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(1024), 0, st, d_hist, 256 * nrsblk_);
      hipLaunchKernelGGL(k_rs_scatter, dim3(nrsblk_), dim3(256), 0, st, (const uint32_t*)d_key[a],
                         (const int*)d_val[a], d_key[b], d_val[b], n, sh, (const uint32_t*)d_hist, nrsblk_);
    }
  }
  hipLaunchKernelGGL(k_tiles, dim3(ntiles_), dim3(64), 0, st, n, (const int*)d_val[0], (const double4*)d_pos_w,
                     d_pos64, d_src32, d_src64, d_tile_c, d_tile_h, d_perm);
  if (host.prm.near_rule == 2) build_tree(st, n);
  const unsigned long long* cullp = nullptr;
  CullView cv{nullptr, nullptr, nullptr};
  if (host.prm.near_rule == 1) {
    const int nd = (int)host.desc_particles.size();
    hipLaunchKernelGGL(k_cull, dim3(ntiles_, nd), dim3(64), 0, st, n, ntiles_, (const double4*)d_pos64,
                       (const Desc*)d_desc_part, (const StepParams*)d_sp, d_cull);
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactThreads), 0, st, nd * ntiles_, ntiles_,
                       (const unsigned long long*)d_cull, d_clist, d_ccount);
    cullp = d_cull;
    cv = CullView{d_cull, d_clist, d_ccount};
  }
  const int ncheck = (int)host.check_axis.size();
  const int ncg = (int)host.check_groups.size();
  const long ccomp = kGroup;
  const size_t cpart_elem = this->cpart_elem();  // the buffer's element size, as reserved
  const long comp = (long)ngroups_ * kGroup;
  const long slot = 5L * comp;
  const int F = host.prm.F;
  // check sums: FP64 in the FP64 path, and also with the sphere near set,
  // whose face rows are differences Phi_B(x+) - Phi_B(x-) of two full sums
  // (a source near x- has its periodic copy near x+; the two large terms
  // cancel exactly, their FP32 rounding would not)
// check sums of the groups [G0, G1) whose far waves are [W0, W1).  A partial
// slot is 5 x kGroup elements of the buffer's element type (cpart_elem
// bytes: 8 when any check sum is FP64, else 4); a float launch into an
// 8-byte buffer uses the first half of each slot, so both precisions can
// share it
#define HSMA_CHECKS(RealC, SC, SRCC, W0, W1, G0, G1)                                                                \
  do {                                                                                                              \
    const long cslot_e = 5L * kGroup * (long)(cpart_elem / sizeof(RealC));                                          \
    if ((W1) > (W0))                                                                                                \
      hipLaunchKernelGGL((k_pair<RealC, false, false>), dim3((W1) - (W0)), dim3(64), 0, st,                         \
                         (const double4*)d_check_pos, (const Group*)d_check_groups, (const CheckSched*)d_csched,    \
                         ncg, (W0), psched_, (const Desc*)d_desc_check, ntiles_, (const double4*)d_tile_c,         \
                         (const float4*)d_tile_h, (const SC*)SRCC, (const double4*)d_pos64,                         \
                         (const StepParams*)d_sp, cv, (RealC*)d_cpart, ccomp, cslot_e);                             \
    if ((G1) > (G0)) {                                                                                              \
      hipLaunchKernelGGL((k_pair<RealC, true, false>), dim3((G1) - (G0)), dim3(64), 0, st,                          \
                         (const double4*)d_check_pos, (const Group*)d_check_groups, (const CheckSched*)d_csched,    \
                         ncg, (G0), psched_, (const Desc*)d_desc_check, ntiles_, (const double4*)d_tile_c,         \
                         (const float4*)d_tile_h, (const SC*)SRCC, (const double4*)d_pos64,                         \
                         (const StepParams*)d_sp, cv, (RealC*)d_cpart, ccomp, cslot_e);                             \
      hipLaunchKernelGGL(k_reduce_check<RealC>, dim3((G1) - (G0)), dim3(kGroup * kCheckParts), 0, st,               \
                         (const Group*)d_check_groups, (const CheckSched*)d_csched, (G0), (const int*)d_check_axis, \
                         (const RealC*)d_cpart, cslot_e, d_v);                                                      \
    }                                                                                                               \
  } while (0)
#define HSMA_PARTICLES_NEAR(Real, S, SRC, NST)                                                                         \
  do {                                                                                                              \
    if ((s = record(st, kStNear, 0, err)) != HSMA_OK) return s;                                                     \
    if (host.prm.near_rule == 2) {                                                                                  \
      if ((s = launch_tree<false>(st, comp, slot, err)) != HSMA_OK) return s;                                       \
    } else {                                                                                                        \
      hipLaunchKernelGGL((k_pair<Real, false, true>),                                                              \
                         dim3(psched_.nch * ((psched_.ngroups + kFarWaves - 1) / kFarWaves)), dim3(kWave * kFarWaves), \
                         0, st,                                                                                     \
                         (const double4*)d_pos64, (const Group*)nullptr, (const CheckSched*)nullptr, 0, 0, psched_,    \
                         (const Desc*)d_desc_part, ntiles_, (const double4*)d_tile_c, (const float4*)d_tile_h,      \
                         (const S*)SRC, (const double4*)d_pos64, (const StepParams*)d_sp, cv, (Real*)d_part, comp, \
                         slot);                                                                                     \
    }                                                                                                               \
    if ((s = record(st, kStNear, 1, err)) != HSMA_OK) return s;                                                     \
    if (psched_.nnear > 0)                                                                                          \
      hipLaunchKernelGGL((k_pair<Real, true, true>), dim3(psched_.nnear * psched_.ngroups), dim3(64), 0, (NST),     \
                         (const double4*)d_pos64, (const Group*)nullptr, (const CheckSched*)nullptr, 0, 0, psched_,    \
                         (const Desc*)d_desc_part, ntiles_, (const double4*)d_tile_c, (const float4*)d_tile_h,      \
                         (const S*)SRC, (const double4*)d_pos64, (const StepParams*)d_sp, cv, (Real*)d_part, comp, \
                         slot);                                                                                     \
  } while (0)
#define HSMA_PARTICLES_SPHERE(Real)                                                                                 \
  do {                                                                                                              \
    if ((s = record(st, kStSphere, 0, err)) != HSMA_OK) return s;                                                   \
    hipLaunchKernelGGL(k_pair_sphere<Real>, dim3(ngroups_, nsphere_), dim3(64), 0, st, (const double4*)d_pos64, n,  \
                       (const double4*)d_surf64, F, sph_chunk_, (Real*)d_part, comp, nchunks_ + psched_.nnear);     \
    if ((s = record(st, kStSphere, 1, err)) != HSMA_OK) return s;                                                   \
  } while (0)
#define HSMA_FINALIZE(Real)                                                                                         \
  do {                                                                                                              \
    hipLaunchKernelGGL(k_finalize<Real>, dim3(nfin), dim3(kWave * fparts), 0, st, n,                              \
                       nchunks_ + psched_.nnear + nsphere_,                                                         \
                       (const Real*)d_part, comp, (const double4*)d_pos64, (const int*)d_perm,                     \
                       (const Desc*)d_desc_part, (int)host.desc_particles.size(), cullp, ntiles_,                   \
                       host.prm.coulomb_k, (const int*)d_status, d_pot, d_force, d_epart);                          \
  } while (0)
  // The check sums, the fit, the sphere sources and the sphere sums at the
  // particles depend only on the tiles, as do the near-set sums at the
  // particles.  The first chain runs
  // on a side stream, forked from and joined back into the call's stream
  // (event edges, so a captured step graph holds all branches), while the
  // far particle sums run on the call's stream (and, above kSmallSort
  // particles, the near pass on a second side stream): the chain's small,
  // latency-bound kernels and the near waves then fill what the far waves
  // leave idle, at every size (50,000 ions: 20.40 -> 20.04 ms per step;
  // 200,000: 313.0 -> 312.1 ms; identical results).
  // the near pass (latency-bound waves) gets a second side stream where it
  // is long enough to pay for the extra fork and join
  const bool near_side = n > kSmallSort;
  {
    HIPCHK(hipEventRecord(ev_fork, st));
    HIPCHK(hipStreamWaitEvent(side, ev_fork, 0));
    if (near_side) HIPCHK(hipStreamWaitEvent(side_near, ev_fork, 0));
    {
      const hipStream_t st = side;  // where the check chain's launches go
      if ((s = record(st, kStCheck, 0, err)) != HSMA_OK) return s;
      if (fp64) {
        HSMA_CHECKS(double, double4, d_src64, 0, ncwork_, 0, ncg);
      } else if (host.prm.near_rule == 1) {
        // sphere near set: the face rows (differences of two full sums) in
        // FP64, the slab's interface rows (single sums) in FP32
        const int gf = host.face_groups;
        HSMA_CHECKS(double, double4, d_src64, 0, cwork_face_, 0, gf);
        HSMA_CHECKS(float, float4, d_src32, cwork_face_, ncwork_, gf, ncg);
      } else if (tree_cwaves_ > 0) {
        // the groups before tree_cgroup0_ direct (none on the slab), the
        // rest by the treecode, then the same row reduction
        const int gf = tree_cgroup0_;
        HSMA_CHECKS(float, float4, d_src32, 0, tree_cbase_, 0, gf);
        if ((s = launch_tree<true>(st, ccomp, 5L * kGroup, err)) != HSMA_OK) return s;
        hipLaunchKernelGGL(k_reduce_check<float>, dim3(ncg - gf), dim3(kGroup * kCheckParts), 0, st,
                           (const Group*)d_check_groups, (const CheckSched*)d_csched, gf, (const int*)d_check_axis,
                           (const float*)d_cpart, 5L * kGroup, d_v);
      } else {
        HSMA_CHECKS(float, float4, d_src32, 0, ncwork_, 0, ncg);
      }
      if ((s = record(st, kStCheck, 1, err)) != HSMA_OK) return s;
      hipLaunchKernelGGL(k_lsq, dim3(host.nb), dim3(256), 0, st, 2 * ncheck, (const double*)d_Praw,
                         (const double*)d_v, d_A);
      hipLaunchKernelGGL(k_sphere_sources, dim3((F + 63) / 64), dim3(64), 0, st, F, host.nb, (const double*)d_SQ,
                         (const double*)d_SD, (const double*)d_A, (const double*)d_ysurf, (const double*)d_nsurf,
                         d_surf32, d_surf64, d_qd);
      // the sphere sums at the particles follow on the same side stream
      // (their own slots; only k_finalize reads them)
      if (fp64) HSMA_PARTICLES_SPHERE(double);
      else HSMA_PARTICLES_SPHERE(float);
      HIPCHK(hipEventRecord(ev_join, st));
    }
  }
  const hipStream_t nst = near_side ? side_near : stream_arg;
  if (fp64) HSMA_PARTICLES_NEAR(double, double4, d_src64, nst);
  else HSMA_PARTICLES_NEAR(float, float4, d_src32, nst);
  if (near_side) HIPCHK(hipEventRecord(ev_join_near, side_near));
  HIPCHK(hipStreamWaitEvent(st, ev_join, 0));
  if (near_side) HIPCHK(hipStreamWaitEvent(st, ev_join_near, 0));
  if (fp64) HSMA_FINALIZE(double);
  else HSMA_FINALIZE(float);
#undef HSMA_CHECKS
#undef HSMA_PARTICLES_NEAR
#undef HSMA_PARTICLES_SPHERE
#undef HSMA_FINALIZE
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, st, nfin, (const double*)d_epart,
                     d_energy ? d_energy : d_energy_scratch);
  HIPCHK(hipGetLastError());
  if ((s = record(st, kStStep, 1, err)) != HSMA_OK) return s;
  if (timing && timed_calls < kMaxTimedCalls) ++timed_calls;
  return HSMA_OK;
}

// Writes the step-parameter block (box, close-pair radii, sphere radius)
// on stream st when it changed since the last write (same stream order as
// the kernels that read it).
hsma_status DevicePlan::set_step_params(hipStream_t st, std::string& err) {
  const bool fp64 = host.prm.precision == HSMA_FP64;
  const int64_t n = std::max<int64_t>(1, cur_n);
  const double3 lo = make_double3(host.lo[0], host.lo[1], host.lo[2]);
  const double3 L = make_double3(host.L[0], host.L[1], host.L[2]);
  const double3 hbox = make_double3(0.5 * host.L[0], 0.5 * host.L[1], 0.5 * host.L[2]);
  // close-pair radius: a tenth of a typical tile extent (FP32 path); the
  // FP64 path needs the near pass only to drop the self pair
  const double vol = host.L[0] * host.L[1] * host.L[2];
  const double ext = std::cbrt(kTile * vol / (double)n);
  const double rc = fp64 ? 1e-9 * ext : close_factor * ext;
  // the step-parameter block is rewritten only when it changes (same
  // stream order as the kernels that read it)
  // sphere radius of the current box, R = lambda |L| / 2 with the diagonal
  // summed left to right (the sphere near set is decided on exactly this R)
  const double R = host.prm.lambda * 0.5 * std::sqrt(host.L[0] * host.L[0] + host.L[1] * host.L[1] + host.L[2] * host.L[2]);
  const double rc2c = rc * rc;
  const double spv[12] = {lo.x, lo.y, lo.z, L.x, L.y, L.z, hbox.x, hbox.y, hbox.z, rc * rc, rc2c, R * R};
  if (!sp_valid || std::memcmp(spv, sp_host, sizeof(spv)) != 0) {
    hipLaunchKernelGGL(k_set_params, dim3(1), dim3(1), 0, st, (StepParams*)d_sp, lo, L, hbox, rc * rc, rc2c, R * R);
    HIPCHK(hipGetLastError());
    std::memcpy(sp_host, spv, sizeof(spv));
    sp_valid = true;
  }
  return HSMA_OK;
}

hsma_status DevicePlan::run(hipStream_t st, int64_t n64, const double* d_xyz, const double* d_q, double* d_energy,
                            double* d_pot, double* d_force, std::string& err) {
  if (n64 > (int64_t)0x3fffffff) {
    err = "too many particles for one call";
    return HSMA_ERR_INVALID_ARG;
  }
  if (host.prm.near_rule == 1 && (n64 + kTile - 1) / kTile > (int64_t)1 << kTileBits) {
    err = "too many particles for the sphere near set (at most 2^26)";
    return HSMA_ERR_INVALID_ARG;
  }
  if (host.prm.near_rule == 2 && (n64 + kTile - 1) / kTile > (int64_t)1 << 20) {
    err = "too many particles for the treecode (at most 2^26)";
    return HSMA_ERR_INVALID_ARG;
  }
  hsma_status s = order_after_previous(st, err);
  if (s != HSMA_OK) return s;
  s = prepare(n64, st, err);
  if (s != HSMA_OK) return s;
  s = set_step_params(st, err);
  if (s != HSMA_OK) return s;
  const int n = (int)n64;
  // Graph replay: a step depends only on (n, buffers, stream) once the box
  // scalars live in d_sp and the check schedule of n has been uploaded
  // (prepare, above, outside any graph).  A key seen among the recent calls
  // is captured on its second call and replayed afterwards; up to
  // kGraphCache captured steps are kept (least recently used out), so
  // replicas that alternate on one plan all replay.
  const GraphKey key{n, d_xyz, d_q, d_energy, d_pot, d_force, st};
  const bool graphable = use_graph && !timing && st != nullptr;
  int hit = -1;
  if (graphable)
    for (size_t i = 0; i < graphs.size(); ++i)
      if (graphs[i].first == key) hit = (int)i;
  if (hit >= 0) {
    std::rotate(graphs.begin(), graphs.begin() + hit, graphs.begin() + hit + 1);  // most recent first
    HIPCHK(hipGraphLaunch(graphs[0].second, st));
    ++graph_replays;
  } else if (graphable && std::find(seen_keys.begin(), seen_keys.end(), key) != seen_keys.end()) {
    if (graphs.size() >= (size_t)kGraphCache) {
      // the evicted step may still run: wait for the plan's previous call
      HIPCHK(hipEventSynchronize(ev_done));
      (void)hipGraphExecDestroy(graphs.back().second);
      graphs.pop_back();
    }
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hsma_status es = enqueue_step(st, n, d_xyz, d_q, d_energy, d_pot, d_force, err);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(st, &graph);
    if (es != HSMA_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return es;
    }
    if (ce != hipSuccess) {
      err = std::string("hipStreamEndCapture: ") + hipGetErrorString(ce);
      return HSMA_ERR_DEVICE;
    }
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      err = std::string("hipGraphInstantiate: ") + hipGetErrorString(ie);
      return HSMA_ERR_DEVICE;
    }
    graphs.insert(graphs.begin(), std::make_pair(key, exec));
    HIPCHK(hipGraphLaunch(exec, st));
  } else {
    if ((s = enqueue_step(st, n, d_xyz, d_q, d_energy, d_pot, d_force, err)) != HSMA_OK) return s;
    if (graphable) {
      seen_keys.insert(seen_keys.begin(), key);
      if (seen_keys.size() > (size_t)kGraphSeen) seen_keys.pop_back();
    }
  }
  if ((s = mark_done(st, err)) != HSMA_OK) return s;
  const long long nd = (long long)host.desc_particles.size();
  near_pairs = (long long)n * nd * n - n;
  long long cp = 0;
  for (const Group& g : host.check_groups) cp += (long long)g.count * g.ndesc * n;
  check_pairs = cp;
  sphere_pairs = (long long)n * host.prm.F;
  return HSMA_OK;
}


// One step whose per-size arena lives in the device's static scratch: no
// device or host allocation.  The decomposition uses the no-allocation
// targets, and the heap arena (if any) is carved back afterwards.  Every
// call on a device shares that device's scratch.
hsma_status DevicePlan::run_noalloc(hipStream_t st, int64_t n, const double* d_xyz, const double* d_q,
                                    double* d_energy, double* d_pot, double* d_force, std::string& err) {
  if (n < 1 || n > kNoAllocMaxN) {
    err = "the no-allocation entry point takes 1 to " + std::to_string(kNoAllocMaxN) + " particles";
    return HSMA_ERR_INVALID_ARG;
  }
  if (!scratch) {
    err = "no scratch address on this device";
    return HSMA_ERR_DEVICE;
  }
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != device) {
    err = "the current device is not the plan's device";
    return HSMA_ERR_INVALID_ARG;
  }
  const int saved[5] = {part_target, check_target, check_target_max, near_target, tree_target};
  const int64_t saved_cap = cap_n;
  auto restore = [&]() {
    part_target = saved[0];
    check_target = saved[1];
    check_target_max = saved[2];
    near_target = saved[3];
    tree_target = saved[4];
    (void)carve(d_arena ? saved_cap : 0, (char*)d_arena);
    cap_n = d_arena ? saved_cap : 0;
    cur_n = -1;  // the next allocating call uploads its schedule again
  };
  part_target = kNoAllocPartTarget;
  check_target = kNoAllocCheckTarget;
  check_target_max = kNoAllocCheckTargetMax;
  near_target = kNoAllocNearTarget;
  tree_target = kNoAllocTreeTarget;
  const size_t need = carve(n, nullptr);
  if (need > kScratchBytes) {
    restore();
    err = "this plan needs " + std::to_string(need) + " bytes of scratch for " + std::to_string(n) +
          " particles; the no-allocation scratch holds " + std::to_string(kScratchBytes);
    return HSMA_ERR_INVALID_ARG;
  }
  (void)carve(n, (char*)scratch);
  cap_n = std::max<int64_t>(n, 64);  // prepare() must not reserve a heap arena
  cur_n = -1;
  const bool timed = timing;
  timing = false;
  hsma_status s = order_after_previous(st, err);
  if (s == HSMA_OK) s = prepare(n, st, err);
  if (s == HSMA_OK) s = set_step_params(st, err);
  if (s == HSMA_OK) s = enqueue_step(st, (int)n, d_xyz, d_q, d_energy, d_pot, d_force, err);
  if (s == HSMA_OK) s = mark_done(st, err);
  timing = timed;
  restore();
  if (s != HSMA_OK) return s;
  const long long nd = (long long)host.desc_particles.size();
  near_pairs = (long long)n * nd * n - n;
  long long cp = 0;
  for (const Group& g : host.check_groups) cp += (long long)g.count * g.ndesc * n;
  check_pairs = cp;
  sphere_pairs = (long long)n * host.prm.F;
  return HSMA_OK;
}

hsma_status DevicePlan::sphere_sources(long long& inside, std::string& err) const {
  inside = 0;
  if (!d_cull || cur_n <= 0) return HSMA_OK;
  if (done_recorded) HIPCHK(hipEventSynchronize(ev_done));
  const size_t nd = host.desc_particles.size();
  std::vector<unsigned long long> m(nd * (size_t)ntiles_);
  HIPCHK(hipMemcpy(m.data(), d_cull, sizeof(unsigned long long) * m.size(), hipMemcpyDeviceToHost));
  for (unsigned long long v : m) inside += __builtin_popcountll(v);
  // padding slots of the last tile read as inside
  inside -= (long long)nd * ((long long)ntiles_ * kTile - cur_n);
  return HSMA_OK;
}

// Keeps a copy of the plan constants for the unit box so that the plan can
// be re-targeted to any box len = s * unit_len with one kernel.
hsma_status DevicePlan::init_scalable(std::string& err) {
  if (scalable) return HSMA_OK;
  const size_t ndp = host.desc_particles.size(), ndc = host.desc_check.size(), nck = host.check_axis.size();
  const size_t npr = host.Praw.size(), nsq = host.SQ.size(), nys = host.ysurf.size();
  HIPCHK(hipMalloc((void**)&d_unit_desc_part, sizeof(Desc) * std::max<size_t>(1, ndp)));
  HIPCHK(hipMalloc((void**)&d_unit_desc_check, sizeof(Desc) * std::max<size_t>(1, ndc)));
  HIPCHK(hipMalloc((void**)&d_unit_check_pos, sizeof(double4) * std::max<size_t>(1, nck)));
  HIPCHK(hipMalloc((void**)&d_unit_Praw, sizeof(double) * std::max<size_t>(1, npr)));
  HIPCHK(hipMalloc((void**)&d_unit_SQ, sizeof(double) * std::max<size_t>(1, nsq)));
  HIPCHK(hipMalloc((void**)&d_unit_SD, sizeof(double) * std::max<size_t>(1, nsq)));
  HIPCHK(hipMalloc((void**)&d_unit_ysurf, sizeof(double) * std::max<size_t>(1, nys)));
  HIPCHK(hipMemcpy(d_unit_desc_part, d_desc_part, sizeof(Desc) * ndp, hipMemcpyDeviceToDevice));
  if (ndc) HIPCHK(hipMemcpy(d_unit_desc_check, d_desc_check, sizeof(Desc) * ndc, hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(d_unit_check_pos, d_check_pos, sizeof(double4) * nck, hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(d_unit_Praw, d_Praw, sizeof(double) * npr, hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(d_unit_SQ, d_SQ, sizeof(double) * nsq, hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(d_unit_SD, d_SD, sizeof(double) * nsq, hipMemcpyDeviceToDevice));
  HIPCHK(hipMemcpy(d_unit_ysurf, d_ysurf, sizeof(double) * nys, hipMemcpyDeviceToDevice));
  for (int k = 0; k < 3; ++k) unit_L[k] = host.L[k];
  unit_R = host.R;
  scalable = true;
  return HSMA_OK;
}

hsma_status DevicePlan::set_box(const double lo[3], double scale, hipStream_t st, std::string& err) {
  if (!scalable) {
    err = "plan is not scalable";
    return HSMA_ERR_INVALID_ARG;
  }
  for (int k = 0; k < 3; ++k) {
    host.lo[k] = lo[k];
    host.L[k] = unit_L[k] * scale;
  }
  host.R = unit_R * scale;
  if (scale == cur_scale) return HSMA_OK;
  const long npr = (long)host.Praw.size(), nsq = (long)host.SQ.size();
  hipLaunchKernelGGL(k_scale_plan, dim3(16, 6), dim3(256), 0, st, scale, (int)host.desc_particles.size(),
                     (const Desc*)d_unit_desc_part, d_desc_part, (int)host.desc_check.size(),
                     (const Desc*)d_unit_desc_check, d_desc_check, (int)host.check_axis.size(),
                     (const double4*)d_unit_check_pos, d_check_pos, npr, (const double*)d_unit_Praw, d_Praw, nsq,
                     (const double*)d_unit_SQ, d_SQ, (const double*)d_unit_SD, d_SD, (int)host.ysurf.size(),
                     (const double*)d_unit_ysurf, d_ysurf);
  HIPCHK(hipGetLastError());
  cur_scale = scale;
  return HSMA_OK;
}

}  // namespace hsma
