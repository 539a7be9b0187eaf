// gfx950 kernels of the HSMA hot path and the per-step launch sequence.
//
// Per step (Sec. 2.2 of the paper, in this order):
//   ingest   wrap into the centred box, validate, spatial (Morton) keys
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

#include "device.h"

namespace hsma {

// ----------------------------------------------------------------- helpers
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

// Knuth's error-free sum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

template <typename Real> struct SrcT;
template <> struct SrcT<float> { typedef float4 T; };
template <> struct SrcT<double> { typedef double4 T; };

__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// ----------------------------------------------------------------- ingest
// Centred, wrapped FP64 positions + charge; 30-bit Morton key of a 1024^3
// cell grid; per-block partial sums (sum q, sum |q|, invalid count).
__global__ __launch_bounds__(256) void k_ingest(int n, const double* __restrict__ xyz, const double* __restrict__ q,
                                                double3 lo, double3 L, int slab, double4* __restrict__ pos,
                                                uint32_t* __restrict__ key, int* __restrict__ val,
                                                double* __restrict__ red) {
  __shared__ double s0[256], s1[256], s2[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
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
    key[i] = (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
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
__global__ __launch_bounds__(256) void k_validate(int nblk, const double* __restrict__ red, int* __restrict__ status) {
  __shared__ double s0[256], s1[256], s2[256];
  double a = 0, b = 0, c = 0;
  for (int i = threadIdx.x; i < nblk; i += 256) {
    a += red[3 * i];
    b += red[3 * i + 1];
    c += red[3 * i + 2];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  s2[threadIdx.x] = c;
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
    int st = HSMA_OK;
    if (s2[0] > 0) st = HSMA_ERR_OUT_OF_DOMAIN;
    else if (!(fabs(s0[0]) <= 1e-12 * s1[0])) st = HSMA_ERR_NOT_NEUTRAL;
    status[0] = st;
  }
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
  __shared__ uint32_t s[1024];
  const int per = (len + 1023) / 1024;
  const int b = threadIdx.x * per;
  const int e = min(len, b + per);
  uint32_t sum = 0;
  for (int i = b; i < e; ++i) sum += a[i];
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t v = threadIdx.x >= o ? s[threadIdx.x - o] : 0u;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - sum;
  for (int i = b; i < e; ++i) {
    const uint32_t v = a[i];
    a[i] = run;
    run += v;
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

__global__ __launch_bounds__(64) void k_tiles(int n, const int* __restrict__ order, const double4* __restrict__ pos,
                                              double4* __restrict__ pos64, float4* __restrict__ src32,
                                              double4* __restrict__ src64, double4* __restrict__ tile_c,
                                              float4* __restrict__ tile_h, int* __restrict__ perm) {
  const int s = blockIdx.x * kTile + threadIdx.x;
  const bool ok = s < n;
  double4 p = make_double4(0, 0, 0, 0);
  int o = 0;
  if (ok) {
    o = order[s];
    p = pos[o];
  }
  const double mnx = wave_min(ok ? p.x : INFINITY), mxx = wave_max(ok ? p.x : -INFINITY);
  const double mny = wave_min(ok ? p.y : INFINITY), mxy = wave_max(ok ? p.y : -INFINITY);
  const double mnz = wave_min(ok ? p.z : INFINITY), mxz = wave_max(ok ? p.z : -INFINITY);
  const double cx = 0.5 * (mnx + mxx), cy = 0.5 * (mny + mxy), cz = 0.5 * (mnz + mxz);
  if (threadIdx.x == 0) {
    tile_c[blockIdx.x] = make_double4(cx, cy, cz, 0.0);
    // half extents rounded up so that the bound stays conservative
    tile_h[blockIdx.x] = make_float4((float)(0.5 * (mxx - mnx)) * 1.0001f + 1e-30f,
                                     (float)(0.5 * (mxy - mny)) * 1.0001f + 1e-30f,
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

// ----------------------------------------------------------------- pair sums
// One wave per work item: a group of up to 128 targets (2 per lane) against
// a contiguous range of (image entry, source tile) pairs.  Sources are read
// with wave-uniform (scalar) loads, so a source costs no VGPRs and no LDS.
// Coordinates: targets are kept as offsets from their group's box centre;
// each tile contributes the FP32-rounded FP64 shift between its image
// centre and the group centre, so close pairs subtract small numbers.
// Pairs closer than sqrt(rc2) (only possible in tiles whose bounding box
// comes within that distance of the group) recompute the difference from
// the FP64 positions, which also removes the self pair.
// Accumulation: plain sums within a tile, error-free (2Sum) folding of the
// tile partials into a (hi, lo) potential across tiles.
template <typename Real, bool PARTICLES>
__global__ __launch_bounds__(64) void k_pair(const double4* __restrict__ tgt, const Group* __restrict__ groups,
                                             const Work* __restrict__ work, const Desc* __restrict__ desc,
                                             int ntiles, const double4* __restrict__ tile_c,
                                             const float4* __restrict__ tile_h,
                                             const typename SrcT<Real>::T* __restrict__ src,
                                             const double4* __restrict__ pos64, double rc2, Real* __restrict__ part,
                                             long comp_stride, long slot_stride) {
  typedef typename SrcT<Real>::T S;
  const Work w = work[blockIdx.x];
  const Group g = groups[w.group];
  const int lane = threadIdx.x;
  double tx[kTPL], ty[kTPL], tz[kTPL];
  bool valid[kTPL];
  double mnx = INFINITY, mny = INFINITY, mnz = INFINITY, mxx = -INFINITY, mxy = -INFINITY, mxz = -INFINITY;
#pragma unroll
  for (int j = 0; j < kTPL; ++j) {
    const int l = j * kWave + lane;
    valid[j] = l < g.count;
    const double4 p = tgt[g.first + (valid[j] ? l : 0)];
    tx[j] = p.x;
    ty[j] = p.y;
    tz[j] = p.z;
    if (valid[j]) {
      mnx = fmin(mnx, p.x); mxx = fmax(mxx, p.x);
      mny = fmin(mny, p.y); mxy = fmax(mxy, p.y);
      mnz = fmin(mnz, p.z); mxz = fmax(mxz, p.z);
    }
  }
  mnx = wave_min(mnx); mxx = wave_max(mxx);
  mny = wave_min(mny); mxy = wave_max(mxy);
  mnz = wave_min(mnz); mxz = wave_max(mxz);
  const double cgx = 0.5 * (mnx + mxx), cgy = 0.5 * (mny + mxy), cgz = 0.5 * (mnz + mxz);
  const double hgx = 0.5 * (mxx - mnx), hgy = 0.5 * (mxy - mny), hgz = 0.5 * (mxz - mnz);
  Real ox[kTPL], oy[kTPL], oz[kTPL];
  Real ph[kTPL], pl[kTPL], ex[kTPL], ey[kTPL], ez[kTPL];
#pragma unroll
  for (int j = 0; j < kTPL; ++j) {
    ox[j] = (Real)(tx[j] - cgx);
    oy[j] = (Real)(ty[j] - cgy);
    oz[j] = (Real)(tz[j] - cgz);
    ph[j] = pl[j] = ex[j] = ey[j] = ez[j] = (Real)0;
  }
  const int tbase = g.first + lane;  // sorted index of this lane's first target

  for (int f = w.f0; f < w.f1; ++f) {
    const int di = f / ntiles;
    const int tile = f - di * ntiles;
    const Desc ds = desc[g.desc_off + di];
    const double4 cs = tile_c[tile];
    const float4 hs = tile_h[tile];
    const double dlx = (cs.x + ds.sx) - cgx;
    const double dly = (cs.y + ds.sy) - cgy;
    const double dlz = (ds.sigma * cs.z + ds.sz) - cgz;
    const double gx = fmax(0.0, fabs(dlx) - hgx - (double)hs.x);
    const double gy = fmax(0.0, fabs(dly) - hgy - (double)hs.y);
    const double gz = fmax(0.0, fabs(dlz) - hgz - (double)hs.z);
    const double gap2 = gx * gx + gy * gy + gz * gz;
    const Real sg = (Real)ds.sigma;
    Real ux[kTPL], uy[kTPL], uz[kTPL];
    Real pp[kTPL], qx[kTPL], qy[kTPL], qz[kTPL];
#pragma unroll
    for (int j = 0; j < kTPL; ++j) {
      ux[j] = ox[j] - (Real)dlx;
      uy[j] = oy[j] - (Real)dly;
      uz[j] = sg * (oz[j] - (Real)dlz);
      pp[j] = qx[j] = qy[j] = qz[j] = (Real)0;
    }
    const S* __restrict__ s = src + (long)tile * kTile;
    if (gap2 >= rc2) {
#pragma unroll 16
      for (int k = 0; k < kTile; ++k) {
        const S v = s[k];
#pragma unroll
        for (int j = 0; j < kTPL; ++j) {
          const Real dx = ux[j] - (Real)v.x;
          const Real dy = uy[j] - (Real)v.y;
          const Real dz = uz[j] - (Real)v.z;
          const Real r2 = dx * dx + dy * dy + dz * dz;
          const Real ri = rsq(r2);
          const Real a = (Real)v.w * ri;
          pp[j] += a;
          const Real b = a * (ri * ri);
          qx[j] += b * dx;
          qy[j] += b * dy;
          qz[j] += b * dz;
        }
      }
    } else {
      const bool ident = ds.sx == 0.0 && ds.sy == 0.0 && ds.sz == 0.0 && ds.sigma > 0.0;
#pragma unroll 4
      for (int k = 0; k < kTile; ++k) {
        const S v = s[k];
#pragma unroll
        for (int j = 0; j < kTPL; ++j) {
          Real dx = ux[j] - (Real)v.x;
          Real dy = uy[j] - (Real)v.y;
          Real dz = uz[j] - (Real)v.z;
          Real r2 = dx * dx + dy * dy + dz * dz;
          Real qq = (Real)v.w;
          if ((double)r2 < rc2) {
            const long si = (long)tile * kTile + k;
            const double4 ps = pos64[si];
            dx = (Real)(tx[j] - (ps.x + ds.sx));
            dy = (Real)(ty[j] - (ps.y + ds.sy));
            dz = sg * (Real)(tz[j] - (ds.sigma * ps.z + ds.sz));
            r2 = dx * dx + dy * dy + dz * dz;
            if (PARTICLES && ident && si == (long)(tbase + j * kWave)) {
              qq = (Real)0;
              r2 = (Real)1;
            }
          }
          const Real ri = rsq(r2);
          const Real a = qq * ri;
          pp[j] += a;
          const Real b = a * (ri * ri);
          qx[j] += b * dx;
          qy[j] += b * dy;
          qz[j] += b * dz;
        }
      }
    }
    const Real sc = (Real)ds.scale;
#pragma unroll
    for (int j = 0; j < kTPL; ++j) {
      const Real t = sc * pp[j];
      if constexpr (sizeof(Real) == 4) {
        float hs2, e;
        two_sum(ph[j], t, hs2, e);
        ph[j] = hs2;
        pl[j] += e;
      } else {
        ph[j] += t;
      }
      ex[j] += sc * qx[j];
      ey[j] += sc * qy[j];
      ez[j] += (sc * sg) * qz[j];
    }
  }
#pragma unroll
  for (int j = 0; j < kTPL; ++j) {
    if (!valid[j]) continue;
    const long o = (long)w.slot * slot_stride + (PARTICLES ? (long)g.first : 0L) + j * kWave + lane;
    part[o] = ph[j];
    part[o + comp_stride] = pl[j];
    part[o + 2 * comp_stride] = ex[j];
    part[o + 3 * comp_stride] = ey[j];
    part[o + 4 * comp_stride] = ez[j];
  }
}

// Sphere sources: charge Q_k and double-layer strength D_k at y_k, normal
// n_k.  phi += Q/|d| - D (n.d)/|d|^3,  E += Q d/|d|^3 + D (n/|d|^3 - 3 (n.d) d/|d|^5).
// Records: surf[2k] = (y, Q), surf[2k+1] = (n, D), box-centred coordinates.
template <typename Real>
__global__ __launch_bounds__(64) void k_pair_sphere(const double4* __restrict__ tgt, int n,
                                                    const typename SrcT<Real>::T* __restrict__ surf, int F,
                                                    Real* __restrict__ part, long comp_stride, long slot_off) {
  typedef typename SrcT<Real>::T S;
  const int lane = threadIdx.x;
  const int first = blockIdx.x * kGroup;
  Real tx[kTPL], ty[kTPL], tz[kTPL];
  Real ph[kTPL], pl[kTPL], ex[kTPL], ey[kTPL], ez[kTPL];
#pragma unroll
  for (int j = 0; j < kTPL; ++j) {
    const int t = min(first + j * kWave + lane, n - 1);
    const double4 p = tgt[t];
    tx[j] = (Real)p.x;
    ty[j] = (Real)p.y;
    tz[j] = (Real)p.z;
    ph[j] = pl[j] = ex[j] = ey[j] = ez[j] = (Real)0;
  }
  for (int k0 = 0; k0 < F; k0 += kTile) {
    const int k1 = min(F, k0 + kTile);
    Real pp[kTPL], qx[kTPL], qy[kTPL], qz[kTPL];
#pragma unroll
    for (int j = 0; j < kTPL; ++j) pp[j] = qx[j] = qy[j] = qz[j] = (Real)0;
    for (int k = k0; k < k1; ++k) {
      const S a0 = surf[2 * k], a1 = surf[2 * k + 1];
#pragma unroll
      for (int j = 0; j < kTPL; ++j) {
        const Real dx = tx[j] - (Real)a0.x, dy = ty[j] - (Real)a0.y, dz = tz[j] - (Real)a0.z;
        const Real r2 = dx * dx + dy * dy + dz * dz;
        const Real ri = rsq(r2);
        const Real ri2 = ri * ri;
        const Real ri3 = ri * ri2;
        const Real a = (Real)a0.w * ri;
        const Real nd = (Real)a1.x * dx + (Real)a1.y * dy + (Real)a1.z * dz;
        const Real t = (Real)a1.w * nd * ri3;
        pp[j] += a - t;
        const Real c1 = ri2 * (a - (Real)3 * t);
        const Real c2 = (Real)a1.w * ri3;
        qx[j] += c1 * dx + c2 * (Real)a1.x;
        qy[j] += c1 * dy + c2 * (Real)a1.y;
        qz[j] += c1 * dz + c2 * (Real)a1.z;
      }
    }
#pragma unroll
    for (int j = 0; j < kTPL; ++j) {
      if constexpr (sizeof(Real) == 4) {
        float hs2, e;
        two_sum(ph[j], pp[j], hs2, e);
        ph[j] = hs2;
        pl[j] += e;
      } else {
        ph[j] += pp[j];
      }
      ex[j] += qx[j];
      ey[j] += qy[j];
      ez[j] += qz[j];
    }
  }
#pragma unroll
  for (int j = 0; j < kTPL; ++j) {
    const int t = first + j * kWave + lane;
    if (t >= n) continue;
    const long o = slot_off + t;
    part[o] = ph[j];
    part[o + comp_stride] = pl[j];
    part[o + 2 * comp_stride] = ex[j];
    part[o + 3 * comp_stride] = ey[j];
    part[o + 4 * comp_stride] = ez[j];
  }
}

// ----------------------------------------------------------------- check / LSQ / sphere
// Sum the work-item partials of every check target in a fixed order:
// v[2t] = potential, v[2t+1] = field component axis[t].
template <typename Real>
__global__ __launch_bounds__(256) void k_reduce_check(int ncheck, const int* __restrict__ t_group,
                                                      const Group* __restrict__ groups,
                                                      const int2* __restrict__ g_work, const int* __restrict__ axis,
                                                      const Real* __restrict__ part, double* __restrict__ v) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= ncheck) return;
  const int gi = t_group[t];
  const int local = t - groups[gi].first;
  const int2 wr = g_work[gi];
  const int ax = axis[t];
  double phi = 0, e = 0;
  if constexpr (sizeof(Real) == 4) {
    float hi = 0, lo = 0, ea = 0, ec = 0;
    for (int w = wr.x; w < wr.x + wr.y; ++w) {
      const Real* p = part + (long)w * 5 * kGroup + local;
      float s, er;
      two_sum(hi, p[0], s, er);
      hi = s;
      lo += er + p[kGroup];
      float y = p[(2 + ax) * kGroup];
      two_sum(ea, y, s, er);
      ea = s;
      ec += er;
    }
    phi = (double)hi + (double)lo;
    e = (double)ea + (double)ec;
  } else {
    for (int w = wr.x; w < wr.x + wr.y; ++w) {
      const Real* p = part + (long)w * 5 * kGroup + local;
      phi += p[0];
      e += p[(2 + ax) * kGroup];
    }
  }
  v[2 * t] = phi;
  v[2 * t + 1] = e;
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
template <typename Real>
__global__ __launch_bounds__(256) void k_finalize(int n, int nslot, const Real* __restrict__ part, long comp_stride,
                                                  const double4* __restrict__ pos64, const int* __restrict__ perm,
                                                  double kc, const int* __restrict__ status, double* __restrict__ pot,
                                                  double* __restrict__ force, double* __restrict__ epart) {
  __shared__ double s[256];
  const int t = blockIdx.x * 256 + threadIdx.x;
  double e = 0;
  if (t < n) {
    double phi, fx, fy, fz;
    if constexpr (sizeof(Real) == 4) {
      float hi = 0, lo = 0, ax = 0, ay = 0, az = 0, cx = 0, cy = 0, cz = 0;
      for (int c = 0; c < nslot; ++c) {
        const Real* p = part + (long)c * 5 * comp_stride + t;
        float sm, er;
        two_sum(hi, p[0], sm, er);
        hi = sm;
        lo += er + p[comp_stride];
        two_sum(ax, p[2 * comp_stride], sm, er); ax = sm; cx += er;
        two_sum(ay, p[3 * comp_stride], sm, er); ay = sm; cy += er;
        two_sum(az, p[4 * comp_stride], sm, er); az = sm; cz += er;
      }
      phi = (double)hi + (double)lo;
      fx = (double)ax + (double)cx;
      fy = (double)ay + (double)cy;
      fz = (double)az + (double)cz;
    } else {
      phi = fx = fy = fz = 0;
      for (int c = 0; c < nslot; ++c) {
        const Real* p = part + (long)c * 5 * comp_stride + t;
        phi += p[0];
        fx += p[2 * comp_stride];
        fy += p[3 * comp_stride];
        fz += p[4 * comp_stride];
      }
    }
    const double q = pos64[t].w;
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
  s[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) epart[blockIdx.x] = s[0];
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

hsma_status DevicePlan::init(std::string& err) {
  HIPCHK(hipGetDevice(&device));
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
  return HSMA_OK;
}

void DevicePlan::free_arena() {
  void* ps[] = {d_key[0], d_key[1], d_val[0], d_val[1], d_hist, d_pos_w, d_pos64, d_src32, d_src64, d_tile_c,
                d_tile_h, d_perm, d_red, d_epart, d_part, d_cpart, d_groups, d_work, d_cwork, d_cg_work};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  d_key[0] = d_key[1] = nullptr;
  d_val[0] = d_val[1] = nullptr;
  d_hist = nullptr;
  d_pos_w = d_pos64 = nullptr;
  d_src32 = nullptr;
  d_src64 = nullptr;
  d_tile_c = nullptr;
  d_tile_h = nullptr;
  d_perm = nullptr;
  d_red = d_epart = nullptr;
  d_part = d_cpart = nullptr;
  d_groups = nullptr;
  d_work = d_cwork = nullptr;
  d_cg_work = nullptr;
  cap_n = 0;
  cur_n = -1;
}

DevicePlan::~DevicePlan() {
  free_arena();
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  void* ps[] = {d_desc_part, d_desc_check, d_check_pos, d_check_axis, d_check_groups, d_check_tgroup, d_Praw,
                d_SQ, d_SD, d_ysurf, d_nsurf, d_v, d_A, d_surf32, d_surf64, d_qd, d_status, d_energy_scratch,
                d_in_xyz, d_in_q, d_out_pot, d_out_force, d_out_energy};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (own_stream) (void)hipStreamDestroy(own_stream);
}

// Work items: every group's (image, tile) range cut into chunks so that a
// launch has about `target` waves.  Particle groups share one chunking
// (slot = chunk index); check groups get one slot per work item.
static void make_work(const std::vector<Group>& groups, int ntiles, int target, bool shared_slots,
                      std::vector<Work>& work, std::vector<int2>* grange, int* nchunks_out) {
  work.clear();
  if (grange) grange->assign(groups.size(), make_int2(0, 0));
  long long total = 0;
  for (const Group& g : groups) total += (long long)g.ndesc * ntiles;
  int nch_shared = 1;
  if (shared_slots && !groups.empty()) {
    const long long per = (long long)groups[0].ndesc * ntiles;
    nch_shared = (int)std::max<long long>(1, std::min<long long>(per / 8 + 1, (target + (long long)groups.size() - 1) / (long long)groups.size()));
    nch_shared = (int)std::min<long long>(nch_shared, per);
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    const long long F = (long long)g.ndesc * ntiles;
    int nch;
    if (shared_slots) nch = nch_shared;
    else nch = (int)std::max<long long>(1, std::min<long long>(F / 4 + 1, (long long)((double)target * F / std::max<long long>(1, total) + 0.5)));
    nch = (int)std::min<long long>(nch, std::max<long long>(1, F));
    const long long chunk = (F + nch - 1) / nch;
    const int first = (int)work.size();
    for (int c = 0; c < nch; ++c) {
      const long long f0 = c * chunk, f1 = std::min(F, f0 + chunk);
      Work w;
      w.group = (int)gi;
      w.f0 = (int)f0;
      w.f1 = (int)f1;
      w.slot = shared_slots ? c : (int)work.size();
      work.push_back(w);
    }
    if (grange) (*grange)[gi] = make_int2(first, (int)work.size() - first);
  }
  // chunk-major order for the shared case: neighbouring waves read the same tiles
  if (shared_slots) {
    std::stable_sort(work.begin(), work.end(), [](const Work& a, const Work& b) { return a.slot < b.slot; });
  }
  if (nchunks_out) *nchunks_out = nch_shared;
}

hsma_status DevicePlan::prepare(int64_t n, std::string& err) {
  if (n == cur_n) return HSMA_OK;
  const int ntiles = (int)((n + kTile - 1) / kTile);
  const int ngroups = (int)((n + kGroup - 1) / kGroup);
  const int npad = ntiles * kTile;
  const int nrsblk = (int)((n + kRsBlock - 1) / kRsBlock);
  // particle groups and work
  std::vector<Group> groups(ngroups);
  for (int g = 0; g < ngroups; ++g)
    groups[g] = Group{g * kGroup, (int)std::min<int64_t>(kGroup, n - (int64_t)g * kGroup), 0,
                      (int)host.desc_particles.size()};
  std::vector<Work> work, cwork;
  int nch = 1;
  make_work(groups, ntiles, part_target, true, work, nullptr, &nch);
  std::vector<int2> cgr;
  make_work(host.check_groups, ntiles, check_target, false, cwork, &cgr, nullptr);
  const size_t rb = host.prm.precision == HSMA_FP64 ? sizeof(double) : sizeof(float);
  const long comp = (long)ngroups * kGroup;
  const size_t part_bytes = rb * 5 * (size_t)comp * (nch + 1);
  const size_t cpart_bytes = rb * 5 * (size_t)kGroup * cwork.size();
  if (n > cap_n || part_bytes > part_cap || cpart_bytes > cpart_cap || work.size() > work_cap ||
      cwork.size() > cwork_cap) {
    free_arena();
    const int64_t cn = std::max<int64_t>(n, 64);
    const int64_t cnt = ((cn + kTile - 1) / kTile);
    const int64_t cpad = cnt * kTile;
    const int64_t crs = (cn + kRsBlock - 1) / kRsBlock;
    HIPCHK(hipMalloc((void**)&d_key[0], sizeof(uint32_t) * cn));
    HIPCHK(hipMalloc((void**)&d_key[1], sizeof(uint32_t) * cn));
    HIPCHK(hipMalloc((void**)&d_val[0], sizeof(int) * cn));
    HIPCHK(hipMalloc((void**)&d_val[1], sizeof(int) * cn));
    HIPCHK(hipMalloc((void**)&d_hist, sizeof(uint32_t) * 256 * crs));
    HIPCHK(hipMalloc((void**)&d_pos_w, sizeof(double4) * cn));
    HIPCHK(hipMalloc((void**)&d_pos64, sizeof(double4) * cpad));
    HIPCHK(hipMalloc((void**)&d_src32, sizeof(float4) * cpad));
    HIPCHK(hipMalloc((void**)&d_src64, sizeof(double4) * cpad));
    HIPCHK(hipMalloc((void**)&d_tile_c, sizeof(double4) * cnt));
    HIPCHK(hipMalloc((void**)&d_tile_h, sizeof(float4) * cnt));
    HIPCHK(hipMalloc((void**)&d_perm, sizeof(int) * cpad));
    HIPCHK(hipMalloc((void**)&d_red, sizeof(double) * 3 * ((cn + 255) / 256)));
    HIPCHK(hipMalloc((void**)&d_epart, sizeof(double) * ((cn + 255) / 256)));
    HIPCHK(hipMalloc(&d_part, part_bytes));
    HIPCHK(hipMalloc(&d_cpart, std::max<size_t>(cpart_bytes, 64)));
    HIPCHK(hipMalloc((void**)&d_groups, sizeof(Group) * groups.size()));
    HIPCHK(hipMalloc((void**)&d_work, sizeof(Work) * work.size()));
    HIPCHK(hipMalloc((void**)&d_cwork, sizeof(Work) * std::max<size_t>(1, cwork.size())));
    HIPCHK(hipMalloc((void**)&d_cg_work, sizeof(int2) * std::max<size_t>(1, cgr.size())));
    cap_n = cn;
    part_cap = part_bytes;
    cpart_cap = cpart_bytes;
    work_cap = work.size();
    cwork_cap = cwork.size();
    group_cap = groups.size();
  }
  if (groups.size() > group_cap) {
    if (d_groups) (void)hipFree(d_groups);
    HIPCHK(hipMalloc((void**)&d_groups, sizeof(Group) * groups.size()));
    group_cap = groups.size();
  }
  HIPCHK(hipMemcpy(d_groups, groups.data(), sizeof(Group) * groups.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(d_work, work.data(), sizeof(Work) * work.size(), hipMemcpyHostToDevice));
  if (!cwork.empty()) {
    HIPCHK(hipMemcpy(d_cwork, cwork.data(), sizeof(Work) * cwork.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d_cg_work, cgr.data(), sizeof(int2) * cgr.size(), hipMemcpyHostToDevice));
  }
  cur_n = n;
  ntiles_ = ntiles;
  ngroups_ = ngroups;
  nwork_ = (int)work.size();
  ncwork_ = (int)cwork.size();
  nchunks_ = nch;
  nrsblk_ = nrsblk;
  (void)npad;
  return HSMA_OK;
}

// Event pair (stage, edge) of the current timed call, created on demand.
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

hsma_status DevicePlan::run(hipStream_t st, int64_t n64, const double* d_xyz, const double* d_q, double* d_energy,
                            double* d_pot, double* d_force, std::string& err) {
  if (n64 > (int64_t)0x3fffffff) {
    err = "too many particles for one call";
    return HSMA_ERR_INVALID_ARG;
  }
  hsma_status s = prepare(n64, err);
  if (s != HSMA_OK) return s;
  const int n = (int)n64;
  const bool fp64 = host.prm.precision == HSMA_FP64;
  const double3 lo = make_double3(host.lo[0], host.lo[1], host.lo[2]);
  const double3 L = make_double3(host.L[0], host.L[1], host.L[2]);
  const int slab = host.prm.geometry == HSMA_GEOM_2D;
  const int nblk = (n + 255) / 256;
  if ((s = record(st, kStStep, 0, err)) != HSMA_OK) return s;
  hipLaunchKernelGGL(k_ingest, dim3(nblk), dim3(256), 0, st, n, d_xyz, d_q, lo, L, slab, d_pos_w, d_key[0],
                     d_val[0], d_red);
  hipLaunchKernelGGL(k_validate, dim3(1), dim3(256), 0, st, nblk, (const double*)d_red, d_status);
  // radix sort: 4 passes of 8 bits over the 30-bit keys (result back in buffer 0)
  for (int pass = 0; pass < 4; ++pass) {
    const int sh = 8 * pass;
    const int a = pass & 1, b = a ^ 1;
    hipLaunchKernelGGL(k_rs_hist, dim3(nrsblk_), dim3(256), 0, st, (const uint32_t*)d_key[a], n, sh, d_hist, nrsblk_);
    hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(1024), 0, st, d_hist, 256 * nrsblk_);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nrsblk_), dim3(256), 0, st, (const uint32_t*)d_key[a],
                       (const int*)d_val[a], d_key[b], d_val[b], n, sh, (const uint32_t*)d_hist, nrsblk_);
  }
  hipLaunchKernelGGL(k_tiles, dim3(ntiles_), dim3(64), 0, st, n, (const int*)d_val[0], (const double4*)d_pos_w,
                     d_pos64, d_src32, d_src64, d_tile_c, d_tile_h, d_perm);
  // close-pair radius for the FP64 coordinate correction (FP32 path):
  // a tenth of a typical tile extent; FP64 path only needs the self pair.
  const double vol = host.L[0] * host.L[1] * host.L[2];
  const double ext = std::cbrt(kTile * vol / std::max(1, n));
  const double rc = fp64 ? 1e-9 * ext : close_factor * ext;
  const double rc2 = rc * rc;
  const int ncheck = (int)host.check_axis.size();
  const long ccomp = kGroup, cslot = 5L * kGroup;
  if ((s = record(st, kStCheck, 0, err)) != HSMA_OK) return s;
  if (fp64) {
    hipLaunchKernelGGL((k_pair<double, false>), dim3(ncwork_), dim3(64), 0, st, (const double4*)d_check_pos,
                       (const Group*)d_check_groups, (const Work*)d_cwork, (const Desc*)d_desc_check, ntiles_,
                       (const double4*)d_tile_c, (const float4*)d_tile_h, (const double4*)d_src64,
                       (const double4*)d_pos64, rc2, (double*)d_cpart, ccomp, cslot);
    if ((s = record(st, kStCheck, 1, err)) != HSMA_OK) return s;
    hipLaunchKernelGGL(k_reduce_check<double>, dim3((ncheck + 255) / 256), dim3(256), 0, st, ncheck,
                       (const int*)d_check_tgroup, (const Group*)d_check_groups, (const int2*)d_cg_work,
                       (const int*)d_check_axis, (const double*)d_cpart, d_v);
  } else {
    hipLaunchKernelGGL((k_pair<float, false>), dim3(ncwork_), dim3(64), 0, st, (const double4*)d_check_pos,
                       (const Group*)d_check_groups, (const Work*)d_cwork, (const Desc*)d_desc_check, ntiles_,
                       (const double4*)d_tile_c, (const float4*)d_tile_h, (const float4*)d_src32,
                       (const double4*)d_pos64, rc2, (float*)d_cpart, ccomp, cslot);
    if ((s = record(st, kStCheck, 1, err)) != HSMA_OK) return s;
    hipLaunchKernelGGL(k_reduce_check<float>, dim3((ncheck + 255) / 256), dim3(256), 0, st, ncheck,
                       (const int*)d_check_tgroup, (const Group*)d_check_groups, (const int2*)d_cg_work,
                       (const int*)d_check_axis, (const float*)d_cpart, d_v);
  }
  hipLaunchKernelGGL(k_lsq, dim3(host.nb), dim3(256), 0, st, 2 * ncheck, (const double*)d_Praw,
                     (const double*)d_v, d_A);
  const int F = host.prm.F;
  hipLaunchKernelGGL(k_sphere_sources, dim3((F + 63) / 64), dim3(64), 0, st, F, host.nb, (const double*)d_SQ,
                     (const double*)d_SD, (const double*)d_A, (const double*)d_ysurf, (const double*)d_nsurf,
                     d_surf32, d_surf64, d_qd);
  const long comp = (long)ngroups_ * kGroup;
  const long slot = 5L * comp;
  if ((s = record(st, kStNear, 0, err)) != HSMA_OK) return s;
  if (fp64) {
    hipLaunchKernelGGL((k_pair<double, true>), dim3(nwork_), dim3(64), 0, st, (const double4*)d_pos64,
                       (const Group*)d_groups, (const Work*)d_work, (const Desc*)d_desc_part, ntiles_,
                       (const double4*)d_tile_c, (const float4*)d_tile_h, (const double4*)d_src64,
                       (const double4*)d_pos64, rc2, (double*)d_part, comp, slot);
    if ((s = record(st, kStNear, 1, err)) != HSMA_OK) return s;
    if ((s = record(st, kStSphere, 0, err)) != HSMA_OK) return s;
    hipLaunchKernelGGL(k_pair_sphere<double>, dim3(ngroups_), dim3(64), 0, st, (const double4*)d_pos64, n,
                       (const double4*)d_surf64, F, (double*)d_part, comp, (long)nchunks_ * slot);
    if ((s = record(st, kStSphere, 1, err)) != HSMA_OK) return s;
    hipLaunchKernelGGL(k_finalize<double>, dim3(nblk), dim3(256), 0, st, n, nchunks_ + 1, (const double*)d_part,
                       comp, (const double4*)d_pos64, (const int*)d_perm, host.prm.coulomb_k,
                       (const int*)d_status, d_pot, d_force, d_epart);
  } else {
    hipLaunchKernelGGL((k_pair<float, true>), dim3(nwork_), dim3(64), 0, st, (const double4*)d_pos64,
                       (const Group*)d_groups, (const Work*)d_work, (const Desc*)d_desc_part, ntiles_,
                       (const double4*)d_tile_c, (const float4*)d_tile_h, (const float4*)d_src32,
                       (const double4*)d_pos64, rc2, (float*)d_part, comp, slot);
    if ((s = record(st, kStNear, 1, err)) != HSMA_OK) return s;
    if ((s = record(st, kStSphere, 0, err)) != HSMA_OK) return s;
    hipLaunchKernelGGL(k_pair_sphere<float>, dim3(ngroups_), dim3(64), 0, st, (const double4*)d_pos64, n,
                       (const float4*)d_surf32, F, (float*)d_part, comp, (long)nchunks_ * slot);
    if ((s = record(st, kStSphere, 1, err)) != HSMA_OK) return s;
    hipLaunchKernelGGL(k_finalize<float>, dim3(nblk), dim3(256), 0, st, n, nchunks_ + 1, (const float*)d_part, comp,
                       (const double4*)d_pos64, (const int*)d_perm, host.prm.coulomb_k, (const int*)d_status,
                       d_pot, d_force, d_epart);
  }
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, st, nblk, (const double*)d_epart,
                     d_energy ? d_energy : d_energy_scratch);
  HIPCHK(hipGetLastError());
  if ((s = record(st, kStStep, 1, err)) != HSMA_OK) return s;
  if (timing && timed_calls < kMaxTimedCalls) ++timed_calls;
  const long long nd = (long long)host.desc_particles.size();
  near_pairs = (long long)n * nd * n - n;
  long long cp = 0;
  for (const Group& g : host.check_groups) cp += (long long)g.count * g.ndesc * n;
  check_pairs = cp;
  sphere_pairs = (long long)n * F;
  return HSMA_OK;
}

}  // namespace hsma
