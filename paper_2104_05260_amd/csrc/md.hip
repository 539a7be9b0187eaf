// Velocity-Verlet molecular dynamics with HSMA electrostatics (see
// include/hsma_md.h): the integration, short-range Lennard-Jones forces and
// thermo kernels, and the C interface.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <new>
#include <string>

#include "../../include/hsma_md.h"
#include "device.h"

namespace hsma {
namespace {

constexpr int kMdBlock = 256;
// Largest system of one driver: the kernels index the n x 3 coordinate
// arrays with 32-bit offsets (3 n < 2^31), and the O(n^2) pair search is
// far past practical long before this bound.
constexpr int64_t kMdMaxParticles = (int64_t)1 << 26;

struct MdBox {
  double lo[3], L[3], iL[3];  // iL = 1 / L
  int slab;  // z not periodic (walls at lo[2] and lo[2] + L[2])
};

struct MdLJ {
  double eps, sig2, rc2, shift;     // pairs: 4 eps [(s/r)^12 - (s/r)^6] + shift, r < rc
  double weps, wsig, wrc, wshift;   // walls, same form in the distance d to a wall
  float rc2_screen;                 // FP32 pre-screen: (rc + the FP32 distance error bound)^2
};

// Nose-Hoover thermostat: target kT, degrees of freedom, thermostat mass
// Q = nf kT tau^2, box volume (pressure's kinetic part).
struct MdNH {
  double dt, kT, nf, Q, vol;
};

// One wave: lane l sums partials l, l + 64, ... in order, then a fixed
// butterfly across the lanes (a single thread walking the partials spent
// 14 us of a 3,000-ion step on dependent loads).
__device__ __forceinline__ double md_wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// v = s v + dt/2 F/m (s: the thermostat's velocity scale, 1 without one);
// then, when dtx != 0, x += dtx v, wrapped into [lo, lo + L) along
// periodic axes.
__global__ __launch_bounds__(kMdBlock) void k_md_kick_drift(int n, double dt, double dtx, double* __restrict__ x,
                                                            double* __restrict__ v, const double* __restrict__ f,
                                                            const double* __restrict__ m, MdBox box,
                                                            const double* __restrict__ scale) {
  const int i = blockIdx.x * kMdBlock + threadIdx.x;
  if (i >= n) return;
  const double h = 0.5 * dt / m[i];
  const double sv = scale ? *scale : 1.0;
  for (int k = 0; k < 3; ++k) {
    const double vk = sv * v[3 * i + k] + h * f[3 * i + k];
    v[3 * i + k] = vk;
    if (dtx != 0.0) {
      double xk = x[3 * i + k] + dtx * vk;
      if (k < 2 || !box.slab) xk -= box.L[k] * floor((xk - box.lo[k]) / box.L[k]);
      x[3 * i + k] = xk;
    }
  }
}

// Lennard-Jones forces (pairs by the minimum image; walls in the slab):
// block (b, c) takes targets b * kMdBlock ... and the sources of chunk c
// (`chunk` sources, a multiple of kMdBlock, staged through LDS in tiles),
// so that small systems still spread over many blocks.  It writes its
// targets' partial forces to fpart[c] (summed in chunk order by the next
// kick) and its sums of the energy (1/2 per pair side, walls in full, by
// the last chunk) and of the pair virial r . F (1/2 per side) to part.
// The image of a source is the nearest one, rint(d / L) taken as
// rint(d * (1 / L)): the two differ only near |d| = L / 2, and the cut-off
// is below half a box edge, so no pair inside it is affected.
__global__ __launch_bounds__(kMdBlock) void k_md_lj(int n, const double* __restrict__ x, MdBox box, MdLJ lj,
                                                    int chunk, double* __restrict__ fpart,
                                                    double* __restrict__ part) {
  __shared__ double sx[kMdBlock], sy[kMdBlock], sz[kMdBlock];
  __shared__ float fsx[kMdBlock], fsy[kMdBlock], fsz[kMdBlock];
  __shared__ double re[kMdBlock], rw[kMdBlock];
  const int i = blockIdx.x * kMdBlock + threadIdx.x;
  const int c = blockIdx.y;
  const bool ok = i < n;
  double xi = 0, yi = 0, zi = 0;
  if (ok) {
    xi = x[3 * i];
    yi = x[3 * i + 1];
    zi = x[3 * i + 2];
  }
  const float xf = (float)xi, yf = (float)yi, zf = (float)zi;
  const float Lf0 = (float)box.L[0], Lf1 = (float)box.L[1], Lf2 = (float)box.L[2];
  const float iLf0 = (float)box.iL[0], iLf1 = (float)box.iL[1], iLf2 = (float)box.iL[2];
  double fx = 0, fy = 0, fz = 0, e = 0, w = 0;
  const int jb = c * chunk, je = min(n, jb + chunk);
  for (int j0 = jb; j0 < je; j0 += kMdBlock) {
    const int j = j0 + threadIdx.x;
    __syncthreads();
    if (j < je) {
      sx[threadIdx.x] = x[3 * j];
      sy[threadIdx.x] = x[3 * j + 1];
      sz[threadIdx.x] = x[3 * j + 2];
      fsx[threadIdx.x] = (float)sx[threadIdx.x];
      fsy[threadIdx.x] = (float)sy[threadIdx.x];
      fsz[threadIdx.x] = (float)sz[threadIdx.x];
    }
    __syncthreads();
    const int jn = min(kMdBlock, je - j0);
    if (!ok) continue;
    for (int jj = 0; jj < jn; ++jj) {
      if (j0 + jj == i) continue;
      // FP32 pre-screen: most pairs lie far beyond the cut-off; the FP64
      // test below decides for every pair the screen lets through, and the
      // screen's radius exceeds rc by a bound on the FP32 distance error
      float ux = xf - fsx[jj], uy = yf - fsy[jj], uz = zf - fsz[jj];
      ux -= Lf0 * rintf(ux * iLf0);
      uy -= Lf1 * rintf(uy * iLf1);
      if (!box.slab) uz -= Lf2 * rintf(uz * iLf2);
      if (ux * ux + uy * uy + uz * uz >= lj.rc2_screen) continue;
      double dx = xi - sx[jj], dy = yi - sy[jj], dz = zi - sz[jj];
      dx -= box.L[0] * rint(dx * box.iL[0]);
      dy -= box.L[1] * rint(dy * box.iL[1]);
      if (!box.slab) dz -= box.L[2] * rint(dz * box.iL[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 >= lj.rc2) continue;
      const double s2 = lj.sig2 / r2, s6 = s2 * s2 * s2;
      const double fr = 24.0 * lj.eps * (2.0 * s6 * s6 - s6) / r2;  // F = fr d
      fx += fr * dx;
      fy += fr * dy;
      fz += fr * dz;
      e += 0.5 * (4.0 * lj.eps * (s6 * s6 - s6) + lj.shift);
      w += 0.5 * fr * r2;
    }
  }
  if (ok && box.slab && lj.weps > 0.0 && c == (int)gridDim.y - 1) {
    // walls at z = lo and z = lo + L, once per particle (last chunk)
    const double dlo = zi - box.lo[2], dhi = box.lo[2] + box.L[2] - zi;
    const double ds[2] = {dlo, dhi};
    for (int s = 0; s < 2; ++s) {
      const double d = ds[s];
      if (d >= lj.wrc) continue;
      const double sd = lj.wsig / d, s6 = sd * sd * sd * sd * sd * sd;
      const double fd = 24.0 * lj.weps * (2.0 * s6 * s6 - s6) / d;  // away from the wall
      fz += s == 0 ? fd : -fd;
      e += 4.0 * lj.weps * (s6 * s6 - s6) + lj.wshift;
    }
  }
  if (ok) {
    double* o = fpart + ((long)c * n + i) * 3;
    o[0] = fx;
    o[1] = fy;
    o[2] = fz;
  }
  re[threadIdx.x] = ok ? e : 0.0;
  rw[threadIdx.x] = ok ? w : 0.0;
  __syncthreads();
  for (int o = kMdBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      re[threadIdx.x] += re[threadIdx.x + o];
      rw[threadIdx.x] += rw[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int b = c * gridDim.x + blockIdx.x;
    part[2 * b] = re[0];
    part[2 * b + 1] = rw[0];
  }
}

// F += the LJ partial forces of the nch chunks in chunk order (fpart not
// NULL), then v += dt/2 F/m (dt = 0: velocities unchanged), and per-block
// sums of the kinetic energy 1/2 m v^2 (v NULL: 0).
__global__ __launch_bounds__(kMdBlock) void k_md_kick(int n, double dt, double* __restrict__ v,
                                                      double* __restrict__ f, const double* __restrict__ m,
                                                      const double* __restrict__ fpart, int nch,
                                                      double* __restrict__ part) {
  __shared__ double rk[kMdBlock];
  const int i = blockIdx.x * kMdBlock + threadIdx.x;
  double ke = 0.0;
  if (i < n && fpart) {
    for (int k = 0; k < 3; ++k) {
      double fk = f[3 * i + k];
      for (int c = 0; c < nch; ++c) fk += fpart[((long)c * n + i) * 3 + k];
      f[3 * i + k] = fk;
    }
  }
  if (i < n && v) {
    const double h = 0.5 * dt / m[i];
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double vk = v[3 * i + k] + h * f[3 * i + k];
      if (dt != 0.0) v[3 * i + k] = vk;
      s += vk * vk;
    }
    ke = 0.5 * m[i] * s;
  }
  rk[threadIdx.x] = ke;
  __syncthreads();
  for (int o = kMdBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) rk[threadIdx.x] += rk[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = rk[0];
}

// Half a step of the Nose-Hoover thermostat (time-reversible splitting):
// xi += dt/4 G(K); s = exp(-dt/2 xi); K -> s^2 K; eta += dt/2 xi;
// xi += dt/4 G(K), with G(K) = (2K - nf kT) / Q.  K: the sum of the
// kinetic-energy block partials (start of a step) or the thermo row's
// (end of a step, whose E_kin and pressure are then updated to the scaled
// velocities).  nh = {xi, eta, E_thermostat = Q xi^2 / 2 + nf kT eta, s};
// the velocities are scaled by s by the next kernel that reads them.
__global__ __launch_bounds__(64) void k_md_nh(int nblk, const double* __restrict__ ke_part, double* __restrict__ row,
                                              double* __restrict__ nh, MdNH p) {
  double K = 0.0;
  if (row) {
    K = row[2];
  } else {
    for (int b = threadIdx.x; b < nblk; b += 64) K += ke_part[b];
    K = md_wave_sum(K);
  }
  if (threadIdx.x != 0) return;
  const double g = p.nf * p.kT;
  double xi = nh[0], eta = nh[1];
  xi += 0.25 * p.dt * (2.0 * K - g) / p.Q;
  const double sc = exp(-0.5 * p.dt * xi);
  const double K2 = K * sc * sc;
  eta += 0.5 * p.dt * xi;
  xi += 0.25 * p.dt * (2.0 * K2 - g) / p.Q;
  nh[0] = xi;
  nh[1] = eta;
  nh[2] = 0.5 * p.Q * xi * xi + g * eta;
  nh[3] = sc;
  if (row) {
    row[3] += 2.0 * (K2 - K) / (3.0 * p.vol);
    row[2] = K2;
  }
}

// out = the LJ partial forces of the nch chunks summed in chunk order
// (multiple time steps keep the short-range forces on their own).
__global__ __launch_bounds__(kMdBlock) void k_md_lj_sum(int n, int nch, const double* __restrict__ fpart,
                                                        double* __restrict__ out) {
  const int i = blockIdx.x * kMdBlock + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) {
    double fk = 0.0;
    for (int c = 0; c < nch; ++c) fk += fpart[((long)c * n + i) * 3 + k];
    out[3 * i + k] = fk;
  }
}

// f = a + b (the caller's total force after a multiple-time-step run).
__global__ __launch_bounds__(kMdBlock) void k_md_add(int n, const double* __restrict__ a, const double* __restrict__ b,
                                                     double* __restrict__ f) {
  const int i = blockIdx.x * kMdBlock + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) f[3 * i + k] = a[3 * i + k] + b[3 * i + k];
}

// v *= s (the end-of-step thermostat scale).
__global__ __launch_bounds__(kMdBlock) void k_md_scale(int n, double* __restrict__ v, const double* __restrict__ nh) {
  const int i = blockIdx.x * kMdBlock + threadIdx.x;
  if (i >= n) return;
  const double sc = nh[3];
  for (int k = 0; k < 3; ++k) v[3 * i + k] *= sc;
}

// Structure of a configuration (the observables of the paper's MD runs).
// Pair-distance histogram: block (b, c) takes targets b * kMdBlock ... and
// the sources of chunk c, counts each pair i < j once, into LDS bins, then
// adds its nonzero bins to the caller's histogram.  Integer atomics: the
// counts do not depend on the order.  Every FP64 operation that decides a
// bin is rounded on its own (no contraction), so a CPU recomputation in the
// same order finds the same bin.
constexpr int kRdfMaxBins = 4096;
__global__ __launch_bounds__(kMdBlock) void k_md_rdf(int n, const double* __restrict__ x,
                                                     const double* __restrict__ q, MdBox box, int chunk,
                                                     int nbins, double rmax2, double dr,
                                                     unsigned long long* __restrict__ hist) {
  extern __shared__ unsigned int bins[];  // 3 x nbins
  for (int k = threadIdx.x; k < 3 * nbins; k += kMdBlock) bins[k] = 0u;
  __shared__ double sx[kMdBlock], sy[kMdBlock], sz[kMdBlock], sq[kMdBlock];
  const int i = blockIdx.x * kMdBlock + threadIdx.x;
  const bool ok = i < n;
  double xi = 0, yi = 0, zi = 0, qi = 0;
  if (ok) {
    xi = x[3 * i];
    yi = x[3 * i + 1];
    zi = x[3 * i + 2];
    qi = q[i];
  }
  const int jb = blockIdx.y * chunk, je = min(n, jb + chunk);
  for (int j0 = jb; j0 < je; j0 += kMdBlock) {
    const int j = j0 + threadIdx.x;
    __syncthreads();
    if (j < je) {
      sx[threadIdx.x] = x[3 * j];
      sy[threadIdx.x] = x[3 * j + 1];
      sz[threadIdx.x] = x[3 * j + 2];
      sq[threadIdx.x] = q[j];
    }
    __syncthreads();
    const int jn = min(kMdBlock, je - j0);
    if (!ok || qi == 0.0) continue;
    for (int jj = 0; jj < jn; ++jj) {
      if (j0 + jj <= i || sq[jj] == 0.0) continue;
      double dx = __dsub_rn(xi, sx[jj]), dy = __dsub_rn(yi, sy[jj]), dz = __dsub_rn(zi, sz[jj]);
      dx = __dsub_rn(dx, __dmul_rn(box.L[0], rint(__dmul_rn(dx, box.iL[0]))));
      dy = __dsub_rn(dy, __dmul_rn(box.L[1], rint(__dmul_rn(dy, box.iL[1]))));
      if (!box.slab) dz = __dsub_rn(dz, __dmul_rn(box.L[2], rint(__dmul_rn(dz, box.iL[2]))));
      const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
      if (!(r2 < rmax2)) continue;
      const int b = min(nbins - 1, (int)__ddiv_rn(__dsqrt_rn(r2), dr));
      const int cls = (qi > 0.0) == (sq[jj] > 0.0) ? (qi > 0.0 ? 0 : 2) : 1;
      atomicAdd(&bins[cls * nbins + b], 1u);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 3 * nbins; k += kMdBlock)
    if (bins[k]) atomicAdd(&hist[k], (unsigned long long)bins[k]);
}

// Density profile along z: bin floor((z - lo_z) / dz), clamped to the
// range; class 0 (q > 0) or 1 (q < 0).
__global__ __launch_bounds__(kMdBlock) void k_md_zprofile(int n, const double* __restrict__ x,
                                                          const double* __restrict__ q, double lo, double dz,
                                                          int nbins, unsigned long long* __restrict__ hist) {
  const int i = blockIdx.x * kMdBlock + threadIdx.x;
  if (i >= n || q[i] == 0.0) return;
  const int b = max(0, min(nbins - 1, (int)floor(__ddiv_rn(__dsub_rn(x[3 * i + 2], lo), dz))));
  atomicAdd(&hist[(q[i] > 0.0 ? 0 : 1) * nbins + b], 1ull);
}

// Thermo row: E_C, E_LJ, E_kin, P (fixed-order sums of the block partials).
__global__ __launch_bounds__(64) void k_md_thermo(int nblk, int nlj, const double* __restrict__ lj_part,
                                                  const double* __restrict__ ke_part,
                                                  const double* __restrict__ e_coul, double volume, int slab,
                                                  double* __restrict__ row) {
  const int lane = threadIdx.x;
  double elj = 0, wlj = 0, ke = 0;
  for (int b = lane; b < nlj; b += 64) {
    elj += lj_part[2 * b];
    wlj += lj_part[2 * b + 1];
  }
  for (int b = lane; b < nblk; b += 64) ke += ke_part[b];
  elj = md_wave_sum(elj);
  wlj = md_wave_sum(wlj);
  ke = md_wave_sum(ke);
  if (lane != 0) return;
  const double ec = *e_coul;
  row[0] = ec;
  row[1] = elj;
  row[2] = ke;
  row[3] = (2.0 * ke + wlj + (slab ? 0.0 : ec)) / (3.0 * volume);
}

}  // namespace
}  // namespace hsma

struct hsma_md {
  hsma_plan* plan = nullptr;
  hsma_md_params prm{};
  int64_t n = 0;
  hsma::MdBox box{};
  hsma::MdLJ lj{};
  int nblk = 0;
  int ljch = 1, ljchunk = 0;    // LJ source chunks and their size (a multiple of kMdBlock)
  double* d_lj_part = nullptr;  // 2 x nblk x ljch
  double* d_ljf = nullptr;      // ljch x n x 3: LJ partial forces by chunk
  double* d_ke_part = nullptr;  // nblk
  double* d_ecoul = nullptr;
  double* d_row = nullptr;      // 4: thermo row when the caller passes none
  double* d_nh = nullptr;       // 4: thermostat state {xi, eta, E_thermostat, scale}
  double* d_fc = nullptr;       // multiple time steps: Coulomb forces, n x 3
  double* d_flj = nullptr;      //   and short-range forces, n x 3, at the current positions
  bool split_valid = false;     //   (left by this driver's last run or forces call)
  bool nh_on = false;
  hsma::MdNH nh{};
  hipEvent_t ev = nullptr;      // end of the driver's last call (its kernels follow the plan's)
  bool recorded = false;
};

namespace {

// Start of a step: the thermostat's first half at the current velocities
// (whose scale the kick-drift applies), then v = s v + dt/2 F/m, x += dt v.
void md_begin_step(hsma_md* md, hipStream_t st, double* x, double* v, const double* f, const double* m) {
  const int n = (int)md->n;
  if (md->nh_on) {
    hipLaunchKernelGGL(hsma::k_md_kick, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, 0.0, v,
                       const_cast<double*>(f), m, (const double*)nullptr, 0, md->d_ke_part);
    hipLaunchKernelGGL(hsma::k_md_nh, dim3(1), dim3(64), 0, st, md->nblk, (const double*)md->d_ke_part,
                       (double*)nullptr, md->d_nh, md->nh);
  }
  hipLaunchKernelGGL(hsma::k_md_kick_drift, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, md->prm.dt, md->prm.dt, x,
                     v, f, m,
                     md->box, md->nh_on ? (const double*)(md->d_nh + 3) : (const double*)nullptr);
}

// F += F_LJ at x (pairs by source chunks, summed into f by the kick),
// v += dt/2 F/m (dt = 0: v unchanged, may be NULL), one thermo row.
void md_lj_kick_thermo(hsma_md* md, hipStream_t st, const double* x, double* v, double* f, const double* m,
                       double dt, const double* e_coul, double* row) {
  const int n = (int)md->n;
  hipLaunchKernelGGL(hsma::k_md_lj, dim3(md->nblk, md->ljch), dim3(hsma::kMdBlock), 0, st, n, x, md->box, md->lj,
                     md->ljchunk, md->d_ljf, md->d_lj_part);
  hipLaunchKernelGGL(hsma::k_md_kick, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, dt, v, f, m,
                     (const double*)md->d_ljf, md->ljch, md->d_ke_part);
  const double vol = md->box.L[0] * md->box.L[1] * md->box.L[2];
  hipLaunchKernelGGL(hsma::k_md_thermo, dim3(1), dim3(64), 0, st, md->nblk, md->nblk * md->ljch,
                     (const double*)md->d_lj_part, (const double*)md->d_ke_part, e_coul, vol, md->box.slab, row);
}

// End of a step, once f holds the Coulomb forces at x and d_e_coulomb their
// energy: F += F_LJ, v += dt/2 F/m, the thermo row, then the thermostat's
// second half (row updated, v scaled).
void md_end_step(hsma_md* md, hipStream_t st, const double* x, double* v, double* f, const double* m,
                 const double* e_coul, double* row) {
  const int n = (int)md->n;
  md_lj_kick_thermo(md, st, x, v, f, m, md->prm.dt, e_coul, row);
  if (md->nh_on) {
    hipLaunchKernelGGL(hsma::k_md_nh, dim3(1), dim3(64), 0, st, 0, (const double*)nullptr, row, md->d_nh, md->nh);
    hipLaunchKernelGGL(hsma::k_md_scale, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, v, (const double*)md->d_nh);
  }
}

// F_LJ at x into d_flj (pairs by source chunks, the chunks summed in order).
void md_short_range_split(hsma_md* md, hipStream_t st, const double* x) {
  const int n = (int)md->n;
  hipLaunchKernelGGL(hsma::k_md_lj, dim3(md->nblk, md->ljch), dim3(hsma::kMdBlock), 0, st, n, x, md->box, md->lj,
                     md->ljchunk, md->d_ljf, md->d_lj_part);
  hipLaunchKernelGGL(hsma::k_md_lj_sum, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, md->ljch,
                     (const double*)md->d_ljf, md->d_flj);
}

// v += dt/2 F/m (dt = 0: v unchanged, may be NULL) with the per-block kinetic
// energies, then the thermo row from the last LJ evaluation and E_C.
void md_kick_thermo(hsma_md* md, hipStream_t st, double* v, const double* f, const double* m, double dt,
                    const double* e_coul, double* row) {
  const int n = (int)md->n;
  hipLaunchKernelGGL(hsma::k_md_kick, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, dt, v, const_cast<double*>(f), m,
                     (const double*)nullptr, 0, md->d_ke_part);
  const double vol = md->box.L[0] * md->box.L[1] * md->box.L[2];
  hipLaunchKernelGGL(hsma::k_md_thermo, dim3(1), dim3(64), 0, st, md->nblk, md->nblk * md->ljch,
                     (const double*)md->d_lj_part, (const double*)md->d_ke_part, e_coul, vol, md->box.slab, row);
}

// One outer step of the multiple-time-step (reversible RESPA) integrator:
// the Coulomb forces kick for dt/2 at both ends of the outer step, and in
// between respa_inner velocity-Verlet steps of dt / respa_inner move the
// particles under the short-range forces alone; the thermostat's halves
// wrap the outer step.  d_fc and d_flj hold the forces at x on entry and
// on exit.
hsma_status md_respa_step(hsma_md* md, hipStream_t st, double* x, double* v, const double* q, const double* m,
                          double* row, std::string& err) {
  const int n = (int)md->n;
  const int k = md->prm.respa_inner;
  const double dt = md->prm.dt, dti = dt / k;
  if (md->nh_on) {
    hipLaunchKernelGGL(hsma::k_md_kick, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, 0.0, v, md->d_fc, m,
                       (const double*)nullptr, 0, md->d_ke_part);
    hipLaunchKernelGGL(hsma::k_md_nh, dim3(1), dim3(64), 0, st, md->nblk, (const double*)md->d_ke_part,
                       (double*)nullptr, md->d_nh, md->nh);
  }
  // v = s v + dt/2 F_C/m
  hipLaunchKernelGGL(hsma::k_md_kick_drift, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, dt, 0.0, x, v,
                     (const double*)md->d_fc, m, md->box, md->nh_on ? (const double*)(md->d_nh + 3) : (const double*)nullptr);
  for (int j = 0; j < k; ++j) {
    hipLaunchKernelGGL(hsma::k_md_kick_drift, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, dti, dti, x, v,
                       (const double*)md->d_flj, m, md->box, (const double*)nullptr);
    md_short_range_split(md, st, x);
    if (j + 1 < k)
      hipLaunchKernelGGL(hsma::k_md_kick, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, dti, v, md->d_flj, m,
                         (const double*)nullptr, 0, md->d_ke_part);
  }
  // the last inner closing kick, then the Coulomb forces at the new x
  hipLaunchKernelGGL(hsma::k_md_kick, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, dti, v, md->d_flj, m,
                     (const double*)nullptr, 0, md->d_ke_part);
  hsma_status s = md->plan->dev.run(st, n, x, q, md->d_ecoul, nullptr, md->d_fc, err);
  if (s != HSMA_OK) return s;
  md_kick_thermo(md, st, v, md->d_fc, m, dt, md->d_ecoul, row);
  if (md->nh_on) {
    hipLaunchKernelGGL(hsma::k_md_nh, dim3(1), dim3(64), 0, st, 0, (const double*)nullptr, row, md->d_nh, md->nh);
    hipLaunchKernelGGL(hsma::k_md_scale, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, v, (const double*)md->d_nh);
  }
  return HSMA_OK;
}

// F = F_Coulomb (the plan's step) + F_LJ at x; one thermo row (E_kin from v).
// With multiple time steps the two parts are also kept apart (d_fc, d_flj).
hsma_status md_forces(hsma_md* md, hipStream_t st, const double* x, const double* v, double* f, const double* q,
                      const double* m, double* row, std::string& err) {
  const int n = (int)md->n;
  if (md->prm.respa_inner >= 2) {
    hsma_status s = md->plan->dev.run(st, n, x, q, md->d_ecoul, nullptr, md->d_fc, err);
    if (s != HSMA_OK) return s;
    md_short_range_split(md, st, x);
    md_kick_thermo(md, st, const_cast<double*>(v), md->d_flj, m, 0.0, md->d_ecoul, row ? row : md->d_row);
    hipLaunchKernelGGL(hsma::k_md_add, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, (const double*)md->d_fc,
                       (const double*)md->d_flj, f);
    md->split_valid = true;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      err = std::string("md kernels: ") + hipGetErrorString(e);
      return HSMA_ERR_DEVICE;
    }
    return HSMA_OK;
  }
  hsma_status s = md->plan->dev.run(st, n, x, q, md->d_ecoul, nullptr, f, err);
  if (s != HSMA_OK) return s;
  md_lj_kick_thermo(md, st, x, const_cast<double*>(v), f, m, 0.0, md->d_ecoul, row ? row : md->d_row);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("md kernels: ") + hipGetErrorString(e);
    return HSMA_ERR_DEVICE;
  }
  return HSMA_OK;
}

}  // namespace

extern "C" {

namespace {
hsma_status md_create(hsma_plan* plan, const hsma_md_params* p, int geometry, const double lo[3],
                      const double L[3], int64_t n, hsma_md** out);
}

hsma_status hsma_md_create(hsma_plan* plan, const hsma_md_params* p, int64_t n, hsma_md** out) {
  if (!plan || !p || !out) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (n < 2 || n > std::min(hsma::max_particles(plan->dev.host.prm.near_rule), hsma::kMdMaxParticles))
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "n out of range (2 to 2^26 particles)");
  const hsma::HostPlan& hp = plan->dev.host;
  const hsma_status s = md_create(plan, p, hp.prm.geometry, hp.lo, hp.L, n, out);
  if (s == HSMA_OK) plan->dev.use_graph = true;  // the Coulomb step replays from a captured graph
  return s;
}

hsma_status hsma_md_create_for_box(const hsma_md_params* p, int geometry, const double box_lo[3],
                                   const double box_len[3], int64_t n, hsma_md** out) {
  if (!p || !out || !box_lo || !box_len) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (n < 2 || n > hsma::kMdMaxParticles)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "n out of range (2 to 2^26 particles)");
  if (geometry != HSMA_GEOM_3D && geometry != HSMA_GEOM_2D)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "geometry must be HSMA_GEOM_3D or HSMA_GEOM_2D");
  for (int k = 0; k < 3; ++k)
    if (!(box_len[k] > 0) || !std::isfinite(box_len[k]) || !std::isfinite(box_lo[k]))
      return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "box lengths must be finite and positive");
  return md_create(nullptr, p, geometry, box_lo, box_len, n, out);
}

namespace {
hsma_status md_create(hsma_plan* plan, const hsma_md_params* p, int geometry, const double lo[3],
                      const double L[3], int64_t n, hsma_md** out) {
  if (!(p->dt > 0) || !std::isfinite(p->dt) || !(p->lj_epsilon >= 0) || !(p->lj_sigma > 0) || !(p->lj_rcut >= 0) ||
      !(p->wall_epsilon >= 0) || !(p->wall_rcut >= 0) || (p->wall_epsilon > 0 && !(p->wall_sigma > 0)) ||
      !(p->nh_kT >= 0) || !(p->nh_damping >= 0) || !std::isfinite(p->nh_kT) || !std::isfinite(p->nh_damping) ||
      ((p->nh_kT > 0) != (p->nh_damping > 0)) || p->respa_inner < 0 || p->respa_inner > 1000)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "invalid MD parameter");
  if (!plan && p->respa_inner >= 2)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "multiple time steps need a plan (hsma_md_run)");
  std::unique_ptr<hsma_md> md(new (std::nothrow) hsma_md());
  if (!md) return hsma::set_last_error(HSMA_ERR_OOM, "host allocation failed");
  md->plan = plan;
  md->prm = *p;
  md->n = n;
  for (int k = 0; k < 3; ++k) {
    md->box.lo[k] = lo[k];
    md->box.L[k] = L[k];
  }
  md->box.slab = geometry == HSMA_GEOM_2D;
  const double k6 = std::pow(2.0, 1.0 / 6.0);
  const double rc = p->lj_rcut > 0 ? p->lj_rcut : k6 * p->lj_sigma;
  const double half = 0.5 * std::min(L[0], std::min(L[1], md->box.slab ? INFINITY : L[2]));
  if (!(rc < half)) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "LJ cut-off must be below half a box edge");
  const double sr6 = std::pow(p->lj_sigma / rc, 6.0);
  md->lj.eps = p->lj_epsilon;
  md->lj.sig2 = p->lj_sigma * p->lj_sigma;
  md->lj.rc2 = rc * rc;
  {
    // FP32 distance error bound: positions rounded to FP32 (relative
    // 2^-24 each), their difference, the image shift and the products, at
    // most a few units of 2^-24 times the largest coordinate; 64 units of
    // margin over the box's largest extent plus its lower corner
    const double ext = std::max(std::max(L[0], L[1]), L[2]) +
                       std::max(std::max(std::fabs(lo[0]), std::fabs(lo[1])), std::fabs(lo[2]));
    const double rs = (rc + 64.0 * std::ldexp(1.0, -24) * ext) * (1.0 + 1e-6);
    md->lj.rc2_screen = (float)(rs * rs) * (1.0f + 1e-6f);
  }
  md->lj.shift = -4.0 * p->lj_epsilon * (sr6 * sr6 - sr6);
  md->lj.weps = p->wall_epsilon;
  md->lj.wsig = p->wall_sigma;
  md->lj.wrc = p->wall_epsilon > 0 ? (p->wall_rcut > 0 ? p->wall_rcut : k6 * p->wall_sigma) : 0.0;
  if (p->wall_epsilon > 0) {
    const double w6 = std::pow(p->wall_sigma / md->lj.wrc, 6.0);
    md->lj.wshift = -4.0 * p->wall_epsilon * (w6 * w6 - w6);
  }
  md->nblk = (int)((n + hsma::kMdBlock - 1) / hsma::kMdBlock);
  for (int k = 0; k < 3; ++k) md->box.iL[k] = 1.0 / L[k];
  // LJ work: about 1024 blocks of (targets, source chunk) where the system
  // is small enough, chunks of whole LDS tiles
  {
    const int want = std::max(1, std::min(md->nblk, (1024 + md->nblk - 1) / md->nblk));
    const int per = (int)((n + want - 1) / want);
    md->ljchunk = (per + hsma::kMdBlock - 1) / hsma::kMdBlock * hsma::kMdBlock;
    md->ljch = (int)((n + md->ljchunk - 1) / md->ljchunk);
  }
  // Nose-Hoover: degrees of freedom without the conserved momentum (3D:
  // 3; slab: x and y), thermostat mass nf kT tau^2
  md->nh_on = p->nh_kT > 0;
  md->nh.dt = p->dt;
  md->nh.kT = p->nh_kT;
  md->nh.nf = 3.0 * (double)n - (md->box.slab ? 2.0 : 3.0);
  md->nh.Q = md->nh.nf * p->nh_kT * p->nh_damping * p->nh_damping;
  md->nh.vol = L[0] * L[1] * L[2];
  if (hipMalloc((void**)&md->d_nh, sizeof(double) * 4) != hipSuccess ||
      hipMemset(md->d_nh, 0, sizeof(double) * 4) != hipSuccess ||
      hipMalloc((void**)&md->d_lj_part, sizeof(double) * 2 * md->nblk * md->ljch) != hipSuccess ||
      hipMalloc((void**)&md->d_ljf, sizeof(double) * 3 * (size_t)n * md->ljch) != hipSuccess ||
      hipMalloc((void**)&md->d_ke_part, sizeof(double) * md->nblk) != hipSuccess ||
      hipMalloc((void**)&md->d_ecoul, sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&md->d_row, sizeof(double) * 4) != hipSuccess ||
      (p->respa_inner >= 2 && (hipMalloc((void**)&md->d_fc, sizeof(double) * 3 * (size_t)n) != hipSuccess ||
                               hipMalloc((void**)&md->d_flj, sizeof(double) * 3 * (size_t)n) != hipSuccess)) ||
      hipEventCreateWithFlags(&md->ev, hipEventDisableTiming) != hipSuccess) {
    hsma_md_destroy(md.release());
    return hsma::set_last_error(HSMA_ERR_OOM, "device allocation failed");
  }
  *out = md.release();
  return HSMA_OK;
}
}  // namespace

hsma_status hsma_md_drift(hsma_md* md, void* stream, double* d_x, double* d_v, const double* d_f,
                          const double* d_m) {
  if (!md || !d_x || !d_v || !d_f || !d_m) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (md->prm.respa_inner >= 2)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "multiple time steps run through hsma_md_run only");
  md_begin_step(md, (hipStream_t)stream, d_x, d_v, d_f, d_m);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hsma::set_last_error(HSMA_ERR_DEVICE, std::string("md kernels: ") + hipGetErrorString(e));
  // the thermostat's half uses the driver's buffers: destroy waits for it
  if (hipEventRecord(md->ev, (hipStream_t)stream) != hipSuccess)
    return hsma::set_last_error(HSMA_ERR_DEVICE, "hipEventRecord failed");
  md->recorded = true;
  return HSMA_OK;
}

hsma_status hsma_md_finish(hsma_md* md, void* stream, const double* d_x, double* d_v, double* d_f,
                           const double* d_m, const double* d_e_coulomb, double* d_thermo_row) {
  if (!md || !d_x || !d_v || !d_f || !d_m || !d_e_coulomb)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (md->prm.respa_inner >= 2)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "multiple time steps run through hsma_md_run only");
  hipStream_t st = (hipStream_t)stream;
  md_end_step(md, st, d_x, d_v, d_f, d_m, d_e_coulomb, d_thermo_row ? d_thermo_row : md->d_row);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hsma::set_last_error(HSMA_ERR_DEVICE, std::string("md kernels: ") + hipGetErrorString(e));
  if (hipEventRecord(md->ev, st) != hipSuccess) return hsma::set_last_error(HSMA_ERR_DEVICE, "hipEventRecord failed");
  md->recorded = true;
  return HSMA_OK;
}

hsma_status hsma_md_short_range(hsma_md* md, void* stream, const double* d_x, const double* d_v, double* d_f,
                                const double* d_m, const double* d_e_coulomb, double* d_thermo_row) {
  if (!md || !d_x || !d_f || !d_m || !d_e_coulomb) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  md_lj_kick_thermo(md, st, d_x, const_cast<double*>(d_v), d_f, d_m, 0.0, d_e_coulomb,
                    d_thermo_row ? d_thermo_row : md->d_row);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hsma::set_last_error(HSMA_ERR_DEVICE, std::string("md kernels: ") + hipGetErrorString(e));
  if (hipEventRecord(md->ev, st) != hipSuccess) return hsma::set_last_error(HSMA_ERR_DEVICE, "hipEventRecord failed");
  md->recorded = true;
  return HSMA_OK;
}

hsma_status hsma_md_forces(hsma_md* md, void* stream, const double* d_x, const double* d_v, double* d_f,
                           const double* d_q, const double* d_m, double* d_thermo_row) {
  if (!md || !d_x || !d_f || !d_q || !d_m) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (!md->plan) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "this driver has no plan (hsma_md_create_for_box)");
  std::string err;
  const hsma_status s = md_forces(md, (hipStream_t)stream, d_x, d_v, d_f, d_q, d_m, d_thermo_row, err);
  if (s != HSMA_OK) return hsma::set_last_error(s, err);
  if (hipEventRecord(md->ev, (hipStream_t)stream) != hipSuccess)
    return hsma::set_last_error(HSMA_ERR_DEVICE, "hipEventRecord failed");
  md->recorded = true;
  return HSMA_OK;
}

hsma_status hsma_md_run(hsma_md* md, void* stream, int nsteps, double* d_x, double* d_v, double* d_f,
                        const double* d_q, const double* d_m, int forces_valid, double* d_thermo) {
  if (!md || !d_x || !d_v || !d_f || !d_q || !d_m) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (nsteps < 0) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (!md->plan) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "this driver has no plan (hsma_md_create_for_box)");
  hipStream_t st = (hipStream_t)stream;
  std::string err;
  hsma_status s;
  const bool respa = md->prm.respa_inner >= 2;
  // multiple time steps need the two force parts, which only this driver's
  // own last run or forces call leaves
  if ((!forces_valid || (respa && !md->split_valid)) &&
      (s = md_forces(md, st, d_x, d_v, d_f, d_q, d_m, nullptr, err)) != HSMA_OK)
    return hsma::set_last_error(s, err);
  const int n = (int)md->n;
  if (respa) {
    for (int step = 0; step < nsteps; ++step) {
      s = md_respa_step(md, st, d_x, d_v, d_q, d_m, d_thermo ? d_thermo + 4 * (size_t)step : md->d_row, err);
      if (s != HSMA_OK) return hsma::set_last_error(s, err);
    }
    hipLaunchKernelGGL(hsma::k_md_add, dim3(md->nblk), dim3(hsma::kMdBlock), 0, st, n, (const double*)md->d_fc,
                       (const double*)md->d_flj, d_f);
    nsteps = 0;
  }
  for (int step = 0; step < nsteps; ++step) {
    md_begin_step(md, st, d_x, d_v, d_f, d_m);
    s = md->plan->dev.run(st, n, d_x, d_q, md->d_ecoul, nullptr, d_f, err);
    if (s != HSMA_OK) return hsma::set_last_error(s, err);
    md_end_step(md, st, d_x, d_v, d_f, d_m, md->d_ecoul, d_thermo ? d_thermo + 4 * (size_t)step : md->d_row);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hsma::set_last_error(HSMA_ERR_DEVICE, std::string("md kernels: ") + hipGetErrorString(e));
  if (hipEventRecord(md->ev, st) != hipSuccess) return hsma::set_last_error(HSMA_ERR_DEVICE, "hipEventRecord failed");
  md->recorded = true;
  return HSMA_OK;
}

hsma_status hsma_md_thermostat(hsma_md* md, void* stream, double* d_state) {
  if (!md || !d_state) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (md->recorded && hipStreamWaitEvent((hipStream_t)stream, md->ev, 0) != hipSuccess)
    return hsma::set_last_error(HSMA_ERR_DEVICE, "hipStreamWaitEvent failed");
  if (hipMemcpyAsync(d_state, md->d_nh, sizeof(double) * 3, hipMemcpyDeviceToDevice, (hipStream_t)stream) !=
      hipSuccess)
    return hsma::set_last_error(HSMA_ERR_DEVICE, "hipMemcpyAsync failed");
  return HSMA_OK;
}

hsma_status hsma_md_rdf(hsma_md* md, void* stream, const double* d_x, const double* d_q, int nbins, double r_max,
                        unsigned long long* d_hist) {
  if (!md || !d_x || !d_q || !d_hist) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (nbins < 1 || nbins > hsma::kRdfMaxBins)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "nbins must be in [1, 4096]");
  const double half = 0.5 * std::min(md->box.L[0], std::min(md->box.L[1], md->box.slab ? INFINITY : md->box.L[2]));
  if (!(r_max > 0) || !(r_max <= half))
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "r_max must be in (0, half the smallest periodic box edge]");
  const int n = (int)md->n;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(hsma::k_md_rdf, dim3(md->nblk, md->ljch), dim3(hsma::kMdBlock),
                     sizeof(unsigned int) * 3 * (size_t)nbins, st, n, d_x, d_q, md->box, md->ljchunk, nbins,
                     r_max * r_max, r_max / nbins, d_hist);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hsma::set_last_error(HSMA_ERR_DEVICE, std::string("md kernels: ") + hipGetErrorString(e));
  return HSMA_OK;
}

hsma_status hsma_md_zprofile(hsma_md* md, void* stream, const double* d_x, const double* d_q, int nbins,
                             unsigned long long* d_hist) {
  if (!md || !d_x || !d_q || !d_hist) return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "NULL argument");
  if (nbins < 1 || nbins > hsma::kRdfMaxBins)
    return hsma::set_last_error(HSMA_ERR_INVALID_ARG, "nbins must be in [1, 4096]");
  const int n = (int)md->n;
  hipLaunchKernelGGL(hsma::k_md_zprofile, dim3(md->nblk), dim3(hsma::kMdBlock), 0, (hipStream_t)stream, n, d_x, d_q,
                     md->box.lo[2], md->box.L[2] / nbins, nbins, d_hist);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hsma::set_last_error(HSMA_ERR_DEVICE, std::string("md kernels: ") + hipGetErrorString(e));
  return HSMA_OK;
}

void hsma_md_destroy(hsma_md* md) {
  if (!md) return;
  if (md->recorded) (void)hipEventSynchronize(md->ev);  // after the plan's work on the same stream
  void* ps[] = {md->d_lj_part, md->d_ljf, md->d_ke_part, md->d_ecoul, md->d_row, md->d_nh, md->d_fc, md->d_flj};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (md->ev) (void)hipEventDestroy(md->ev);
  delete md;
}

}  // extern "C"
