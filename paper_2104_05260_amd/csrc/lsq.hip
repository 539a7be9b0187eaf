// Least-squares pseudo-inverse on the device: CholeskyQR2 in FP64, the Gram
// matrices on the matrix cores (v_mfma_f64_16x16x4f64), grouped over
// several matrices (plan classes with different p, rows, geometry) per
// launch.
//
// For a fitting matrix M (rows x cols, full column rank) of Eq. 6 the plan
// needs P = R^-1 Q^T with M = Q R.  CholeskyQR2: G = M^T M = R1^T R1
// (Cholesky), Q1 = M R1^-1; G2 = Q1^T Q1 = R2^T R2, Q = Q1 R2^-1; R = R2 R1.
// One pass loses accuracy like cond(M)^2; the second pass restores
// orthogonality to rounding for cond(M) up to about 1e8 (the plans here have
// cond 1e2 - 1e4).  P = R^-1 Q^T by back substitution, one row of Q per
// thread.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "device.h"

namespace hsma {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// One matrix of the group: M (rows x cols, row-major), work arrays.
struct LsqDesc {
  const double* M;
  double* Q;     // rows x cols
  double* G;     // cols x cols
  double* R1;    // cols x cols (upper)
  double* R2;    // cols x cols (upper)
  double* P;     // cols x rows
  int* bad;      // set when a Cholesky pivot is not positive
  int rows, cols;
};

// A 16 x 16 tile (ti, tj), ti <= tj, of one group's Gram matrix.
struct GramTile {
  int g, ti, tj;
};

// G = A^T A for the tiles of the work list, one wave per tile.  Per step of
// four rows the matrix core takes a 16 x 4 block of A^T and a 4 x 16 block
// of A: lane l supplies A^T[l % 16][l / 16] = A[r0 + l / 16][16 ti + l % 16]
// and A[r0 + l / 16][16 tj + l % 16]; it receives G rows 4 v + l / 16,
// column l % 16 (v = 0..3; layout checked on gfx950).  The tile is written
// to (ti, tj) and mirrored.
__global__ __launch_bounds__(64) void k_gram(const LsqDesc* __restrict__ gd, const GramTile* __restrict__ tiles,
                                             int use_q) {
  const GramTile t = tiles[blockIdx.x];
  const LsqDesc d = gd[t.g];
  const double* __restrict__ A = use_q ? d.Q : d.M;
  const int l = threadIdx.x;
  const int ci = 16 * t.ti + (l & 15), cj = 16 * t.tj + (l & 15);
  const bool okI = ci < d.cols, okJ = cj < d.cols;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = 0; r0 < d.rows; r0 += 4) {
    const int r = r0 + (l >> 4);
    const bool okr = r < d.rows;
    const double a = (okr && okI) ? A[(long)r * d.cols + ci] : 0.0;
    const double b = (okr && okJ) ? A[(long)r * d.cols + cj] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  for (int v = 0; v < 4; ++v) {
    const int row = 16 * t.ti + 4 * v + (l >> 4);
    if (row < d.cols && okJ) {
      d.G[(long)row * d.cols + cj] = acc[v];
      d.G[(long)cj * d.cols + row] = acc[v];
    }
  }
}

// Cholesky G = R^T R (R upper), one block per group, column by column:
// R[j][j] = sqrt(G[j][j] - sum_k<j R[k][j]^2),
// R[j][i] = (G[j][i] - sum_k<j R[k][j] R[k][i]) / R[j][j], i > j.
__global__ __launch_bounds__(256) void k_chol(const LsqDesc* __restrict__ gd, int second) {
  const LsqDesc d = gd[blockIdx.x];
  double* __restrict__ R = second ? d.R2 : d.R1;
  const int n = d.cols, tid = threadIdx.x;
  __shared__ double red[256];
  __shared__ double diag;
  for (int i = tid; i < n * n; i += 256) R[i] = 0.0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int k = tid; k < j; k += 256) s += R[(long)k * n + j] * R[(long)k * n + j];
    red[tid] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    if (tid == 0) {
      const double g = d.G[(long)j * n + j];
      const double p = g - red[0];
      if (!(p > 1e-28 * fabs(g)) || !(p > 0.0)) *d.bad = 1;
      diag = sqrt(fmax(p, 1e-300));
      R[(long)j * n + j] = diag;
    }
    __syncthreads();
    const double rjj = diag;
    for (int i = j + 1 + tid; i < n; i += 256) {
      double a = d.G[(long)j * n + i];
      for (int k = 0; k < j; ++k) a -= R[(long)k * n + j] * R[(long)k * n + i];
      R[(long)j * n + i] = a / rjj;
    }
    __syncthreads();
  }
}

// One row of A per thread, over the flat row list of all groups:
// mode 0: Q[r] = M[r] R1^-1;  mode 1: Q[r] = Q[r] R2^-1 (in place);
// mode 2: P[:, r] = R^-1 Q[r]^T with R = R2 R1 held in R1.
struct RowItem {
  int g, r;
};
__global__ __launch_bounds__(256) void k_rows(const LsqDesc* __restrict__ gd, const RowItem* __restrict__ items,
                                              int nitems, int mode) {
  const int it = blockIdx.x * 256 + threadIdx.x;
  if (it >= nitems) return;
  const RowItem ri = items[it];
  const LsqDesc d = gd[ri.g];
  const int n = d.cols;
  if (mode <= 1) {
    // forward substitution q R = a, written into Q's row
    const double* __restrict__ R = mode == 0 ? d.R1 : d.R2;
    const double* __restrict__ a = (mode == 0 ? d.M : d.Q) + (long)ri.r * n;
    double* __restrict__ q = d.Q + (long)ri.r * n;
    for (int i = 0; i < n; ++i) {
      double s = a[i];
      for (int k = 0; k < i; ++k) s -= q[k] * R[(long)k * n + i];
      q[i] = s / R[(long)i * n + i];
    }
  } else {
    // back substitution R x = q; x is column r of P (cols x rows)
    const double* __restrict__ R = d.R1;
    const double* __restrict__ q = d.Q + (long)ri.r * n;
    double* __restrict__ P = d.P;
    const long ld = d.rows;
    for (int i = n - 1; i >= 0; --i) {
      double s = q[i];
      for (int k = i + 1; k < n; ++k) s -= R[(long)i * n + k] * P[(long)k * ld + ri.r];
      P[(long)i * ld + ri.r] = s / R[(long)i * n + i];
    }
  }
}

// R1 <- R2 R1 (both upper triangular), one block per group; the product is
// built in G (free after the second Cholesky) and copied back.
__global__ __launch_bounds__(256) void k_rmul(const LsqDesc* __restrict__ gd) {
  const LsqDesc d = gd[blockIdx.x];
  const int n = d.cols;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i = e / n, j = e - i * n;
    double s = 0.0;
    for (int k = i; k <= j; ++k) s += d.R2[(long)i * n + k] * d.R1[(long)k * n + j];
    d.G[e] = j >= i ? s : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += 256) d.R1[e] = d.G[e];
}

#define LSQCHK(x)                                                      \
  do {                                                                 \
    hipError_t e_ = (x);                                               \
    if (e_ != hipSuccess) {                                            \
      err = std::string(#x) + ": " + hipGetErrorString(e_);            \
      status = e_ == hipErrorOutOfMemory ? HSMA_ERR_OOM : HSMA_ERR_DEVICE; \
      goto done;                                                       \
    }                                                                  \
  } while (0)

}  // namespace

hsma_status device_pinv_batch(std::vector<LsqJob>& jobs, std::string& err) {
  hsma_status status = HSMA_OK;
  const int ng = (int)jobs.size();
  if (ng == 0) return HSMA_OK;
  std::vector<LsqDesc> gd(ng);
  std::vector<GramTile> tiles;
  std::vector<RowItem> rows;
  std::vector<void*> owned;
  hipStream_t st = nullptr;
  LsqDesc* d_gd = nullptr;
  GramTile* d_tiles = nullptr;
  RowItem* d_rows = nullptr;
  int* d_bad = nullptr;
  std::vector<int> bad(ng, 0);
  auto dalloc = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 8)) != hipSuccess) return nullptr;
    owned.push_back(p);
    return p;
  };
  for (const LsqJob& j : jobs) {
    if (j.rows < j.cols || j.cols < 1) {
      err = "least-squares matrix has fewer rows than columns";
      return HSMA_ERR_RANK;
    }
  }
  LSQCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  LSQCHK(hipMalloc((void**)&d_bad, sizeof(int) * ng));
  LSQCHK(hipMemsetAsync(d_bad, 0, sizeof(int) * ng, st));
  for (int g = 0; g < ng; ++g) {
    const LsqJob& j = jobs[g];
    const size_t rc = (size_t)j.rows * j.cols, cc = (size_t)j.cols * j.cols;
    LsqDesc& d = gd[g];
    d.rows = j.rows;
    d.cols = j.cols;
    double* M = (double*)dalloc(sizeof(double) * rc);
    d.Q = (double*)dalloc(sizeof(double) * rc);
    d.G = (double*)dalloc(sizeof(double) * cc);
    d.R1 = (double*)dalloc(sizeof(double) * cc);
    d.R2 = (double*)dalloc(sizeof(double) * cc);
    d.P = (double*)dalloc(sizeof(double) * rc);
    if (!M || !d.Q || !d.G || !d.R1 || !d.R2 || !d.P) {
      err = "device allocation for the least-squares factorisation failed";
      status = HSMA_ERR_OOM;
      goto done;
    }
    d.M = M;
    d.bad = d_bad + g;
    LSQCHK(hipMemcpyAsync(M, j.M->data(), sizeof(double) * rc, hipMemcpyHostToDevice, st));
    const int nt = (j.cols + 15) / 16;
    for (int ti = 0; ti < nt; ++ti)
      for (int tj = ti; tj < nt; ++tj) tiles.push_back(GramTile{g, ti, tj});
    for (int r = 0; r < j.rows; ++r) rows.push_back(RowItem{g, r});
  }
  d_gd = (LsqDesc*)dalloc(sizeof(LsqDesc) * ng);
  d_tiles = (GramTile*)dalloc(sizeof(GramTile) * tiles.size());
  d_rows = (RowItem*)dalloc(sizeof(RowItem) * rows.size());
  if (!d_gd || !d_tiles || !d_rows) {
    err = "device allocation for the least-squares factorisation failed";
    status = HSMA_ERR_OOM;
    goto done;
  }
  LSQCHK(hipMemcpyAsync(d_gd, gd.data(), sizeof(LsqDesc) * ng, hipMemcpyHostToDevice, st));
  LSQCHK(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(GramTile) * tiles.size(), hipMemcpyHostToDevice, st));
  LSQCHK(hipMemcpyAsync(d_rows, rows.data(), sizeof(RowItem) * rows.size(), hipMemcpyHostToDevice, st));
  {
    const int nrow = (int)rows.size(), rblk = (nrow + 255) / 256;
    // pass 1: G = M^T M, R1, Q1 = M R1^-1
    hipLaunchKernelGGL(k_gram, dim3((unsigned)tiles.size()), dim3(64), 0, st, (const LsqDesc*)d_gd,
                       (const GramTile*)d_tiles, 0);
    hipLaunchKernelGGL(k_chol, dim3(ng), dim3(256), 0, st, (const LsqDesc*)d_gd, 0);
    hipLaunchKernelGGL(k_rows, dim3(rblk), dim3(256), 0, st, (const LsqDesc*)d_gd, (const RowItem*)d_rows, nrow, 0);
    // pass 2: G2 = Q1^T Q1, R2, Q = Q1 R2^-1, R = R2 R1
    hipLaunchKernelGGL(k_gram, dim3((unsigned)tiles.size()), dim3(64), 0, st, (const LsqDesc*)d_gd,
                       (const GramTile*)d_tiles, 1);
    hipLaunchKernelGGL(k_chol, dim3(ng), dim3(256), 0, st, (const LsqDesc*)d_gd, 1);
    hipLaunchKernelGGL(k_rows, dim3(rblk), dim3(256), 0, st, (const LsqDesc*)d_gd, (const RowItem*)d_rows, nrow, 1);
    hipLaunchKernelGGL(k_rmul, dim3(ng), dim3(256), 0, st, (const LsqDesc*)d_gd);
    // P = R^-1 Q^T
    hipLaunchKernelGGL(k_rows, dim3(rblk), dim3(256), 0, st, (const LsqDesc*)d_gd, (const RowItem*)d_rows, nrow, 2);
    LSQCHK(hipGetLastError());
  }
  for (int g = 0; g < ng; ++g) {
    LsqJob& j = jobs[g];
    j.P->assign((size_t)j.rows * j.cols, 0.0);
    j.Rdiag.assign(j.cols, 0.0);
    LSQCHK(hipMemcpyAsync(j.P->data(), gd[g].P, sizeof(double) * j.P->size(), hipMemcpyDeviceToHost, st));
    for (int i = 0; i < j.cols; ++i)
      LSQCHK(hipMemcpyAsync(&j.Rdiag[i], gd[g].R1 + (size_t)i * j.cols + i, sizeof(double), hipMemcpyDeviceToHost,
                            st));
  }
  LSQCHK(hipMemcpyAsync(bad.data(), d_bad, sizeof(int) * ng, hipMemcpyDeviceToHost, st));
  LSQCHK(hipStreamSynchronize(st));
  for (int g = 0; g < ng; ++g) {
    LsqJob& j = jobs[g];
    double dmax = 0, dmin = 1e300;
    for (double v : j.Rdiag) {
      dmax = std::max(dmax, std::fabs(v));
      dmin = std::min(dmin, std::fabs(v));
    }
    j.cond = dmin > 0 ? dmax / dmin : INFINITY;
    j.ok = !bad[g] && dmin > 1e-12 * dmax;
  }
done:
  if (st) (void)hipStreamSynchronize(st);
  for (void* p : owned) (void)hipFree(p);
  if (d_bad) (void)hipFree(d_bad);
  if (st) (void)hipStreamDestroy(st);
  return status;
}

}  // namespace hsma
