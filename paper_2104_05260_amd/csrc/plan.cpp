// Host FP64 plan of the HSMA hot path: check points, image tables, the
// harmonic basis, the least-squares pseudo-inverse and the surface maps.
// Runs once per (box, parameters); nothing here is on the per-step path.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "hsma_internal.h"

namespace hsma {

namespace {

constexpr double kPi = 3.14159265358979323846;

bool is_fibonacci(int F, int* prev) {
  int a = 1, b = 2;
  while (b < F) {
    int c = a + b;
    a = b;
    b = c;
  }
  if (b == F && F > 2) {
    *prev = a;
    return true;
  }
  return false;
}

int zaremba(int F, int g) {
  int best = F;
  for (int h2 = 1; h2 <= F / 2; ++h2) {
    long long h1 = (-(long long)g * h2) % F;
    if (h1 < 0) h1 += F;
    if (h1 > F / 2) h1 -= F;
    long long v = std::max<long long>(1, std::llabs(h1)) * h2;
    if (v < best) best = (int)v;
  }
  return best;
}

}  // namespace

int lattice_generator(int F, int Fw) {
  if (Fw > 0) return Fw;
  int prev;
  if (is_fibonacci(F, &prev)) return prev;
  int best_g = 1, best = -1;
  for (int g = 1; g <= F / 2; ++g) {
    int z = zaremba(F, g);
    if (z > best) {
      best = z;
      best_g = g;
    }
  }
  return best_g;
}

// Regular solid harmonics R_n^m = r^n P_n^m(cos t) e^{i m phi} / (n+m)!
// through the three-term recurrence
//   R_m^m     = -(x + i y)/(2m) R_{m-1}^{m-1}
//   R_{m+1}^m = z R_m^m
//   R_n^m     = ((2n-1) z R_{n-1}^m - r^2 R_{n-2}^m) / ((n+m)(n-m)),
// differentiated term by term for the gradients.  Each real part is scaled
// by sqrt((2n+1)(n-m)!(n+m)!/(4 pi)) (times sqrt 2 for m > 0) so that the
// functions are orthonormal on the unit sphere.
void solid_harmonics(int p, const double xi[3], double* val, double* grad) {
  typedef std::complex<double> C;
  const double x = xi[0], y = xi[1], z = xi[2];
  const double r2 = x * x + y * y + z * z;
  const int W = p + 1;
  std::vector<C> Rv(W * W, C(0, 0));
  std::vector<C> Rg(grad ? 3 * W * W : 0, C(0, 0));
  auto at = [W](int n, int m) { return n * W + m; };
  Rv[at(0, 0)] = 1.0;
  const C xpiy(x, y);
  for (int m = 0; m <= p; ++m) {
    if (m > 0) {
      Rv[at(m, m)] = -xpiy / (2.0 * m) * Rv[at(m - 1, m - 1)];
      if (grad) {
        for (int k = 0; k < 3; ++k) {
          C e = (k == 0) ? C(1, 0) : (k == 1 ? C(0, 1) : C(0, 0));
          Rg[3 * at(m, m) + k] = -(e * Rv[at(m - 1, m - 1)] + xpiy * Rg[3 * at(m - 1, m - 1) + k]) / (2.0 * m);
        }
      }
    }
    if (m + 1 <= p) {
      Rv[at(m + 1, m)] = z * Rv[at(m, m)];
      if (grad)
        for (int k = 0; k < 3; ++k)
          Rg[3 * at(m + 1, m) + k] = (k == 2 ? Rv[at(m, m)] : C(0, 0)) + z * Rg[3 * at(m, m) + k];
    }
    for (int n = m + 2; n <= p; ++n) {
      const double den = double(n + m) * double(n - m);
      Rv[at(n, m)] = ((2.0 * n - 1.0) * z * Rv[at(n - 1, m)] - r2 * Rv[at(n - 2, m)]) / den;
      if (grad) {
        for (int k = 0; k < 3; ++k) {
          const double xk = xi[k];
          C t = (2.0 * n - 1.0) * ((k == 2 ? Rv[at(n - 1, m)] : C(0, 0)) + z * Rg[3 * at(n - 1, m) + k]) -
                2.0 * xk * Rv[at(n - 2, m)] - r2 * Rg[3 * at(n - 2, m) + k];
          Rg[3 * at(n, m) + k] = t / den;
        }
      }
    }
  }
  int j = 0;
  for (int n = 1; n <= p; ++n) {
    for (int m = 0; m <= n; ++m) {
      double lf = std::lgamma(n - m + 1.0) + std::lgamma(n + m + 1.0);
      double c = std::sqrt((2.0 * n + 1.0) / (4.0 * kPi)) * std::exp(0.5 * lf);
      if (m > 0) c *= std::sqrt(2.0);
      const C v = Rv[at(n, m)];
      val[j] = c * v.real();
      if (grad)
        for (int k = 0; k < 3; ++k) grad[3 * j + k] = c * Rg[3 * at(n, m) + k].real();
      ++j;
      if (m > 0) {
        val[j] = c * v.imag();
        if (grad)
          for (int k = 0; k < 3; ++k) grad[3 * j + k] = c * Rg[3 * at(n, m) + k].imag();
        ++j;
      }
    }
  }
}

namespace {

// Householder QR of a (rows x cols, row-major) with cols <= rows.  Returns
// the thin-Q pseudo-inverse P = R^{-1} Q^T (cols x rows, row-major).
bool pseudo_inverse(std::vector<double> a, int rows, int cols, std::vector<double>& P, double& cond) {
  std::vector<double> vs(size_t(rows) * cols, 0.0);  // Householder vectors (column j in vs[:, j])
  std::vector<double> beta(cols, 0.0);
  std::vector<double> Rdiag(cols);
  for (int j = 0; j < cols; ++j) {
    double nrm = 0;
    for (int i = j; i < rows; ++i) nrm += a[size_t(i) * cols + j] * a[size_t(i) * cols + j];
    nrm = std::sqrt(nrm);
    double a0 = a[size_t(j) * cols + j];
    double alpha = (a0 > 0) ? -nrm : nrm;
    // v = x - alpha e1
    double vnorm2 = 0;
    for (int i = j; i < rows; ++i) {
      double v = a[size_t(i) * cols + j] - (i == j ? alpha : 0.0);
      vs[size_t(i) * cols + j] = v;
      vnorm2 += v * v;
    }
    beta[j] = vnorm2 > 0 ? 2.0 / vnorm2 : 0.0;
    for (int c = j; c < cols; ++c) {
      double s = 0;
      for (int i = j; i < rows; ++i) s += vs[size_t(i) * cols + j] * a[size_t(i) * cols + c];
      s *= beta[j];
      for (int i = j; i < rows; ++i) a[size_t(i) * cols + c] -= s * vs[size_t(i) * cols + j];
    }
    Rdiag[j] = a[size_t(j) * cols + j];
  }
  double dmax = 0, dmin = 1e300;
  for (int j = 0; j < cols; ++j) {
    dmax = std::max(dmax, std::fabs(Rdiag[j]));
    dmin = std::min(dmin, std::fabs(Rdiag[j]));
  }
  cond = dmin > 0 ? dmax / dmin : INFINITY;
  if (!(dmin > 1e-12 * dmax)) return false;
  // Q^T (cols x rows): apply the reflections H_{cols-1} ... H_0 to e_r for
  // every r is costly; instead build Qthin (rows x cols) = H_0 ... H_{cols-1} [I; 0].
  std::vector<double> Q(size_t(rows) * cols, 0.0);
  for (int j = 0; j < cols; ++j) Q[size_t(j) * cols + j] = 1.0;
  for (int j = cols - 1; j >= 0; --j) {
    for (int c = 0; c < cols; ++c) {
      double s = 0;
      for (int i = j; i < rows; ++i) s += vs[size_t(i) * cols + j] * Q[size_t(i) * cols + c];
      s *= beta[j];
      for (int i = j; i < rows; ++i) Q[size_t(i) * cols + c] -= s * vs[size_t(i) * cols + j];
    }
  }
  // P = R^{-1} Q^T: for every row index r, solve R p = Q[r, :]^T.
  P.assign(size_t(cols) * rows, 0.0);
  std::vector<double> rhs(cols);
  for (int r = 0; r < rows; ++r) {
    for (int c = 0; c < cols; ++c) rhs[c] = Q[size_t(r) * cols + c];
    for (int c = cols - 1; c >= 0; --c) {
      double s = rhs[c];
      for (int k = c + 1; k < cols; ++k) s -= a[size_t(c) * cols + k] * rhs[k];
      rhs[c] = s / a[size_t(c) * cols + c];
    }
    for (int c = 0; c < cols; ++c) P[size_t(c) * rows + r] = rhs[c];
  }
  return true;
}

// Periodic spectral Dirichlet-to-Neumann operator on an nz x nz interface
// grid (index ix * nz + iy): out = DFT^-1 diag(|G|) DFT f, with
// G = 2 pi (mx / Lx, my / Ly), mx, my the signed frequencies.  Separable
// direct transforms with cosine/sine tables.
struct DtN {
  int nz;
  std::vector<double> cs, sn, G;
  DtN(int n, double Lx, double Ly) : nz(n), cs(size_t(n) * n), sn(size_t(n) * n), G(size_t(n) * n) {
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        const double t = 2.0 * kPi * double((long long)a * b % n) / n;
        cs[size_t(a) * n + b] = std::cos(t);
        sn[size_t(a) * n + b] = std::sin(t);
      }
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        const double ma = (a <= n / 2) ? a : a - n;
        const double mb = (b <= n / 2) ? b : b - n;
        G[size_t(a) * n + b] = 2.0 * kPi * std::sqrt((ma / Lx) * (ma / Lx) + (mb / Ly) * (mb / Ly));
      }
  }
  void apply(const double* f, double* out) const {
    const int n = nz;
    std::vector<double> ar(size_t(n) * n), ai(size_t(n) * n), br(size_t(n) * n), bi(size_t(n) * n);
    // forward along iy: A[ix][my] = sum_iy f e^{-i 2pi my iy / n}
    for (int ix = 0; ix < n; ++ix)
      for (int my = 0; my < n; ++my) {
        double sr = 0, si = 0;
        for (int iy = 0; iy < n; ++iy) {
          const double v = f[size_t(ix) * n + iy];
          sr += v * cs[size_t(my) * n + iy];
          si -= v * sn[size_t(my) * n + iy];
        }
        ar[size_t(ix) * n + my] = sr;
        ai[size_t(ix) * n + my] = si;
      }
    // forward along ix, times |G|
    for (int mx = 0; mx < n; ++mx)
      for (int my = 0; my < n; ++my) {
        double sr = 0, si = 0;
        for (int ix = 0; ix < n; ++ix) {
          const double c = cs[size_t(mx) * n + ix], s = sn[size_t(mx) * n + ix];
          const double xr = ar[size_t(ix) * n + my], xi = ai[size_t(ix) * n + my];
          sr += xr * c + xi * s;
          si += xi * c - xr * s;
        }
        const double g = G[size_t(mx) * n + my];
        br[size_t(mx) * n + my] = g * sr;
        bi[size_t(mx) * n + my] = g * si;
      }
    // inverse along mx
    for (int ix = 0; ix < n; ++ix)
      for (int my = 0; my < n; ++my) {
        double sr = 0, si = 0;
        for (int mx = 0; mx < n; ++mx) {
          const double c = cs[size_t(mx) * n + ix], s = sn[size_t(mx) * n + ix];
          const double xr = br[size_t(mx) * n + my], xi = bi[size_t(mx) * n + my];
          sr += xr * c - xi * s;
          si += xi * c + xr * s;
        }
        ar[size_t(ix) * n + my] = sr;
        ai[size_t(ix) * n + my] = si;
      }
    // inverse along my, real part
    const double scale = 1.0 / (double(n) * n);
    for (int ix = 0; ix < n; ++ix)
      for (int iy = 0; iy < n; ++iy) {
        double sr = 0;
        for (int my = 0; my < n; ++my) {
          const double c = cs[size_t(my) * n + iy], s = sn[size_t(my) * n + iy];
          sr += ar[size_t(ix) * n + my] * c - ai[size_t(ix) * n + my] * s;
        }
        out[size_t(ix) * n + iy] = sr * scale;
      }
  }
};

void surface_rule(int F, int Fw, int rule, double R, std::vector<double>& y, std::vector<double>& n,
                  std::vector<double>& w) {
  y.resize(3 * size_t(F));
  n.resize(3 * size_t(F));
  w.resize(F);
  std::vector<double> th(F), ph(F);
  if (rule == 0) {
    const int g = lattice_generator(F, Fw);
    for (int k = 0; k < F; ++k) {
      const double t = double(k) / F;
      const double psi = t * t * t * (10.0 + t * (-15.0 + 6.0 * t));
      const double dpsi = 30.0 * t * t * (1.0 - t) * (1.0 - t);
      th[k] = kPi * psi;
      ph[k] = 2.0 * kPi * double((long long)k * g % F) / F;
      w[k] = R * R * std::sin(th[k]) * kPi * dpsi * 2.0 * kPi / F;
    }
  } else {
    const int m = (int)std::lround(std::sqrt(F / 2.0));
    // Gauss-Legendre nodes by Newton iteration on P_m
    std::vector<double> xs(m), ws(m);
    for (int i = 0; i < m; ++i) {
      double x = -std::cos(kPi * (i + 0.75) / (m + 0.5));  // ascending nodes
      for (int it = 0; it < 100; ++it) {
        double p0 = 1, p1 = x;
        for (int k = 2; k <= m; ++k) {
          double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        double dp = m * (x * p1 - p0) / (x * x - 1.0);
        double dx = p1 / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-16) {
          ws[i] = 2.0 / ((1.0 - x * x) * dp * dp);
          break;
        }
        ws[i] = 2.0 / ((1.0 - x * x) * dp * dp);
      }
      xs[i] = x;
    }
    int k = 0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < 2 * m; ++j, ++k) {
        th[k] = std::acos(xs[i]);
        ph[k] = 2.0 * kPi * j / (2 * m);
        w[k] = R * R * ws[i] * kPi / m;
      }
  }
  for (int k = 0; k < F; ++k) {
    n[3 * k] = std::sin(th[k]) * std::cos(ph[k]);
    n[3 * k + 1] = std::sin(th[k]) * std::sin(ph[k]);
    n[3 * k + 2] = std::cos(th[k]);
    for (int c = 0; c < 3; ++c) y[3 * k + c] = R * n[3 * k + c];
  }
}

// Face pairs: pair t on axis axes[t % na], j = t / na, in-face coordinates
// u = (j + 1/2)/K_d - 1/2 and v = frac(j (sqrt5 - 1)/2) - 1/2 along the two
// other axes (increasing order).  Only x- (on the face at -L_d/2) is stored.
void face_pairs(const double L[3], int K, const int* axes, int na, std::vector<double>& xm,
                std::vector<int>& axis) {
  const double gfrac = (std::sqrt(5.0) - 1.0) / 2.0;
  xm.assign(3 * size_t(K), 0.0);
  axis.assign(K, 0);
  for (int t = 0; t < K; ++t) {
    const int d = axes[t % na];
    const int j = t / na;
    const int Kd = (K - (t % na) + na - 1) / na;
    int o[2], c = 0;
    for (int a = 0; a < 3; ++a)
      if (a != d) o[c++] = a;
    const double u = (j + 0.5) / Kd - 0.5;
    const double jg = j * gfrac;
    const double v = (jg - std::floor(jg)) - 0.5;
    xm[3 * t + d] = -0.5 * L[d];
    xm[3 * t + o[0]] = u * L[o[0]];
    xm[3 * t + o[1]] = v * L[o[1]];
    axis[t] = d;
  }
}

double image_strength(int l, double gu, double gl, bool upper) {
  // l-th upper image: gu^ceil(l/2) gl^floor(l/2); lower: gl^ceil gu^floor
  const int c = (l + 1) / 2, f = l / 2;
  return upper ? std::pow(gu, c) * std::pow(gl, f) : std::pow(gl, c) * std::pow(gu, f);
}

}  // namespace

hsma_status build_host_plan(const hsma_params& prm, const double lo[3], const double L[3], HostPlan& P,
                            std::string& msg, const PinvFn* pinv) {
  P = HostPlan();
  P.prm = prm;
  for (int k = 0; k < 3; ++k) {
    P.lo[k] = lo[k];
    P.L[k] = L[k];
    if (!(L[k] > 0) || !std::isfinite(L[k]) || !std::isfinite(lo[k])) {
      msg = "box lengths must be finite and positive";
      return HSMA_ERR_INVALID_ARG;
    }
  }
  if (prm.lsq_solver != 0 && prm.lsq_solver != 1) {
    msg = "lsq_solver must be 0 (host QR) or 1 (device CholeskyQR2)";
    return HSMA_ERR_INVALID_ARG;
  }
  // the least-squares pseudo-inverse: given, host Householder QR, or the
  // device's CholeskyQR2 (FP64 matrix cores)
  auto solve_pinv = [&](const std::vector<double>& M, int rows, int cols, std::vector<double>& Pi, double& cond,
                        std::string& m) -> hsma_status {
    bool ok = false;
    if (pinv) {
      ok = (*pinv)(M, rows, cols, Pi, cond);
    } else if (prm.lsq_solver == 1) {
      std::vector<LsqJob> jobs(1);
      jobs[0].M = &M;
      jobs[0].rows = rows;
      jobs[0].cols = cols;
      jobs[0].P = &Pi;
      const hsma_status ds = device_pinv_batch(jobs, m);
      if (ds != HSMA_OK) return ds;
      ok = jobs[0].ok;
      cond = jobs[0].cond;
    } else {
      ok = pseudo_inverse(M, rows, cols, Pi, cond);
    }
    if (!ok) {
      m = "least-squares matrix is rank deficient";
      return HSMA_ERR_RANK;
    }
    return HSMA_OK;
  };
  const bool slab = prm.geometry == HSMA_GEOM_2D;
  if (prm.geometry != HSMA_GEOM_3D && !slab) {
    msg = "geometry must be HSMA_GEOM_3D or HSMA_GEOM_2D";
    return HSMA_ERR_INVALID_ARG;
  }
  if (prm.p < 1 || prm.p > 24 || prm.K < 1 || prm.F < 4 || prm.F > 1000000 ||
      (prm.surface_rule != 0 && prm.surface_rule != 1) || prm.near_rule < 0 || prm.near_rule > 2 ||
      (prm.precision != HSMA_FP64 && prm.precision != HSMA_FP32C) || !(prm.lambda > 0)) {
    msg = "invalid method parameter (p in 1..24, K >= 1, F >= 4, surface rule 0/1, near rule 0/1/2, precision, "
          "lambda > 0)";
    return HSMA_ERR_INVALID_ARG;
  }
  if (prm.near_rule == 2 &&
      (prm.precision != HSMA_FP32C || prm.tree_order < 4 || prm.tree_order > 12 || prm.tree_order % 2 != 0 ||
       !(prm.tree_theta > 0 && prm.tree_theta <= 0.75))) {
    msg = "near rule 2 (treecode): FP32C, tree order 4/6/8/10/12, 0 < tree theta <= 0.75";
    return HSMA_ERR_INVALID_ARG;
  }
  if (prm.surface_rule == 1) {
    const int m = (int)std::lround(std::sqrt(prm.F / 2.0));
    if (2 * m * m != prm.F) {
      msg = "surface_rule 1 needs F = 2 n^2";
      return HSMA_ERR_INVALID_ARG;
    }
  }
  if (slab && (prm.M < 0 || prm.M > 200 || prm.nz < 2 || prm.nz > 512 || !(std::fabs(prm.gamma_up) < 1) ||
               !(std::fabs(prm.gamma_low) < 1))) {
    msg = "slab parameters: 0 <= M <= 200, 2 <= nz <= 512, |gamma| < 1";
    return HSMA_ERR_INVALID_ARG;
  }
  const double diag = std::sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
  P.R = prm.lambda * 0.5 * diag;
  const double Lmin = std::min(L[0], std::min(L[1], L[2]));
  const double Rmax = slab ? std::min(1.5 * std::min(L[0], L[1]), (prm.M + 0.5) * L[2]) : 1.5 * Lmin;
  if (!(P.R > 0.5 * diag && P.R < Rmax)) {
    msg = "sphere radius R = lambda*|L|/2 must exceed the half diagonal and stay inside the near cells";
    return HSMA_ERR_GEOMETRY;
  }
  const int p = prm.p;
  const int nb = (p + 1) * (p + 1) - 1;
  P.nb = nb;
  const double R = P.R;

  // ---- image tables
  auto push = [](std::vector<Desc>& v, double sx, double sy, double sz, double sg, double sc) {
    v.push_back(Desc{sx, sy, sz, sg, sc});
  };
  const int naxes = slab ? 2 : 3;
  std::vector<Desc> axis_tables[3];
  if (!slab) {
    for (int a = -1; a <= 1; ++a)
      for (int b = -1; b <= 1; ++b)
        for (int c = -1; c <= 1; ++c) push(P.desc_particles, a * L[0], b * L[1], c * L[2], 1.0, 1.0);
    // Telescoped difference sets: Phi_B(x+) - Phi_B(x-) for x+ = x- + L_d e_d
    // equals the potential at x- of the cells at k_d = -2 minus the cells at
    // k_d = +1 (the other two indices over {-1,0,1}).
    for (int d = 0; d < 3; ++d)
      for (int kd : {-2, 1})
        for (int a = -1; a <= 1; ++a)
          for (int b = -1; b <= 1; ++b) {
            int k[3];
            k[d] = kd;
            int o[2], c = 0;
            for (int e = 0; e < 3; ++e)
              if (e != d) o[c++] = e;
            k[o[0]] = a;
            k[o[1]] = b;
            push(axis_tables[d], k[0] * L[0], k[1] * L[1], k[2] * L[2], 1.0, kd == -2 ? 1.0 : -1.0);
          }
  } else {
    auto layers = [&](std::vector<Desc>& v, double sx, double sy, double sgn) {
      push(v, sx, sy, 0.0, 1.0, sgn);
      for (int l = 1; l <= prm.M; ++l) {
        const double sig = (l % 2) ? -1.0 : 1.0;
        push(v, sx, sy, l * L[2], sig, sgn * image_strength(l, prm.gamma_up, prm.gamma_low, true));
        push(v, sx, sy, -l * L[2], sig, sgn * image_strength(l, prm.gamma_up, prm.gamma_low, false));
      }
    };
    for (int a = -1; a <= 1; ++a)
      for (int b = -1; b <= 1; ++b) layers(P.desc_particles, a * L[0], b * L[1], 1.0);
    for (int d = 0; d < 2; ++d)
      for (int kd : {-2, 1})
        for (int a = -1; a <= 1; ++a) {
          double s[2];
          s[d] = kd * L[d];
          s[1 - d] = a * L[1 - d];
          layers(axis_tables[d], s[0], s[1], kd == -2 ? 1.0 : -1.0);
        }
  }

  if (prm.near_rule == 1) {
    // sphere near set: drop the image cells that cannot reach into the
    // sphere (nearest point of [s - L/2, s + L/2] at least R from the
    // centre, with a margin against rounding); the kernels test the rest
    // source by source
    std::vector<Desc> kept;
    for (const Desc& d : P.desc_particles) {
      const double sh[3] = {d.sx, d.sy, d.sz};
      double m2 = 0;
      for (int c = 0; c < 3; ++c) {
        const double g = std::max(0.0, std::fabs(sh[c]) - 0.5 * L[c]);
        m2 += g * g;
      }
      if (m2 <= R * R * (1 + 1e-9)) kept.push_back(d);
    }
    P.desc_particles.swap(kept);
  }

  // ---- check targets and fitting rows
  const int K = prm.K;
  std::vector<double> xm;
  std::vector<int> pax;
  const int axes3[3] = {0, 1, 2};
  face_pairs(L, K, axes3, naxes, xm, pax);
  const int nz = slab ? prm.nz : 0;
  const int ngrid = nz * nz;
  P.nrows = 2 * K + 2 * ngrid;
  if (P.nrows < nb) {
    msg = "fewer least-squares rows than unknowns";
    return HSMA_ERR_RANK;
  }
  std::vector<double> M(size_t(P.nrows) * nb, 0.0);
  std::vector<double> bv(nb), bg(3 * size_t(nb)), bv2(nb), bg2(3 * size_t(nb));
  for (int t = 0; t < K; ++t) {
    const int d = pax[t];
    double xi_m[3], xi_p[3];
    for (int c = 0; c < 3; ++c) {
      xi_m[c] = xm[3 * t + c] / R;
      xi_p[c] = xi_m[c] + (c == d ? L[d] / R : 0.0);
    }
    solid_harmonics(p, xi_m, bv.data(), bg.data());
    solid_harmonics(p, xi_p, bv2.data(), bg2.data());
    for (int j = 0; j < nb; ++j) {
      M[size_t(t) * nb + j] = bv2[j] - bv[j];
      // L_d (d_d b(x+) - d_d b(x-)), gradients w.r.t. xi carry 1/R
      M[size_t(K + t) * nb + j] = L[d] / R * (bg2[3 * j + d] - bg[3 * j + d]);
    }
  }
  // Face-pair check targets, grouped by axis, and their columns of Praw
  // (A = Praw v, v = raw potential and field component at every target).
  // Stencil rule: one target x- per pair, summed over the telescoped sets
  // (cells at k_d = -2 minus cells at k_d = +1 give Phi_B(x+) - Phi_B(x-)
  // at x-).  Sphere rule: the set B is no union of cells, so both x- and
  // x+ = x- + L_d e_d are targets over the near set and the row difference
  // is taken in Praw (+ for x+, - for x-).
  // Rows: Y_val = -(Phi+ - Phi-);  Y_der = -L_d d_d(Phi+ - Phi-) = L_d (E_d+ - E_d-).
  const bool sphere_near = prm.near_rule == 1;
  const int nface = sphere_near ? 2 * K : K;
  auto face_targets = [&](const std::vector<double>& Pinv, int ncheck, int& tcount) {
    for (int side = sphere_near ? 0 : 1; side < 2; ++side) {
      const double sgn = sphere_near ? (side == 0 ? -1.0 : 1.0) : 1.0;
      for (int d = 0; d < naxes; ++d) {
        std::vector<int> ts;
        for (int t = 0; t < K; ++t)
          if (pax[t] == d) ts.push_back(t);
        const std::vector<Desc>& set = sphere_near ? P.desc_particles : axis_tables[d];
        for (size_t g0 = 0; g0 < ts.size(); g0 += kGroup) {
          Group grp{tcount, (int)std::min<size_t>(kGroup, ts.size() - g0), (int)P.desc_check.size(),
                    (int)set.size()};
          for (int i = 0; i < grp.count; ++i) {
            const int t = ts[g0 + i];
            for (int c = 0; c < 3; ++c)
              P.check_pos.push_back(xm[3 * t + c] + (sphere_near && side == 1 && c == d ? L[d] : 0.0));
            P.check_axis.push_back(d);
            for (int j = 0; j < nb; ++j) {
              P.Praw[size_t(j) * 2 * ncheck + 2 * tcount] += -sgn * Pinv[size_t(j) * P.nrows + t];
              P.Praw[size_t(j) * 2 * ncheck + 2 * tcount + 1] += sgn * L[d] * Pinv[size_t(j) * P.nrows + K + t];
            }
            ++tcount;
          }
          P.check_groups.push_back(grp);
          P.desc_check.insert(P.desc_check.end(), set.begin(), set.end());
        }
      }
    }
  };
  std::vector<std::vector<double>> Tb;  // per interface: T applied to basis columns
  if (slab) {
    DtN T(nz, L[0], L[1]);
    const double h = 0.5 * L[2];
    std::vector<double> grid(2 * size_t(ngrid) * 3);
    for (int s = 0; s < 2; ++s)
      for (int ix = 0; ix < nz; ++ix)
        for (int iy = 0; iy < nz; ++iy) {
          double* g = &grid[(size_t(s) * ngrid + size_t(ix) * nz + iy) * 3];
          g[0] = (ix + 0.5) * L[0] / nz - 0.5 * L[0];
          g[1] = (iy + 0.5) * L[1] / nz - 0.5 * L[1];
          g[2] = s == 0 ? h : -h;
        }
    std::vector<double> col(ngrid), tcol(ngrid);
    for (int s = 0; s < 2; ++s) {
      const double gam = s == 0 ? prm.gamma_up : prm.gamma_low;
      const double sgn = s == 0 ? 1.0 : -1.0;
      std::vector<double> vals(size_t(ngrid) * nb), dz(size_t(ngrid) * nb);
      for (int g = 0; g < ngrid; ++g) {
        double xi[3];
        for (int c = 0; c < 3; ++c) xi[c] = grid[(size_t(s) * ngrid + g) * 3 + c] / R;
        solid_harmonics(p, xi, bv.data(), bg.data());
        for (int j = 0; j < nb; ++j) {
          vals[size_t(g) * nb + j] = bv[j];
          dz[size_t(g) * nb + j] = bg[3 * j + 2] / R;
        }
      }
      for (int j = 0; j < nb; ++j) {
        for (int g = 0; g < ngrid; ++g) col[g] = vals[size_t(g) * nb + j];
        T.apply(col.data(), tcol.data());
        for (int g = 0; g < ngrid; ++g)
          M[size_t(2 * K + s * ngrid + g) * nb + j] = h * ((1 + gam) * dz[size_t(g) * nb + j] + sgn * (1 - gam) * tcol[g]);
      }
    }
    // check targets on the interfaces, in 8x8 blocks for spatially compact groups
    // (filled below together with the face pairs)
    std::vector<double> Pinv;
    {
      const hsma_status ls = solve_pinv(M, P.nrows, nb, Pinv, P.cond, msg);
      if (ls != HSMA_OK) return ls;
    }
    // ---- targets: face pairs grouped by axis, then the two interface grids
    const int ncheck = nface + 2 * ngrid;
    P.Praw.assign(size_t(nb) * 2 * ncheck, 0.0);
    int tcount = 0;
    face_targets(Pinv, ncheck, tcount);
    P.face_groups = (int)P.check_groups.size();
    for (int s = 0; s < 2; ++s) {
      const double gam = s == 0 ? prm.gamma_up : prm.gamma_low;
      const double sgn = s == 0 ? 1.0 : -1.0;
      // slot of grid point (ix, iy) once ordered in 8x8 blocks
      std::vector<int> slot(ngrid);
      const int first_slot = tcount;
      std::vector<int> order;
      for (int bx = 0; bx < nz; bx += 8)
        for (int by = 0; by < nz; by += 8)
          for (int ix = bx; ix < std::min(nz, bx + 8); ++ix)
            for (int iy = by; iy < std::min(nz, by + 8); ++iy) order.push_back(ix * nz + iy);
      for (size_t i = 0; i < order.size(); ++i) slot[order[i]] = first_slot + (int)i;
      for (size_t g0 = 0; g0 < order.size(); g0 += kGroup) {
        Group grp{first_slot + (int)g0, (int)std::min<size_t>(kGroup, order.size() - g0),
                  (int)P.desc_check.size(), (int)P.desc_particles.size()};
        P.check_groups.push_back(grp);
        P.desc_check.insert(P.desc_check.end(), P.desc_particles.begin(), P.desc_particles.end());
      }
      for (size_t i = 0; i < order.size(); ++i) {
        const int g = order[i];
        for (int c = 0; c < 3; ++c) P.check_pos.push_back(grid[(size_t(s) * ngrid + g) * 3 + c]);
        P.check_axis.push_back(2);
      }
      tcount += ngrid;
      // Y_g = -h[(1+gam)(-Ez_g) + sgn (1-gam) (T Phi)_g]
      //     = h(1+gam) v[2 slot(g)+1] - sgn h (1-gam) sum_g' T[g,g'] v[2 slot(g')]
      const int row0 = 2 * K + s * ngrid;
      for (int j = 0; j < nb; ++j) {
        for (int g = 0; g < ngrid; ++g) {
          const double pj = Pinv[size_t(j) * P.nrows + row0 + g];
          P.Praw[size_t(j) * 2 * ncheck + 2 * slot[g] + 1] += h * (1 + gam) * pj;
          col[g] = pj;
        }
        T.apply(col.data(), tcol.data());  // T symmetric: (P_rows T)[j, g'] = T (P_rows^T)[g']
        for (int g = 0; g < ngrid; ++g)
          P.Praw[size_t(j) * 2 * ncheck + 2 * slot[g]] += -sgn * h * (1 - gam) * tcol[g];
      }
    }
  } else {
    std::vector<double> Pinv;
    {
      const hsma_status ls = solve_pinv(M, P.nrows, nb, Pinv, P.cond, msg);
      if (ls != HSMA_OK) return ls;
    }
    const int ncheck = nface;
    P.Praw.assign(size_t(nb) * 2 * ncheck, 0.0);
    int tcount = 0;
    face_targets(Pinv, ncheck, tcount);
    P.face_groups = (int)P.check_groups.size();
  }

  // ---- sphere quadrature and the maps A -> (Q, D)
  std::vector<double> w;
  surface_rule(prm.F, prm.Fw, prm.surface_rule, R, P.ysurf, P.nsurf, w);
  P.SQ.assign(size_t(prm.F) * nb, 0.0);
  P.SD.assign(size_t(prm.F) * nb, 0.0);
  std::vector<int> deg(nb);
  {
    int j = 0;
    for (int n = 1; n <= p; ++n)
      for (int m = 0; m < 2 * n + 1; ++m) deg[j++] = n;
  }
  for (int k = 0; k < prm.F; ++k) {
    double xi[3] = {P.nsurf[3 * k], P.nsurf[3 * k + 1], P.nsurf[3 * k + 2]};
    solid_harmonics(p, xi, bv.data(), nullptr);
    for (int j = 0; j < nb; ++j) {
      // u = sum A b; d_n u = sum A (n_deg / R) b on |r| = R (b homogeneous)
      P.SD[size_t(k) * nb + j] = w[k] * bv[j] / (4.0 * kPi);
      P.SQ[size_t(k) * nb + j] = w[k] * deg[j] / R * bv[j] / (4.0 * kPi);
    }
  }
  return HSMA_OK;
}

// Host-side input validation of the host-memory calls: finite coordinates
// and charges, every ion strictly between the slab's interfaces, charge
// neutrality (the constant mode A_0^0 is undetermined otherwise).
hsma_status validate_host_input(const hsma_params& prm, const double lo[3], const double L[3], int64_t n,
                                const double* xyz, const double* q, std::string& msg) {
  double sq = 0, sa = 0;
  const bool slab = prm.geometry == HSMA_GEOM_2D;
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(xyz[3 * i + c])) {
        msg = "non-finite coordinate";
        return HSMA_ERR_OUT_OF_DOMAIN;
      }
    if (!std::isfinite(q[i])) {
      msg = "non-finite charge";
      return HSMA_ERR_OUT_OF_DOMAIN;
    }
    if (slab) {
      const double z = xyz[3 * i + 2] - lo[2];
      if (!(z > 0.0 && z < L[2])) {
        msg = "particle outside the slab";
        return HSMA_ERR_OUT_OF_DOMAIN;
      }
    }
    sq += q[i];
    sa += std::fabs(q[i]);
  }
  if (!(std::fabs(sq) <= 1e-12 * sa)) {
    msg = "system is not charge neutral";
    return HSMA_ERR_NOT_NEUTRAL;
  }
  return HSMA_OK;
}

}  // namespace hsma
