/* Direct fp64 Coulomb sums for the HSMA oracle (test infrastructure only).
 *
 * Plain double loops, one target at a time, sources in the order given.
 * Units: Coulomb constant 1, so a charge q at distance r has potential q/r
 * (Eq. 2 with eps_c = 1).
 */
#include <math.h>
#include <stdint.h>

/* For every target t:
 *   phi[t]       = sum_s q_s / |x_t - y_s|
 *   field[3t+k]  = sum_s q_s (x_t - y_s)_k / |x_t - y_s|^3   (E = -grad phi)
 * skipping source index skip[t] when skip != NULL and skip[t] >= 0.
 * tx: nt*3, sy: ns*3 (row-major xyz), sq: ns.                             */
void oracle_charge_sums(int64_t nt, const double* tx, int64_t ns, const double* sy,
                        const double* sq, const int64_t* skip, double* phi, double* field) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t t = 0; t < nt; ++t) {
    const double x = tx[3 * t], y = tx[3 * t + 1], z = tx[3 * t + 2];
    const int64_t sk = skip ? skip[t] : -1;
    double p = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    for (int64_t s = 0; s < ns; ++s) {
      if (s == sk) continue;
      const double dx = x - sy[3 * s], dy = y - sy[3 * s + 1], dz = z - sy[3 * s + 2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double pot = sq[s] / r;
      const double e = pot / (r * r);
      p += pot;
      ex += e * dx;
      ey += e * dy;
      ez += e * dz;
    }
    phi[t] = p;
    field[3 * t] = ex;
    field[3 * t + 1] = ey;
    field[3 * t + 2] = ez;
  }
}

/* Single + double layer point sources on the auxiliary sphere:
 *   phi  += Q_k/|d| - D_k (n_k.d)/|d|^3
 *   E    += Q_k d/|d|^3 + D_k ( n_k/|d|^3 - 3 (n_k.d) d/|d|^5 ),  d = x_t - y_k
 * (the potential of a charge Q_k and of a dipole of moment -D_k n_k). */
void oracle_layer_sums(int64_t nt, const double* tx, int64_t nk, const double* yk,
                       const double* nrm, const double* Q, const double* D,
                       double* phi, double* field) {
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nt; ++t) {
    const double x = tx[3 * t], y = tx[3 * t + 1], z = tx[3 * t + 2];
    double p = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
    for (int64_t k = 0; k < nk; ++k) {
      const double dx = x - yk[3 * k], dy = y - yk[3 * k + 1], dz = z - yk[3 * k + 2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double r = sqrt(r2);
      const double r3 = r2 * r;
      const double r5 = r3 * r2;
      const double nd = nrm[3 * k] * dx + nrm[3 * k + 1] * dy + nrm[3 * k + 2] * dz;
      p += Q[k] / r - D[k] * nd / r3;
      ex += Q[k] * dx / r3 + D[k] * (nrm[3 * k] / r3 - 3.0 * nd * dx / r5);
      ey += Q[k] * dy / r3 + D[k] * (nrm[3 * k + 1] / r3 - 3.0 * nd * dy / r5);
      ez += Q[k] * dz / r3 + D[k] * (nrm[3 * k + 2] / r3 - 3.0 * nd * dz / r5);
    }
    phi[t] = p;
    field[3 * t] = ex;
    field[3 * t + 1] = ey;
    field[3 * t + 2] = ez;
  }
}
