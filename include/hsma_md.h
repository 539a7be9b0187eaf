/*
 * hsma_md.h -- molecular dynamics on top of the HSMA hot path.
 *
 * Velocity-Verlet integration of charged soft spheres, the systems the
 * paper integrates with HSMA as the electrostatics of an MD engine: the
 * primitive electrolytes of Sec. 4.1 (ions as purely repulsive
 * Lennard-Jones spheres, cut at the potential minimum) and, in the slab
 * geometry, the ions between two dielectric interfaces of Sec. 4.3 (kept
 * inside by repulsive Lennard-Jones walls).  Per step:
 *   v += dt/2 F/m;  x += dt v (wrapped along the periodic axes);
 *   F = F_Coulomb (the plan's step, F_i = q_i E_i) + F_LJ (pairs, walls);
 *   v += dt/2 F/m;  thermo row.
 * With respa_inner = k >= 2 a step of dt is: v += dt/2 F_C/m; k times
 * { v += dt/(2k) F_LJ/m; x += dt/k v; F_LJ at x; v += dt/(2k) F_LJ/m };
 * F_C at x; v += dt/2 F_C/m; thermo row (F_C: the plan's Coulomb forces,
 * F_LJ: pairs and walls).  The driver keeps the two force parts between
 * its calls (forces_valid = 1 reuses them after its own last run).
 * With the Nose-Hoover thermostat (the paper's runs are NVT), half a
 * thermostat step before and after, in the time-reversible splitting:
 *   xi += dt/4 G;  v *= exp(-xi dt/2);  eta += dt/2 xi;  xi += dt/4 G,
 *   G = (2 E_kin - nf kT) / Q,
 * and the thermo row's E_kin and pressure are those after it.
 * Everything runs on the device on the caller's buffers; the plan's step is
 * replayed from a captured HIP graph after the first steps.
 *
 * Thermo row per step (4 doubles): E_Coulomb, E_LJ (pairs + walls),
 * E_kinetic, and the pressure P = (2 E_kin + W_LJ + W_C) / (3 V) of the
 * fully periodic geometry, with W_LJ = sum over pairs r_ij . F_ij and
 * W_C = E_Coulomb: the HSMA energy is homogeneous of degree -1 under
 * scaling of positions and box together (E(s r, s L) = E / s), so its
 * volume derivative gives exactly that virial.  In the slab geometry the
 * fourth value is the LJ part (2 E_kin + W_LJ) / (3 V) only.
 *
 * The LJ pairs are found by testing all N^2 minimum-image distances (LDS
 * tiles of 256 sources; small systems split the sources into chunks over
 * more blocks and sum the chunks' forces in a fixed order): meant for the
 * ensembles served here (up to about 10^4 - 10^5 ions per replica), not
 * for large single systems.
 *
 * Layouts as in hsma.h: positions, velocities, forces n x 3 row-major FP64;
 * charges and masses n FP64.  Positions must lie in the plan's box (slab: z
 * strictly between the walls).  Units: those of the plan (its coulomb_k is
 * the Coulomb prefactor, e.g. the Bjerrum length in units of kT).
 */
#ifndef HSMA_MD_H
#define HSMA_MD_H

#include <stdint.h>

#include "hsma.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsma_md_params {
  double dt;            /* time step                                            */
  double lj_epsilon;    /* pair potential 4 eps [(sig/r)^12 - (sig/r)^6] + eps   */
  double lj_sigma;      /*   for r < lj_rcut (shifted to 0 at the cut)           */
  double lj_rcut;       /*   (0: 2^(1/6) sigma, purely repulsive)  must be below
                             half the shortest periodic box edge                  */
  double wall_epsilon;  /* slab: the same form in the distance to each wall      */
  double wall_sigma;    /*   (wall_epsilon 0: no walls)                          */
  double wall_rcut;     /*   (0: 2^(1/6) wall_sigma)                             */
  double nh_kT;         /* Nose-Hoover thermostat (NVT, as the paper's runs of
                             Sec. 4.1 and 4.3): target kT, with               */
  double nh_damping;    /*   damping time tau (thermostat mass nf kT tau^2, nf =
                             3n - 3, slab 3n - 2); both 0: constant energy (NVE) */
  int respa_inner;      /* 0 or 1: velocity Verlet.  k >= 2 (at most 1000):
                             multiple time steps (reversible RESPA, as the
                             paper's slab runs of Sec. 4.3): the Coulomb forces
                             act every dt, the short-range forces every dt / k
                             (hsma_md_run with a plan only)                    */
} hsma_md_params;

typedef struct hsma_md hsma_md;

/* A driver for n particles integrated with `plan` (which must outlive it);
 * 2 <= n <= 2^26 (and within the plan's own particle limit).
 * Errors: INVALID_ARG (n, parameters, a cut-off above half a box edge),
 * OOM, DEVICE.                                                           */
hsma_status hsma_md_create(hsma_plan* plan, const hsma_md_params* params, int64_t n, hsma_md** out);

/* Runs nsteps steps on `stream` (a hipStream_t; asynchronous).  d_f holds
 * the forces at d_x on return; forces_valid = 1 says it already holds them
 * on entry (from the previous call), else they are computed first.
 * d_thermo: nsteps x 4 device doubles, or NULL.                          */
hsma_status hsma_md_run(hsma_md* md, void* stream, int nsteps, double* d_x, double* d_v, double* d_f,
                        const double* d_q, const double* d_m, int forces_valid, double* d_thermo);

/* Forces (Coulomb + LJ) at d_x into d_f, and one thermo row whose kinetic
 * energy is taken from d_v (may be NULL: 0).                            */
hsma_status hsma_md_forces(hsma_md* md, void* stream, const double* d_x, const double* d_v, double* d_f,
                           const double* d_q, const double* d_m, double* d_thermo_row);

/* A driver without a plan, for steps whose Coulomb forces come from
 * elsewhere (e.g. a device request to hsma_server): geometry and box as in
 * hsma_plan_create; 2 <= n <= 2^26.  hsma_md_run and hsma_md_forces need a plan and refuse
 * it (INVALID_ARG); the two halves of a step below work on any driver.   */
hsma_status hsma_md_create_for_box(const hsma_md_params* params, int geometry, const double box_lo[3],
                                   const double box_len[3], int64_t n, hsma_md** out);

/* First half of a step: the thermostat's first half if one is set, then
 * v += dt/2 F/m, x += dt v (wrapped).                                    */
hsma_status hsma_md_drift(hsma_md* md, void* stream, double* d_x, double* d_v, const double* d_f,
                          const double* d_m);

/* Second half, once d_f holds the Coulomb forces at the new d_x and
 * d_e_coulomb their energy (device scalar): F += F_LJ, v += dt/2 F/m, one
 * thermo row (device, 4 doubles, or NULL), then the thermostat's closing
 * half if one is set.                                                   */
hsma_status hsma_md_finish(hsma_md* md, void* stream, const double* d_x, double* d_v, double* d_f,
                           const double* d_m, const double* d_e_coulomb, double* d_thermo_row);

/* Forces at the start of a run for a driver without a plan: once d_f
 * holds the Coulomb forces at d_x and d_e_coulomb their energy, F += F_LJ
 * and one thermo row (E_kin from d_v, which may be NULL: 0), with no kick
 * and no thermostat (what hsma_md_forces does after the plan's step).   */
hsma_status hsma_md_short_range(hsma_md* md, void* stream, const double* d_x, const double* d_v, double* d_f,
                                const double* d_m, const double* d_e_coulomb, double* d_thermo_row);

/* Thermostat state after the driver's last enqueued call, copied on
 * `stream` (which first waits for that call) into d_state (3 device
 * doubles): xi (thermostat velocity), eta (its position) and its energy
 * Q xi^2 / 2 + nf kT eta, so that E_Coulomb + E_LJ + E_kin + that energy
 * is conserved by the integration (all 0 without a thermostat).  A later
 * call of the driver on another stream must be ordered after this copy by
 * the caller, as for any two calls of one driver.                       */
hsma_status hsma_md_thermostat(hsma_md* md, void* stream, double* d_state);

/* Structure of a configuration: the observables of the paper's MD runs
 * (Sec. 4: radial distribution functions of the 3D electrolytes, ion
 * density profiles between the dielectric interfaces).  Both add counts to
 * the caller's device histogram (uint64, not cleared: accumulate over
 * snapshots) with integer atomics, so the counts do not depend on the
 * order of the work; asynchronous on `stream`.  Errors: INVALID_ARG.
 *
 * Pair distances: every pair i < j with both charges nonzero at
 * minimum-image distance r < r_max goes to bin floor(r / dr), dr = r_max /
 * nbins, of class 0 (both q > 0), 1 (opposite signs) or 2 (both q < 0);
 * d_hist holds 3 x nbins counts.  Per periodic axis (x and y; z too in 3D)
 * d = (x_i - x_j) - L rint((x_i - x_j) * (1 / L)), then r =
 * sqrt((dx^2 + dy^2) + dz^2), each FP64 operation rounded on its own (no
 * fused multiply-add), so that a CPU recomputation in this order finds the
 * same bins.  1 <= nbins <= 4096; 0 < r_max <= half the smallest periodic
 * box edge.  O(n^2) pair tests, as for the LJ pairs.                    */
hsma_status hsma_md_rdf(hsma_md* md, void* stream, const double* d_x, const double* d_q, int nbins, double r_max,
                        unsigned long long* d_hist);

/* Density profile along z: particle i with q_i != 0 goes to bin
 * floor((z_i - lo_z) / (L_z / nbins)) (clamped to [0, nbins - 1]) of class
 * 0 (q > 0) or 1 (q < 0); d_hist holds 2 x nbins counts; 1 <= nbins <= 4096. */
hsma_status hsma_md_zprofile(hsma_md* md, void* stream, const double* d_x, const double* d_q, int nbins,
                             unsigned long long* d_hist);

void hsma_md_destroy(hsma_md* md);

#ifdef __cplusplus
}
#endif
#endif /* HSMA_MD_H */
