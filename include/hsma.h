/*
 * hsma.h -- C ABI of the MI355X (gfx950) HSMA hot path.
 *
 * Harmonic surface mapping (HSMA) Coulomb solver for N point charges in a
 * box that is either fully periodic (HSMA3D, Eq. 3 of the paper) or periodic
 * in x and y with two planar dielectric interfaces at the z faces of the box
 * (HSMA2D, Eq. 4).  One call computes, for one configuration:
 *   the electrostatic energy E = 1/2 sum_i q_i Phi_i,
 *   the potential Phi_i at every particle (own self term excluded, all of its
 *     periodic / dielectric images included),
 *   the force F_i = q_i E_i with E_i = -grad Phi at r_i.
 * The method (Sec. 2.2): the charges and images inside an auxiliary region
 * are summed directly; the rest is a harmonic series of degree <= p whose
 * coefficients are fitted by least squares at check points (Eqs. 5-6), then
 * mapped to charges and dipoles on a sphere of radius R = lambda * half box
 * diagonal (integrated with a lattice "Fibonacci" rule) and summed at the
 * particles.  Units: Coulomb constant coulomb_k (1 by default), eps_c = 1.
 *
 * Conventions
 *  - Every buffer belongs to the caller.  Host entry points copy inputs in
 *    and results out and keep no caller pointer after they return.  Device
 *    entry points read and write the caller's device buffers asynchronously
 *    on the given stream; they must stay valid until that work completes.
 *  - Layouts: positions are n x 3 row-major (x0 y0 z0 x1 ...), FP64;
 *    charges n FP64; potential n FP64; force n x 3 FP64; energy 1 FP64.
 *    Any output pointer may be NULL (that output is skipped).
 *  - Two charges at zero distance (coincident ions, or an ion on a periodic
 *    image of another) have no finite energy.  This is not checked: the
 *    call returns OK, and the energy and those ions' outputs are not finite.
 *  - A plan is not thread-safe; distinct plans are independent.  No C++
 *    exception crosses this interface.  On error the call returns a negative
 *    hsma_status and hsma_last_error() describes it.
 */
#ifndef HSMA_H
#define HSMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HSMA_OK = 0,
  HSMA_ERR_INVALID_ARG = -1,   /* NULL pointer, bad size or parameter          */
  HSMA_ERR_NOT_NEUTRAL = -2,   /* |sum q| > 1e-12 sum |q|: A_0^0 undetermined  */
  HSMA_ERR_OUT_OF_DOMAIN = -3, /* slab: a particle z not strictly inside; or a
                                  non-finite coordinate / charge               */
  HSMA_ERR_GEOMETRY = -4,      /* sphere radius outside its admissible range   */
  HSMA_ERR_RANK = -5,          /* fewer fitting rows than unknowns, or the
                                  fitting matrix is rank deficient             */
  HSMA_ERR_NO_DEVICE = -6,     /* no usable gfx950 device                      */
  HSMA_ERR_OOM = -7,           /* device allocation failed / over budget       */
  HSMA_ERR_DEVICE = -8,        /* a HIP runtime call failed                    */
  HSMA_ERR_BUSY = -9,          /* server queue full                            */
  HSMA_ERR_CANCELLED = -10     /* server shut down before the request ran      */
} hsma_status;

enum { HSMA_GEOM_3D = 0, HSMA_GEOM_2D = 1 };
enum { HSMA_FP64 = 0, HSMA_FP32C = 1 };

/* Method parameters (cf. the kspace_style arguments of Sec. 3.2).          */
typedef struct hsma_params {
  int geometry;        /* HSMA_GEOM_3D or HSMA_GEOM_2D                          */
  int precision;       /* HSMA_FP64: all sums in FP64.  HSMA_FP32C: pair and
                          surface sums in FP32 with compensated accumulation;
                          FP64 in the least-squares solve, the energy reduction
                          and the close-pair coordinate correction            */
  double lambda;       /* R = lambda * |L| / 2 (sphere radius over half the
                          box diagonal); 3D: |L|/2 < R < 1.5 min L;
                          2D: |L|/2 < R < min(1.5 Lx, 1.5 Ly, (M+1/2) Lz)     */
  int p;               /* harmonic degree; (p+1)^2 - 1 unknowns (A_0^0 = 0)  */
  int K;               /* 3D: check-point pairs on opposite faces (2K rows);
                          2D: x/y face pairs                                  */
  int F;               /* points on the sphere                                */
  int Fw;              /* lattice generator of the surface rule (0 = auto)   */
  int surface_rule;    /* 0: periodised rank-1 (Fibonacci) lattice;
                          1: Gauss-Legendre x trapezoid (F = 2 n^2)          */
  int near_rule;       /* near set of Sec. 2.2.  0: the cell stencil (3D: 27
                          cells; 2D: 9 cells x (2M+1) image layers).
                          1: only the images of that stencil strictly inside
                          the sphere, |y - box centre| < R (FP64 test on the
                          image position); the stencil covers the sphere for
                          every admissible R.  Rule 1 sums about a third of
                          the pairs (3D, lambda 1.5) but its far field starts
                          at R, so it needs a higher p for the same error.
                          2: the stencil of rule 0, summed at the particles
                          and at the check points by a treecode (multipole
                          expansions, up to order tree_order, of the source
                          nodes that satisfy (r_node + r_group) < tree_theta
                          * distance; direct sums elsewhere).  FP32C only.
                          An approximation of rule 0.  At the default order
                          12, theta 0.5 the energy is within 4.5e-7 (50,000
                          ions) and 1.5e-7 (999,999 ions) of the direct FP64
                          sums and the RMS force within 5e-7; the 20,000-ion
                          slab stays at 1.6e-6 in energy.  Order 8 is 1.5x
                          faster at 1.3e-5 energy, 3e-6 RMS force            */
  int M;               /* 2D: image layers above and below                    */
  double gamma_up;     /* 2D: (eps_c - eps_up)/(eps_c + eps_up), |gamma| < 1  */
  double gamma_low;    /* 2D: (eps_c - eps_low)/(eps_c + eps_low)             */
  int nz;              /* 2D: interface grid points per dimension (DtN rows)  */
  double coulomb_k;    /* prefactor of q_i q_j / r (default 1)                */
  int tree_order;      /* near rule 2: multipole order, 4, 6, 8, 10 or 12     */
  double tree_theta;   /* near rule 2: opening parameter, 0 < theta <= 0.75   */
  int lsq_solver;      /* least-squares pseudo-inverse of Eq. 6, built once per
                          plan: 0 host Householder QR (FP64); 1 CholeskyQR2
                          on the device (FP64, Gram matrices on the matrix
                          cores; the plan's device must be current)          */
} hsma_params;

typedef struct hsma_plan hsma_plan;

/* Fills *p with defaults: 3D, FP32C, lambda 1.5, p 10, K 2(p+1)^2, F 800,
 * Fw 0, surface rule 0, near rule 0, M 10, gammas 0, nz 80, coulomb_k 1,
 * tree order 12, tree theta 0.5, lsq solver 0.                            */
void hsma_params_default(hsma_params* p);

/* Builds the per-geometry plan (the set-up parts of Sec. 2.2 and the
 * parameters of Sec. 3.2): check points on the box faces (and, in 2D, the
 * interface grids), the sphere quadrature, the harmonic basis, the
 * least-squares pseudo-inverse of Eq. 6 (host FP64 Householder QR, or the
 * device's FP64 matrix cores with lsq_solver 1) and the image tables of
 * Eqs. 3-4; uploads them to the current HIP device.
 * box_lo: lower box corner; box_len: edge lengths (all > 0).  In 2D the
 * dielectric interfaces are the planes z = box_lo[2] and z = box_lo[2] +
 * box_len[2].  Errors: INVALID_ARG, GEOMETRY, RANK, NO_DEVICE, OOM, DEVICE. */
hsma_status hsma_plan_create(const hsma_params* params, const double box_lo[3],
                             const double box_len[3], hsma_plan** out);

void hsma_plan_destroy(hsma_plan* plan);

/* Particle count of one call: 1 <= n <= 2^30 - 1 with near rule 0, and
 * n <= 2^26 (2^20 tiles of 64) with near rules 1 and 2.  Larger counts fail
 * with INVALID_ARG before any buffer is read or any work is enqueued.      */

/* One step of the method (Sec. 2.2, Eqs. 3-6): near-set sums at the check
 * points, the least-squares fit, the sphere charges and dipoles, the sums
 * at the particles, then E = 1/2 sum q_i Phi_i and F_i = q_i E_i.
 * Host-memory call (synchronous): xyz (n x 3) and q (n) are read, energy
 * (1), potential (n) and force (n x 3) written, each output optional
 * (NULL).  Validates the input on the host first:
 * n within the limits above, finite values, neutrality (NOT_NEUTRAL), slab
 * domain (OUT_OF_DOMAIN).  Positions outside the box are wrapped along
 * periodic axes.                                                          */
hsma_status hsma_compute(hsma_plan* plan, int64_t n, const double* xyz, const double* q,
                         double* energy, double* potential, double* force);

/* The same step (Sec. 2.2, Eqs. 3-6) on device memory: d_xyz, d_q, d_energy,
 * d_potential, d_force are device pointers in the layouts above (outputs
 * optional), owned by the caller and in use until the stream reaches the
 * end of the step.  Enqueues the whole step on `stream` (a hipStream_t;
 * NULL = default stream) and returns without waiting.  Validation runs on
 * the device; an invalid input makes every requested output NaN and is
 * reported by the next hsma_plan_device_status() on this plan.             */
hsma_status hsma_compute_device(hsma_plan* plan, void* stream, int64_t n, const double* d_xyz,
                                const double* d_q, double* d_energy, double* d_potential,
                                double* d_force);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving or MD loops, harnesses that forbid allocation): the same step as
 * hsma_compute_device, with its per-call working memory (sort keys, tiles,
 * partial sums) taken from a static device array of 48 MiB that the library
 * holds on every GPU it runs on until the process ends, instead of from an
 * allocation.  The call makes no device or host allocation.  The plan must
 * have been created on the current device (plan creation allocates the
 * plan's constants and looks up the array's address).
 * Limits: 1 <= n <= 16384 particles, else HSMA_ERR_INVALID_ARG; a plan whose
 * parameters need more working memory for n than the array holds is also
 * refused with HSMA_ERR_INVALID_ARG and a message giving both sizes.
 * Sharing: every call on a GPU uses that GPU's one array, which keeps the
 * last call's contents; calls that overlap on one GPU (different streams,
 * plans or threads, without ordering between them) race and give wrong
 * results.  Calls of one plan are ordered by the plan itself.
 * The work decomposition differs from hsma_compute_device's (fewer, longer
 * waves), so FP32C results agree with it to the FP32C tolerances, FP64
 * results to rounding.  Validation and outputs as hsma_compute_device.    */
hsma_status hsma_compute_device_noalloc(hsma_plan* plan, void* stream, int64_t n, const double* d_xyz,
                                        const double* d_q, double* d_energy, double* d_potential,
                                        double* d_force);

/* Waits for the plan's last device call and returns the status that its
 * device-side validation recorded (OK, NOT_NEUTRAL or OUT_OF_DOMAIN).      */
hsma_status hsma_plan_device_status(hsma_plan* plan);

/* Per-stage device times (ms) of the last hsma_compute on this plan and
 * plan facts.  Fields set to -1 when unavailable.                          */
typedef struct hsma_plan_info {
  int nb;                /* unknowns (p+1)^2 - 1                                */
  int n_rows;            /* least-squares rows                                  */
  int n_check;           /* check targets evaluated per step                    */
  int n_desc;            /* near-set image descriptors per particle             */
  double radius;         /* R                                                   */
  double cond;           /* condition number estimate of the (scaled) fit       */
  int64_t near_pairs;    /* pair interactions of the last step: particles      */
  int64_t check_pairs;   /*   check targets (sphere near set: counted from the
                              last step's masks; the call waits for that step;
                              treecode: the stencil pairs it approximates)      */
  int64_t surface_pairs; /*   sphere sources                                    */
} hsma_plan_info;
hsma_status hsma_plan_get_info(const hsma_plan* plan, hsma_plan_info* info);

/* Device time of the main stages, summed over the device or host calls
 * made on this plan since timing was (re)enabled, from HIP events recorded
 * on the call's stream around each stage (at most 4096 calls are timed).
 * hsma_plan_get_timing waits for those calls to finish.                   */
typedef struct hsma_timing {
  int64_t calls;      /* timed calls                                           */
  double step_ms;     /* whole step, first to last kernel                      */
  double check_ms;    /* check-target near sums (before their reduction)       */
  double near_ms;     /* particle near-set sums (the dominant kernel)          */
  double sphere_ms;   /* particle sphere-source sums                           */
} hsma_timing;
hsma_status hsma_plan_set_timing(hsma_plan* plan, int enable);
hsma_status hsma_plan_get_timing(hsma_plan* plan, hsma_timing* out);

/* Step graphs (default off).  When on, a device call on a non-NULL stream
 * whose (particle count, buffers, stream) repeats one of the plan's recent
 * calls is captured into a HIP graph (on that second call) and replayed on
 * later calls with the same key, so a repeated step costs one graph launch
 * instead of ~20 kernel launches.  Up to 8 captured steps are kept per plan
 * (least recently used out), so replicas that alternate on one plan all
 * replay.  Positions, charges and box may change between calls: the graph
 * reads them from the buffers and from a device parameter block written by
 * an ordinary launch before each replay.  Results are identical to eager
 * execution.  Timing (hsma_plan_set_timing) forces eager launches.        */
hsma_status hsma_plan_set_graph(hsma_plan* plan, int enable);

/* Thread-local description of the last error on this thread.               */
const char* hsma_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HSMA_H */
