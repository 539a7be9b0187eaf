/*
 * hsma_debug.h -- host-only views of the HSMA plan, for tests.
 *
 * These calls build the host FP64 part of a plan (check points, image
 * tables, least-squares pseudo-inverse, sphere maps; see hsma_plan_create
 * in hsma.h) without touching a GPU, so that it can be compared with an
 * independent implementation.  Not part of the per-step path.
 */
#ifndef HSMA_DEBUG_H
#define HSMA_DEBUG_H

#include <stdint.h>

#include "hsma.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsma_host_plan hsma_host_plan;

/* Real regular solid harmonics of degree 1..p at scaled point xi = r/R,
 * orthonormal on the unit sphere (the plan's basis for the harmonic series
 * of Eq. 5).  val: (p+1)^2-1 values; grad (optional): 3 per value, w.r.t. xi. */
hsma_status hsma_debug_solid_harmonics(int p, const double xi[3], double* val, double* grad);

/* Sort key of cell (x, y, z) of the 1024^3 grid (10 bits per axis) that
 * orders the particles each step: the position along a 3D Hilbert curve.  */
uint32_t hsma_debug_hilbert_key(uint32_t x, uint32_t y, uint32_t z);

/* Builds only the host part of a plan.  Same parameter checks and errors as
 * hsma_plan_create except that no device is used.                         */
hsma_status hsma_debug_host_plan_create(const hsma_params* params, const double box_lo[3],
                                        const double box_len[3], hsma_host_plan** out);
void hsma_debug_host_plan_destroy(hsma_host_plan* hp);

/* Copies the named plan array into out[0..cap) (as doubles, row-major) and
 * returns its full length; -1 for an unknown name.  Names: "Praw" (nb x
 * 2*ncheck), "check_pos" (ncheck x 3, box-centred), "check_axis",
 * "check_groups" (first, count, desc_off, ndesc), "desc_particles" and
 * "desc_check" (sx, sy, sz, sigma, scale per entry), "ysurf", "nsurf"
 * (F x 3), "SQ", "SD" (F x nb), "scalars" (R, nb, nrows, cond).          */
int64_t hsma_debug_host_plan_get(const hsma_host_plan* hp, const char* name, double* out, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif /* HSMA_DEBUG_H */
