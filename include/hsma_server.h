/*
 * hsma_server.h -- continuous-batching request server for the HSMA hot path.
 *
 * Serves many independent systems of one plan class (the same method
 * parameters and the same box shape, any size: box_len = s * the class's
 * box) on one GPU, e.g. the replicas of a Monte Carlo or MD ensemble.  A
 * request is one evaluation (energy, potentials, forces; see hsma.h) of one
 * configuration.
 *
 * Scheduling: a scheduler thread owns the device.  Requests wait in a FIFO
 * queue; a request is admitted into a device slot as soon as a slot is free
 * (the HBM budget fixes the number of slots), and its step is enqueued at
 * once on that slot's stream, so requests that arrive while others run join the
 * device work without waiting for a batch boundary and the steps of
 * different systems overlap on the GPU.  A slot keeps its arena and its
 * device copy of the plan between requests; the plan is re-targeted to each
 * request's box by one kernel (no host least-squares work per request).
 * A request's kernels and their order do not depend on what else runs, so
 * its result is bitwise the same alone and in a mix.
 *
 * Ownership: inputs are copied at submit; output buffers given to submit
 * belong to the caller and must stay valid until the request is waited for.
 * Errors are per request: an invalid or oversized request fails alone.
 */
#ifndef HSMA_SERVER_H
#define HSMA_SERVER_H

#include <stdint.h>

#include "hsma.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsma_server hsma_server;

typedef struct hsma_server_cfg {
  hsma_params params;     /* method parameters shared by every request            */
  double box_len[3];      /* box shape of the class (requests: s * box_len)       */
  int64_t max_n;          /* largest particle count a slot must hold (within the
                             per-call limit of hsma.h, else INVALID_ARG)        */
  int max_slots;          /* upper bound on resident requests                     */
  int64_t hbm_budget;     /* device bytes for the slots' arenas and plans
                             (0: half of the free device memory); the number of
                             slots is min(max_slots, budget / bytes per slot)     */
  int queue_capacity;     /* pending requests beyond which submit is refused
                             with HSMA_ERR_BUSY (0: unlimited)                    */
} hsma_server_cfg;

typedef struct hsma_request {
  int64_t n;              /* particles, 1 <= n <= cfg.max_n (else HSMA_ERR_OOM)   */
  const double* xyz;      /* n x 3 host positions, copied at submit               */
  const double* q;        /* n host charges, copied at submit                     */
  double box_lo[3];
  double scale;           /* box = scale * cfg.box_len, scale > 0                 */
  double* potential;      /* n host doubles or NULL, written before wait returns  */
  double* force;          /* n x 3 host doubles or NULL                           */
} hsma_request;

typedef struct hsma_result {
  hsma_status status;     /* per-request outcome                                  */
  double energy;
  double t_submit;        /* seconds on a steady clock                            */
  double t_start;         /* admitted and enqueued on the device                  */
  double t_done;          /* results available on the host                        */
  int slot;               /* device slot that ran it (-1 if never admitted)       */
} hsma_result;

/* Creates the plan class, the slots (arena + plan each) and the scheduler.
 * Errors: INVALID_ARG, GEOMETRY, RANK, NO_DEVICE, OOM (not even one slot
 * fits the budget), DEVICE.                                               */
hsma_status hsma_server_create(const hsma_server_cfg* cfg, hsma_server** out);

/* Queues a request; *ticket identifies it.  Host-side validation as in
 * hsma_compute (NOT_NEUTRAL, OUT_OF_DOMAIN) happens here and is returned
 * directly; OOM if n > max_n; BUSY if the queue is full.                  */
hsma_status hsma_server_submit(hsma_server* s, const hsma_request* req, uint64_t* ticket);

/* Blocks until the request is done, fills *out and forgets the ticket.
 * Returns out->status (HSMA_ERR_INVALID_ARG for an unknown ticket).       */
hsma_status hsma_server_wait(hsma_server* s, uint64_t ticket, hsma_result* out);

/* Number of slots the budget allowed, and bytes per slot.                  */
hsma_status hsma_server_get_slots(const hsma_server* s, int* nslots, int64_t* bytes_per_slot);

/* Stops admitting: requests still queued complete with HSMA_ERR_CANCELLED,
 * admitted ones run to completion, then the scheduler exits.  The server
 * stays valid for hsma_server_wait (results and cancellations can still be
 * collected); hsma_server_submit returns HSMA_ERR_CANCELLED.               */
void hsma_server_shutdown(hsma_server* s);

/* Shuts down (as above), waits for threads already blocked in
 * hsma_server_wait to return, and frees everything.  No call on `s` may
 * start once destroy has begun.                                           */
void hsma_server_destroy(hsma_server* s);

#ifdef __cplusplus
}
#endif
#endif /* HSMA_SERVER_H */
