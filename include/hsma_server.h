/*
 * hsma_server.h -- continuous-batching request server for the HSMA hot path.
 *
 * Serves many independent systems on one GPU, e.g. the replicas of a Monte
 * Carlo or MD ensemble.  A request is one evaluation (energy, potentials,
 * forces; see hsma.h) of one configuration, with its own method parameters
 * (Sec. 3.2 of the paper: each system carries its kspace parameters) and its
 * own box.
 *
 * Plan classes: requests with the same parameters and the same box shape
 * (box_len / box_len[0], equal to 1e-14 relative; the request's box is then
 * the class's shape times box_len[0]) share one plan class, whose least-squares
 * pseudo-inverse (Eq. 6) is built once for the class's unit box and
 * re-targeted to each request's box by one kernel; a box of any size of
 * that shape costs no host least-squares work.  Classes are created when
 * the server starts (cfg.classes: all their factorisations in one grouped
 * device launch) or when a request first names a new one.
 *
 * Scheduling: a scheduler thread owns the device.  Requests wait in a FIFO
 * queue; a request is admitted into a device slot as soon as a slot is free
 * (the HBM budget fixes the number of slots), and its step is enqueued at
 * once on that slot's stream, so requests that arrive while others run join
 * the device work without waiting for a batch boundary and the steps of
 * different systems overlap on the GPU.  A request carrying a system id is
 * preferably given a free slot among whose last 8 requests the same system
 * and class ran (as many as a slot keeps captured steps for); a slot
 * that sees the same system again (same size, same buffers) replays the
 * step it captured in a HIP graph instead of launching it kernel by kernel.
 * Completion: each slot has a thread blocked on the slot's end-of-step
 * event, which reports the slot done (no polling, no host callbacks).
 * A request's kernels and their order do not depend on what else
 * runs, so its result is bitwise the same alone and in a mix.
 *
 * Device-resident systems: with HSMA_REQ_DEVICE the request's pointers are
 * device pointers; the step reads the caller's positions and charges and
 * writes the caller's outputs in place, so a replica's state never leaves
 * HBM.  Inputs must be complete when the step starts: either before submit,
 * or signalled by ready_event (a hipEvent_t the slot's stream waits for).
 *
 * Ownership: host inputs are copied at submit; every output buffer (host or
 * device) and every device input belongs to the caller and must stay valid
 * (and device inputs unmodified) until the request is waited for.  Errors
 * are per request: an invalid or oversized request fails alone.
 */
#ifndef HSMA_SERVER_H
#define HSMA_SERVER_H

#include <stdint.h>

#include "hsma.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsma_server hsma_server;

/* A plan class: method parameters and a box shape (any size of the shape). */
typedef struct hsma_class {
  hsma_params params;
  double box_len[3];
} hsma_class;

typedef struct hsma_server_cfg {
  hsma_params params;     /* default parameters (requests with params NULL)     */
  double box_len[3];      /* default box shape (requests with box_len 0, scale) */
  int64_t max_n;          /* largest particle count a slot must hold (within the
                             per-call limit of hsma.h, else INVALID_ARG)        */
  int max_slots;          /* upper bound on resident requests                     */
  int64_t hbm_budget;     /* device bytes for the slots' arenas and plans
                             (0: half of the free device memory); the number of
                             slots is min(max_slots, budget / bytes per slot)     */
  int queue_capacity;     /* pending requests beyond which submit is refused
                             with HSMA_ERR_BUSY (0: unlimited)                    */
  int n_classes;          /* further plan classes created at start (0: none)   */
  const hsma_class* classes; /* n_classes classes; their least-squares
                             factorisations run together (grouped FP64 matrix-
                             core launches) when their lsq_solver is 1          */
} hsma_server_cfg;

enum { HSMA_REQ_DEVICE = 1 };

typedef struct hsma_request {
  int64_t n;              /* particles, 1 <= n <= cfg.max_n (else HSMA_ERR_OOM)   */
  const double* xyz;      /* n x 3 positions: host (copied at submit) or device  */
  const double* q;        /* n charges: host (copied at submit) or device        */
  double box_lo[3];
  double box_len[3];      /* box edges; all zero: scale * cfg.box_len           */
  double scale;           /* used when box_len is zero; > 0                      */
  const hsma_params* params; /* NULL: cfg.params; copied at submit               */
  double* potential;      /* n doubles or NULL (host, or device with the flag)  */
  double* force;          /* n x 3 doubles or NULL                               */
  double* energy;         /* device requests: 1 device double or NULL (the
                             energy is also returned in hsma_result)           */
  int flags;              /* HSMA_REQ_DEVICE: pointers are device pointers       */
  uint64_t system_id;     /* nonzero: slot affinity key (graph replay)           */
  void* ready_event;      /* device requests: hipEvent_t the step waits for, or NULL */
} hsma_request;

typedef struct hsma_result {
  hsma_status status;     /* per-request outcome (device validation included)    */
  double energy;
  double t_submit;        /* seconds on a steady clock                            */
  double t_start;         /* admitted and enqueued on the device                  */
  double t_done;          /* results available to the caller                      */
  int slot;               /* device slot that ran it (-1 if never admitted)       */
  int replayed;           /* 1 if the step was a replay of a captured graph       */
  int plan_class;         /* index of the request's plan class                    */
} hsma_result;

typedef struct hsma_server_stats {
  int64_t completed;      /* requests finished (any status)                       */
  int64_t graph_replays;  /* steps run as graph replays                           */
  int64_t affinity_hits;  /* requests given a slot that recently ran their system */
  int classes;            /* plan classes created                                 */
  int slots;
} hsma_server_stats;

/* Creates the default class and cfg.classes, the slots and the scheduler.
 * Errors: INVALID_ARG, GEOMETRY, RANK, NO_DEVICE, OOM (not even one slot
 * fits the budget), DEVICE.                                               */
hsma_status hsma_server_create(const hsma_server_cfg* cfg, hsma_server** out);

/* Queues a request; *ticket identifies it.  Host requests are validated
 * here as in hsma_compute (NOT_NEUTRAL, OUT_OF_DOMAIN); device requests on
 * the device (their status is the result's).  A new parameter set or box
 * shape creates its plan class here (errors of hsma_plan_create).  OOM if
 * n > max_n; BUSY if the queue is full; CANCELLED after shutdown.          */
hsma_status hsma_server_submit(hsma_server* s, const hsma_request* req, uint64_t* ticket);

/* Blocks until the request is done, fills *out and forgets the ticket.
 * Returns out->status (HSMA_ERR_INVALID_ARG for an unknown ticket).       */
hsma_status hsma_server_wait(hsma_server* s, uint64_t ticket, hsma_result* out);

/* Number of slots the budget allowed, and bytes per slot.                  */
hsma_status hsma_server_get_slots(const hsma_server* s, int* nslots, int64_t* bytes_per_slot);

hsma_status hsma_server_get_stats(const hsma_server* s, hsma_server_stats* out);

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
