/* cptr_serve.h -- a solve server: many CPTR-(F)GMRES linear solves in flight
 * on one GPU, with continuous admission.
 *
 * Each request is one linear system of a fully implicit simulator's Newton
 * step (the setting of Sec. 1 and Sec. 3 of the paper): a 3x3 block-sparse
 * Jacobian, a right-hand side and a tolerance.  A request runs through
 *   queued -> host setup (AMG hierarchy, ILU(0); cptr_setup's host half)
 *          -> ready (its exact device footprint is known)
 *          -> admitted (a slot is free and the footprint fits the HBM budget)
 *          -> device setup + (F)GMRES on the slot's own stream -> done.
 * Requests are admitted in arrival order as slots and memory free up, while
 * others are on the GPU; their kernels overlap on the device.  All device
 * memory of admitted requests comes from one arena of `hbm_budget_bytes`
 * allocated when the server is created, so admission never calls hipMalloc or
 * hipFree.  A request's result does not depend on what else is in flight:
 * every kernel is deterministic and a request only touches its own memory.
 *
 * Threads: `setup_workers` host threads run host setups (each with
 * `setup.setup_threads` threads of its own, or a number sized to the request
 * when that is 0); `max_inflight` slot threads each own one non-blocking HIP
 * stream.  The server's functions are thread-safe.
 */
#ifndef CPTR_SERVE_H
#define CPTR_SERVE_H

#include <stdint.h>

#include "cptr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cptr_server_s* cptr_server;

typedef struct {
  int32_t max_inflight;      /* slots: requests on the GPU at once (default 4, 1..64) */
  int32_t setup_workers;     /* concurrent host setups (default 8, 1..64) */
  int64_t hbm_budget_bytes;  /* device bytes for all admitted requests (default 16 GiB) */
  int32_t device;            /* HIP device ordinal (default 0) */
  cptr_setup_opts setup;     /* setup options of every request (default cptr_setup_opts_default,
                                with precond_precision = CPTR_PRECISION_FP32 and setup_threads = 0:
                                per request, one thread per 400k block rows, 1 to 4) */
} cptr_server_opts;

typedef struct {
  int32_t status;          /* cptr_status of the request (setup or solve) */
  int32_t iterations;
  int32_t converged;
  int32_t pad_;
  double rel_res_true;
  double queue_s;          /* submitted -> host setup started */
  double host_setup_s;     /* host setup and footprint */
  double admit_wait_s;     /* ready -> admitted (waiting for a slot and HBM) */
  double device_setup_s;   /* device layouts and uploads */
  double solve_s;          /* right-hand side upload, (F)GMRES, solution download */
  double latency_s;        /* submitted -> done */
  int64_t device_bytes;    /* HBM footprint the request was admitted with */
  double admitted_at_s;    /* when the request was admitted, seconds since the server was
                              created (0 if never admitted) */
  double done_at_s;        /* when its solution was back on the host, same clock */
} cptr_serve_info;

typedef struct {
  int64_t submitted, completed, failed;
  int32_t peak_inflight;       /* most requests admitted at once */
  int32_t pad_;
  int64_t peak_reserved_bytes; /* most HBM reserved by admitted requests at once (<= budget) */
  int64_t hbm_budget_bytes;
} cptr_server_stats;

void cptr_server_opts_default(cptr_server_opts* o);

/* Creates the server: validates the options, allocates the HBM arena on
 * `device` and starts the threads.  CPTR_E_INVALID for options out of range,
 * CPTR_E_NOMEM when the arena cannot be allocated. */
cptr_status cptr_server_create(const cptr_server_opts* o, cptr_server* out);

/* Queues one request and returns at once with its id (> 0).  The server copies
 * A (host arrays, on_device = 0, block size 3, elliptic_idx/n_elliptic as for
 * cptr_setup) and b (host, 3 * A->n_block_rows doubles) before returning; `so`
 * NULL means cptr_solve_opts_default.  x0 is zero.  CPTR_E_INVALID for NULL
 * arguments or device arrays; problems found in A itself are reported by the
 * request's status. */
cptr_status cptr_server_submit(cptr_server sv, const cptr_bsr* A, const int32_t* elliptic_idx,
                               int32_t n_elliptic, const double* b, const cptr_solve_opts* so,
                               int64_t* id);

/* Waits for request `id` (timeout_ms < 0: no limit).  On completion copies the
 * solution into x (host, 3 * n_block_rows doubles; may be NULL), fills `info`
 * (may be NULL), forgets the request and returns its status (CPTR_OK or
 * CPTR_NOT_CONVERGED for a finished solve, the error of a failed setup or
 * solve, e.g. CPTR_E_NOMEM when its footprint exceeds the whole budget).
 * CPTR_E_STATE when the timeout expires first (the request stays), CPTR_E_INVALID
 * for an unknown id. */
cptr_status cptr_server_wait(cptr_server sv, int64_t id, double* x, cptr_serve_info* info,
                             int32_t timeout_ms);

/* Message of the last failed request that cptr_server_wait returned. */
const char* cptr_server_last_error(cptr_server sv);

cptr_status cptr_server_get_stats(cptr_server sv, cptr_server_stats* st);

/* Finishes every queued and admitted request, stops the threads and frees the
 * arena.  Results not yet waited for are dropped. */
cptr_status cptr_server_destroy(cptr_server sv);

#ifdef __cplusplus
}
#endif

#endif /* CPTR_SERVE_H */
