/*
 * fgt_serve.h -- C ABI of the request loop that serves many box fast Gauss
 * transforms (fgt.h) on one device.
 *
 * A caller submits requests; each names a request type by an integer key.
 * All requests with one key share the tree, p, delta, tol, boundary condition
 * and precision of the first submission with that key (the caller's promise;
 * a mismatch in the scalar parameters or the leaf count is rejected).  The
 * server keeps, per key, the plan of Algorithm 4 -- the flat tree, the lists
 * and the precomputed 1D tables of Section 4 -- resident in device memory, so
 * later requests of the same type skip planning and uploads.
 *
 * Scheduling (continuous admission, not a FIFO queue):
 *  - a scheduler thread inside the server admits waiting requests in arrival
 *    order, skipping any that cannot start yet, whenever a slot (one of
 *    `nslots` HIP streams at the default priority) is free;
 *  - a request can start when its type's plan is resident and one of the
 *    plan's workspaces (the per-execution intermediates) is idle; a second,
 *    third, ... workspace of a busy plan is added while memory allows, so
 *    requests of one type can overlap too;
 *  - device memory held by the server (tables, lists, workspaces and, for
 *    host-memory requests, staging for sigma and u) never exceeds
 *    `hbm_budget`.  When admission needs room, idle extra workspaces and then
 *    idle plans with no waiting requests are released, least recently used
 *    first; a request whose type alone exceeds the budget fails with
 *    FGT_ERR_OOM;
 *  - new request types are planned on the host by `nbuilders` builder threads
 *    while the device keeps running other requests.
 *
 * Results are bitwise identical to fgt_execute of the same plan: every
 * request runs the same kernels in the same order on its own workspace, and
 * the kernels reduce with gathers in a fixed order (no atomics).
 *
 * Every function returns FGT_OK (0) or a negative FGT_ERR_* code (fgt.h).
 * Functions may be called from several threads; fgt_last_error() is per thread.
 */
#ifndef FGT_SERVE_H
#define FGT_SERVE_H

#include "fgt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fgt_server fgt_server_t;

typedef struct fgt_server_opts {
  int32_t nslots;      /* concurrent executions (HIP streams), 1..64; 0 = 4 */
  int32_t nbuilders;   /* host threads that plan new request types, 1..16; 0 = 2 */
  int64_t hbm_budget;  /* device bytes the server may hold; 0 = 90% of the free
                          device memory when the server is created */
} fgt_server_opts_t;

typedef struct fgt_request {
  int64_t key;               /* request type, see above */
  const fgt_tree_t* tree;    /* needed only for the first request of a key (the
                                tree is copied); may be NULL afterwards */
  int32_t p;
  double delta, tol;
  int32_t bc;                /* FGT_FREE or FGT_PERIODIC */
  int32_t precision;         /* FGT_FP64 or FGT_FP32 */
  const double* sigma;       /* [nleaves][p^d] as in fgt.h */
  double* u;                 /* [nleaves][p^d] result */
  int32_t host_io;           /* 0: sigma and u are device memory that the caller keeps
                                valid until the request completes; 1: they are host
                                memory (pinned memory keeps the copies asynchronous),
                                staged through server-owned device buffers that count
                                against the budget */
} fgt_request_t;

typedef struct fgt_completion {
  int64_t id;                /* as returned by fgt_server_submit */
  int64_t key;
  int32_t status;            /* FGT_OK or the error that ended the request */
  int32_t cache_hit;         /* 1 if the key's plan had been built before this request */
  int64_t npoints;           /* nleaves * p^d */
  double queue_ms;           /* submit -> launch on a slot */
  double total_ms;           /* submit -> completion seen by the scheduler */
  double device_ms;          /* the transform's kernels on the slot stream (HIP events;
                                host-memory copies excluded) */
} fgt_completion_t;

typedef struct fgt_server_stats {
  int64_t submitted, completed, failed;
  int64_t plans_built;        /* host plans built (one per new key) */
  int64_t plans_uploaded;     /* uploads to the device, re-uploads after eviction included */
  int64_t plans_evicted;
  int64_t workspaces_added;   /* workspaces beyond each plan's first */
  int64_t resident_bytes, peak_resident_bytes, budget_bytes;
  int32_t nslots, running, waiting;
} fgt_server_stats_t;

/* Creates a server on the current HIP device and starts its threads.  opts may
   be NULL for the defaults. */
int fgt_server_create(const fgt_server_opts_t* opts, fgt_server_t** out);

/* Queues one request and returns at once with its id (ids start at 1 and
   increase).  Errors found here (bad arguments, a key reused with other
   parameters, the server shutting down) are returned and nothing is queued;
   errors found later are reported in the request's completion. */
int fgt_server_submit(fgt_server_t* srv, const fgt_request_t* req, int64_t* id);

/* Moves up to `max` completions, oldest first, into out[] and sets *n.  Never
   blocks. */
int fgt_server_poll(fgt_server_t* srv, fgt_completion_t* out, int32_t max, int32_t* n);

/* As fgt_server_poll, but first waits until a completion is available, the
   server is idle (nothing waiting or running) or timeout_ms has passed
   (timeout_ms < 0: no limit). */
int fgt_server_wait(fgt_server_t* srv, fgt_completion_t* out, int32_t max, int32_t* n,
                    double timeout_ms);

/* Blocks until every submitted request has completed.  Completions stay
   available to fgt_server_poll. */
int fgt_server_drain(fgt_server_t* srv);

int fgt_server_stats(fgt_server_t* srv, fgt_server_stats_t* out);

/* Drains, stops the threads and releases every plan, workspace and stream.
   srv may be NULL. */
int fgt_server_destroy(fgt_server_t* srv);

#ifdef __cplusplus
}
#endif

#endif /* FGT_SERVE_H */
