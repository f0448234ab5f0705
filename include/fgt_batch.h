/*
 * fgt_batch.h -- C ABI for running many independent box fast Gauss
 * transforms (fgt.h) together on one device.
 *
 * A batch groups resident plans (Algorithm 4 each, with its own tree, p, delta,
 * tol, boundary condition and precision) by kernel class -- dimension, compute
 * precision, plane-wave mode tiles ceil(nr/16) and node steps -- and runs each
 * stage of the method (formation, merge, out->in translation, evaluation, near
 * field) once per class for all its transforms: a launch covers every
 * transform of the class, each workgroup finding its transform from a table
 * of block ranges.  The launches of one execution are captured once in a HIP
 * graph and replayed.  Results are bitwise identical to fgt_execute of each
 * plan alone (the same kernel bodies, the same fixed-order reductions).
 *
 * The schedule -- how many streams the classes are spread over and whether a
 * stream runs its classes stage by stage or class by class -- and the tile
 * shape of the d = 3 box formation are chosen at fgt_batch_create.  Tile
 * shapes change neither the columns nor the order of any sum: results stay
 * bitwise identical.
 *
 * 1D plans are accepted and run with their own (non-batched) launches inside
 * the same graph.  Every function returns FGT_OK or a negative FGT_ERR_* code.
 */
#ifndef FGT_BATCH_H
#define FGT_BATCH_H

#include "fgt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fgt_batch fgt_batch_t;

typedef struct fgt_batch_opts {
  void* stream;        /* hipStream_t the batch runs on; NULL = the HIP default stream */
  int32_t use_graph;   /* 1 (default when opts is NULL) = capture and replay a HIP graph;
                          0 = launch directly every time */
  int32_t nstreams;    /* schedule: streams the classes are spread over (1..8; 0 = 1) */
  int32_t class_major; /* schedule: 1 = each stream runs its classes one after the other,
                          0 = stage by stage across its classes */
  int32_t form_tile;   /* box-formation tile shape of every d = 3 class: 0 (default) = four
                          16-column slabs per wave, as fgt_execute; 1 = two */
  int32_t persistent;  /* 1 = one persistent launch per kernel class running every stage of
                          every transform of the class (a work queue in stage order; a block
                          waits, with a device-scope acquire, for its transform's previous
                          stage).  Switched off: fgt_batch_create returns FGT_ERR_UNSUPPORTED
                          (on the device such a batch did not finish).  0 (default) = one
                          launch per class and stage */
} fgt_batch_opts_t;

typedef struct fgt_batch_info {
  int64_t njobs, npoints;
  int32_t nclasses;     /* kernel classes of d = 2, 3 */
  int32_t nsingle;      /* 1D plans run one by one */
  int32_t nlaunches;    /* kernel launches per execution */
  int32_t nstreams, class_major, use_graph;
  double tuned_ms;      /* 0: the autotuner is switched off (fgt_batch_tune) */
  int32_t tile_alt_classes; /* classes whose box formation runs the alternative tile shape */
  int32_t persistent;       /* classes run as one persistent launch each */
  int32_t persistent_error; /* 1 if a persistent launch's bounded wait ran out since the batch
                               was created (read after a device synchronize; its results are
                               then not to be used) */
} fgt_batch_info_t;

/* Builds a batch over nplans resident plans (not host-only, all on the current
   device).  The batch keeps pointers to the plans, which must outlive it and
   must not be executed concurrently with it. */
int fgt_batch_create(fgt_plan_t* const* plans, int64_t nplans, const fgt_batch_opts_t* opts,
                     fgt_batch_t** out);

/* Sets the device arrays of every transform: sigma[i] and u[i] (host arrays of
   nplans device pointers, layout as in fgt.h).  Waits for earlier executions
   of the batch to finish; the graph is kept. */
int fgt_batch_bind(fgt_batch_t* b, const double* const* sigma, double* const* u);

/* Enqueues one execution of every transform of the batch on its stream. */
int fgt_batch_execute(fgt_batch_t* b);

/* Schedule autotuner: switched off.  It re-captured the batch graph once per
   trial schedule and crashed the host process intermittently on large batches,
   for a reason not established; it now returns FGT_ERR_UNSUPPORTED (and 0 in
   *best_ms, which may be NULL) without touching the device. */
int fgt_batch_tune(fgt_batch_t* b, int32_t reps, double* best_ms);

int fgt_batch_info(const fgt_batch_t* b, fgt_batch_info_t* info);

/* Waits for the batch's work and releases it (not its plans).  b may be NULL. */
int fgt_batch_destroy(fgt_batch_t* b);

#ifdef __cplusplus
}
#endif

#endif /* FGT_BATCH_H */
