/*
 * fgt_point.h -- the discrete (point) Gauss transform on MI355X.
 *
 * Computes Section 1, Eq. (pgt),
 *
 *     u(x_i) = sum_j exp(-|x_i - y_j|^2 / delta) q_j,   i = 1..M, j = 1..N,
 *
 * for sources y_j and targets x_i in [-1/2, 1/2]^d (d = 2, 3; free space),
 * by the scheme of Section 3 with the paper's closing remark applied: the
 * points are sorted on Algorithm 1's level-restricted tree (boxes with more
 * than n_s sources or targets split down to the cutoff level, whose boxes have
 * side >= D0 sqrt(delta)); a target in a cutoff-level box takes its dense
 * colleagues (more than n_s points, the P-list) by plane waves (Theorem 1,
 * Eqs. (multipoleexpansion), (diagonaltranslation), (localexpansion)) and the
 * rest of its neighbor list (the D-list) directly, Eq. (pgt2).  Instead of
 * NUFFTs, the points of a plane-wave box are represented on tensor grids of
 * p Gauss-Legendre "proxy" nodes per axis on the boxes of a finer level:
 * charges are spread to the grid with Lagrange weights, the grid forms and
 * evaluates expansions in tensor form (the box transform's kernels), and the
 * grid's potential is interpolated back to the targets.  The proxy level is
 * chosen so that p nodes interpolate every plane wave of the expansion to
 * tol / (10 d).
 *
 * Points are given on the host at planning time (the tree is built there);
 * charges and potentials are device arrays at execution time.  Every
 * function returns FGT_OK or a negative FGT_ERR_* code (fgt.h) and never
 * throws; fgt_last_error() gives detail.
 */
#ifndef FGT_POINT_H
#define FGT_POINT_H

#include <stdint.h>

#include "fgt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fgt_point_opts {
  int32_t p;          /* proxy nodes per axis, 4..16 (0: 16) */
  int32_t ns;         /* Algorithm 1's n_s: boxes with more sources or targets are split,
                         and a cutoff-level box with more is dense (0: 64) */
  int32_t host_only;  /* 1: build the host plan only (fgt_point_info / fgt_point_array work,
                         fgt_point_execute refuses) */
  void* stream;       /* HIP stream of every execution (NULL: the default stream) */
} fgt_point_opts_t;

typedef struct fgt_point_info {
  int32_t dim, p, ns;
  int32_t lc;          /* cutoff level */
  int32_t lp;          /* proxy level (boxes carrying the proxy grids) */
  int32_t nr;          /* real plane-wave modes per axis, 2M - 1 */
  int64_t nsrc, ntgt;
  int64_t nleaves;     /* leaves of Algorithm 1's tree */
  int64_t ndense;      /* cutoff-level leaves with more than n_s points */
  int64_t npwbox;      /* boxes with incoming expansions (dense ones also form them) */
  int64_t nproxy;      /* proxy grids */
  int64_t nplist;      /* translations */
  int64_t ndirect_terms; /* source-target pairs summed directly */
  double delta, tol;
  double proxy_err;    /* largest interpolation error of a plane wave on a proxy box */
  int64_t device_bytes;
} fgt_point_info_t;

typedef struct fgt_point_plan fgt_point_plan_t;

/*
 * Plans the transform for src [nsrc][dim] and tgt [ntgt][dim] (host arrays,
 * copied; every coordinate in [-1/2, 1/2]).  delta > 0, tol in [1e-12, 0.1).
 * FGT_ERR_UNSUPPORTED when delta is so small that the cutoff level exceeds
 * the build's depth, or p cannot reach tol at any proxy level this build
 * allows.  opts may be NULL.  *out is owned by the caller (fgt_point_destroy).
 */
int fgt_point_plan(int dim, int64_t nsrc, const double* src, int64_t ntgt, const double* tgt,
                   double delta, double tol, const fgt_point_opts_t* opts, fgt_point_plan_t** out);

/*
 * u_dev [ntgt] = the transform of the charges q_dev [nsrc] (device arrays in
 * the caller's point order, owned by the caller; u is overwritten).
 * Asynchronous on the plan's stream; calls on one plan are serialized by it.
 */
int fgt_point_execute(fgt_point_plan_t* plan, const double* q_dev, double* u_dev);

int fgt_point_info(const fgt_point_plan_t* plan, fgt_point_info_t* info);

/*
 * Copies a host array of the plan for inspection (int32 unless noted):
 * "leaf_level", "leaf_coord", "leaf_dense", "src_perm", "tgt_perm",
 * "leaf_src_start", "leaf_tgt_start", "dl_tgt", "dl_haspw", "dl_start",
 * "dl_src", "px_coord", "px_src_start", "px_tgt_start", "plist_start",
 * "plist_src", "plist_dir", "pw_start", "pwleaf_id".  Writes at most cap
 * elements (dst may be NULL to query) and returns the length, or a negative code.
 */
int64_t fgt_point_array(const fgt_point_plan_t* plan, const char* name, void* dst, int64_t cap);

/* Releases the plan.  NULL is ignored. */
void fgt_point_destroy(fgt_point_plan_t* plan);

#ifdef __cplusplus
}
#endif

#endif /* FGT_POINT_H */
