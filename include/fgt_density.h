/*
 * fgt_density.h -- C ABI for building the input of the box fast Gauss
 * transform on the device: an adaptive, level-restricted tree that resolves a
 * density, with the density sampled at every leaf's tensor Gauss-Legendre
 * nodes (Algorithm 3).
 *
 * The density is a sum of Gaussians, sigma(x) = sum_i a_i exp(-|x - c_i|^2 /
 * w_i^2), optionally periodized over the 3^d nearest images: the family the
 * benchmark workloads are drawn from.  Algorithm 3 runs level by level: the
 * boxes of a level are sampled at their nodes (a kernel), the error of each
 * box's degree p-1 interpolant is estimated from its Legendre tail (Eq.
 * (funerr), the same kernel as the output trees of fgt_output.h), and boxes
 * with e > eps * ||sigma||_2 are split; the leaf tree is then 2:1 balanced
 * (corner adjacency, wrapped when periodic) and sampled.  ||sigma||_2 is the
 * closed form (int_{R^d} sigma^2)^(1/2) of the non-periodized sum unless the
 * caller gives one.
 *
 * Every function returns FGT_OK or a negative FGT_ERR_* code (fgt.h).
 */
#ifndef FGT_DENSITY_H
#define FGT_DENSITY_H

#include "fgt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fgt_gaussians {
  int32_t dim;            /* 1, 2 or 3 */
  int64_t n;              /* number of Gaussians, >= 1 */
  const double* centers;  /* [n][dim], host */
  const double* widths;   /* [n], w_i > 0 (host) */
  const double* amps;     /* [n], host */
  int32_t periodic;       /* 1 = each Gaussian summed over the shifts {-1,0,1}^dim */
} fgt_gaussians_t;

typedef struct fgt_resolve_opts {
  int32_t min_level;      /* boxes above this level are always split (default 0) */
  int32_t max_level;      /* boxes at this level are never split (default 12, at most
                             19 / 28 / 30 for d = 3 / 2 / 1) */
  int64_t max_leaves;     /* 0 = no limit; else FGT_ERR_UNSUPPORTED when the unbalanced
                             tree would exceed it */
  double norm;            /* ||sigma||_2 of the split test; 0 = the closed form */
  void* stream;           /* hipStream_t; NULL = the default stream */
} fgt_resolve_opts_t;

typedef struct fgt_density_info {
  int32_t dim, p;
  int64_t nleaves;        /* leaves of the balanced tree */
  int64_t nleaves_unbalanced;
  int64_t boxes_sampled;  /* boxes whose nodes were sampled for the split test */
  int32_t lmin, lmax;
  double norm, threshold; /* ||sigma||_2 and eps * ||sigma||_2 */
} fgt_density_info_t;

typedef struct fgt_density fgt_density_t;

/*
 * Runs Algorithm 3 for the Gaussian sum g at p nodes per axis and tolerance
 * eps in (0, 1).  Synchronous on opts->stream.  *out receives the tree (host)
 * and sigma on its leaves (device), owned by the caller (fgt_density_destroy).
 * opts may be NULL.
 */
int fgt_resolve_gaussians(const fgt_gaussians_t* g, int p, double eps, const fgt_resolve_opts_t* opts,
                          fgt_density_t** out);

int fgt_density_info(const fgt_density_t* r, fgt_density_info_t* info);

/* Copies the leaves (Morton order of the lower corners) to host arrays
   level[nleaves], coord[nleaves*dim]. */
int fgt_density_tree(const fgt_density_t* r, int32_t* level, int32_t* coord);

/* Copies sigma on the leaves to sigma_dev ([nleaves][p^dim], device) and waits. */
int fgt_density_values(const fgt_density_t* r, double* sigma_dev);

/* Releases the result and its device memory.  NULL is ignored. */
void fgt_density_destroy(fgt_density_t* r);

/*
 * Samples the Gaussian sum g at the tensor Gauss-Legendre nodes of the leaves
 * of `tree` into sigma_dev ([nleaves][p^dim], device, layout of fgt.h).
 * Waits for `stream` (NULL = default stream) before returning.  Levels and
 * coordinates are range-checked; the leaves need not tile the box.
 */
int fgt_sample_gaussians(const fgt_gaussians_t* g, const fgt_tree_t* tree, int p, double* sigma_dev,
                         void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FGT_DENSITY_H */
