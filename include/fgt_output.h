/*
 * fgt_output.h -- C ABI for resolving the output of the box fast Gauss
 * transform (fgt.h) on its own adaptive tree, and for evaluating a tree's
 * piecewise polynomial at arbitrary points.
 *
 * The tree that resolves sigma need not resolve u = G * sigma: a sharp
 * feature diffused a short distance can stay too sharp for the input leaves
 * (Section 4.2).  fgt_output_resolve builds a new tree for u:
 *
 *  - Refinement (Algorithm 5): the error of each leaf's degree p-1 tensor
 *    interpolant of u is estimated from the tail of its Legendre coefficients
 *    (Eq. (funerr): e = sqrt(mean of c_alpha^2 over ||alpha||_2 >= p); for
 *    d = 1 the last two orders).  Leaves with e > eps * ||u||_2 are split,
 *    never below the finest level of the input tree (the remark after
 *    Algorithm 5), the tree is rebalanced, and u is computed on the new leaves.
 *    Repeated until no leaf is flagged.
 *  - Coarsening (Algorithm 6): level by level from the finest, a box whose
 *    2^d children are all leaves gets u at its own nodes from the children's
 *    interpolants; if its e <= eps * ||u||_2 the children are deleted.  The
 *    tree is then rebalanced (Algorithm 6, last step), new leaves taking u
 *    from the interpolant of the leaf they split.
 *
 * ||u||_2 = (int_B u^2)^(1/2) by Gauss-Legendre quadrature on the leaves.
 *
 * How u reaches the new leaves differs from Algorithm 5, which pushes each
 * split box's plane-wave expansion to its children and adds direct terms:
 * here sigma is carried to the new leaves exactly (a degree p-1 polynomial on
 * a leaf is the same polynomial on each of its descendants, sampled at their
 * nodes) and the whole transform (fgt_execute) runs again on the refined tree.
 * Both give the transform of the same piecewise polynomial density.
 *
 * Every function returns FGT_OK or a negative FGT_ERR_* code (fgt.h).  Device
 * arrays are FP64 in the layout of fgt.h.
 */
#ifndef FGT_OUTPUT_H
#define FGT_OUTPUT_H

#include "fgt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fgt_output fgt_output_t;

typedef struct fgt_output_opts {
  double eps;          /* resolution of u: 0 = the transform's tol */
  int32_t refine;      /* 1 = Algorithm 5 (default when opts is NULL) */
  int32_t coarsen;     /* 1 = Algorithm 6 and rebalancing (default when opts is NULL) */
  int32_t max_passes;  /* refinement passes; 0 = until no leaf is flagged */
} fgt_output_opts_t;

typedef struct fgt_output_info {
  int32_t dim, p;
  int32_t passes;               /* transforms run (1 + refinement passes that split leaves) */
  int64_t nleaves_in, nleaves;  /* leaves of the input and of the output tree */
  int64_t nboxes_in, nboxes;    /* all boxes (leaves and their ancestors) */
  int64_t added_refine;         /* boxes added by splitting flagged leaves (2^d per split) */
  int64_t added_refine_balance; /* boxes added to rebalance the refined trees */
  int64_t deleted_coarsen;      /* boxes deleted by coarsening (2^d per merge) */
  int64_t added_balance;        /* boxes added by the final rebalancing */
  double u_l2;                  /* ||u||_2 on the last refined tree */
  double threshold;             /* eps * u_l2, the bound on e per leaf */
  double max_leaf_error;        /* largest e over the output leaves */
} fgt_output_info_t;

/*
 * Runs the transform of sigma_dev ([nleaves][p^d], device) on `tree` (p,
 * delta, tol, bc and opts as in fgt_plan) and resolves u on an output tree as
 * described above.  Synchronous on opts->stream (NULL = the default stream).
 * *out receives an object owned by the caller (fgt_output_destroy) holding
 * the output tree (host) and u on its leaves (device).  oopts may be NULL.
 */
int fgt_output_resolve(const fgt_tree_t* tree, int p, double delta, double tol, int bc,
                       const fgt_opts_t* opts, const fgt_output_opts_t* oopts,
                       const double* sigma_dev, fgt_output_t** out);

int fgt_output_info(const fgt_output_t* o, fgt_output_info_t* info);

/* Copies the output tree's leaves to host arrays level[nleaves],
   coord[nleaves*dim] (Morton order of the lower corners). */
int fgt_output_tree(const fgt_output_t* o, int32_t* level, int32_t* coord);

/* Copies u on the output leaves to u_dev ([nleaves][p^d], device) and waits. */
int fgt_output_values(const fgt_output_t* o, double* u_dev);

/* Releases the object and its device memory.  NULL is ignored. */
void fgt_output_destroy(fgt_output_t* o);

/*
 * Evaluates the piecewise polynomial given by values u_dev ([nleaves][p^d],
 * device) at the tensor Gauss-Legendre nodes of the leaves of `tree` (the
 * leaf model of Eq. (papprox)) at npts points x_dev ([npts][dim], device, in
 * [-1/2, 1/2]^dim), writing out_dev[npts] (device).  A point on a face shared
 * by two leaves takes the leaf on its upper side; points outside the unit box
 * are clamped to it.  The leaves must tile the unit box (as fgt_plan checks;
 * here only levels and coordinates are range-checked).  Asynchronous on
 * `stream` (hipStream_t, NULL = default stream); the tree is copied.
 */
int fgt_interp(const fgt_tree_t* tree, int p, const double* u_dev, int64_t npts,
               const double* x_dev, double* out_dev, void* stream);

/*
 * 2:1 balances a tree (corner adjacency, wrapped when bc = FGT_PERIODIC) by
 * splitting coarse leaves, as the level restriction of Algorithms 3, 5 and 6
 * requires.  Writes at most cap leaves (Morton order) to level_out[cap],
 * coord_out[cap*dim] (host; may be NULL to query) and returns the number of
 * leaves of the balanced tree, or a negative code.  Host only.
 */
int64_t fgt_tree_balance(const fgt_tree_t* tree, int bc, int32_t* level_out, int32_t* coord_out,
                         int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* FGT_OUTPUT_H */
