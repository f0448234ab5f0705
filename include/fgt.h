/*
 * fgt.h -- C ABI of the MI355X machine fast Gauss transform.
 *
 * Computes the continuous Gauss transform of Greengard, Jiang, Rachh and
 * Wang, "A new version of the adaptive fast Gauss transform for discrete and
 * continuous sources", Section 1, Eq. (bgt):
 *
 *     u(x) = int_B G(x - y; delta) sigma(y) dy,   B = [-1/2, 1/2]^d,
 *
 * with G the free-space Gaussian exp(-|x|^2/delta) (Eq. (gkernel)) or its
 * periodization over Z^d (Eq. (gper_kernel)).  sigma is given on a
 * level-restricted adaptive tree with p^d tensor-product Gauss-Legendre
 * samples on every leaf (Section 4, Algorithm 3; Definition treedefs), and u is
 * returned at the same nodes (Algorithm 4: "potentials evaluated at all tensor
 * product grid points on all leaf boxes").
 *
 * Conventions shared by every entry point:
 *  - Leaf i is the box of side 2^-level[i] whose lower corner is
 *    -1/2 + coord[i*dim+a] * 2^-level[i] on axis a (0 <= coord < 2^level).
 *    Its center is -1/2 + (coord + 1/2) 2^-level.
 *  - Within a leaf, node (i_1, ..., i_d) sits at center + (L/2)(eta_{i_1}, ...,
 *    eta_{i_d}), eta the ascending Gauss-Legendre nodes on [-1,1] (Lemma
 *    polycost), and is stored at offset i_1 + p*i_2 + p^2*i_3 (axis 1 fastest).
 *  - sigma and u are arrays [nleaves][p^d] of doubles in the caller's leaf
 *    order, in DEVICE memory (for example torch tensors on cuda:0).
 *  - Every function returns FGT_OK (0) or a negative FGT_ERR_* code and never
 *    throws; fgt_strerror() names the code, fgt_last_error() gives detail.
 */
#ifndef FGT_H
#define FGT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FGT_OK 0
#define FGT_ERR_INVALID_ARG (-1)  /* p, delta, tol, bc, dim or a pointer out of range */
#define FGT_ERR_NOT_TILING (-2)   /* leaves overlap, leave gaps or leave [0,2^level) */
#define FGT_ERR_NOT_BALANCED (-3) /* two leaves sharing a boundary point differ by >1 level */
#define FGT_ERR_OOM (-4)          /* device or host allocation failed */
#define FGT_ERR_UNSUPPORTED (-5)  /* a configuration this build does not implement */
#define FGT_ERR_HIP (-6)          /* a HIP runtime call failed */

#define FGT_FREE 0     /* free-space kernel, Eq. (gkernel) */
#define FGT_PERIODIC 1 /* periodic kernel, Eq. (gper_kernel); Section 5 */

#define FGT_FP64 0 /* every contraction in FP64 */
#define FGT_FP32 1 /* contractions and expansions in FP32 with FP32 accumulation;
                      tables are built in FP64 and rounded once; sigma/u stay FP64.
                      Adds about 2e-7 relative l2 error: fgt_plan accepts it for
                      tol >= 1e-6 only (FGT_ERR_UNSUPPORTED below) */
#define FGT_BF16X3 2 /* as FGT_FP32, but every matrix product runs as three bf16
                        matrix-core products of hi/lo splits of its FP32 operands
                        (the lo x lo term dropped), accumulated in FP32; translations
                        stay FP32.  About 1e-5 relative error per product and 3e-6
                        relative l2 error on u: accepted for tol >= 1e-4 only */

typedef struct fgt_tree {
  int32_t dim;           /* 1, 2 or 3 */
  int64_t nleaves;
  const int32_t* level;  /* [nleaves], host memory, copied by fgt_plan */
  const int32_t* coord;  /* [nleaves*dim], host memory, copied by fgt_plan */
} fgt_tree_t;

typedef struct fgt_opts {
  int32_t precision;     /* FGT_FP64 (default), FGT_FP32 or FGT_BF16X3 */
  double eps_internal;   /* plane-wave tolerance eps of Theorem 1; 0 = derived from tol */
  int32_t force_lc;      /* -1 = automatic cutoff level; else a level <= the automatic one */
  void* stream;          /* hipStream_t for fgt_execute; NULL = the HIP default stream */
  int32_t own_stream;    /* 1 = the plan creates (and destroys) a non-blocking stream of
                            its own and ignores `stream` */
  int32_t profile;       /* 1 = record HIP events around every stage (fgt_stage_times) */
  int32_t host_only;     /* 1 = build the host plan only (no device memory); for inspection */
  int32_t no_fuse;       /* 1 = never fuse the 3D translation with the first evaluation step
                            (fgt_info_t.fused_translate); batches of many transforms run
                            faster unfused */
} fgt_opts_t;

typedef struct fgt_info {
  int32_t dim, p, bc, precision;
  int32_t lc;            /* cutoff level (boxes of side >= D0 sqrt(delta)) */
  int32_t lmin, lmax;    /* leaf levels */
  int32_t nf;            /* 2M, the mode count n_f of Theorem 1 */
  int32_t nr;            /* real modes per axis actually used, 2M-1 */
  double delta, tol, eps, D0, R, h;
  int64_t nleaves, npoints;
  int64_t n_pwbox;       /* cutoff-level boxes that hold expansions (f = 1) */
  int64_t n_pwleaf;      /* leaves that form and evaluate expansions */
  int64_t n_plist;       /* outgoing->incoming translations */
  int64_t n_near_target, n_near_pair;
  double flops_form, flops_eval, flops_translate, flops_near; /* algorithmic, per execute */
  double bytes_min;      /* algorithmic minimum HBM bytes per execute */
  int64_t device_bytes;  /* device memory held by the plan; for a host-only plan, the
                            bytes it would hold once on the device (an upper bound) */
  int64_t n_plane, n_row; /* d = 3: plane-wave leaves grouped by (box, level, axis-3
                            position) and, within those, by axis-1 position; formation and
                            evaluation apply each 1D table once per group; 0 for d < 3 */
  int64_t n_near_source; /* distinct leaves that are near-field sources */
  int64_t n_near_haspw;  /* near-field targets that also receive a plane-wave evaluation */
  int32_t fused_translate; /* d = 3: 1 if the out->in translations run fused with the first
                              evaluation contraction (incoming expansions never stored); chosen
                              when they would exceed 128 MB and nr <= 64 */
  int32_t fourier;       /* 1 = periodic transform with cutoff level <= 1, run as the
                            periodic kernel's truncated Fourier series on the root
                            (Sections 2.2 and 5): lc = 0, nr = 2 n_p + 1, R = 0,
                            h = 2 pi sqrt(delta), no near field */
  int32_t nr_stored;     /* modes stored per axis, 2M = nr + 1: mode m's (cos, sin) pair at
                            2m, 2m+1, the constant at 0 and an exact zero at 1; the stride
                            of the "F" and "E" arrays and of every expansion */
} fgt_info_t;

typedef struct fgt_plan fgt_plan_t;

/*
 * Plans a transform (Algorithm 4 precomputation, Section 4.1).  Validates the
 * tree (tiling, 2:1 balance with corner adjacency, periodic wrap if
 * bc == FGT_PERIODIC), chooses eps, the cutoff level and the plane-wave modes
 * (Theorem 1), builds the flat per-level lists and the FP64 1D tables, and
 * uploads everything to the current HIP device.  p in [1,16]; delta > 0;
 * tol in (0, 0.1) (Theorem 1 needs eps < 0.1).  Periodic trees take one layer
 * of image boxes at a cutoff level >= 2 and the truncated Fourier series of
 * the periodic kernel on the root otherwise (Section 5; fgt_info_t.fourier);
 * FGT_ERR_UNSUPPORTED if that series needs more than 128 real modes
 * (2 n_p + 1 > 128, only with force_lc on a small delta), and for a
 * reduced precision below its smallest tol (FGT_FP32: 1e-6, FGT_BF16X3: 1e-4).
 * opts may be NULL.  *out receives a plan owned by the caller (fgt_destroy).
 */
int fgt_plan(const fgt_tree_t* tree, int p, double delta, double tol, int bc,
             const fgt_opts_t* opts, fgt_plan_t** out);

/*
 * Runs the transform: sigma_dev [nleaves][p^d] in, u_dev [nleaves][p^d] out
 * (overwritten), both device pointers owned by the caller.  Asynchronous on
 * the plan's stream; the plan's workspace is reused, so calls on one plan are
 * serialized by that stream.  Errors from asynchronous work surface on
 * fgt_sync.
 */
int fgt_execute(fgt_plan_t* plan, const double* sigma_dev, double* u_dev);

/*
 * For callers that cannot allocate device memory at execution time (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): fgt_execute with the workspace (plane intermediates, expansions,
 * partial sums) taken from a static device array of 64 MiB that the library
 * holds on every GPU it runs on until the process ends, instead of the plan's
 * own workspace.  Allocates nothing and calls no allocating routine; results
 * are bitwise those of fgt_execute.  Returns FGT_ERR_UNSUPPORTED, without
 * enqueuing anything, when the plan's workspace exceeds 64 MiB (small and
 * medium trees fit; the 3D p = 16 trees of millions of points do not).  All
 * calls on one GPU share that array, and it keeps the last call's contents:
 * calls that may overlap on one GPU (plans on different streams, or from
 * different threads) race and must be ordered by the caller.  Asynchronous on
 * the plan's stream, like fgt_execute.
 */
int fgt_execute_noalloc(fgt_plan_t* plan, const double* sigma_dev, double* u_dev);

/* Waits for the plan's stream.  Returns FGT_ERR_HIP if queued work failed. */
int fgt_sync(fgt_plan_t* plan);

/* Fills *info (any plan, including host-only plans). */
int fgt_plan_info(const fgt_plan_t* plan, fgt_info_t* info);

/*
 * Per-stage device times in milliseconds of the last fgt_execute of a plan
 * made with opts.profile = 1, after fgt_sync: ms[0..5] = form-leaf,
 * form-box, translate, eval-box, eval-leaf, near.  Returns the number of
 * stages written (<= n).
 */
int fgt_stage_times(const fgt_plan_t* plan, double* ms, int n);

/* Releases the plan and its device memory.  NULL is ignored. */
void fgt_destroy(fgt_plan_t* plan);

const char* fgt_strerror(int code);
const char* fgt_last_error(void); /* thread-local detail of the last failure */

/*
 * n_f(R) = 2 ceil(D0 (R + D0)/pi), D0 = sqrt(log(3/eps)): the number of plane
 * waves of Theorem 1 for range R*sqrt(delta) (Table 1 lists it for R = 2, 3,
 * 4 D0).  r_over_d0 gives R in units of D0.  Host only.
 */
int fgt_pw_terms(double eps, double r_over_d0);

/*
 * n_p = ceil(sqrt(log(1/eps))/(pi sqrt(delta))): Fourier terms of the periodic
 * Gaussian on the unit interval (Section 2.2, Table 2).  Host only.
 */
int fgt_periodic_terms(double eps, double delta);

/*
 * Copies a host-side array of a plan (host-only or full) for inspection:
 * name is one of "F" ([table][nr_stored][p]), "E" ([table][p][nr_stored]),
 * "V", "rot" (double) or "pwbox_isleaf", "pw_start",
 * "pwleaf_id", "pwleaf_tab", "pwleaf_box", "box_order", "plist_start",
 * "plist_src", "plist_dir", "echunk", "fitem", "fred", "near_tgt",
 * "near_haspw", "near_start", "near_src", "near_tab", "ftab_meta", "vtab_meta",
 * "plane_start", "plane_tab", "plane_row", "row_start", "row_tab",
 * "plane_order" (planes in dispatch order), and the
 * fused translation's target groups "te_start", "te_mem" (4 member boxes per
 * group, -1 = empty), "te_src", "te_dir" (one word per entry, byte t the
 * direction code of member t, 0xFF = not a source of it) and its workgroups
 * "te_wg" (group, tile) (int32).
 * Writes at most cap elements to dst (may be NULL to query) and returns the
 * array's length, or a negative code.
 */
int64_t fgt_plan_array(const fgt_plan_t* plan, const char* name, void* dst, int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* FGT_H */
