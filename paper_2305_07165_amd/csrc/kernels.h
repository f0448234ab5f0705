// Device-side arguments of one transform and the stage launcher.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fgt_host.h"

namespace fgt {

// phi of a fused d = 3 plan is stored tile-major, so that the translation's
// workgroup reads one contiguous block per source box: with tp (m1, m2) mode
// pairs per tile (the plan's te_tp), a box holds ceil(M^2 / tp) blocks of nr
// rows (r3) by 4 tp columns, and column (r1, r2), pair j = (r1 / 2) M + r2 / 2,
// sits in block j / tp at (r1 & 1) 2 tp + 2 (j % tp) + (r2 & 1).  Other plans
// (tp = 0) store [r3][r1][r2] (d = 3).
__host__ __device__ inline int64_t phi_box_coefs(int d, int M, int nr, int tp) {
  if (tp <= 0) {
    int64_t n = nr;
    for (int a = 1; a < d; a++) n *= nr;
    return n;
  }
  return (int64_t)((M * M + tp - 1) / tp) * nr * 4 * tp;
}
// offset of column (r1, r2) of row 0 inside a tiled box; rows are 4 tp apart
__host__ __device__ inline int64_t phi_tiled_col(int M, int tp, int nr, int r1, int r2) {
  const int j = (r1 >> 1) * M + (r2 >> 1);
  const int tile = j / tp;
  return (int64_t)tile * nr * 4 * tp + (r1 & 1) * 2 * tp + 2 * (j - tile * tp) + (r2 & 1);
}

struct DeviceArgs {
  int d = 0, p = 0, nr = 0, M = 0;
  bool fp32 = false;  // FP32 storage (FP32 or BF16x3 products)
  bool bf3 = false;   // products as split bf16 matrix-core steps (Bf16x3 in mfma.h)
  bool fuse_te = false;  // d = 3: translation fused with the first evaluation step (no psi)
  int64_t nA = 0, nL = 0, nE = 0, nT = 0;
  // tables (compute precision)
  const void *F = nullptr, *E = nullptr, *V = nullptr, *rot = nullptr;
  // lists
  const int32_t *pw_start = nullptr, *pwleaf_id = nullptr, *pwleaf_tab = nullptr;
  const int32_t* pwleaf_box = nullptr;
  const int32_t* box_order = nullptr;  // plane-wave boxes, most leaves first
  const int32_t *plist_start = nullptr, *plist_src = nullptr, *plist_dir = nullptr;
  // d = 3 fused translation: target groups and workgroups (fgt_host.h te_*)
  const int32_t *te_start = nullptr, *te_mem = nullptr, *te_src = nullptr, *te_dir = nullptr;
  const int32_t* te_wg = nullptr;
  int64_t nTG = 0, nTW = 0;
  const int32_t* echunk = nullptr;
  // formation work items (box, first leaf, end leaf, partial slot or -1) and
  // the reductions of split boxes (box, first slot, slot count)
  const int32_t *fitem = nullptr, *fred = nullptr;
  int64_t nFI = 0, nFR = 0;
  // d = 3 planes and rows of pw leaves (fgt_host.h)
  int64_t nPl = 0;
  const int32_t *plane_start = nullptr, *plane_tab = nullptr, *plane_row = nullptr;
  const int32_t *row_start = nullptr, *row_tab = nullptr;
  const int32_t* plane_order = nullptr;  // planes, most work first
  const int32_t *near_tgt = nullptr, *near_haspw = nullptr, *near_start = nullptr;
  const int32_t *near_src = nullptr, *near_tab = nullptr;
  // workspace (compute precision): Y/Z [nU][p*nr^(d-1)] (nU = planes for d = 3,
  // pw leaves otherwise), phi [nA][ncoef_phi], psi [nA][nr^d]
  void *Y = nullptr, *phi = nullptr, *psi = nullptr;
  int64_t ncoef_phi = 0;    // coefficients per box of phi and partial (phi_box_coefs)
  int phi_tp = 0;           // tile-major phi with this many pairs per tile; 0: [r3][r1][r2]
  void* partial = nullptr;  // [nslots][nr^d] partial sums of split boxes
};

// One transform of a batch: its arguments and its sigma / u.
struct BatchJob {
  DeviceArgs a;
  const double* sigma = nullptr;
  double* u = nullptr;
};

// The device stages in launch order.
enum Stage { kFormLeaf = 0, kFormBox, kReduce, kTranslate, kEvalBox, kEvalLeaf, kNear, kNumStages };

// Transforms of one kernel class share every kernel instantiation: dimension,
// compute precision (FP64, FP32, BF16x3), mode tiles per axis NT = ceil(nr/16),
// node steps KS.
struct KernelClass {
  int d = 0;
  bool fp32 = false, bf3 = false, fuse_te = false;
  int nt = 0, ks = 0;
  bool operator<(const KernelClass& o) const {
    if (d != o.d) return d < o.d;
    if (fp32 != o.fp32) return fp32 < o.fp32;
    if (bf3 != o.bf3) return bf3 < o.bf3;
    if (fuse_te != o.fuse_te) return fuse_te < o.fuse_te;
    if (nt != o.nt) return nt < o.nt;
    return ks < o.ks;
  }
};
KernelClass kernel_class(const DeviceArgs& a);

// Workgroups `stage` takes for one transform of d = 2 or 3 (0: the stage does
// not run); the grids of launch_fast.
int64_t stage_blocks(const DeviceArgs& a, int stage);
int64_t translate_blocks(const DeviceArgs& a);
// Workgroups of the d = 3 box formation with `slabs` 16-column slabs per wave
// (tile 0 of a batched launch: 2 slabs, as fgt_execute; tile 1: 4 slabs).
int64_t form_box_blocks(const DeviceArgs& a, int slabs);
constexpr int kFormBoxTiles = 2;
constexpr int kFormBoxTileSlabs[kFormBoxTiles] = {2, 4};

// Block b of a batched launch belongs to the last job j with start[j] <= b.
__device__ __forceinline__ int batch_job_of(const int32_t* __restrict__ start, int njobs, int b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Launches one stage for njobs transforms of class c.  jobs, start and count
// are device arrays: job j owns blocks [start[j], start[j] + count[j]) of a
// grid of `grid` blocks, start[j] a multiple of 8 (blocks past count[j] exit).
// tile selects the tile shape of stages that have two (the d = 3 box
// formation: kFormBoxTileSlabs[tile] slabs per wave); the grid must match it.
hipError_t launch_stage_batched(const KernelClass& c, int stage, const BatchJob* jobs,
                                const int32_t* start, const int32_t* count, int njobs,
                                int64_t grid, hipStream_t st, int tile = 0);
template <typename T>
void launch_translate_batched(int d, const BatchJob* jobs, const int32_t* start,
                              const int32_t* count, int njobs, int64_t grid, hipStream_t st);

// Persistent batched execution (persist.hip): one launch of `grid` workgroups
// runs every stage of the njobs transforms of class c.  start/count hold the
// per-stage block ranges ([kNumStages][njobs], as launch_stage_batched takes
// them, tile 0), stage_base[s] the first work item of stage s (stage_base
// [kNumStages] = all items), head the work queue (zero before the launch) and
// ctl[0] an error flag and ctl[1 + j kNumStages + s] the finished blocks of
// stage s of job j (zero before the launch).
bool persistent_supported(const KernelClass& c);
hipError_t launch_class_persistent(const KernelClass& c, const BatchJob* jobs, const int32_t* start,
                                   const int32_t* count, int njobs, const int64_t* stage_base, uint64_t* head,
                                   int32_t* ctl, int spin_limit, int grid, hipStream_t st);
// Zeroes n int32 by a kernel (graph-capture safe, unlike a memset node).
hipError_t zero_i32(int32_t* p, int64_t n, hipStream_t st);

// Dynamic LDS bytes of the stages that stage data in LDS.
size_t lds_form_leaf(int d, int p, int nr, size_t tsize);
size_t lds_eval_leaf(int d, int p, int nr, size_t tsize);
size_t lds_near(int d, int p, size_t tsize);
size_t lds_transeval(int tp, int nr, size_t tsize);  // the fused d = 3 translation

// Enqueues every stage on st.  ev (7 events or NULL) brackets the stages.
hipError_t launch_transform(const DeviceArgs& a, const double* sigma, double* u,
                            hipStream_t st, hipEvent_t* ev);
// The d = 2 and d = 3 stages (kernels_fast.hip).
hipError_t launch_fast(const DeviceArgs& a, const double* sigma, double* u, hipStream_t st,
                       hipEvent_t* ev);
// The outgoing -> incoming translations (kernels.hip).
template <typename T>
void launch_translate(const DeviceArgs& a, hipStream_t st);

}  // namespace fgt
