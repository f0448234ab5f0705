// Tuned device stages of the box Gauss transform for d = 2 and d = 3.
//
// Tile counts are compile time: NT = ceil(nr/16) mode tiles per axis and
// KS = ceil(p/4) node steps (FP32 always runs 4 node steps, see mfma.h).
// Node axes are padded to 16 inside a tile.  Chained contractions pass result
// tiles from one matrix-core product to the next in registers (mfma.h); LDS is
// used where a contraction runs across the tiles held by different waves, and
// to share one plane's 1D tables among the waves of the plane formation.
//
// d = 3:
//   form3_plane Y_P[j3][r1][r2] = sum_{rows} F1_row[r1][j1] (sum_{s in row} sum_j2 sigma_s[j3][j2][j1] F2_s[r2][j2])
//   form_box    phi_A[r3][c]    = sum_{P in A} sum_j3 F3_P[r3][j3] Y_P[j3][c]
//   translate   psi_A = sum_{B in P(A)} Rot(c_B - c_A) phi_B        (kernels.hip)
//   eval_box    Z_P[i3][c]      = sum_r3 E3_P[i3][r3] psi_A[r3][c]
//   eval3_plane u_s[i3][i2][i1] = sum_r2 E2_s[i2][r2] (sum_r1 Z_P[i3][r1][r2] E1_row[i1][r1])
// (P: a plane of leaves sharing level and axis-3 table; row: leaves of a plane
// sharing the axis-1 table.  Grouping the sums this way is exact: each table
// factor is applied once to the sum of everything it multiplies.)
//   near3       u_T (+)= sum_S (V3 (x) V2 (x) V1) sigma_S, grouped by tables
// The mode tensors phi, psi, Y, Z of d = 3 are stored with the r2 index fastest
// ([r3][r1][r2]), so that every global operand load runs along a contiguous axis.
// d = 2 fuses formation and evaluation per box / per leaf (no intermediate).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "kernels.h"
#include "mfma.h"
#include "stage_bodies.h"

namespace fgt {

// kernels: one transform per launch (blockIdx.x is the stage's block), and
// many transforms of one kernel class per launch (BatchJob tables; the block
// is found in the job's range, see batch_job_of).

#define FGT_BATCH_PROLOGUE                               \
  const int j = batch_job_of(start, njobs, blockIdx.x); \
  const int bid = blockIdx.x - start[j];                 \
  if (bid >= count[j]) return;                           \
  const DeviceArgs& a = jobs[j].a;
#define FGT_BATCH_PARAMS \
  const BatchJob* __restrict__ jobs, const int32_t* __restrict__ start, const int32_t* __restrict__ count, int njobs

template <typename C, int NT, int KS>
__global__ __launch_bounds__(256) void form3_plane(
    const double* __restrict__ sigma, const int32_t* __restrict__ leaf_id, const int32_t* __restrict__ leaf_tab,
    const int32_t* __restrict__ plane_order, const int32_t* __restrict__ plane_row,
    const int32_t* __restrict__ row_start, const int32_t* __restrict__ row_tab, const elem_t<C>* __restrict__ F,
    int p, int nr, elem_t<C>* __restrict__ Y) {
  typedef elem_t<C> T;
  form3_plane_body<C, NT, KS>(sigma, leaf_id, leaf_tab, plane_order, plane_row, row_start, row_tab, F, p, nr, Y,
                              blockIdx.x);
}
template <typename C, int NT, int KS>
__global__ __launch_bounds__(256) void form3_plane_b(FGT_BATCH_PARAMS) {
  typedef elem_t<C> T;
  FGT_BATCH_PROLOGUE
  form3_plane_body<C, NT, KS>(jobs[j].sigma, a.pwleaf_id, a.pwleaf_tab, a.plane_order, a.plane_row, a.row_start,
                              a.row_tab,
                              cptr<T>(a.F), a.p, a.nr, mptr<T>(a.Y), bid);
}

template <typename C, int D, int NT, int KS>
__global__ __launch_bounds__(256) void form_box(const elem_t<C>* __restrict__ Y, const int32_t* __restrict__ fitem,
                                                const int32_t* __restrict__ leaf_tab, const elem_t<C>* __restrict__ F,
                                                int p, int nr, int ncoltiles, int M, int tp, int64_t ncoef_phi,
                                                elem_t<C>* __restrict__ phi, elem_t<C>* __restrict__ partial) {
  typedef elem_t<C> T;
  form_box_body<C, D, NT, KS, kFormBoxSlabs>(Y, fitem, leaf_tab, F, p, nr, ncoltiles, M, tp, ncoef_phi, phi, partial,
                                             blockIdx.x);
}
template <typename C, int D, int NT, int KS, int H>
__global__ __launch_bounds__(256) void form_box_b(FGT_BATCH_PARAMS) {
  typedef elem_t<C> T;
  FGT_BATCH_PROLOGUE
  const int ncol128 = (n2_of(D, a.nr) + form_box_cols_of(H) - 1) / form_box_cols_of(H);
  form_box_body<C, D, NT, KS, H>(cptr<T>(a.Y), a.fitem, D == 3 ? a.plane_tab : a.pwleaf_tab, cptr<T>(a.F), a.p, a.nr,
                                 ncol128, a.M, a.phi_tp, a.ncoef_phi, mptr<T>(a.phi), mptr<T>(a.partial), bid);
}

template <typename T>
__global__ __launch_bounds__(256) void reduce_partials(const T* __restrict__ partial, const int32_t* __restrict__ fred,
                                                       int64_t ncoef, int nchunk, T* __restrict__ phi) {
  reduce_partials_body<T>(partial, fred, ncoef, nchunk, phi, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(256) void reduce_partials_b(FGT_BATCH_PARAMS) {
  FGT_BATCH_PROLOGUE
  const int64_t ncoef = a.ncoef_phi;
  reduce_partials_body<T>(cptr<T>(a.partial), a.fred, ncoef, (int)((ncoef + 255) / 256), mptr<T>(a.phi), bid);
}

template <typename C, int D, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT <= 4 ? 2 : 1))) void eval_box(
    const elem_t<C>* __restrict__ psi, const int32_t* __restrict__ box_order, const int32_t* __restrict__ pw_start,
    const int32_t* __restrict__ leaf_tab, const elem_t<C>* __restrict__ E, int p, int nr, int ncoltiles,
    uint32_t pmagic, elem_t<C>* __restrict__ Z) {
  typedef elem_t<C> T;
  eval_box_body<C, D, NT>(psi, box_order, pw_start, leaf_tab, E, p, nr, ncoltiles, pmagic, Z, blockIdx.x);
}
template <typename C, int D, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT <= 4 ? 2 : 1))) void eval_box_b(
    FGT_BATCH_PARAMS) {
  typedef elem_t<C> T;
  FGT_BATCH_PROLOGUE
  const int ncol = (n2_of(D, a.nr) + 63) / 64;
  eval_box_body<C, D, NT>(cptr<T>(a.psi), a.box_order, D == 3 ? a.plane_start : a.pw_start,
                          D == 3 ? a.plane_tab : a.pwleaf_tab, cptr<T>(a.E), a.p, a.nr, ncol,
                          pmagic_of(a.p), mptr<T>(a.Y), bid);
}

template <typename C, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT <= 3 ? 2 : 1))) void eval3_plane(
    const elem_t<C>* __restrict__ Z, const int32_t* __restrict__ leaf_id, const int32_t* __restrict__ leaf_tab,
    const int32_t* __restrict__ plane_order, const int32_t* __restrict__ plane_row,
    const int32_t* __restrict__ row_start, const int32_t* __restrict__ row_tab, const elem_t<C>* __restrict__ E,
    int p, int nr, double* __restrict__ u) {
  typedef elem_t<C> T;
  eval3_plane_body<C, NT>(Z, leaf_id, leaf_tab, plane_order, plane_row, row_start, row_tab, E, p, nr, u, blockIdx.x);
}
template <typename C, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT <= 3 ? 2 : 1))) void eval3_plane_b(
    FGT_BATCH_PARAMS) {
  typedef elem_t<C> T;
  FGT_BATCH_PROLOGUE
  eval3_plane_body<C, NT>(cptr<T>(a.Y), a.pwleaf_id, a.pwleaf_tab, a.plane_order, a.plane_row, a.row_start,
                          a.row_tab,
                          cptr<T>(a.E), a.p, a.nr, jobs[j].u, bid);
}

template <typename C, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void near3(
    const double* __restrict__ sigma, const int32_t* __restrict__ near_tgt, const int32_t* __restrict__ near_haspw,
    const int32_t* __restrict__ near_start, const int32_t* __restrict__ near_src,
    const int32_t* __restrict__ near_tab, const elem_t<C>* __restrict__ V, int p, double* __restrict__ u) {
  typedef elem_t<C> T;
  near3_body<C, KS>(sigma, near_tgt, near_haspw, near_start, near_src, near_tab, V, p, u, blockIdx.x);
}
template <typename C, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void near3_b(FGT_BATCH_PARAMS) {
  typedef elem_t<C> T;
  FGT_BATCH_PROLOGUE
  near3_body<C, KS>(jobs[j].sigma, a.near_tgt, a.near_haspw, a.near_start, a.near_src, a.near_tab, cptr<T>(a.V),
                    a.p, jobs[j].u, bid);
}

template <typename C, int NT, int KS>
__global__ __launch_bounds__(256) void form2_box(const double* __restrict__ sigma, const int32_t* __restrict__ fitem,
                                                 const int32_t* __restrict__ leaf_id,
                                                 const int32_t* __restrict__ leaf_tab, const elem_t<C>* __restrict__ F,
                                                 int p, int nr, elem_t<C>* __restrict__ phi, elem_t<C>* __restrict__ partial) {
  typedef elem_t<C> T;
  form2_box_body<C, NT, KS>(sigma, fitem, leaf_id, leaf_tab, F, p, nr, phi, partial, blockIdx.x);
}
template <typename C, int NT, int KS>
__global__ __launch_bounds__(256) void form2_box_b(FGT_BATCH_PARAMS) {
  typedef elem_t<C> T;
  FGT_BATCH_PROLOGUE
  form2_box_body<C, NT, KS>(jobs[j].sigma, a.fitem, a.pwleaf_id, a.pwleaf_tab, cptr<T>(a.F), a.p, a.nr,
                            mptr<T>(a.phi), mptr<T>(a.partial), bid);
}

template <typename C, int NT>
__global__ __launch_bounds__(256) void eval2_leaf(const elem_t<C>* __restrict__ psi, const int32_t* __restrict__ leaf_box,
                                                  const int32_t* __restrict__ leaf_id,
                                                  const int32_t* __restrict__ leaf_tab, const elem_t<C>* __restrict__ E,
                                                  int p, int nr, int nleaf, double* __restrict__ u) {
  typedef elem_t<C> T;
  eval2_leaf_body<C, NT>(psi, leaf_box, leaf_id, leaf_tab, E, p, nr, nleaf, u, blockIdx.x);
}
template <typename C, int NT>
__global__ __launch_bounds__(256) void eval2_leaf_b(FGT_BATCH_PARAMS) {
  typedef elem_t<C> T;
  FGT_BATCH_PROLOGUE
  eval2_leaf_body<C, NT>(cptr<T>(a.psi), a.pwleaf_box, a.pwleaf_id, a.pwleaf_tab, cptr<T>(a.E), a.p, a.nr,
                         (int)a.nL, jobs[j].u, bid);
}

template <typename C, int KS>
__global__ __launch_bounds__(256) void near2(const double* __restrict__ sigma, const int32_t* __restrict__ near_tgt,
                                             const int32_t* __restrict__ near_haspw,
                                             const int32_t* __restrict__ near_start,
                                             const int32_t* __restrict__ near_src,
                                             const int32_t* __restrict__ near_tab, const elem_t<C>* __restrict__ V, int p,
                                             int ntgt, double* __restrict__ u) {
  typedef elem_t<C> T;
  near2_body<C, KS>(sigma, near_tgt, near_haspw, near_start, near_src, near_tab, V, p, ntgt, u, blockIdx.x);
}
template <typename C, int KS>
__global__ __launch_bounds__(256) void near2_b(FGT_BATCH_PARAMS) {
  typedef elem_t<C> T;
  FGT_BATCH_PROLOGUE
  near2_body<C, KS>(jobs[j].sigma, a.near_tgt, a.near_haspw, a.near_start, a.near_src, a.near_tab, cptr<T>(a.V),
                    a.p, (int)a.nT, jobs[j].u, bid);
}

template <typename C, int NT>
__global__ __launch_bounds__(256) void transeval3(
    const elem_t<C>* __restrict__ phi, const int32_t* __restrict__ te_start, const int32_t* __restrict__ te_mem,
    const int32_t* __restrict__ te_src, const int32_t* __restrict__ te_dir, const int32_t* __restrict__ te_wg,
    const elem_t<C>* __restrict__ rot, const int32_t* __restrict__ plane_start,
    const int32_t* __restrict__ plane_tab, const elem_t<C>* __restrict__ E, int p, int M, int nr, int tp,
    elem_t<C>* __restrict__ Z) {
  extern __shared__ __align__(16) unsigned char te_lds[];
  transeval3_body<C, NT>(phi, te_start, te_mem, te_src, te_dir, te_wg, rot, plane_start, plane_tab, E, p, M, nr, tp,
                         Z, reinterpret_cast<elem_t<C>*>(te_lds), blockIdx.x);
}
// batched: the launch provides the LDS of the class's largest plan (transeval_lds_max)
template <typename C, int NT>
__global__ __launch_bounds__(256) void transeval3_b(FGT_BATCH_PARAMS) {
  extern __shared__ __align__(16) unsigned char te_lds[];
  FGT_BATCH_PROLOGUE
  typedef elem_t<C> T;
  transeval3_body<C, NT>(cptr<T>(a.phi), a.te_start, a.te_mem, a.te_src, a.te_dir, a.te_wg, cptr<T>(a.rot),
                         a.plane_start, a.plane_tab, cptr<T>(a.E), a.p, a.M, a.nr, a.phi_tp, mptr<T>(a.Y),
                         reinterpret_cast<T*>(te_lds), bid);
}

#undef FGT_BATCH_PROLOGUE
#undef FGT_BATCH_PARAMS

// ---------------------------------------------------------------------------
// grids

size_t lds_transeval(int tp, int nr, size_t tsize) { return transeval_lds(tp, nr, tsize); }

KernelClass kernel_class(const DeviceArgs& a) {
  KernelClass c;
  c.d = a.d;
  c.fp32 = a.fp32;
  c.bf3 = a.bf3;
  c.fuse_te = a.fuse_te;
  c.nt = std::min(8, std::max(1, (a.nr + 15) / 16));
  c.ks = a.p <= 8 ? 2 : 4;
  return c;
}

int64_t form_box_blocks(const DeviceArgs& a, int slabs) {
  if (a.nL <= 0) return 0;
  if (a.d != 3) return a.nFI;
  const int64_t N2 = (int64_t)a.nr * a.nr, cols = form_box_cols_of(slabs);
  return a.nFI * ((N2 + cols - 1) / cols);
}

int64_t stage_blocks(const DeviceArgs& a, int stage) {
  const int64_t nr = a.nr;
  const int64_t N2 = a.d == 3 ? nr * nr : nr;
  const bool pw = a.nL > 0;
  switch (stage) {
    case kFormLeaf: {
      if (!pw || a.d != 3) return 0;
      const int nt = kernel_class(a).nt, tg = form3_tile_group(nt);
      return a.nPl * ((a.p * ((nt + tg - 1) / tg) + 3) / 4);
    }
    case kFormBox: return form_box_blocks(a, kFormBoxSlabs);
    case kReduce: return pw && a.nFR > 0 ? a.nFR * ((a.ncoef_phi + 255) / 256) : 0;
    case kTranslate: return pw ? (a.d == 3 && a.fuse_te ? transeval3_blocks(a) : translate_blocks(a)) : 0;
    // d = 3: a separate stage unless fused into the translation; d = 2: fused into eval2_leaf
    case kEvalBox: return pw && a.d == 3 && !a.fuse_te ? a.nA * ((N2 + 63) / 64) : 0;
    case kEvalLeaf: return pw ? (a.d == 3 ? a.nPl * ((a.p + 3) / 4) : (a.nL + 3) / 4) : 0;
    case kNear: return a.nT > 0 ? (a.d == 3 ? a.nT : (a.nT + 3) / 4) : 0;
    default: return 0;
  }
}

template <typename C, int NT, int KS>
static void launch_batched_nt(int d, bool fuse, int stage, const BatchJob* jobs, const int32_t* start,
                              const int32_t* count, int njobs, int64_t grid, hipStream_t st, int tile) {
  typedef elem_t<C> T;
  const dim3 g((unsigned)grid), b(256);
  if (d == 3) {
    switch (stage) {
      case kFormLeaf: hipLaunchKernelGGL((form3_plane_b<C, NT, KS>), g, b, 0, st, jobs, start, count, njobs); break;
      case kFormBox:
        if (tile == 1)
          hipLaunchKernelGGL((form_box_b<C, 3, NT, KS, kFormBoxSlabsAlt>), g, b, 0, st, jobs, start, count, njobs);
        else
          hipLaunchKernelGGL((form_box_b<C, 3, NT, KS, kFormBoxSlabs>), g, b, 0, st, jobs, start, count, njobs);
        break;
      case kReduce: hipLaunchKernelGGL((reduce_partials_b<T>), g, b, 0, st, jobs, start, count, njobs); break;
      case kTranslate:
        if (fuse)
          hipLaunchKernelGGL((transeval3_b<C, NT>), g, b, transeval_lds_max(NT, sizeof(T)), st, jobs, start, count,
                             njobs);
        else launch_translate_batched<T>(3, jobs, start, count, njobs, grid, st);
        break;
      case kEvalBox: hipLaunchKernelGGL((eval_box_b<C, 3, NT>), g, b, 0, st, jobs, start, count, njobs); break;
      case kEvalLeaf: hipLaunchKernelGGL((eval3_plane_b<C, NT>), g, b, 0, st, jobs, start, count, njobs); break;
      case kNear: hipLaunchKernelGGL((near3_b<C, KS>), g, b, 0, st, jobs, start, count, njobs); break;
    }
  } else {
    switch (stage) {
      case kFormBox: hipLaunchKernelGGL((form2_box_b<C, NT, KS>), g, b, 0, st, jobs, start, count, njobs); break;
      case kReduce: hipLaunchKernelGGL((reduce_partials_b<T>), g, b, 0, st, jobs, start, count, njobs); break;
      case kTranslate: launch_translate_batched<T>(2, jobs, start, count, njobs, grid, st); break;
      case kEvalLeaf: hipLaunchKernelGGL((eval2_leaf_b<C, NT>), g, b, 0, st, jobs, start, count, njobs); break;
      case kNear: hipLaunchKernelGGL((near2_b<C, KS>), g, b, 0, st, jobs, start, count, njobs); break;
      default: break;
    }
  }
}

template <typename C, int KS>
static void launch_batched_ks(const KernelClass& c, int stage, const BatchJob* jobs, const int32_t* start,
                              const int32_t* count, int njobs, int64_t grid, hipStream_t st, int tile) {
  typedef elem_t<C> T;
  switch (c.nt) {
    case 1: launch_batched_nt<C, 1, KS>(c.d, c.fuse_te, stage, jobs, start, count, njobs, grid, st, tile); break;
    case 2: launch_batched_nt<C, 2, KS>(c.d, c.fuse_te, stage, jobs, start, count, njobs, grid, st, tile); break;
    case 3: launch_batched_nt<C, 3, KS>(c.d, c.fuse_te, stage, jobs, start, count, njobs, grid, st, tile); break;
    case 4: launch_batched_nt<C, 4, KS>(c.d, c.fuse_te, stage, jobs, start, count, njobs, grid, st, tile); break;
    case 5: launch_batched_nt<C, 5, KS>(c.d, c.fuse_te, stage, jobs, start, count, njobs, grid, st, tile); break;
    case 6: launch_batched_nt<C, 6, KS>(c.d, c.fuse_te, stage, jobs, start, count, njobs, grid, st, tile); break;
    case 7: launch_batched_nt<C, 7, KS>(c.d, c.fuse_te, stage, jobs, start, count, njobs, grid, st, tile); break;
    default: launch_batched_nt<C, 8, KS>(c.d, c.fuse_te, stage, jobs, start, count, njobs, grid, st, tile); break;
  }
}

hipError_t launch_stage_batched(const KernelClass& c, int stage, const BatchJob* jobs, const int32_t* start,
                                const int32_t* count, int njobs, int64_t grid, hipStream_t st, int tile) {
  if (grid <= 0 || njobs <= 0) return hipSuccess;
  if (c.d != 2 && c.d != 3) return hipErrorInvalidValue;
  if (c.bf3) {
    if (c.ks == 2) launch_batched_ks<Bf16x3, 2>(c, stage, jobs, start, count, njobs, grid, st, tile);
    else launch_batched_ks<Bf16x3, 4>(c, stage, jobs, start, count, njobs, grid, st, tile);
  } else if (c.fp32) {
    if (c.ks == 2) launch_batched_ks<float, 2>(c, stage, jobs, start, count, njobs, grid, st, tile);
    else launch_batched_ks<float, 4>(c, stage, jobs, start, count, njobs, grid, st, tile);
  } else {
    if (c.ks == 2) launch_batched_ks<double, 2>(c, stage, jobs, start, count, njobs, grid, st, tile);
    else launch_batched_ks<double, 4>(c, stage, jobs, start, count, njobs, grid, st, tile);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launch

template <typename T>
static void launch_reduce(const DeviceArgs& a, hipStream_t st) {
  if (a.nFR == 0) return;
  const int64_t ncoef = a.ncoef_phi;
  const int nchunk = (int)((ncoef + 255) / 256);
  hipLaunchKernelGGL((reduce_partials<T>), dim3((unsigned)stage_blocks(a, kReduce)), dim3(256), 0, st,
                     static_cast<const T*>(a.partial), a.fred, ncoef, nchunk, static_cast<T*>(a.phi));
}

template <typename C, int NT, int KS>
static void launch_nt(const DeviceArgs& a, const double* sigma, double* u, hipStream_t st,
                      hipEvent_t* ev, int D) {
  typedef elem_t<C> T;
  const int p = a.p, nr = a.nr;
  const T* F = static_cast<const T*>(a.F);
  const T* E = static_cast<const T*>(a.E);
  const T* V = static_cast<const T*>(a.V);
  T* Y = static_cast<T*>(a.Y);
  T* phi = static_cast<T*>(a.phi);
  T* psi = static_cast<T*>(a.psi);
  auto rec = [&](int i) { if (ev) (void)hipEventRecord(ev[i], st); };
  rec(0);
  if (a.nL > 0) {
    if (D == 3) {
      const int N2 = nr * nr, ncol = (N2 + 63) / 64;
      const int ncol128 = (N2 + form_box_cols_of(kFormBoxSlabs) - 1) / form_box_cols_of(kFormBoxSlabs);
      hipLaunchKernelGGL((form3_plane<C, NT, KS>), dim3((unsigned)stage_blocks(a, kFormLeaf)), dim3(256), 0, st, sigma,
                         a.pwleaf_id, a.pwleaf_tab, a.plane_order, a.plane_row, a.row_start, a.row_tab, F, p, nr, Y);
      rec(1);
      hipLaunchKernelGGL((form_box<C, 3, NT, KS>), dim3((unsigned)stage_blocks(a, kFormBox)), dim3(256), 0, st, Y,
                         a.fitem, a.plane_tab, F, p, nr, ncol128, a.M, a.phi_tp, a.ncoef_phi, phi, static_cast<T*>(a.partial));
      launch_reduce<T>(a, st);
      rec(2);
      if (a.fuse_te) {
        hipLaunchKernelGGL((transeval3<C, NT>), dim3((unsigned)stage_blocks(a, kTranslate)), dim3(256),
                           transeval_lds(a.phi_tp, nr, sizeof(T)), st, static_cast<const T*>(a.phi), a.te_start,
                           a.te_mem, a.te_src, a.te_dir, a.te_wg, static_cast<const T*>(a.rot), a.plane_start,
                           a.plane_tab, E, p, a.M, nr, a.phi_tp, Y);
        rec(3);
        rec(4);
      } else {
        launch_translate<T>(a, st);
        rec(3);
        const uint32_t pmagic = (uint32_t)((0x100000000ull + p - 1) / p);  // ceil(2^32 / p)
        hipLaunchKernelGGL((eval_box<C, 3, NT>), dim3((unsigned)stage_blocks(a, kEvalBox)), dim3(256), 0, st, psi,
                           a.box_order, a.plane_start, a.plane_tab, E, p, nr, ncol, pmagic, Y);
        rec(4);
      }
      hipLaunchKernelGGL((eval3_plane<C, NT>), dim3((unsigned)stage_blocks(a, kEvalLeaf)), dim3(256), 0, st, Y,
                         a.pwleaf_id, a.pwleaf_tab, a.plane_order, a.plane_row, a.row_start, a.row_tab, E, p, nr, u);
      rec(5);
    } else {
      rec(1);
      hipLaunchKernelGGL((form2_box<C, NT, KS>), dim3((unsigned)stage_blocks(a, kFormBox)), dim3(256), 0, st, sigma, a.fitem,
                         a.pwleaf_id, a.pwleaf_tab, F, p, nr, phi, static_cast<T*>(a.partial));
      launch_reduce<T>(a, st);
      rec(2);
      launch_translate<T>(a, st);
      rec(3);
      rec(4);
      hipLaunchKernelGGL((eval2_leaf<C, NT>), dim3((unsigned)stage_blocks(a, kEvalLeaf)), dim3(256), 0, st, psi,
                         a.pwleaf_box, a.pwleaf_id, a.pwleaf_tab, E, p, nr, (int)a.nL, u);
      rec(5);
    }
  } else {
    for (int i = 1; i <= 5; i++) rec(i);
  }
  if (a.nT > 0) {
    if (D == 3)
      hipLaunchKernelGGL((near3<C, KS>), dim3((unsigned)stage_blocks(a, kNear)), dim3(256), 0, st, sigma, a.near_tgt, a.near_haspw,
                         a.near_start, a.near_src, a.near_tab, V, p, u);
    else
      hipLaunchKernelGGL((near2<C, KS>), dim3((unsigned)stage_blocks(a, kNear)), dim3(256), 0, st, sigma,
                         a.near_tgt, a.near_haspw, a.near_start, a.near_src, a.near_tab, V, p,
                         (int)a.nT, u);
  }
  rec(6);
}

template <typename C, int KS>
static void launch_ks(const DeviceArgs& a, const double* sigma, double* u, hipStream_t st,
                      hipEvent_t* ev) {
  typedef elem_t<C> T;
  const int nt = (a.nr + 15) / 16;
  switch (nt) {
    case 1: launch_nt<C, 1, KS>(a, sigma, u, st, ev, a.d); break;
    case 2: launch_nt<C, 2, KS>(a, sigma, u, st, ev, a.d); break;
    case 3: launch_nt<C, 3, KS>(a, sigma, u, st, ev, a.d); break;
    case 4: launch_nt<C, 4, KS>(a, sigma, u, st, ev, a.d); break;
    case 5: launch_nt<C, 5, KS>(a, sigma, u, st, ev, a.d); break;
    case 6: launch_nt<C, 6, KS>(a, sigma, u, st, ev, a.d); break;
    case 7: launch_nt<C, 7, KS>(a, sigma, u, st, ev, a.d); break;
    default: launch_nt<C, 8, KS>(a, sigma, u, st, ev, a.d); break;
  }
}

hipError_t launch_fast(const DeviceArgs& a, const double* sigma, double* u, hipStream_t st,
                       hipEvent_t* ev) {
  const bool ks2 = a.p <= 8;
  if (a.bf3) {
    if (ks2) launch_ks<Bf16x3, 2>(a, sigma, u, st, ev);
    else launch_ks<Bf16x3, 4>(a, sigma, u, st, ev);
  } else if (a.fp32) {
    if (ks2) launch_ks<float, 2>(a, sigma, u, st, ev);
    else launch_ks<float, 4>(a, sigma, u, st, ev);
  } else {
    if (ks2) launch_ks<double, 2>(a, sigma, u, st, ev);
    else launch_ks<double, 4>(a, sigma, u, st, ev);
  }
  return hipGetLastError();
}

}  // namespace fgt
