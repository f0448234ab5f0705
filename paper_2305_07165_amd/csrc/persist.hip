// Persistent batched execution of one kernel class (fgt_batch.h, opts.persistent):
// one launch runs every stage of every transform of the class.
//
// Work items are the blocks of the class's per-stage launches laid end to end
// in stage order (all transforms' first stage, then their second, ...), and
// workgroups take them from a queue in increasing order.  Before running a
// block of stage s of transform j, the workgroup waits until every block of
// j's previous stage has finished; after it, it publishes its writes with a
// device-scope release and counts itself done.  An item only ever waits for
// items of lower index, which workgroups that are already running hold, so the
// queue drains whatever the grid size and whatever else runs on the device;
// the wait is still bounded (spin_limit), and a wait that runs out sets the
// error flag instead of hanging.  The stage bodies are the per-stage kernels'
// own (stage_bodies.h, translate.h): results are bitwise those of fgt_execute.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "mfma.h"
#include "stage_bodies.h"
#include "translate.h"

namespace fgt {

namespace {

__global__ void k_zero_i32(int32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <typename C, int D, int NT, int KS, bool FUSE>
__global__ __launch_bounds__(256) void class_persistent(const BatchJob* __restrict__ jobs,
                                                        const int32_t* __restrict__ start,
                                                        const int32_t* __restrict__ count, int njobs,
                                                        const int64_t* __restrict__ stage_base,
                                                        uint64_t* __restrict__ head, int32_t* __restrict__ ctl,
                                                        int spin_limit) {
  typedef elem_t<C> T;
  extern __shared__ __align__(16) unsigned char te_lds[];
  __shared__ int64_t s_item;
  const int64_t total = stage_base[kNumStages];
  int32_t* done = ctl + 1;  // ctl[0]: error flag; then done[njobs][kNumStages]
  for (;;) {
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd((unsigned long long*)head, 1ull);
    __syncthreads();
    const int64_t g = s_item;
    __syncthreads();
    if (g >= total) break;
    int stage = 0;
    while (g >= stage_base[stage + 1]) stage++;
    const int local = (int)(g - stage_base[stage]);
    const int32_t* st = start + (size_t)stage * njobs;
    const int j = batch_job_of(st, njobs, local);
    const int bid = local - st[j];
    if (bid >= count[(size_t)stage * njobs + j]) continue;  // alignment gap between transforms
    if (threadIdx.x == 0) {
      for (int ps = stage - 1; ps >= 0; ps--) {
        const int need = count[(size_t)ps * njobs + j];
        if (need == 0) continue;
        // poll with relaxed loads (an acquire load would invalidate this XCD's
        // L2 on every poll, under every other workgroup on it), then acquire
        // once
        int spins = 0;
        while (__hip_atomic_load(&done[(size_t)j * kNumStages + ps], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               need) {
          // a wait that runs out flags the launch, and every later wait then
          // gives up at once: the kernel always finishes
          if (++spins > spin_limit || __hip_atomic_load(&ctl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(&ctl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(8);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        break;
      }
    }
    __syncthreads();
    const DeviceArgs& a = jobs[j].a;
    switch (stage) {
      case kFormLeaf:
        if constexpr (D == 3)
          form3_plane_body<C, NT, KS>(jobs[j].sigma, a.pwleaf_id, a.pwleaf_tab, a.plane_order, a.plane_row,
                                      a.row_start,
                                      a.row_tab, cptr<T>(a.F), a.p, a.nr, mptr<T>(a.Y), bid);
        break;
      case kFormBox:
        if constexpr (D == 3) {
          const int ncol = (n2_of(D, a.nr) + form_box_cols_of(kFormBoxSlabs) - 1) / form_box_cols_of(kFormBoxSlabs);
          form_box_body<C, D, NT, KS, kFormBoxSlabs>(cptr<T>(a.Y), a.fitem, a.plane_tab, cptr<T>(a.F), a.p, a.nr,
                                                     ncol, a.M, a.phi_tp, a.ncoef_phi, mptr<T>(a.phi), mptr<T>(a.partial),
                                                     bid);
        } else {
          form2_box_body<C, NT, KS>(jobs[j].sigma, a.fitem, a.pwleaf_id, a.pwleaf_tab, cptr<T>(a.F), a.p, a.nr,
                                    mptr<T>(a.phi), mptr<T>(a.partial), bid);
        }
        break;
      case kReduce: {
        const int64_t ncoef = a.ncoef_phi;
        reduce_partials_body<T>(cptr<T>(a.partial), a.fred, ncoef, (int)((ncoef + 255) / 256), mptr<T>(a.phi), bid);
        break;
      }
      case kTranslate:
        if constexpr (D == 3 && FUSE)
          transeval3_body<C, NT>(cptr<T>(a.phi), a.te_start, a.te_mem, a.te_src, a.te_dir, a.te_wg, cptr<T>(a.rot),
                                 a.plane_start, a.plane_tab, cptr<T>(a.E), a.p, a.M, a.nr, a.phi_tp, mptr<T>(a.Y),
                                 reinterpret_cast<T*>(te_lds), bid);
        else
          translate_body<T, D, D == 3>(cptr<T>(a.phi), a.plist_start, a.plist_src, a.plist_dir, cptr<T>(a.rot), a.M,
                                       a.nr, (int)a.nA, static_cast<T*>(const_cast<void*>(a.psi)), bid);
        break;
      case kEvalBox:
        if constexpr (D == 3 && !FUSE)
          eval_box_body<C, D, NT>(cptr<T>(a.psi), a.box_order, a.plane_start, a.plane_tab, cptr<T>(a.E), a.p, a.nr,
                                  (n2_of(D, a.nr) + 63) / 64, pmagic_of(a.p), mptr<T>(a.Y), bid);
        break;
      case kEvalLeaf:
        if constexpr (D == 3)
          eval3_plane_body<C, NT>(cptr<T>(a.Y), a.pwleaf_id, a.pwleaf_tab, a.plane_order, a.plane_row, a.row_start,
                                  a.row_tab,
                                  cptr<T>(a.E), a.p, a.nr, jobs[j].u, bid);
        else
          eval2_leaf_body<C, NT>(cptr<T>(a.psi), a.pwleaf_box, a.pwleaf_id, a.pwleaf_tab, cptr<T>(a.E), a.p, a.nr,
                                 (int)a.nL, jobs[j].u, bid);
        break;
      case kNear:
        if constexpr (D == 3)
          near3_body<C, KS>(jobs[j].sigma, a.near_tgt, a.near_haspw, a.near_start, a.near_src, a.near_tab,
                            cptr<T>(a.V), a.p, jobs[j].u, bid);
        else
          near2_body<C, KS>(jobs[j].sigma, a.near_tgt, a.near_haspw, a.near_start, a.near_src, a.near_tab,
                            cptr<T>(a.V), a.p, (int)a.nT, jobs[j].u, bid);
        break;
      default:
        break;
    }
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(&done[(size_t)j * kNumStages + stage], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename C, int D, int NT, int KS>
void launch_d(bool fuse, const BatchJob* jobs, const int32_t* start, const int32_t* count, int njobs,
              const int64_t* stage_base, uint64_t* head, int32_t* ctl, int spin_limit, int grid, hipStream_t st) {
  typedef elem_t<C> T;
  if (D == 3 && fuse)
    hipLaunchKernelGGL((class_persistent<C, D, NT, KS, true>), dim3(grid), dim3(256), transeval_lds_max(NT, sizeof(T)),
                       st, jobs, start, count, njobs, stage_base, head, ctl, spin_limit);
  else
    hipLaunchKernelGGL((class_persistent<C, D, NT, KS, false>), dim3(grid), dim3(256), 0, st, jobs, start, count,
                       njobs, stage_base, head, ctl, spin_limit);
}

template <typename C, int KS>
void launch_nt(const KernelClass& c, const BatchJob* jobs, const int32_t* start, const int32_t* count, int njobs,
               const int64_t* stage_base, uint64_t* head, int32_t* ctl, int spin_limit, int grid, hipStream_t st) {
#define FGT_PERSIST_CASE(NTV)                                                                                   \
  case NTV:                                                                                                     \
    if (c.d == 3)                                                                                               \
      launch_d<C, 3, NTV, KS>(c.fuse_te, jobs, start, count, njobs, stage_base, head, ctl, spin_limit, grid, st); \
    else                                                                                                        \
      launch_d<C, 2, NTV, KS>(false, jobs, start, count, njobs, stage_base, head, ctl, spin_limit, grid, st);   \
    break;
  switch (c.nt) {
    FGT_PERSIST_CASE(1)
    FGT_PERSIST_CASE(2)
    FGT_PERSIST_CASE(3)
    FGT_PERSIST_CASE(4)
    FGT_PERSIST_CASE(5)
    FGT_PERSIST_CASE(6)
    FGT_PERSIST_CASE(7)
    default:
      FGT_PERSIST_CASE(8)
  }
#undef FGT_PERSIST_CASE
}

}  // namespace

bool persistent_supported(const KernelClass& c) { return (c.d == 2 || c.d == 3) && !c.bf3; }

hipError_t zero_i32(int32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_class_persistent(const KernelClass& c, const BatchJob* jobs, const int32_t* start,
                                   const int32_t* count, int njobs, const int64_t* stage_base, uint64_t* head,
                                   int32_t* ctl, int spin_limit, int grid, hipStream_t st) {
  if (!persistent_supported(c) || grid <= 0) return hipErrorInvalidValue;
  if (c.fp32) {
    if (c.ks == 2) launch_nt<float, 2>(c, jobs, start, count, njobs, stage_base, head, ctl, spin_limit, grid, st);
    else launch_nt<float, 4>(c, jobs, start, count, njobs, stage_base, head, ctl, spin_limit, grid, st);
  } else {
    if (c.ks == 2) launch_nt<double, 2>(c, jobs, start, count, njobs, stage_base, head, ctl, spin_limit, grid, st);
    else launch_nt<double, 4>(c, jobs, start, count, njobs, stage_base, head, ctl, spin_limit, grid, st);
  }
  return hipGetLastError();
}

}  // namespace fgt
