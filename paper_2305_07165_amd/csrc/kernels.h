// Device-side arguments of one transform and the stage launcher.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fgt_host.h"

namespace fgt {

struct DeviceArgs {
  int d = 0, p = 0, nr = 0, M = 0;
  bool fp32 = false;
  int64_t nA = 0, nL = 0, nE = 0, nT = 0;
  // tables (compute precision)
  const void *F = nullptr, *E = nullptr, *V = nullptr, *rot = nullptr;
  // lists
  const int32_t *pw_start = nullptr, *pwleaf_id = nullptr, *pwleaf_tab = nullptr;
  const int32_t* pwleaf_box = nullptr;
  const int32_t* box_order = nullptr;  // plane-wave boxes, most leaves first
  const int32_t *plist_start = nullptr, *plist_src = nullptr, *plist_dir = nullptr;
  const int32_t* echunk = nullptr;
  // formation work items (box, first leaf, end leaf, partial slot or -1) and
  // the reductions of split boxes (box, first slot, slot count)
  const int32_t *fitem = nullptr, *fred = nullptr;
  int64_t nFI = 0, nFR = 0;
  const int32_t *near_tgt = nullptr, *near_haspw = nullptr, *near_start = nullptr;
  const int32_t *near_src = nullptr, *near_tab = nullptr;
  // workspace (compute precision): Y/Z [nL][p*nr^(d-1)], phi/psi [nA][nr^d]
  void *Y = nullptr, *phi = nullptr, *psi = nullptr;
  void* partial = nullptr;  // [nslots][nr^d] partial sums of split boxes
};

// Dynamic LDS bytes of the stages that stage data in LDS.
size_t lds_form_leaf(int d, int p, int nr, size_t tsize);
size_t lds_eval_leaf(int d, int p, int nr, size_t tsize);
size_t lds_near(int d, int p, size_t tsize);

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
