// The plan object behind the opaque fgt_plan_t, shared by the ABI and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fgt.h"
#include "fgt_host.h"
#include "kernels.h"

struct fgt_plan {
  fgt::HostPlan hp;
  bool host_only = true;
  int device = -1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool profile = false;
  bool ev_ready = false;
  hipEvent_t ev[7] = {};
  std::vector<void*> allocs;
  int64_t device_bytes = 0;
  fgt::DeviceArgs args;
};

namespace fgt {
// Records msg as this thread's fgt_last_error() and returns code.
int set_error(int code, const std::string& msg);
// Device bytes a plan holds once uploaded: tables, lists and one workspace.
int64_t plan_device_bytes(const HostPlan& hp);
// Device bytes of one workspace (the per-execution intermediates Y, phi, psi
// and the partial slots).
int64_t plan_workspace_bytes(const HostPlan& hp);
// Allocates and uploads a host-only plan; fgt_execute then uses `stream`.
int plan_upload(fgt_plan_t* pl, hipStream_t stream);
// Frees a resident plan's device memory and returns it to the host-only state
// (the host plan stays, so plan_upload can bring it back).
int plan_unload(fgt_plan_t* pl);
// A second workspace for a resident plan: *args becomes the plan's arguments
// with its own intermediates in one allocation *mem (released with hipFree),
// so two executions of one plan may overlap.
int plan_alloc_workspace(const fgt_plan_t* pl, DeviceArgs* args, void** mem);
// Enqueues one transform with the given device arguments on `stream`.
int execute_args(const DeviceArgs& a, const double* sigma, double* u, hipStream_t stream);
}  // namespace fgt
