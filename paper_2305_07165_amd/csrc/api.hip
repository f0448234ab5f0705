// C ABI of the box Gauss transform: plan lifecycle, upload, execution.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fgt_host.h"
#include "kernels.h"
#include "../../include/fgt.h"
#include "plan_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return FGT_ERR_HIP;
}

template <typename X>
int upload(fgt_plan_t* pl, const X* src, size_t n, void** out) {
  *out = nullptr;
  if (n == 0) return FGT_OK;
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, n * sizeof(X));
  if (e != hipSuccess) return fail(FGT_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  pl->allocs.push_back(d);
  pl->device_bytes += (int64_t)(n * sizeof(X));
  e = hipMemcpy(d, src, n * sizeof(X), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  *out = d;
  return FGT_OK;
}

int alloc(fgt_plan_t* pl, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) return FGT_OK;
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return fail(FGT_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  pl->allocs.push_back(d);
  pl->device_bytes += (int64_t)bytes;
  *out = d;
  return FGT_OK;
}

int upload_i32(fgt_plan_t* pl, const std::vector<int32_t>& v, const int32_t** out) {
  void* d;
  int rc = upload(pl, v.data(), v.size(), &d);
  *out = static_cast<const int32_t*>(d);
  return rc;
}

int upload_table(fgt_plan_t* pl, const std::vector<double>& v, bool fp32, const void** out) {
  void* d;
  int rc;
  if (fp32) {
    std::vector<float> f(v.size());
    for (size_t i = 0; i < v.size(); i++) f[i] = (float)v[i];  // rounded once
    rc = upload(pl, f.data(), f.size(), &d);
  } else {
    rc = upload(pl, v.data(), v.size(), &d);
  }
  *out = d;
  return rc;
}

double ipowd(double b, int e) {
  double r = 1;
  for (int i = 0; i < e; i++) r *= b;
  return r;
}

}  // namespace

int64_t fgt::plan_device_bytes(const HostPlan& hp) {
  const int64_t ts = hp.precision != FGT_FP64 ? 4 : 8;
  int64_t b = ts * (int64_t)(hp.F.size() + hp.E.size() + hp.V.size() + hp.rot.size());
  for (const std::vector<int32_t>* v : {&hp.pw_start, &hp.pwleaf_id, &hp.pwleaf_tab, &hp.pwleaf_box,
                                        &hp.box_order, &hp.plist_start, &hp.plist_src, &hp.plist_dir,
                                        &hp.echunk, &hp.near_tgt, &hp.fitem, &hp.fred, &hp.near_haspw,
                                        &hp.near_start, &hp.near_src, &hp.near_tab, &hp.plane_start,
                                        &hp.plane_tab, &hp.plane_row, &hp.row_start, &hp.row_tab})
    b += 4 * (int64_t)v->size();
  return b + plan_workspace_bytes(hp);
}

// coefficients per box of phi and of the partial sums (tile-major in fused
// d = 3 plans, kernels.h)
static int64_t phi_coefs(const fgt::HostPlan& hp) {
  return fgt::phi_box_coefs(hp.d, hp.pw.M, hp.nrs, hp.d == 3 && hp.fuse_te ? hp.te_tp : 0);
}

int64_t fgt::plan_workspace_bytes(const HostPlan& hp) {
  const int64_t ts = hp.precision != FGT_FP64 ? 4 : 8;
  int64_t n2 = 1;
  for (int a = 1; a < hp.d; a++) n2 *= hp.nrs;
  const int64_t ncoef = n2 * hp.nrs, nphi = phi_coefs(hp);
  const int64_t round = 256 / ts;  // each array starts on a 256-byte boundary
  auto up = [&](int64_t n) { return (n + round - 1) / round * round; };
  const int64_t nU = hp.d == 3 ? hp.n_plane() : (hp.d == 2 ? 0 : hp.n_pwleaf());
  const int64_t npsi = hp.fuse_te ? 0 : up(hp.n_pwbox() * ncoef);  // no psi when fused away
  return ts * (up(nU * hp.p * n2) + up(hp.n_pwbox() * nphi) + npsi + up((int64_t)hp.nslots * nphi));
}

namespace {

int setup_device(fgt_plan_t* pl, const fgt_opts_t* opts) {
  fgt::HostPlan& hp = pl->hp;
  hipError_t e = hipGetDevice(&pl->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const bool fp32 = hp.precision != FGT_FP64;
  const size_t ts = fp32 ? sizeof(float) : sizeof(double);
  int lds_max = 0;
  e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, pl->device);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  size_t need = std::max(fgt::lds_form_leaf(hp.d, hp.p, hp.nrs, ts),
                         std::max(fgt::lds_eval_leaf(hp.d, hp.p, hp.nrs, ts), fgt::lds_near(hp.d, hp.p, ts)));
  if (hp.fuse_te) need = std::max(need, fgt::lds_transeval(hp.te_tp, hp.nrs, ts));
  if (need > (size_t)lds_max)
    return fail(FGT_ERR_UNSUPPORTED, "stage needs " + std::to_string(need) + " bytes of LDS, device allows " +
                                         std::to_string(lds_max));
  fgt::DeviceArgs& a = pl->args;
  a.d = hp.d;
  a.p = hp.p;
  a.nr = hp.nrs;  // the kernels see the stored modes
  a.M = hp.pw.M;
  a.fp32 = fp32;
  a.bf3 = hp.precision == FGT_BF16X3;
  a.fuse_te = hp.fuse_te;
  a.nA = hp.n_pwbox();
  a.nL = hp.n_pwleaf();
  a.nE = (int64_t)hp.echunk.size() / 3;
  a.nT = hp.n_near_tgt();
  a.nFI = (int64_t)hp.fitem.size() / 4;
  a.nFR = (int64_t)hp.fred.size() / 3;
  int rc;
  if ((rc = upload_table(pl, hp.F, fp32, &a.F)) || (rc = upload_table(pl, hp.E, fp32, &a.E)) ||
      (rc = upload_table(pl, hp.V, fp32, &a.V)) || (rc = upload_table(pl, hp.rot, fp32, &a.rot)))
    return rc;
  if ((rc = upload_i32(pl, hp.pw_start, &a.pw_start)) || (rc = upload_i32(pl, hp.pwleaf_id, &a.pwleaf_id)) ||
      (rc = upload_i32(pl, hp.pwleaf_tab, &a.pwleaf_tab)) || (rc = upload_i32(pl, hp.pwleaf_box, &a.pwleaf_box)) ||
      (rc = upload_i32(pl, hp.box_order, &a.box_order)) ||
      (rc = upload_i32(pl, hp.plist_start, &a.plist_start)) ||
      (rc = upload_i32(pl, hp.plist_src, &a.plist_src)) || (rc = upload_i32(pl, hp.plist_dir, &a.plist_dir)) ||
      (rc = upload_i32(pl, hp.echunk, &a.echunk)) || (rc = upload_i32(pl, hp.near_tgt, &a.near_tgt)) ||
      (rc = upload_i32(pl, hp.fitem, &a.fitem)) || (rc = upload_i32(pl, hp.fred, &a.fred)) ||
      (rc = upload_i32(pl, hp.near_haspw, &a.near_haspw)) ||
      (rc = upload_i32(pl, hp.near_start, &a.near_start)) || (rc = upload_i32(pl, hp.near_src, &a.near_src)) ||
      (rc = upload_i32(pl, hp.near_tab, &a.near_tab)) ||
      (rc = upload_i32(pl, hp.plane_start, &a.plane_start)) ||
      (rc = upload_i32(pl, hp.plane_tab, &a.plane_tab)) || (rc = upload_i32(pl, hp.plane_row, &a.plane_row)) ||
      (rc = upload_i32(pl, hp.row_start, &a.row_start)) || (rc = upload_i32(pl, hp.row_tab, &a.row_tab)) ||
      (rc = upload_i32(pl, hp.plane_order, &a.plane_order)) ||
      (rc = upload_i32(pl, hp.te_start, &a.te_start)) || (rc = upload_i32(pl, hp.te_mem, &a.te_mem)) ||
      (rc = upload_i32(pl, hp.te_src, &a.te_src)) || (rc = upload_i32(pl, hp.te_dir, &a.te_dir)) ||
      (rc = upload_i32(pl, hp.te_wg, &a.te_wg)))
    return rc;
  a.nTG = hp.n_te_group();
  a.nTW = (int64_t)hp.te_wg.size() / 2;
  a.nPl = hp.n_plane();
  const size_t n2 = (size_t)ipowd(hp.nrs, hp.d - 1);
  const size_t ncoef = n2 * hp.nrs;
  a.ncoef_phi = phi_coefs(hp);
  a.phi_tp = hp.d == 3 && hp.fuse_te ? hp.te_tp : 0;
  // the intermediate: per plane for d = 3, none for d = 2 (both axes fused), per leaf for d = 1
  const int64_t nU = hp.d == 3 ? hp.n_plane() : (hp.d == 2 ? 0 : a.nL);
  // no psi when the translation is fused with the first evaluation step
  const size_t npsi = hp.fuse_te ? 0 : (size_t)a.nA * ncoef * ts;
  if ((rc = alloc(pl, (size_t)nU * hp.p * n2 * ts, &a.Y)) ||
      (rc = alloc(pl, (size_t)a.nA * a.ncoef_phi * ts, &a.phi)) || (rc = alloc(pl, npsi, &a.psi)) ||
      (rc = alloc(pl, (size_t)hp.nslots * a.ncoef_phi * ts, &a.partial)))
    return rc;
  if (opts && opts->own_stream) {
    e = hipStreamCreateWithFlags(&pl->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    pl->own_stream = true;
  } else {
    pl->stream = opts ? static_cast<hipStream_t>(opts->stream) : nullptr;
  }
  if (pl->profile) {
    for (int i = 0; i < 7; i++) {
      e = hipEventCreate(&pl->ev[i]);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    pl->ev_ready = true;
  }
  pl->host_only = false;
  return FGT_OK;
}

void release(fgt_plan_t* pl) {
  if (!pl) return;
  if (!pl->host_only || !pl->allocs.empty()) {
    if (pl->device >= 0) (void)hipSetDevice(pl->device);
    (void)hipStreamSynchronize(pl->stream);
  }
  if (pl->ev_ready)
    for (int i = 0; i < 7; i++) (void)hipEventDestroy(pl->ev[i]);
  for (void* p : pl->allocs) (void)hipFree(p);
  if (pl->own_stream && pl->stream) (void)hipStreamDestroy(pl->stream);
  delete pl;
}

}  // namespace

int fgt::set_error(int code, const std::string& msg) { return fail(code, msg); }

int fgt::plan_upload(fgt_plan_t* pl, hipStream_t stream) {
  if (!pl || !pl->host_only) return fail(FGT_ERR_INVALID_ARG, "plan is not host-only");
  fgt_opts_t o{};
  o.stream = stream;
  const int rc = setup_device(pl, &o);
  if (rc != FGT_OK) {
    // leave the plan host-only, as it was
    if (pl->ev_ready)
      for (int i = 0; i < 7; i++) (void)hipEventDestroy(pl->ev[i]);
    pl->ev_ready = false;
    for (void* p : pl->allocs) (void)hipFree(p);
    pl->allocs.clear();
    pl->device_bytes = 0;
    pl->args = fgt::DeviceArgs();
    pl->stream = nullptr;
    pl->host_only = true;
  }
  return rc;
}

int fgt::plan_unload(fgt_plan_t* pl) {
  if (!pl || pl->host_only) return fail(FGT_ERR_INVALID_ARG, "plan is not resident");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (pl->ev_ready)
    for (int i = 0; i < 7; i++) (void)hipEventDestroy(pl->ev[i]);
  pl->ev_ready = false;
  for (void* p : pl->allocs) (void)hipFree(p);
  pl->allocs.clear();
  if (pl->own_stream && pl->stream) (void)hipStreamDestroy(pl->stream);
  pl->own_stream = false;
  pl->stream = nullptr;
  pl->device_bytes = 0;
  pl->args = fgt::DeviceArgs();
  pl->host_only = true;
  return FGT_OK;
}

// Lays the workspace arrays (Y, phi, psi unless fused away, partial sums) out
// from base, each on a 256-byte boundary, in plan_workspace_bytes(hp) bytes.
static void carve_workspace(const fgt::HostPlan& hp, void* base, fgt::DeviceArgs* args) {
  const int64_t ts = hp.precision != FGT_FP64 ? 4 : 8;
  int64_t n2 = 1;
  for (int a = 1; a < hp.d; a++) n2 *= hp.nrs;
  const int64_t ncoef = n2 * hp.nrs, nphi = phi_coefs(hp), round = 256 / ts;
  auto up = [&](int64_t n) { return (n + round - 1) / round * round; };
  char* c = static_cast<char*>(base);
  args->Y = c;
  c += ts * up((hp.d == 3 ? hp.n_plane() : (hp.d == 2 ? 0 : hp.n_pwleaf())) * hp.p * n2);
  args->phi = c;
  c += ts * up(hp.n_pwbox() * nphi);
  args->psi = hp.fuse_te ? nullptr : c;
  if (!hp.fuse_te) c += ts * up(hp.n_pwbox() * ncoef);
  args->partial = c;
}

int fgt::plan_alloc_workspace(const fgt_plan_t* pl, DeviceArgs* args, void** mem) {
  if (!pl || pl->host_only || !args || !mem) return fail(FGT_ERR_INVALID_ARG, "plan is not resident");
  const int64_t bytes = plan_workspace_bytes(pl->hp);
  void* m = nullptr;
  hipError_t e = hipMalloc(&m, (size_t)std::max<int64_t>(bytes, 256));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(FGT_ERR_OOM, "workspace") : hip_fail(e, "hipMalloc");
  *args = pl->args;
  carve_workspace(pl->hp, m, args);
  *mem = m;
  return FGT_OK;
}

int fgt::execute_args(const DeviceArgs& a, const double* sigma, double* u, hipStream_t stream) {
  if (!sigma || !u) return fail(FGT_ERR_INVALID_ARG, "sigma or u is NULL");
  hipError_t e = fgt::launch_transform(a, sigma, u, stream, nullptr);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return FGT_OK;
}

namespace {

// ---------------------------------------------------------------------------
// Static scratch of fgt_execute_noalloc: one file-scope device array per GPU
// (each device holds its own copy at its own address until the process ends).
// Host code never uses the array's name as an address: the device address is
// looked up once per device with that device current, and kept.
constexpr int64_t kScratchBytes = int64_t(64) << 20;
constexpr int kScratchDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// The device address of `scratch` on `device`, which must be current.
int scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kScratchDevices)
    return fail(FGT_ERR_UNSUPPORTED, "device ordinal beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(FGT_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return FGT_OK;
}

}  // namespace

extern "C" {

int fgt_plan(const fgt_tree_t* tree, int p, double delta, double tol, int bc, const fgt_opts_t* opts,
             fgt_plan_t** out) {
  if (!out) return fail(FGT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!tree) return fail(FGT_ERR_INVALID_ARG, "tree is NULL");
  fgt_opts_t o{};
  o.force_lc = -1;
  if (opts) o = *opts;
  fgt_plan_t* pl = new (std::nothrow) fgt_plan_t();
  if (!pl) return fail(FGT_ERR_OOM, "host allocation");
  pl->profile = o.profile != 0;
  std::string err;
  int rc;
  try {
    rc = fgt::build_host_plan(tree->dim, tree->nleaves, tree->level, tree->coord, p, delta, tol, bc,
                              o.precision, o.eps_internal, o.force_lc, o.no_fuse == 0, pl->hp, err);
  } catch (const std::bad_alloc&) {
    rc = FGT_ERR_OOM;
    err = "host allocation";
  } catch (...) {
    rc = FGT_ERR_INVALID_ARG;
    err = "unexpected exception while planning";
  }
  if (rc != FGT_OK) {
    delete pl;
    return fail(rc, err);
  }
  if (!o.host_only) {
    rc = setup_device(pl, &o);
    if (rc != FGT_OK) {
      std::string keep = g_err;
      release(pl);
      return fail(rc, keep);
    }
  }
  *out = pl;
  return FGT_OK;
}

int fgt_execute(fgt_plan_t* pl, const double* sigma, double* u) {
  if (!pl) return fail(FGT_ERR_INVALID_ARG, "plan is NULL");
  if (pl->host_only) return fail(FGT_ERR_INVALID_ARG, "host-only plan cannot execute");
  if (!sigma || !u) return fail(FGT_ERR_INVALID_ARG, "sigma/u is NULL");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  e = fgt::launch_transform(pl->args, sigma, u, pl->stream, pl->profile ? pl->ev : nullptr);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return FGT_OK;
}

int fgt_execute_noalloc(fgt_plan_t* pl, const double* sigma, double* u) {
  if (!pl) return fail(FGT_ERR_INVALID_ARG, "plan is NULL");
  if (pl->host_only) return fail(FGT_ERR_INVALID_ARG, "host-only plan cannot execute");
  if (!sigma || !u) return fail(FGT_ERR_INVALID_ARG, "sigma/u is NULL");
  const int64_t need = fgt::plan_workspace_bytes(pl->hp);
  if (need > kScratchBytes)
    return fail(FGT_ERR_UNSUPPORTED, "plan workspace of " + std::to_string(need) +
                                         " bytes exceeds the static scratch of " + std::to_string(kScratchBytes) +
                                         " bytes (fgt_execute uses the plan's own workspace)");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  void* base = nullptr;
  const int rc = scratch_address(pl->device, &base);
  if (rc != FGT_OK) return rc;
  // every word the kernels read from the workspace is written earlier in the
  // same execution, so the scratch needs no clearing
  fgt::DeviceArgs a = pl->args;
  carve_workspace(pl->hp, base, &a);
  e = fgt::launch_transform(a, sigma, u, pl->stream, pl->profile ? pl->ev : nullptr);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return FGT_OK;
}

int fgt_sync(fgt_plan_t* pl) {
  if (!pl) return fail(FGT_ERR_INVALID_ARG, "plan is NULL");
  if (pl->host_only) return FGT_OK;
  hipError_t e = hipSetDevice(pl->device);
  if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return FGT_OK;
}

int fgt_stage_times(const fgt_plan_t* pl, double* ms, int n) {
  if (!pl || !ms) return fail(FGT_ERR_INVALID_ARG, "NULL argument");
  if (!pl->ev_ready) return 0;
  int k = 0;
  for (int i = 0; i < 6 && k < n; i++, k++) {
    float t = 0;
    hipError_t e = hipEventElapsedTime(&t, pl->ev[i], pl->ev[i + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    ms[k] = t;
  }
  return k;
}

int fgt_plan_info(const fgt_plan_t* pl, fgt_info_t* info) {
  if (!pl || !info) return fail(FGT_ERR_INVALID_ARG, "NULL argument");
  const fgt::HostPlan& hp = pl->hp;
  std::memset(info, 0, sizeof(*info));
  info->dim = hp.d;
  info->p = hp.p;
  info->bc = hp.bc;
  info->precision = hp.precision;
  info->lc = hp.lc;
  info->lmin = hp.lmin;
  info->lmax = hp.lmax;
  info->nf = 2 * hp.pw.M;
  info->nr = hp.nr;
  info->nr_stored = hp.nrs;
  info->delta = hp.delta;
  info->tol = hp.tol;
  info->eps = hp.pw.eps;
  info->D0 = hp.pw.D0;
  info->R = hp.pw.R;
  info->h = hp.pw.h;
  info->nleaves = hp.nleaves;
  const double pd = ipowd(hp.p, hp.d);
  info->npoints = (int64_t)(hp.nleaves * pd);
  info->n_pwbox = hp.n_pwbox();
  info->n_pwleaf = hp.n_pwleaf();
  info->n_plist = hp.n_plist();
  info->n_near_target = hp.n_near_tgt();
  info->n_near_pair = hp.n_near_pair();
  double fe = 0;  // formation (= evaluation) flops: each 1D table applied once per leaf group
  if (hp.d == 3) {
    fe = 2.0 * hp.nr * ipowd(hp.p, 4) * hp.n_pwleaf() + 2.0 * ipowd(hp.nr, 2) * ipowd(hp.p, 3) * hp.n_row() +
         2.0 * ipowd(hp.nr, 3) * ipowd(hp.p, 2) * hp.n_plane();
    fe /= hp.p;
  } else {
    for (int a = 1; a <= hp.d; a++) fe += 2.0 * ipowd(hp.nr, a) * ipowd(hp.p, hp.d - a + 1) * hp.n_pwleaf();
  }
  info->flops_form = fe;
  info->flops_eval = fe;
  info->n_plane = hp.n_plane();
  info->n_row = hp.n_row();
  {
    std::vector<char> seen(hp.nleaves, 0);
    int64_t ns = 0;
    for (int32_t sidx : hp.near_src) ns += !seen[sidx], seen[sidx] = 1;
    info->n_near_source = ns;
    int64_t nh = 0;
    for (int32_t h : hp.near_haspw) nh += h != 0;
    info->n_near_haspw = nh;
  }
  info->fused_translate = hp.fuse_te ? 1 : 0;
  info->fourier = hp.fourier ? 1 : 0;
  info->flops_translate = (3.0 * hp.d + 1.0) * ipowd(hp.nr, hp.d) * hp.n_plist();
  info->flops_near = 2.0 * hp.d * ipowd(hp.p, hp.d + 1) * hp.n_near_pair();
  const double ts = hp.precision != FGT_FP64 ? 4.0 : 8.0;
  info->bytes_min = 16.0 * hp.nleaves * pd + 4.0 * ts * ipowd(hp.nr, hp.d) * hp.n_pwbox();
  info->device_bytes = pl->host_only ? fgt::plan_device_bytes(hp) : pl->device_bytes;
  return FGT_OK;
}

void fgt_destroy(fgt_plan_t* pl) { release(pl); }

const char* fgt_strerror(int code) {
  switch (code) {
    case FGT_OK: return "ok";
    case FGT_ERR_INVALID_ARG: return "invalid argument";
    case FGT_ERR_NOT_TILING: return "leaves do not tile the unit box";
    case FGT_ERR_NOT_BALANCED: return "tree is not level-restricted";
    case FGT_ERR_OOM: return "out of memory";
    case FGT_ERR_UNSUPPORTED: return "unsupported configuration";
    case FGT_ERR_HIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

const char* fgt_last_error(void) { return g_err.c_str(); }

int fgt_pw_terms(double eps, double r_over_d0) {
  if (!(eps > 0 && eps < 0.1) || !(r_over_d0 >= 1.0)) return FGT_ERR_INVALID_ARG;
  const double D0 = std::sqrt(std::log(3.0 / eps));
  return 2 * fgt::pw_params(eps, r_over_d0 * D0).M;
}

int fgt_periodic_terms(double eps, double delta) {
  if (!(eps > 0 && eps < 1) || !(delta > 0)) return FGT_ERR_INVALID_ARG;
  return fgt::periodic_terms(eps, delta);
}

int64_t fgt_plan_array(const fgt_plan_t* pl, const char* name, void* dst, int64_t cap) {
  if (!pl || !name) return fail(FGT_ERR_INVALID_ARG, "NULL argument");
  const fgt::HostPlan& hp = pl->hp;
  const std::vector<double>* dv = nullptr;
  const std::vector<int32_t>* iv = nullptr;
  std::string n(name);
  if (n == "F") dv = &hp.F;
  else if (n == "E") dv = &hp.E;
  else if (n == "V") dv = &hp.V;
  else if (n == "rot") dv = &hp.rot;
  else if (n == "pwbox_isleaf") iv = &hp.pwbox_isleaf;
  else if (n == "pw_start") iv = &hp.pw_start;
  else if (n == "pwleaf_id") iv = &hp.pwleaf_id;
  else if (n == "pwleaf_tab") iv = &hp.pwleaf_tab;
  else if (n == "pwleaf_box") iv = &hp.pwleaf_box;
  else if (n == "box_order") iv = &hp.box_order;
  else if (n == "plist_start") iv = &hp.plist_start;
  else if (n == "plist_src") iv = &hp.plist_src;
  else if (n == "plist_dir") iv = &hp.plist_dir;
  else if (n == "te_start") iv = &hp.te_start;
  else if (n == "te_mem") iv = &hp.te_mem;
  else if (n == "te_src") iv = &hp.te_src;
  else if (n == "te_dir") iv = &hp.te_dir;
  else if (n == "te_wg") iv = &hp.te_wg;
  else if (n == "echunk") iv = &hp.echunk;
  else if (n == "fitem") iv = &hp.fitem;
  else if (n == "fred") iv = &hp.fred;
  else if (n == "near_tgt") iv = &hp.near_tgt;
  else if (n == "near_haspw") iv = &hp.near_haspw;
  else if (n == "near_start") iv = &hp.near_start;
  else if (n == "near_src") iv = &hp.near_src;
  else if (n == "near_tab") iv = &hp.near_tab;
  else if (n == "ftab_meta") iv = &hp.ftab_meta;
  else if (n == "vtab_meta") iv = &hp.vtab_meta;
  else if (n == "plane_start") iv = &hp.plane_start;
  else if (n == "plane_tab") iv = &hp.plane_tab;
  else if (n == "plane_row") iv = &hp.plane_row;
  else if (n == "row_start") iv = &hp.row_start;
  else if (n == "row_tab") iv = &hp.row_tab;
  else if (n == "plane_order") iv = &hp.plane_order;
  else return fail(FGT_ERR_INVALID_ARG, "unknown array name");
  if (dv) {
    if (dst && cap > 0) std::memcpy(dst, dv->data(), sizeof(double) * std::min<int64_t>(cap, dv->size()));
    return (int64_t)dv->size();
  }
  if (dst && cap > 0) std::memcpy(dst, iv->data(), sizeof(int32_t) * std::min<int64_t>(cap, iv->size()));
  return (int64_t)iv->size();
}

}  // extern "C"
