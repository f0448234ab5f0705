// Many transforms per launch (declared in fgt_batch.h).
//
// Plans are grouped by kernel class; for every class and stage one launch
// covers all the class's transforms (kernels_fast.hip, *_b kernels).  The
// launch sequence of an execution is captured into a HIP graph on a private
// stream and replayed on the batch's stream.  A schedule spreads the classes
// over one or more streams (a fork/join inside the graph) and orders each
// stream's launches stage by stage or class by class; the caller picks it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/fgt.h"
#include "../../include/fgt_batch.h"
#include "plan_internal.h"

namespace {

struct ClassRun {
  fgt::KernelClass kc;
  std::vector<int> members;                 // plan indices
  int64_t grid[fgt::kNumStages] = {};       // blocks of each stage's launch
  std::vector<int32_t> start, count;        // [kNumStages + 1][n], host copies; the last
                                            // row: box formation with tile 1
  int64_t grid_alt = 0;                     // blocks of box formation with tile 1
  int tile = 0;                             // box-formation tile shape (kFormBoxTileSlabs)
  double work = 0;                          // blocks over all stages (schedule weight)
  fgt::BatchJob* jobs = nullptr;            // device [n]
  int32_t* dstart = nullptr;                // device [kNumStages + 1][n]
  int32_t* dcount = nullptr;
  bool persistent = false;                  // one persistent launch for all stages
  int64_t items = 0;                        // its work items (tile-0 blocks of every stage)
  int64_t* dbase = nullptr;                 // device [kNumStages + 1] first item per stage
  uint64_t* dhead = nullptr;                // device work queue
  int32_t* dctl = nullptr;                  // device [1 + n kNumStages] error flag, done counts
  bool has_tiles() const { return kc.d == 3 && grid[fgt::kFormBox] > 0; }
};

// Persistent launches: workgroups per class launch (4 per CU of 256 CUs; more
// only queue) and the bound of a block's wait for its transform's previous
// stage, in polls of about 0.1 us (under a second).
constexpr int64_t kPersistentGrid = 1024;
constexpr int kSpinLimit = 1 << 22;

int herr(hipError_t e, const char* what) {
  return fgt::set_error(FGT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

struct fgt_batch {
  int device = 0;
  hipStream_t stream = nullptr;   // the caller's (may be the default stream)
  hipStream_t cap = nullptr;      // private stream used for graph capture
  std::vector<fgt_plan_t*> plans;
  std::vector<ClassRun> classes;
  std::vector<int> singles;       // 1D plans
  std::vector<const double*> sigma;
  std::vector<double*> u;
  bool bound = false;
  bool use_graph = true;
  int nstreams = 1;
  bool class_major = false;
  bool persistent = false;
  std::vector<hipStream_t> side;  // nstreams - 1 streams of the fork/join
  std::vector<hipEvent_t> ev;     // fork + joins
  hipGraphExec_t exec = nullptr;
  int nlaunch = 0;
  double tuned_ms = 0;
  std::vector<void*> allocs;
};

namespace {

// Destroys the instantiated graph once no replay of it is in flight.
void drop_graph(fgt_batch* b) {
  if (b->exec) {
    (void)hipStreamSynchronize(b->stream);
    (void)hipGraphExecDestroy(b->exec);
  }
  b->exec = nullptr;
}

// Creates side streams up to nstreams - 1; streams beyond that (left by a
// tuning run) stay idle until the batch is released.
int ensure_side_streams(fgt_batch* b) {
  while ((int)b->side.size() < b->nstreams - 1) {
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return herr(e, "hipStreamCreate");
    b->side.push_back(s);
  }
  while ((int)b->ev.size() < b->nstreams) {
    hipEvent_t x = nullptr;
    hipError_t e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
    if (e != hipSuccess) return herr(e, "hipEventCreate");
    b->ev.push_back(x);
  }
  return FGT_OK;
}

// Longest-processing-time assignment of classes to streams.
std::vector<std::vector<int>> assign(const fgt_batch* b) {
  std::vector<int> order(b->classes.size());
  for (size_t i = 0; i < order.size(); i++) order[i] = (int)i;
  std::sort(order.begin(), order.end(),
            [&](int x, int y) { return b->classes[x].work > b->classes[y].work; });
  std::vector<std::vector<int>> per(b->nstreams);
  std::vector<double> load(b->nstreams, 0.0);
  for (int c : order) {
    const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    per[s].push_back(c);
    load[s] += b->classes[c].work;
  }
  return per;
}

// Enqueues one execution on `st` (the capture stream or the caller's stream).
int enqueue(fgt_batch* b, hipStream_t st) {
  const std::vector<std::vector<int>> per = assign(b);
  hipError_t e;
  int launches = 0;
  // fork exactly the nstreams - 1 side streams that are joined below: under
  // capture, a stream that waits on the fork event joins the capture
  if (b->nstreams > 1) {
    if ((e = hipEventRecord(b->ev[0], st)) != hipSuccess) return herr(e, "hipEventRecord");
    for (int si = 1; si < b->nstreams; si++)
      if ((e = hipStreamWaitEvent(b->side[si - 1], b->ev[0], 0)) != hipSuccess)
        return herr(e, "hipStreamWaitEvent");
  }
  for (int si = 0; si < b->nstreams; si++) {
    hipStream_t s = si == 0 ? st : b->side[si - 1];
    auto run = [&](int c, int stage) -> int {
      ClassRun& cr = b->classes[c];
      if (cr.persistent) {
        // the class's single launch, issued in the slot of its first stage
        if (stage != 0) return FGT_OK;
        const int n = (int)cr.members.size();
        const int64_t nctl = 1 + (int64_t)n * fgt::kNumStages;
        hipError_t le = fgt::zero_i32(cr.dctl, nctl, s);
        if (le == hipSuccess) le = fgt::zero_i32(reinterpret_cast<int32_t*>(cr.dhead), 2, s);
        if (le != hipSuccess) return herr(le, "zero counters");
        const int grid = (int)std::min<int64_t>(cr.items, kPersistentGrid);
        le = fgt::launch_class_persistent(cr.kc, cr.jobs, cr.dstart, cr.dcount, n, cr.dbase, cr.dhead, cr.dctl,
                                          kSpinLimit, grid, s);
        if (le != hipSuccess) return herr(le, "persistent launch");
        launches += 3;
        return FGT_OK;
      }
      if (cr.grid[stage] == 0) return FGT_OK;
      const int n = (int)cr.members.size();
      const bool alt = stage == fgt::kFormBox && cr.tile == 1;
      const size_t row = alt ? (size_t)fgt::kNumStages : (size_t)stage;
      hipError_t le = fgt::launch_stage_batched(cr.kc, stage, cr.jobs, cr.dstart + row * n, cr.dcount + row * n, n,
                                                alt ? cr.grid_alt : cr.grid[stage], s, alt ? 1 : 0);
      if (le != hipSuccess) return herr(le, "batched launch");
      launches++;
      return FGT_OK;
    };
    int rc;
    if (b->class_major) {
      for (int c : per[si])
        for (int stage = 0; stage < fgt::kNumStages; stage++)
          if ((rc = run(c, stage)) != FGT_OK) return rc;
    } else {
      for (int stage = 0; stage < fgt::kNumStages; stage++)
        for (int c : per[si])
          if ((rc = run(c, stage)) != FGT_OK) return rc;
    }
  }
  for (int i : b->singles) {
    const int rc = fgt::execute_args(b->plans[i]->args, b->sigma[i], b->u[i], st);
    if (rc != FGT_OK) return rc;
    launches += 7;
  }
  if (b->nstreams > 1) {
    for (int si = 1; si < b->nstreams; si++) {
      if ((e = hipEventRecord(b->ev[si], b->side[si - 1])) != hipSuccess) return herr(e, "hipEventRecord");
      if ((e = hipStreamWaitEvent(st, b->ev[si], 0)) != hipSuccess) return herr(e, "hipStreamWaitEvent");
    }
  }
  b->nlaunch = launches;
  return FGT_OK;
}

int build_graph(fgt_batch* b) {
  drop_graph(b);
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return herr(e, "hipStreamBeginCapture");
  const int rc = enqueue(b, b->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);
  if (rc != FGT_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return herr(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->exec = nullptr;
    return herr(e, "hipGraphInstantiate");
  }
  return FGT_OK;
}

int launch(fgt_batch* b) {
  if (!b->use_graph) return enqueue(b, b->stream);
  if (!b->exec) {
    const int rc = build_graph(b);
    if (rc != FGT_OK) return rc;
  }
  const hipError_t e = hipGraphLaunch(b->exec, b->stream);
  return e == hipSuccess ? FGT_OK : herr(e, "hipGraphLaunch");
}

void release(fgt_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
  for (hipEvent_t x : b->ev) (void)hipEventDestroy(x);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (void* p : b->allocs) (void)hipFree(p);
  delete b;
}

}  // namespace

extern "C" {

int fgt_batch_create(fgt_plan_t* const* plans, int64_t nplans, const fgt_batch_opts_t* opts,
                     fgt_batch_t** out) {
  if (!out) return fgt::set_error(FGT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!plans || nplans < 1 || nplans > (1 << 20))
    return fgt::set_error(FGT_ERR_INVALID_ARG, "need 1..2^20 plans");
  fgt_batch_opts_t o{};
  o.use_graph = 1;
  if (opts) o = *opts;
  if (o.nstreams == 0) o.nstreams = 1;
  if (o.nstreams < 1 || o.nstreams > 8) return fgt::set_error(FGT_ERR_INVALID_ARG, "nstreams must be 1..8");
  if (o.form_tile < 0 || o.form_tile >= fgt::kFormBoxTiles)
    return fgt::set_error(FGT_ERR_INVALID_ARG, "form_tile must be 0 or 1");
  if (o.persistent)
    // Switched off: on the device, a batch of 13 classes with this option did
    // not finish its first execution within three minutes, twice (with the
    // waits polled by acquire loads, then by relaxed loads and one acquire);
    // the cause is not established and the path stays off.
    return fgt::set_error(FGT_ERR_UNSUPPORTED,
                          "persistent batched launches are switched off (they did not finish on the device)");
  fgt_batch* b = new (std::nothrow) fgt_batch();
  if (!b) return fgt::set_error(FGT_ERR_OOM, "host allocation");
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) {
    delete b;
    return herr(e, "hipGetDevice");
  }
  b->stream = static_cast<hipStream_t>(o.stream);
  b->use_graph = o.use_graph != 0;
  b->nstreams = o.nstreams;
  b->class_major = o.class_major != 0;
  b->persistent = o.persistent != 0;
  b->plans.assign(plans, plans + nplans);
  for (int64_t i = 0; i < nplans; i++) {
    const fgt_plan_t* pl = plans[i];
    if (!pl || pl->host_only || pl->device != b->device) {
      delete b;
      return fgt::set_error(FGT_ERR_INVALID_ARG, "plan " + std::to_string(i) +
                                                     " is NULL, host-only or on another device");
    }
  }
  // classes
  std::vector<fgt::KernelClass> keys;
  for (int64_t i = 0; i < nplans; i++) {
    const fgt::DeviceArgs& a = plans[i]->args;
    if (a.d == 1) {
      b->singles.push_back((int)i);
      continue;
    }
    const fgt::KernelClass kc = fgt::kernel_class(a);
    size_t c = 0;
    while (c < keys.size() && (keys[c] < kc || kc < keys[c])) c++;
    if (c == keys.size()) {
      keys.push_back(kc);
      b->classes.emplace_back();
      b->classes.back().kc = kc;
    }
    b->classes[c].members.push_back((int)i);
  }
  for (ClassRun& cr : b->classes) {
    const int n = (int)cr.members.size();
    cr.start.assign((size_t)(fgt::kNumStages + 1) * n, 0);
    cr.count.assign((size_t)(fgt::kNumStages + 1) * n, 0);
    // row kNumStages: box formation with the alternative tile shape
    for (int stage = 0; stage <= fgt::kNumStages; stage++) {
      int64_t at = 0;
      for (int j = 0; j < n; j++) {
        const fgt::DeviceArgs& ja = plans[cr.members[j]]->args;
        const int64_t nb = stage < fgt::kNumStages ? fgt::stage_blocks(ja, stage)
                                                   : (cr.kc.d == 3 ? fgt::form_box_blocks(ja, fgt::kFormBoxTileSlabs[1])
                                                                   : fgt::stage_blocks(ja, fgt::kFormBox));
        at = (at + 7) / 8 * 8;  // keep block % 8 == XCD of the transform's own blocks
        cr.start[(size_t)stage * n + j] = (int32_t)at;
        cr.count[(size_t)stage * n + j] = (int32_t)nb;
        at += nb;
        if (stage < fgt::kNumStages) cr.work += (double)nb;
      }
      if (at > 0x7fffffff) {
        release(b);
        return fgt::set_error(FGT_ERR_UNSUPPORTED, "a batched launch would exceed 2^31 workgroups");
      }
      if (stage < fgt::kNumStages) cr.grid[stage] = at;
      else cr.grid_alt = at;
    }
    void* m = nullptr;
    const size_t jb = sizeof(fgt::BatchJob) * n, ib = sizeof(int32_t) * cr.start.size();
    cr.persistent = b->persistent && fgt::persistent_supported(cr.kc);
    if (cr.persistent) {
      std::vector<int64_t> base(fgt::kNumStages + 1, 0);
      for (int stage = 0; stage < fgt::kNumStages; stage++) base[stage + 1] = base[stage] + cr.grid[stage];
      cr.items = base[fgt::kNumStages];
      const size_t nctl = 1 + (size_t)n * fgt::kNumStages;
      void* pm = nullptr;
      e = hipMalloc(&pm, sizeof(int64_t) * base.size() + 16 + sizeof(int32_t) * nctl);
      if (e != hipSuccess) {
        release(b);
        return fgt::set_error(FGT_ERR_OOM, "persistent counters");
      }
      b->allocs.push_back(pm);
      cr.dbase = static_cast<int64_t*>(pm);
      cr.dhead = reinterpret_cast<uint64_t*>(cr.dbase + base.size());
      cr.dctl = reinterpret_cast<int32_t*>(cr.dhead + 2);
      if ((e = hipMemcpy(cr.dbase, base.data(), sizeof(int64_t) * base.size(), hipMemcpyHostToDevice)) !=
          hipSuccess) {
        release(b);
        return herr(e, "hipMemcpy");
      }
    }
    e = hipMalloc(&m, jb + 2 * ib + 256);
    if (e != hipSuccess) {
      release(b);
      return fgt::set_error(FGT_ERR_OOM, "batch tables");
    }
    b->allocs.push_back(m);
    cr.jobs = static_cast<fgt::BatchJob*>(m);
    cr.dstart = reinterpret_cast<int32_t*>(static_cast<char*>(m) + (jb + 255) / 256 * 256);
    cr.dcount = cr.dstart + cr.start.size();
    if ((e = hipMemcpy(cr.dstart, cr.start.data(), ib, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(cr.dcount, cr.count.data(), ib, hipMemcpyHostToDevice)) != hipSuccess) {
      release(b);
      return herr(e, "hipMemcpy");
    }
  }
  for (ClassRun& cr : b->classes)
    if (cr.has_tiles()) cr.tile = o.form_tile;
  b->sigma.assign(nplans, nullptr);
  b->u.assign(nplans, nullptr);
  int rc;
  if ((e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) {
    release(b);
    return herr(e, "hipStreamCreate");
  }
  if ((rc = ensure_side_streams(b)) != FGT_OK) {
    release(b);
    return rc;
  }
  *out = b;
  return FGT_OK;
}

int fgt_batch_bind(fgt_batch_t* b, const double* const* sigma, double* const* u) {
  if (!b || !sigma || !u) return fgt::set_error(FGT_ERR_INVALID_ARG, "batch, sigma or u is NULL");
  for (size_t i = 0; i < b->plans.size(); i++)
    if (!sigma[i] || !u[i]) return fgt::set_error(FGT_ERR_INVALID_ARG, "sigma[i] or u[i] is NULL");
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return herr(e, "hipSetDevice");
  if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return herr(e, "hipStreamSynchronize");
  for (size_t i = 0; i < b->plans.size(); i++) {
    b->sigma[i] = sigma[i];
    b->u[i] = u[i];
  }
  for (ClassRun& cr : b->classes) {
    std::vector<fgt::BatchJob> jobs(cr.members.size());
    for (size_t j = 0; j < jobs.size(); j++) {
      const int i = cr.members[j];
      jobs[j].a = b->plans[i]->args;
      jobs[j].sigma = sigma[i];
      jobs[j].u = u[i];
    }
    if ((e = hipMemcpy(cr.jobs, jobs.data(), sizeof(fgt::BatchJob) * jobs.size(), hipMemcpyHostToDevice)) !=
        hipSuccess)
      return herr(e, "hipMemcpy");
  }
  // 1D plans take sigma/u as kernel arguments: their captured launches change
  if (!b->singles.empty()) drop_graph(b);
  b->bound = true;
  return FGT_OK;
}

int fgt_batch_execute(fgt_batch_t* b) {
  if (!b) return fgt::set_error(FGT_ERR_INVALID_ARG, "batch is NULL");
  if (!b->bound) return fgt::set_error(FGT_ERR_INVALID_ARG, "batch is not bound (fgt_batch_bind)");
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return herr(e, "hipSetDevice");
  return launch(b);
}

int fgt_batch_tune(fgt_batch_t* b, int32_t reps, double* best_ms) {
  if (!b || reps < 1) return fgt::set_error(FGT_ERR_INVALID_ARG, "batch is NULL or reps < 1");
  if (best_ms) *best_ms = 0;
  // The tuner re-captured and re-instantiated the batch graph once per trial
  // schedule (with a fork/join over side streams) and crashed the host process
  // intermittently on large batches; its cause is not established, so the
  // schedule stays the one given at fgt_batch_create.
  return fgt::set_error(FGT_ERR_UNSUPPORTED,
                        "fgt_batch_tune is switched off; pick the schedule in fgt_batch_opts_t");
}

int fgt_batch_info(const fgt_batch_t* b, fgt_batch_info_t* info) {
  if (!b || !info) return fgt::set_error(FGT_ERR_INVALID_ARG, "batch or info is NULL");
  *info = fgt_batch_info_t{};
  info->njobs = (int64_t)b->plans.size();
  for (const fgt_plan_t* pl : b->plans) {
    int64_t pd = 1;
    for (int a = 0; a < pl->hp.d; a++) pd *= pl->hp.p;
    info->npoints += pl->hp.nleaves * pd;
  }
  info->nclasses = (int32_t)b->classes.size();
  info->nsingle = (int32_t)b->singles.size();
  int nl = 7 * (int)b->singles.size();
  for (const ClassRun& cr : b->classes)
    if (cr.persistent) nl += 3;  // two counter clears and the persistent kernel
    else
      for (int s = 0; s < fgt::kNumStages; s++) nl += cr.grid[s] > 0;
  info->nlaunches = nl;
  info->nstreams = b->nstreams;
  info->class_major = b->class_major ? 1 : 0;
  info->use_graph = b->use_graph ? 1 : 0;
  info->tuned_ms = b->tuned_ms;
  for (const ClassRun& cr : b->classes) info->tile_alt_classes += cr.tile == 1;
  for (const ClassRun& cr : b->classes) {
    if (!cr.persistent) continue;
    info->persistent++;
    int32_t flag = 0;
    if (hipMemcpy(&flag, cr.dctl, sizeof(flag), hipMemcpyDeviceToHost) == hipSuccess && flag)
      info->persistent_error = 1;
  }
  return FGT_OK;
}

int fgt_batch_destroy(fgt_batch_t* b) {
  release(b);
  return FGT_OK;
}

}  // extern "C"
