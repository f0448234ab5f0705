// Request loop serving many transforms on one device (declared in fgt_serve.h).
//
// One scheduler thread owns the device side: it admits waiting requests onto
// free slot streams, uploads plans within the memory budget, and reaps
// completions by polling each slot's completion event.  Builder threads build
// host plans of new request types.  All shared state sits behind one mutex;
// HIP calls that may take long (uploads, allocations) are made by the
// scheduler with the mutex held, which only delays submitters briefly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fgt.h"
#include "../../include/fgt_serve.h"
#include "plan_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Workspace {
  fgt::DeviceArgs args;
  void* mem = nullptr;   // own allocation; null for the plan's first workspace
  double* io = nullptr;  // staging of host-memory requests: sigma, then u
  bool busy = false;
};

enum class State { Building, Built, Resident, Failed };

struct Entry {
  int64_t key = 0;
  State state = State::Building;
  int err = FGT_OK;
  std::string msg;
  // request type, as first submitted
  int dim = 0, p = 0, bc = 0, precision = 0;
  int64_t nleaves = 0, npoints = 0;
  double delta = 0, tol = 0;
  std::vector<int32_t> level, coord;  // released once the host plan exists
  fgt_plan_t* plan = nullptr;
  int64_t base_bytes = 0;  // tables, lists and the first workspace
  int64_t ws_bytes = 0;    // one more workspace
  int64_t io_bytes = 0;    // sigma + u staging
  std::vector<Workspace> ws;
  int64_t held = 0;        // device bytes this entry holds now
  uint64_t last_use = 0;
  int waiting = 0;         // queued requests of this type
};

struct Request {
  int64_t id = 0;
  Entry* entry = nullptr;
  const double* sigma = nullptr;
  double* u = nullptr;
  bool host_io = false;
  bool cache_hit = false;
  int ws = -1;
  Clock::time_point t_submit, t_launch;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t k0 = nullptr, k1 = nullptr, done = nullptr;
  std::unique_ptr<Request> req;  // null when the slot is free
};

}  // namespace

struct fgt_server {
  int device = 0;
  int64_t budget = 0;
  int64_t resident = 0, peak = 0;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_build;
  uint64_t epoch = 0;  // bumped on every event the scheduler must look at
  bool stopping = false, builders_stop = false, sched_stop = false;
  std::vector<Slot> slots;
  std::map<int64_t, std::unique_ptr<Entry>> entries;
  std::deque<Entry*> build_queue;
  int building = 0;
  std::list<std::unique_ptr<Request>> waiting;  // arrival order
  int running = 0;
  std::deque<fgt_completion_t> done;
  int64_t next_id = 1;
  uint64_t tick = 0;
  fgt_server_stats_t st{};
  std::thread sched;
  std::vector<std::thread> builders;
};

namespace {

void finish(fgt_server* s, const Request& r, int status, float device_ms) {
  fgt_completion_t c{};
  c.id = r.id;
  c.key = r.entry->key;
  c.status = status;
  c.cache_hit = r.cache_hit ? 1 : 0;
  c.npoints = r.entry->npoints;
  const Clock::time_point now = Clock::now();
  c.queue_ms = r.ws >= 0 ? ms_between(r.t_submit, r.t_launch) : ms_between(r.t_submit, now);
  c.total_ms = ms_between(r.t_submit, now);
  c.device_ms = device_ms;
  s->done.push_back(c);
  s->st.completed++;
  if (status != FGT_OK) s->st.failed++;
  s->cv_done.notify_all();
}

void hold(fgt_server* s, Entry* e, int64_t bytes) {
  e->held += bytes;
  s->resident += bytes;
  s->peak = std::max(s->peak, s->resident);
}

// Releases one unit of idle memory held by an entry other than `keep`: first
// the newest idle extra workspace of the least recently used entry, then a
// whole idle plan with no waiting requests; with `any`, also an idle plan
// that has waiting requests.  Returns false if nothing can be released.
bool evict_one(fgt_server* s, const Entry* keep, bool any) {
  Entry* best = nullptr;
  for (auto& kv : s->entries) {
    Entry* e = kv.second.get();
    if (e == keep || e->state != State::Resident || e->ws.size() < 2 || e->ws.back().busy) continue;
    if (!best || e->last_use < best->last_use) best = e;
  }
  if (best) {
    Workspace& w = best->ws.back();
    const int64_t b = best->ws_bytes + (w.io ? best->io_bytes : 0);
    (void)hipFree(w.mem);
    if (w.io) (void)hipFree(w.io);
    best->held -= b;
    s->resident -= b;
    best->ws.pop_back();
    return true;
  }
  for (int pass = 0; pass < (any ? 2 : 1) && !best; pass++) {
    for (auto& kv : s->entries) {
      Entry* e = kv.second.get();
      if (e == keep || e->state != State::Resident || (pass == 0 && e->waiting > 0)) continue;
      bool idle = true;
      for (const Workspace& w : e->ws) idle = idle && !w.busy;
      if (!idle) continue;
      if (!best || e->last_use < best->last_use) best = e;
    }
  }
  if (!best) return false;
  for (Workspace& w : best->ws) {
    if (w.mem) (void)hipFree(w.mem);
    if (w.io) (void)hipFree(w.io);
  }
  best->ws.clear();
  (void)fgt::plan_unload(best->plan);
  s->resident -= best->held;
  best->held = 0;
  best->state = State::Built;
  s->st.plans_evicted++;
  return true;
}

// Makes room for `bytes` more device bytes; false if it cannot be done now.
bool make_room(fgt_server* s, const Entry* keep, int64_t bytes, bool any) {
  while (s->resident + bytes > s->budget)
    if (!evict_one(s, keep, any)) return false;
  return true;
}

void fail_entry(Entry* e, int code, const std::string& msg) {
  e->state = State::Failed;
  e->err = code;
  e->msg = msg;
}

// Admission outcomes of one waiting request.
constexpr int kWaitBusy = -1;   // every workspace of its plan is in use
constexpr int kWaitRoom = -2;   // the budget has no room now
constexpr int kFailOom = -3;    // a device allocation failed

// Uploads a built plan.
int make_resident(fgt_server* s, Entry* e, bool any) {
  if (e->base_bytes > s->budget) {
    fail_entry(e, FGT_ERR_OOM, "request type needs " + std::to_string(e->base_bytes) +
                                   " device bytes, over the server budget");
    return kFailOom;
  }
  if (!make_room(s, e, e->base_bytes, any)) return kWaitRoom;
  const int rc = fgt::plan_upload(e->plan, nullptr);
  if (rc != FGT_OK) {
    const std::string msg = fgt_last_error();
    // a failed allocation may succeed later, once running requests end or
    // other plans are released
    if (rc == FGT_ERR_OOM && (s->running > 0 || s->resident > 0)) return kWaitRoom;
    fail_entry(e, rc, msg);
    return kFailOom;
  }
  e->ws.assign(1, Workspace());
  e->ws[0].args = e->plan->args;
  hold(s, e, e->base_bytes);
  e->state = State::Resident;
  s->st.plans_uploaded++;
  return FGT_OK;
}

// Index of an idle workspace of e ready for the request, adding one (or its
// staging) if allowed and memory permits; else one of the kWait/kFail codes.
int pick_workspace(fgt_server* s, Entry* e, bool host_io, bool alloc, bool any) {
  for (size_t k = 0; k < e->ws.size(); k++) {
    Workspace& w = e->ws[k];
    if (w.busy) continue;
    if (host_io && !w.io) {
      if (!alloc || !make_room(s, e, e->io_bytes, any)) return kWaitRoom;
      void* m = nullptr;
      if (hipMalloc(&m, (size_t)e->io_bytes) != hipSuccess) return kFailOom;
      w.io = static_cast<double*>(m);
      hold(s, e, e->io_bytes);
    }
    return (int)k;
  }
  if (e->ws.size() >= s->slots.size()) return kWaitBusy;
  if (!alloc) return kWaitRoom;
  const int64_t need = e->ws_bytes + (host_io ? e->io_bytes : 0);
  if (!make_room(s, e, need, any)) return kWaitBusy;  // an existing workspace frees up first
  Workspace w;
  if (fgt::plan_alloc_workspace(e->plan, &w.args, &w.mem) != FGT_OK) return kWaitBusy;
  if (host_io) {
    void* m = nullptr;
    if (hipMalloc(&m, (size_t)e->io_bytes) != hipSuccess) {
      (void)hipFree(w.mem);
      return kWaitBusy;
    }
    w.io = static_cast<double*>(m);
  }
  e->ws.push_back(w);
  hold(s, e, need);
  s->st.workspaces_added++;
  return (int)e->ws.size() - 1;
}

// Enqueues the request on slot `k`.
void launch(fgt_server* s, std::unique_ptr<Request> r, int k) {
  Slot& sl = s->slots[k];
  Entry* e = r->entry;
  Workspace& w = e->ws[r->ws];
  w.busy = true;
  e->last_use = ++s->tick;
  const size_t bytes = (size_t)e->npoints * sizeof(double);
  const double* sg = r->sigma;
  double* uu = r->u;
  hipError_t he = hipSuccess;
  if (r->host_io) {
    sg = w.io;
    uu = w.io + e->npoints;
    he = hipMemcpyAsync(w.io, r->sigma, bytes, hipMemcpyHostToDevice, sl.stream);
  }
  int rc = he == hipSuccess ? FGT_OK : FGT_ERR_HIP;
  if (rc == FGT_OK && hipEventRecord(sl.k0, sl.stream) != hipSuccess) rc = FGT_ERR_HIP;
  if (rc == FGT_OK) rc = fgt::execute_args(w.args, sg, uu, sl.stream);
  if (rc == FGT_OK && hipEventRecord(sl.k1, sl.stream) != hipSuccess) rc = FGT_ERR_HIP;
  if (rc == FGT_OK && r->host_io &&
      hipMemcpyAsync(r->u, uu, bytes, hipMemcpyDeviceToHost, sl.stream) != hipSuccess)
    rc = FGT_ERR_HIP;
  if (rc == FGT_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess) rc = FGT_ERR_HIP;
  r->t_launch = Clock::now();
  if (rc != FGT_OK) {
    // work already queued on the stream must end before the workspace is reused
    (void)hipStreamSynchronize(sl.stream);
    w.busy = false;
    finish(s, *r, rc, 0.0f);
    return;
  }
  sl.req = std::move(r);
  s->running++;
}

void reap(fgt_server* s) {
  for (Slot& sl : s->slots) {
    if (!sl.req) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    float ms = 0.0f;
    if (q == hipSuccess) (void)hipEventElapsedTime(&ms, sl.k0, sl.k1);
    std::unique_ptr<Request> r = std::move(sl.req);
    Entry* e = r->entry;
    e->ws[r->ws].busy = false;
    e->last_use = ++s->tick;
    s->running--;
    finish(s, *r, q == hipSuccess ? FGT_OK : FGT_ERR_HIP, ms);
  }
}

// One pass over the waiting requests in arrival order.  A request that
// cannot start yet is skipped, so later ones may start first; once a request
// has been refused memory, later requests may only use workspaces that
// already exist, so small requests cannot keep an older large one out.  The
// oldest request may also release idle plans that have waiting requests.
void admit(fgt_server* s) {
  std::vector<int> free_slots;
  for (int k = (int)s->slots.size() - 1; k >= 0; k--)
    if (!s->slots[k].req) free_slots.push_back(k);
  bool blocked = false;
  for (auto it = s->waiting.begin(); it != s->waiting.end() && !free_slots.empty();) {
    Request* r = it->get();
    Entry* e = r->entry;
    const bool head = it == s->waiting.begin();
    int w = kWaitBusy;
    if (e->state == State::Built) {
      const int rc = blocked ? kWaitRoom : make_resident(s, e, head);
      if (rc == kWaitRoom) blocked = true;
    }
    if (e->state == State::Resident) {
      w = pick_workspace(s, e, r->host_io, !blocked, head);
      if (w == kWaitRoom) blocked = true;
      if (w == kFailOom) {
        e->waiting--;
        fgt::set_error(FGT_ERR_OOM, "device allocation for host-memory staging");
        finish(s, *r, FGT_ERR_OOM, 0.0f);
        it = s->waiting.erase(it);
        continue;
      }
    }
    if (e->state == State::Failed) {
      e->waiting--;
      fgt::set_error(e->err, e->msg);
      finish(s, *r, e->err, 0.0f);
      it = s->waiting.erase(it);
      continue;
    }
    if (w < 0) {
      ++it;
      continue;
    }
    r->ws = w;
    e->waiting--;
    std::unique_ptr<Request> own = std::move(*it);
    it = s->waiting.erase(it);
    const int k = free_slots.back();
    free_slots.pop_back();
    launch(s, std::move(own), k);
  }
}

void scheduler_main(fgt_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    reap(s);
    admit(s);
    if (s->sched_stop && s->running == 0) break;
    if (s->running > 0) {
      // poll the slot events; keep the lock free meanwhile
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else {
      const uint64_t seen = s->epoch;
      s->cv_sched.wait_for(lk, std::chrono::milliseconds(5),
                           [&] { return s->epoch != seen || s->sched_stop; });
    }
  }
}

void builder_main(fgt_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_build.wait(lk, [&] { return s->builders_stop || !s->build_queue.empty(); });
    if (s->build_queue.empty()) return;
    Entry* e = s->build_queue.front();
    s->build_queue.pop_front();
    s->building++;
    lk.unlock();
    fgt_tree_t t{e->dim, e->nleaves, e->level.data(), e->coord.data()};
    fgt_opts_t o{};
    o.force_lc = -1;
    o.precision = e->precision;
    o.host_only = 1;
    fgt_plan_t* pl = nullptr;
    const int rc = fgt_plan(&t, e->p, e->delta, e->tol, e->bc, &o, &pl);
    const std::string msg = rc == FGT_OK ? std::string() : std::string(fgt_last_error());
    lk.lock();
    s->building--;
    if (rc != FGT_OK) {
      fail_entry(e, rc, msg);
    } else {
      e->plan = pl;
      e->base_bytes = fgt::plan_device_bytes(pl->hp);
      e->ws_bytes = fgt::plan_workspace_bytes(pl->hp);
      e->io_bytes = 2 * e->npoints * (int64_t)sizeof(double);
      e->state = State::Built;
      s->st.plans_built++;
    }
    std::vector<int32_t>().swap(e->level);
    std::vector<int32_t>().swap(e->coord);
    s->epoch++;
    s->cv_sched.notify_one();
    s->cv_done.notify_all();
  }
}

bool idle(const fgt_server* s) { return s->waiting.empty() && s->running == 0; }

int take(fgt_server* s, fgt_completion_t* out, int32_t max, int32_t* n) {
  int32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n = k;
  return FGT_OK;
}

}  // namespace

extern "C" {

int fgt_server_create(const fgt_server_opts_t* opts, fgt_server_t** out) {
  if (!out) return fgt::set_error(FGT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  fgt_server_opts_t o{};
  if (opts) o = *opts;
  if (o.nslots == 0) o.nslots = 4;
  if (o.nbuilders == 0) o.nbuilders = 2;
  if (o.nslots < 1 || o.nslots > 64 || o.nbuilders < 1 || o.nbuilders > 16 || o.hbm_budget < 0)
    return fgt::set_error(FGT_ERR_INVALID_ARG, "nslots must be 1..64, nbuilders 1..16, hbm_budget >= 0");
  std::unique_ptr<fgt_server> s(new (std::nothrow) fgt_server());
  if (!s) return fgt::set_error(FGT_ERR_OOM, "host allocation");
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) return fgt::set_error(FGT_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  size_t free_b = 0, total_b = 0;
  e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) return fgt::set_error(FGT_ERR_HIP, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
  s->budget = o.hbm_budget > 0 ? o.hbm_budget : (int64_t)(0.9 * (double)free_b);
  s->slots.resize(o.nslots);
  for (Slot& sl : s->slots) {
    if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreate(&sl.k0)) != hipSuccess || (e = hipEventCreate(&sl.k1)) != hipSuccess ||
        (e = hipEventCreate(&sl.done)) != hipSuccess) {
      for (Slot& t : s->slots) {
        if (t.stream) (void)hipStreamDestroy(t.stream);
        if (t.k0) (void)hipEventDestroy(t.k0);
        if (t.k1) (void)hipEventDestroy(t.k1);
        if (t.done) (void)hipEventDestroy(t.done);
      }
      return fgt::set_error(FGT_ERR_HIP, std::string("stream/event creation: ") + hipGetErrorString(e));
    }
  }
  s->st.nslots = o.nslots;
  fgt_server* raw = s.get();
  raw->sched = std::thread(scheduler_main, raw);
  for (int i = 0; i < o.nbuilders; i++) raw->builders.emplace_back(builder_main, raw);
  *out = s.release();
  return FGT_OK;
}

int fgt_server_submit(fgt_server_t* s, const fgt_request_t* q, int64_t* id) {
  if (!s || !q || !id) return fgt::set_error(FGT_ERR_INVALID_ARG, "server, request or id is NULL");
  *id = 0;
  if (!q->sigma || !q->u) return fgt::set_error(FGT_ERR_INVALID_ARG, "sigma or u is NULL");
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return fgt::set_error(FGT_ERR_OOM, "host allocation");
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return fgt::set_error(FGT_ERR_INVALID_ARG, "server is shutting down");
  auto it = s->entries.find(q->key);
  Entry* e;
  if (it == s->entries.end()) {
    const fgt_tree_t* t = q->tree;
    if (!t || !t->level || !t->coord || t->dim < 1 || t->dim > 3 || t->nleaves < 1)
      return fgt::set_error(FGT_ERR_INVALID_ARG, "the first request of a key needs a valid tree");
    if (q->p < 1 || q->p > 16) return fgt::set_error(FGT_ERR_INVALID_ARG, "p out of range");
    std::unique_ptr<Entry> ne(new (std::nothrow) Entry());
    if (!ne) return fgt::set_error(FGT_ERR_OOM, "host allocation");
    ne->key = q->key;
    ne->dim = t->dim;
    ne->nleaves = t->nleaves;
    ne->p = q->p;
    ne->delta = q->delta;
    ne->tol = q->tol;
    ne->bc = q->bc;
    ne->precision = q->precision;
    int64_t pd = 1;
    for (int a = 0; a < t->dim; a++) pd *= q->p;
    ne->npoints = t->nleaves * pd;
    ne->level.assign(t->level, t->level + t->nleaves);
    ne->coord.assign(t->coord, t->coord + t->nleaves * t->dim);
    e = ne.get();
    s->entries[q->key] = std::move(ne);
    s->build_queue.push_back(e);
    s->cv_build.notify_one();
  } else {
    e = it->second.get();
    if (e->p != q->p || e->delta != q->delta || e->tol != q->tol || e->bc != q->bc ||
        e->precision != q->precision || (q->tree && (q->tree->dim != e->dim || q->tree->nleaves != e->nleaves)))
      return fgt::set_error(FGT_ERR_INVALID_ARG, "key " + std::to_string(q->key) +
                                                     " was first submitted with other parameters");
    r->cache_hit = e->state == State::Built || e->state == State::Resident;
  }
  r->id = s->next_id++;
  r->entry = e;
  r->sigma = q->sigma;
  r->u = q->u;
  r->host_io = q->host_io != 0;
  e->waiting++;
  *id = r->id;
  s->waiting.push_back(std::move(r));
  s->st.submitted++;
  s->epoch++;
  s->cv_sched.notify_one();
  return FGT_OK;
}

int fgt_server_poll(fgt_server_t* s, fgt_completion_t* out, int32_t max, int32_t* n) {
  if (!s || !n || (max > 0 && !out)) return fgt::set_error(FGT_ERR_INVALID_ARG, "bad poll arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  return take(s, out, max, n);
}

int fgt_server_wait(fgt_server_t* s, fgt_completion_t* out, int32_t max, int32_t* n, double timeout_ms) {
  if (!s || !n || (max > 0 && !out)) return fgt::set_error(FGT_ERR_INVALID_ARG, "bad wait arguments");
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] { return !s->done.empty() || idle(s); };
  if (timeout_ms < 0)
    s->cv_done.wait(lk, ready);
  else
    s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready);
  return take(s, out, max, n);
}

int fgt_server_drain(fgt_server_t* s) {
  if (!s) return fgt::set_error(FGT_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return idle(s); });
  return FGT_OK;
}

int fgt_server_stats(fgt_server_t* s, fgt_server_stats_t* out) {
  if (!s || !out) return fgt::set_error(FGT_ERR_INVALID_ARG, "server or out is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->resident_bytes = s->resident;
  out->peak_resident_bytes = s->peak;
  out->budget_bytes = s->budget;
  out->running = s->running;
  out->waiting = (int32_t)s->waiting.size();
  return FGT_OK;
}

int fgt_server_destroy(fgt_server_t* s) {
  if (!s) return FGT_OK;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->stopping = true;
    s->cv_done.wait(lk, [&] { return idle(s); });
    s->builders_stop = true;
    s->sched_stop = true;
    s->cv_build.notify_all();
    s->cv_sched.notify_all();
  }
  for (std::thread& t : s->builders) t.join();
  s->sched.join();
  (void)hipSetDevice(s->device);
  for (Slot& sl : s->slots) {
    (void)hipStreamSynchronize(sl.stream);
    (void)hipStreamDestroy(sl.stream);
    (void)hipEventDestroy(sl.k0);
    (void)hipEventDestroy(sl.k1);
    (void)hipEventDestroy(sl.done);
  }
  for (auto& kv : s->entries) {
    Entry* e = kv.second.get();
    for (Workspace& w : e->ws) {
      if (w.mem) (void)hipFree(w.mem);
      if (w.io) (void)hipFree(w.io);
    }
    if (e->plan) fgt_destroy(e->plan);
  }
  delete s;
  return FGT_OK;
}

}  // extern "C"
