// Continuous-batching request server (rpca_server_* in include/rpca.h).
//
// Requests queue in arrival order.  Each step of the server
//   1. admits queued requests in FIFO order while the number of active
//      solves is below max_active and the admission footprint of the active
//      set (library workspace plus the request's M, L and S) stays within the
//      HBM budget; the request at the head waits until enough finishes (no
//      overtaking), and a request larger than the whole budget is completed
//      at once with RPCA_ERR_NOMEM;
//   2. gives each admitted request its device workspace (held until it
//      finishes, so its S, Y, eigenvectors and state stay resident between
//      steps) and runs its init pass;
//   3. runs `quantum` iterations of every active solve together, on the
//      lanes of the engine (a solve that has stopped exits its launches at
//      once), then reads back all solve states with one gather and copy;
//   4. retires the solves that stopped: the finalize pass writes L and S,
//      the workspace is freed and a completion is reported.
// A solve's arithmetic depends only on its own data and shape, so its result
// is bitwise the same whatever else is active.
//
// A request may carry a timeout (rpca_server_set_timeout before submitting):
// once that much time has passed since its submission, it is completed with
// RPCA_ERR_TIMEOUT at the next step, whether it is still queued or active
// (an active solve is dropped after the quantum that was running, its
// workspace freed and its L and S left unspecified).
//
// With RPCA_SERVER_SIMULATE no HIP call is made: admission and retirement run
// as above and every request finishes after maxit iterations, counted in
// quanta, on a clock that advances by exactly 1 ms per step.  This exercises
// the queueing, timeout and failure logic without a device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <vector>

#include "rpca.h"
#include "common.h"
#include "engine.h"
#include "launch.h"

namespace rpca {
namespace {

struct Req {
  rpca_problem p{};
  int64_t tag = 0;
  size_t footprint = 0;  // admission footprint
  SolveRec rec;
  int sim_iter = 0;      // simulate: iterations run
  int64_t deadline = 0;  // server clock (ns) after which it times out; 0 = never
};

size_t io_bytes(int64_t m, int64_t n, int dtype) {
  return 3 * static_cast<size_t>(m) * static_cast<size_t>(n) * (dtype == RPCA_F32 ? 4 : 8);
}

}  // namespace
}  // namespace rpca

struct rpca_server {
  int dtype = RPCA_F32;
  int gram_mode = RPCA_GRAM_DEFAULT;
  size_t budget = 0, used = 0, peak = 0;
  int max_active = 1, quantum = 1;
  bool simulate = false;
  bool broken = false;
  hipStream_t user = nullptr;
  std::deque<rpca::Req*> queue;
  std::vector<rpca::Req*> active;
  std::deque<rpca_completion> ready;
  rpca::Lanes lanes;
  bool lanes_ok = false;
  rpca::Plan plan;
  bool plan_valid = false;
  double timeout_s = 0.0;   // applied to requests submitted from now on
  int64_t sim_clock = 0;    // simulate: ns, +1 ms per step
  int inject_init = 0;      // fail the next init stage with this code (0 = none)
  std::mutex mu;
};

namespace rpca {
namespace {

#define SV(expr)                  \
  do {                            \
    const hipError_t e_ = (expr); \
    if (e_ != hipSuccess) {       \
      set_error(#expr, e_);       \
      return RPCA_ERR_DEVICE;     \
    }                             \
  } while (0)

void complete(rpca_server* s, Req* r, int status, int iters, double resid) {
  rpca_completion c;
  c.tag = r->tag;
  c.status = status;
  c.iterations = iters;
  c.residual = resid;
  s->ready.push_back(c);
}

// Server clock in ns: steady time, or the simulated clock.
int64_t now_ns(const rpca_server* s) {
  if (s->simulate) return s->sim_clock;
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

bool expired(const rpca_server* s, const Req* r, int64_t now) {
  return r->deadline != 0 && now >= r->deadline;
}

// Complete every queued request whose deadline has passed.
void expire_queued(rpca_server* s, int64_t now) {
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    if (expired(s, *it, now)) {
      complete(s, *it, RPCA_ERR_TIMEOUT, 0, 0.0);
      delete *it;
      it = s->queue.erase(it);
    } else {
      ++it;
    }
  }
}

// Newly admitted requests whose set-up failed: give back their workspace
// (if they got one) and their share of the budget, and complete them with
// the failure's code.
void fail_admitted(rpca_server* s, std::vector<Req*>& reqs, int code, hipStream_t stream) {
  for (Req* r : reqs) {
    if (r->rec.mem) {
      (void)hipFreeAsync(r->rec.mem, stream);
      r->rec.mem = nullptr;
    }
    s->used -= r->footprint;
    complete(s, r, code, 0, 0.0);
    delete r;
  }
  reqs.clear();
}

// FIFO admission under max_active and the footprint budget.
void admit(rpca_server* s, std::vector<Req*>& fresh) {
  while (!s->queue.empty() && static_cast<int>(s->active.size() + fresh.size()) < s->max_active) {
    Req* r = s->queue.front();
    if (r->footprint > s->budget) {
      s->queue.pop_front();
      complete(s, r, RPCA_ERR_NOMEM, 0, 0.0);
      delete r;
      continue;
    }
    if (s->used + r->footprint > s->budget) break;
    s->queue.pop_front();
    s->used += r->footprint;
    s->peak = std::max(s->peak, s->used);
    fresh.push_back(r);
  }
}

int step_simulated(rpca_server* s) {
  s->sim_clock += 1000000;  // 1 ms per step
  const int64_t now = now_ns(s);
  expire_queued(s, now);
  std::vector<Req*> fresh;
  admit(s, fresh);
  if (!fresh.empty() && s->inject_init != 0) {
    const int code = s->inject_init;
    s->inject_init = 0;
    fail_admitted(s, fresh, code, nullptr);
  }
  for (Req* r : fresh) s->active.push_back(r);
  std::vector<Req*> keep;
  for (Req* r : s->active) {
    r->sim_iter = std::min(r->p.maxit, r->sim_iter + s->quantum);
    if (expired(s, r, now) && r->sim_iter < r->p.maxit) {
      complete(s, r, RPCA_ERR_TIMEOUT, r->sim_iter, 0.0);
      s->used -= r->footprint;
      delete r;
    } else if (r->sim_iter >= r->p.maxit) {
      complete(s, r, RPCA_NOT_CONVERGED, r->sim_iter, 0.0);
      s->used -= r->footprint;
      delete r;
    } else {
      keep.push_back(r);
    }
  }
  s->active.swap(keep);
  return RPCA_OK;
}

std::vector<SolveRec*> recs_of(const std::vector<Req*>& v) {
  std::vector<SolveRec*> out;
  out.reserve(v.size());
  for (Req* r : v) out.push_back(&r->rec);
  return out;
}

int nlanes_for(size_t count) { return static_cast<int>(std::min<size_t>(count, kServeLanes)); }

// Fork the lanes from lane 0 (each lane waits for lane 0's work so far).
hipError_t fork_from0(const Lanes& L) {
  if (L.s.size() <= 1) return hipSuccess;
  hipError_t e = hipEventRecord(L.fork, L.s[0]);
  for (size_t i = 1; i < L.s.size() && e == hipSuccess; ++i) e = hipStreamWaitEvent(L.s[i], L.fork, 0);
  return e;
}

hipError_t join_to0(const Lanes& L) {
  hipError_t e = hipSuccess;
  for (size_t i = 1; i < L.s.size() && e == hipSuccess; ++i) {
    e = hipEventRecord(L.join[i], L.s[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(L.s[0], L.join[i], 0);
  }
  return e;
}

// Set-up of newly admitted requests: workspace, then their init pass.  On a
// failure the requests of this stage are released (fail_admitted) before the
// code is returned, so nothing leaks and the budget is given back.
int start_admitted(rpca_server* s, std::vector<Req*>& fresh) {
  Lanes& L = s->lanes;
  hipStream_t s0 = L.s[0];
  if (s->inject_init != 0) {
    const int code = s->inject_init;
    s->inject_init = 0;
    fail_admitted(s, fresh, code, s0);
    return code == RPCA_ERR_DEVICE ? code : RPCA_OK;
  }
  {
    const hipError_t e = hipStreamSynchronize(s->user);  // inputs come from the caller's stream
    if (e != hipSuccess) {
      set_error("hipStreamSynchronize(caller stream)", e);
      fail_admitted(s, fresh, RPCA_ERR_DEVICE, s0);
      return RPCA_ERR_DEVICE;
    }
  }
  std::vector<Req*> ok;
  for (Req* r : fresh) {
    void* mem = nullptr;
    const hipError_t e = hipMallocAsync(&mem, r->rec.big.total, s0);
    if (e != hipSuccess || mem == nullptr) {
      (void)hipGetLastError();
      s->used -= r->footprint;
      complete(s, r, RPCA_ERR_NOMEM, 0, 0.0);
      delete r;
      continue;
    }
    r->rec.mem = static_cast<char*>(mem);
    ok.push_back(r);
  }
  fresh.clear();
  if (ok.empty()) return RPCA_OK;
  std::vector<SolveRec*> recs = recs_of(ok);
  const int nl = nlanes_for(recs.size());
  assign_lanes(recs, nl);
  Plan pn;
  const int rc = plan_build(pn, recs, nl, s->dtype, s0);
  if (rc != RPCA_OK) {
    plan_free(pn, s0);
    fail_admitted(s, ok, rc, s0);
    return rc == RPCA_ERR_DEVICE ? rc : RPCA_OK;
  }
  Lanes sub;  // the first nl lanes
  sub.s.assign(L.s.begin(), L.s.begin() + nl);
  sub.join.assign(L.join.begin(), L.join.begin() + nl);
  sub.fork = L.fork;
  hipError_t e = enqueue_reset_states(pn, s0);
  if (e == hipSuccess) e = enqueue_init(pn, sub);
  if (e == hipSuccess) e = join_to0(sub);
  if (e != hipSuccess) {
    set_error("server init stage", e);
    plan_free(pn, s0);
    fail_admitted(s, ok, RPCA_ERR_DEVICE, s0);
    return RPCA_ERR_DEVICE;
  }
  plan_free(pn, s0);
  for (Req* r : ok) s->active.push_back(r);
  s->plan_valid = false;
  return RPCA_OK;
}

int step_device(rpca_server* s) {
  if (!s->lanes_ok) {
    const int rc = lanes_create(s->lanes, kServeLanes);
    if (rc != RPCA_OK) return rc;
    s->lanes_ok = true;
  }
  Lanes& L = s->lanes;
  hipStream_t s0 = L.s[0];

  // 1-2. timeouts of queued requests; admission, workspace and init pass of
  // the newly admitted solves
  expire_queued(s, now_ns(s));
  std::vector<Req*> fresh;
  admit(s, fresh);
  if (!fresh.empty()) {
    const int rc = start_admitted(s, fresh);
    if (rc != RPCA_OK) return rc;
  }
  if (s->active.empty()) return RPCA_OK;

  // 3. one quantum of iterations for every active solve
  if (!s->plan_valid) {
    plan_free(s->plan, s0);
    s->plan = Plan{};
    std::vector<SolveRec*> recs = recs_of(s->active);
    assign_lanes(recs, nlanes_for(recs.size()));
    const int rc = plan_build(s->plan, recs, nlanes_for(recs.size()), s->dtype, s0);
    if (rc != RPCA_OK) return rc;  // the active solves stay; the next step retries
    s->plan_valid = true;
  }
  const int rcp = lanes_reserve_pinned(L, static_cast<int>(s->active.size()));
  if (rcp != RPCA_OK) return rcp;
  {
    const int nl = static_cast<int>(s->plan.lanes.size());
    Lanes sub;
    sub.s.assign(L.s.begin(), L.s.begin() + nl);
    sub.join.assign(L.join.begin(), L.join.begin() + nl);
    sub.fork = L.fork;
    sub.pinned[0] = L.pinned[0];
    sub.pinned[1] = L.pinned[1];
    sub.snap[0] = L.snap[0];
    sub.snap[1] = L.snap[1];
    sub.pinned_count = L.pinned_count;
    SV(fork_from0(sub));
    SV(enqueue_iterations(s->plan, sub, s->quantum));
    SV(enqueue_snapshot(s->plan, sub, 0));
    SV(hipEventSynchronize(L.snap[0]));
  }
  for (size_t i = 0; i < s->active.size(); ++i) s->active[i]->rec.st = L.pinned[0][i];

  // 4. retire the solves that stopped, and drop those past their deadline
  const int64_t now = now_ns(s);
  std::vector<Req*> done, late, keep;
  for (Req* r : s->active) {
    if (r->rec.st.done) done.push_back(r);
    else if (expired(s, r, now)) late.push_back(r);
    else keep.push_back(r);
  }
  if (!late.empty()) {
    // every lane joined lane 0 in the snapshot, so their work on these
    // workspaces is ordered before the frees
    for (Req* r : late) {
      SV(hipFreeAsync(r->rec.mem, s0));
      r->rec.mem = nullptr;
      complete(s, r, RPCA_ERR_TIMEOUT, r->rec.st.iter, r->rec.st.resid);
      s->used -= r->footprint;
      delete r;
    }
    late.clear();
    s->plan_valid = false;
  }
  if (!done.empty()) {
    std::vector<SolveRec*> recs = recs_of(done);
    const int nl = nlanes_for(recs.size());
    assign_lanes(recs, nl);
    Plan pd;
    const int rc = plan_build(pd, recs, nl, s->dtype, s0);
    if (rc != RPCA_OK) {
      // keep them active (they exit their launches at once); retried next step
      plan_free(pd, s0);
      for (Req* r : done) keep.push_back(r);
      s->active.swap(keep);
      return rc;
    }
    Lanes sub;
    sub.s.assign(L.s.begin(), L.s.begin() + nl);
    sub.join.assign(L.join.begin(), L.join.begin() + nl);
    sub.fork = L.fork;
    SV(fork_from0(sub));
    SV(enqueue_finalize(pd, sub));
    SV(join_to0(sub));
    plan_free(pd, s0);
    for (Req* r : done) {
      SV(hipFreeAsync(r->rec.mem, s0));
      r->rec.mem = nullptr;
    }
    SV(hipStreamSynchronize(s0));  // L and S are complete before they are reported
    for (Req* r : done) {
      complete(s, r, r->rec.st.status, r->rec.st.iter, r->rec.st.resid);
      s->used -= r->footprint;
      delete r;
    }
    s->plan_valid = false;
  }
  s->active.swap(keep);
  return RPCA_OK;
}

#undef SV

}  // namespace
}  // namespace rpca

using namespace rpca;

extern "C" {

size_t rpca_server_request_bytes(int64_t m, int64_t n, int32_t dtype) {
  const size_t ws = rpca_footprint_bytes(m, n, dtype);
  return ws == 0 ? 0 : ws + io_bytes(m, n, dtype);
}

rpca_server* rpca_server_create(int32_t dtype, int32_t gram_mode, size_t hbm_budget,
                                int32_t max_active, int32_t quantum, int32_t flags, void* stream) {
  if (dtype != RPCA_F32 && dtype != RPCA_F64) return nullptr;
  if (gram_mode != RPCA_GRAM_DEFAULT && gram_mode != RPCA_GRAM_BF16X3 &&
      gram_mode != RPCA_GRAM_BF16X6)
    return nullptr;
  if (gram_mode != RPCA_GRAM_DEFAULT && dtype != RPCA_F32) return nullptr;
  if (hbm_budget == 0 || max_active < 1 || quantum < 1) return nullptr;
  if (flags & ~RPCA_SERVER_SIMULATE) return nullptr;
  rpca_server* s = new (std::nothrow) rpca_server();
  if (!s) return nullptr;
  s->dtype = dtype;
  s->gram_mode = gram_mode;
  s->budget = hbm_budget;
  s->max_active = max_active;
  s->quantum = quantum;
  s->simulate = (flags & RPCA_SERVER_SIMULATE) != 0;
  s->user = static_cast<hipStream_t>(stream);
  if (!s->simulate) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
      delete s;
      return nullptr;
    }
    setup_pool(dev);
  }
  return s;
}

int rpca_server_submit(rpca_server* s, const rpca_problem* p, int64_t tag) {
  if (!s || !p) return RPCA_ERR_ARG;
  Req* r = new (std::nothrow) Req();
  if (!r) return RPCA_ERR_NOMEM;
  r->p = *p;
  r->tag = tag;
  const int rc = make_rec(r->p, s->dtype, s->gram_mode, r->rec);
  if (rc != RPCA_OK) {
    delete r;
    return rc;
  }
  r->footprint = rpca_server_request_bytes(p->m, p->n, s->dtype);
  std::lock_guard<std::mutex> lk(s->mu);
  // a tag names one request until its completion has been reported
  bool dup = false;
  for (const Req* q : s->queue) dup = dup || q->tag == tag;
  for (const Req* q : s->active) dup = dup || q->tag == tag;
  for (const rpca_completion& c : s->ready) dup = dup || c.tag == tag;
  if (dup) {
    delete r;
    set_error_text("rpca_server_submit: tag already in use");
    return RPCA_ERR_ARG;
  }
  if (s->timeout_s > 0.0)
    r->deadline = now_ns(s) + static_cast<int64_t>(s->timeout_s * 1e9 + 0.5);
  s->queue.push_back(r);
  return RPCA_OK;
}

int rpca_server_set_timeout(rpca_server* s, double seconds) {
  if (!s || !(seconds >= 0.0) || seconds > 1e9) return RPCA_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  s->timeout_s = seconds;
  return RPCA_OK;
}

int rpca_server_inject_failure(rpca_server* s, int32_t stage, int32_t code) {
  if (!s || stage != RPCA_SERVER_STAGE_INIT || code >= 0) return RPCA_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  s->inject_init = code;
  return RPCA_OK;
}

int rpca_server_step(rpca_server* s, rpca_completion* out, int32_t capacity, int32_t* count) {
  if (!s || !count || capacity < 0 || (capacity > 0 && !out)) return RPCA_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *count = 0;
  if (s->broken) return RPCA_ERR_DEVICE;
  const int rc = s->simulate ? step_simulated(s) : step_device(s);
  if (rc == RPCA_ERR_DEVICE) s->broken = true;
  int k = 0;
  while (k < capacity && !s->ready.empty()) {
    out[k++] = s->ready.front();
    s->ready.pop_front();
  }
  *count = k;
  return rc;
}

int rpca_server_pending(rpca_server* s, int32_t* queued, int32_t* active, size_t* bytes_in_use) {
  if (!s) return RPCA_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = static_cast<int32_t>(s->queue.size());
  if (active) *active = static_cast<int32_t>(s->active.size());
  if (bytes_in_use) *bytes_in_use = s->used;
  return static_cast<int>(s->queue.size() + s->active.size() + s->ready.size());
}

size_t rpca_server_peak_bytes(rpca_server* s) {
  if (!s) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  return s->peak;
}

void rpca_server_destroy(rpca_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->simulate && s->lanes_ok) {
      for (auto st : s->lanes.s) (void)hipStreamSynchronize(st);
      plan_free(s->plan, s->lanes.s[0]);
      for (Req* r : s->active)
        if (r->rec.mem) (void)hipFreeAsync(r->rec.mem, s->lanes.s[0]);
      (void)hipStreamSynchronize(s->lanes.s[0]);
      lanes_destroy(s->lanes);
    }
    for (Req* r : s->active) delete r;
    for (Req* r : s->queue) delete r;
    s->active.clear();
    s->queue.clear();
  }
  delete s;
}

}  // extern "C"
