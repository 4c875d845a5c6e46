// rpca_solve_noalloc: one solve whose workspace lives in a fixed device array
// of the library instead of memory allocated per call, for callers that
// cannot allocate (see include/rpca.h).
//
// The array `scratch` below holds, for the solve of the call, everything the
// allocating entry points put in their stream-ordered allocations: the
// iterate buffers, partial sums, projector, eigenvectors and state (the
// solve's workspace, at the head of the array) and then the control block
// (descriptor, work items, group items, eigensolver id list, state gather).
// The kernels are those of rpca_solve_f32 / rpca_solve_f64, launched directly
// on the caller's stream in the same order and with the same per-solve
// reduction order, so the results are bitwise the same.
//
// In host code `scratch` names a host-side stand-in of the array, not its
// device address.  The address is asked for once per device, with that
// device current, through hipGetSymbolAddress and kept per device; only that
// address is used afterwards (descriptors, uploads).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "rpca.h"
#include "common.h"
#include "engine.h"
#include "launch.h"

namespace rpca {
namespace {

static __device__ __align__(256) unsigned char scratch[RPCA_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
constexpr int kChunkFirst = 8;   // iterations between state reads, doubling ...
constexpr int kChunkMax = 32;    // ... up to this

std::mutex g_dev_mu[kMaxDevices];   // one call at a time per device
std::mutex g_addr_mu;
char* g_addr[kMaxDevices] = {};     // device address of `scratch`, per device

size_t al256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Device address of this device's copy of `scratch` (set-up on first use).
char* scratch_address(int dev) {
  std::lock_guard<std::mutex> lk(g_addr_mu);
  if (g_addr[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      set_error("hipGetSymbolAddress(scratch)", e);
      (void)hipGetLastError();
      return nullptr;
    }
    g_addr[dev] = static_cast<char*>(ptr);
  }
  return g_addr[dev];
}

// Read the solve's state: gather kernel into the control block, copy to the
// host, wait for the stream.
hipError_t read_state(const Plan& plan, hipStream_t s, SolveState& out) {
  hipError_t e = launch_gather_states(1, s, plan.descs, plan.gathered);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&out, plan.gathered, sizeof(SolveState), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) set_error("state read-back", e);
  return e;
}

int solve_noalloc(const rpca_problem& p, int dtype, hipStream_t stream, int32_t* iterations) {
  set_error_text("");
  SolveRec rec;
  const int vrc = make_rec(p, dtype, RPCA_GRAM_DEFAULT, rec);
  if (vrc != RPCA_OK) return vrc;

  // Lay out the workspace and the control block in the array; reject what
  // does not fit before any device call.
  Plan plan;
  std::vector<SolveRec*> recs{&rec};
  rec.lane = 0;
  rec.mem = nullptr;  // the descriptors are written once the address is known
  const size_t ws = al256(rec.big.total);
  const size_t ctrl_bytes = plan_prepare(plan, recs, 1, dtype);
  if (ws + ctrl_bytes > static_cast<size_t>(RPCA_NOALLOC_MAX_BYTES)) {
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "rpca_solve_noalloc: the solve needs %zu bytes of workspace, more than the "
                  "%zu bytes of the static scratch (RPCA_NOALLOC_MAX_BYTES)",
                  ws + ctrl_bytes, static_cast<size_t>(RPCA_NOALLOC_MAX_BYTES));
    set_error_text(msg);
    return RPCA_ERR_ARG;
  }

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error("hipGetDevice", e);
    return RPCA_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_dev_mu[dev]);
  char* base = scratch_address(dev);
  if (base == nullptr) return RPCA_ERR_DEVICE;

  rec.mem = base;
  plan = Plan{};
  (void)plan_prepare(plan, recs, 1, dtype);
  Lanes L;
  L.s.assign(1, stream);
  L.join.assign(1, nullptr);

  int rc = RPCA_OK;
  SolveState st{};
#define NA(expr)                \
  do {                          \
    const hipError_t e_ = (expr); \
    if (e_ != hipSuccess) {     \
      set_error(#expr, e_);     \
      rc = RPCA_ERR_DEVICE;     \
      goto done;                \
    }                           \
  } while (0)
  {
    // the caller's stream orders the previous call's work (and the inputs)
    // before this one's use of the array
    rc = plan_upload(plan, base + ws, stream);
    if (rc != RPCA_OK) goto done;
    NA(enqueue_reset_states(plan, stream));
    NA(enqueue_init(plan, L));
    int launched = 0, chunk = kChunkFirst;
    for (;;) {
      // a solve that stops after k passes needs k + 1 eigensolve launches
      // (the last one records the stop); at most maxit + 1
      const int c = std::min(chunk, rec.maxit + 1 - launched);
      if (c <= 0) {
        set_error_text("rpca_solve_noalloc: the solve did not stop after maxit + 1 launches");
        rc = RPCA_ERR_DEVICE;
        goto done;
      }
      NA(enqueue_iterations(plan, L, c));
      launched += c;
      NA(read_state(plan, stream, st));
      if (st.done) break;
      chunk = std::min(chunk * 2, kChunkMax);
    }
    NA(enqueue_finalize(plan, L));
    NA(read_state(plan, stream, st));
    rc = st.status;
    if (iterations) *iterations = rc >= 0 ? st.iter : 0;
  }
#undef NA
done:
  if (rc == RPCA_ERR_DEVICE) (void)hipGetLastError();
  // nothing may still read the host copy of the control block
  (void)hipStreamSynchronize(stream);
  return rc;
}

}  // namespace
}  // namespace rpca

extern "C" int rpca_solve_noalloc(const void* M, int64_t m, int64_t n, int32_t dtype,
                                  double lambda, double mu, double tol, int32_t maxit, void* L,
                                  void* S, int32_t* iterations, void* stream) {
  if (iterations) *iterations = 0;
  if (dtype != RPCA_F32 && dtype != RPCA_F64) return RPCA_ERR_ARG;
  rpca_problem p;
  std::memset(&p, 0, sizeof(p));
  p.M = M;
  p.m = m;
  p.n = n;
  p.lambda = lambda;
  p.mu = mu;
  p.tol = tol;
  p.maxit = maxit;
  p.L = L;
  p.S = S;
  return rpca::solve_noalloc(p, dtype, static_cast<hipStream_t>(stream), iterations);
}
