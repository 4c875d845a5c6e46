// Host runtime of librpca_mi355x: the C ABI declared in include/rpca.h.
//
// A call (one solve or a batch) is laid out as follows:
//   * one stream-ordered device allocation holds the control block (solve
//     descriptors, the work-item and group tables, solve states) and
//     every solve's iterate buffers, reduction partials, Gram, projector and
//     eigenvectors;
//   * the init pass runs once per frame class, then iterations are enqueued
//     in chunks of [eigensolve per eigensolver class, update pass per frame
//     class, group reduction];
//     a solve that has finished makes its later launches exit at once, so the
//     host only reads the solve states back between chunks;
//   * the finalize pass writes L and S, the states are read back, and the
//     allocation is returned to the pool.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "rpca.h"
#include "common.h"
#include "launch.h"

using namespace rpca;

namespace {

constexpr int kChunkFirst = 8;
constexpr int kChunkMax = 64;

int nb_class(int64_t n, int dtype) {
  if (dtype == RPCA_F32) {
    for (int c : kClassesF32)
      if (n <= c) return c;
  } else {
    for (int c : kClassesF64)
      if (n <= c) return c;
  }
  return 0;
}

struct Geo {
  int nb = 0, tiles = 0, tps = 1, slots = 0, groups = 0, pstride = 0;
  size_t es = 0;
};

// Tiles per workgroup: one.  Each workgroup then holds its Gram accumulators
// only for its own tile (fewer live registers, more resident workgroups), and
// the hardware overlaps one workgroup's loads with another's arithmetic.  The
// partial-slot layout depends only on the solve's own shape, so a solve
// reduces in the same order alone and inside any batch.
int tiles_per_slot(int) { return 1; }

bool geometry(int64_t m, int64_t n, int dtype, Geo& g) {
  if (m < 1 || n < 1 || n > RPCA_N_MAX) return false;
  g.nb = nb_class(n, dtype);
  if (g.nb == 0 || n > kEigMaxN) return false;
  if (m >= (int64_t(1) << 30)) return false;  // row offsets are 32-bit byte offsets
  const int64_t tiles = (m + kTile - 1) / kTile;
  g.tiles = static_cast<int>(tiles);
  g.tps = tiles_per_slot(g.tiles);
  g.slots = (g.tiles + g.tps - 1) / g.tps;
  g.groups = (g.slots + kGroup - 1) / kGroup;
  g.pstride = pstride_for(g.nb);
  g.es = dtype == RPCA_F32 ? 4 : 8;
  return true;
}

size_t al256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct Big {
  size_t S0, S1, Y0, Y1, part, gpart, P, V, trace, total;
};

Big big_layout(int64_t m, int64_t n, const Geo& g) {
  Big b{};
  size_t o = 0;
  const size_t mat = al256(static_cast<size_t>(m) * static_cast<size_t>(n) * g.es);
  b.S0 = o; o += mat;
  b.S1 = o; o += mat;
  b.Y0 = o; o += mat;
  b.Y1 = o; o += mat;
  b.part = o; o += al256(static_cast<size_t>(g.slots) * g.pstride * sizeof(double));
  b.gpart = o; o += al256(static_cast<size_t>(g.groups) * g.pstride * sizeof(double));
  b.P = o; o += al256(static_cast<size_t>(g.nb) * g.nb * g.es);
  b.V = o; o += al256(static_cast<size_t>(g.nb) * g.nb * sizeof(double));
  b.trace = o;
#ifdef RPCA_TRACE
  o += al256(static_cast<size_t>(g.slots) * 4 * sizeof(int64_t));
#endif
  b.total = o;
  return b;
}

bool overlap(const void* a, const void* b, size_t bytes) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + bytes && y < x + bytes;
}

// ---------------------------------------------------------------- profiling
struct Profile {
  std::mutex mu;
  bool on = false;
  double init_ms = 0, eig_ms = 0, update_ms = 0, finalize_ms = 0;
  int64_t eig_launches = 0, update_launches = 0, solves = 0, iterations = 0;
  double update_bytes = 0;
};
Profile g_prof;

struct EvPair {
  hipEvent_t a = nullptr, b = nullptr;
  int kind = 0;        // 0 init, 1 eig, 2 update, 3 finalize
  int iter = 0;        // eig/update: 1-based launch index
  int cls = -1;        // update: class index
};

// ------------------------------------------------------------- device pool
std::once_flag g_pool_once[64];
void setup_pool(int dev) {
  if (dev < 0 || dev >= 64) return;
  std::call_once(g_pool_once[dev], [dev] {
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  });
}

struct ClassRun {
  int nb;
  int item_off, item_cnt;
  std::vector<int> solves;
};

#ifdef RPCA_TRACE
// Trace builds: per-phase eigensolve times and the workgroup timeline of the
// last update pass of the first solve, printed to stderr (10 ns ticks).
void trace_report(const SolveState& st, const void* dtrace, int slots, hipStream_t stream) {
  std::vector<int64_t> t(static_cast<size_t>(slots) * 4);
  if (hipMemcpyAsync(t.data(), dtrace, t.size() * sizeof(int64_t), hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return;
  const double it = st.iter > 0 ? st.iter : 1;
  std::fprintf(stderr,
               "[trace] eig us/iter: reduce+control %.2f warm %.2f jacobi %.2f project %.2f "
               "(sweeps/iter %.2f)\n",
               st.trace[0] * 0.01 / it, st.trace[1] * 0.01 / it, st.trace[2] * 0.01 / it,
               st.trace[3] * 0.01 / it, st.sweeps_total / it);
  int64_t b0 = INT64_MAX, b1 = 0, e1 = 0, e2 = 0;
  double sum_tiles = 0;
  for (int s = 0; s < slots; ++s) {
    b0 = std::min(b0, t[s * 4 + 0]);
    b1 = std::max(b1, t[s * 4 + 0]);
    e1 = std::max(e1, t[s * 4 + 1]);
    e2 = std::max(e2, t[s * 4 + 2]);
    sum_tiles += static_cast<double>(t[s * 4 + 1] - t[s * 4 + 0]);
  }
  std::fprintf(stderr,
               "[trace] update us: last WG start %.2f, tiles done %.2f, partials %.2f; "
               "mean WG tile time %.2f\n",
               (b1 - b0) * 0.01, (e1 - b0) * 0.01, (e2 - b0) * 0.01, sum_tiles / slots * 0.01);
}
#endif

thread_local char g_last_error[512] = "";

void set_error(const char* what, hipError_t e) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", what, hipGetErrorString(e),
                static_cast<int>(e));
}

#define CK(expr)                          \
  do {                                    \
    hipError_t e_ = (expr);               \
    if (e_ != hipSuccess) {               \
      set_error(#expr, e_);               \
      rc = RPCA_ERR_DEVICE;               \
      goto done;                          \
    }                                     \
  } while (0)

int run_batch(rpca_problem* probs, int count, int dtype, int gram_mode, hipStream_t stream) {
  g_last_error[0] = '\0';
  if (count < 1 || probs == nullptr) return RPCA_ERR_ARG;
  if (dtype != RPCA_F32 && dtype != RPCA_F64) return RPCA_ERR_ARG;
  if (gram_mode != RPCA_GRAM_DEFAULT && gram_mode != RPCA_GRAM_BF16X3) return RPCA_ERR_ARG;
  if (gram_mode == RPCA_GRAM_BF16X3) return RPCA_ERR_UNSUPPORTED;

  std::vector<Geo> geo(count);
  std::vector<Big> big(count);
  for (int i = 0; i < count; ++i) {
    rpca_problem& p = probs[i];
    if (!p.M || !p.L || !p.S || p.m < 1 || p.n < 1 || p.n > RPCA_N_MAX || p.maxit < 1)
      return RPCA_ERR_ARG;
    if (!std::isfinite(p.lambda) || !std::isfinite(p.mu) || std::isnan(p.tol)) return RPCA_ERR_ARG;
    const size_t bytes = static_cast<size_t>(p.m) * static_cast<size_t>(p.n) * (dtype == RPCA_F32 ? 4 : 8);
    if (overlap(p.M, p.L, bytes) || overlap(p.M, p.S, bytes) || overlap(p.L, p.S, bytes))
      return RPCA_ERR_ARG;
    if (!geometry(p.m, p.n, dtype, geo[i])) return RPCA_ERR_UNSUPPORTED;
    big[i] = big_layout(p.m, p.n, geo[i]);
  }

  // Frame classes and the work-item table.
  std::vector<ClassRun> classes;
  for (int i = 0; i < count; ++i) {
    auto it = std::find_if(classes.begin(), classes.end(),
                           [&](const ClassRun& c) { return c.nb == geo[i].nb; });
    if (it == classes.end()) {
      classes.push_back(ClassRun{geo[i].nb, 0, 0, {}});
      it = classes.end() - 1;
    }
    it->solves.push_back(i);
  }
  std::vector<WorkItem> items;
  for (auto& c : classes) {
    c.item_off = static_cast<int>(items.size());
    for (int s : c.solves)
      for (int q = 0; q < geo[s].slots; ++q) items.push_back(WorkItem{s, q});
    c.item_cnt = static_cast<int>(items.size()) - c.item_off;
  }

  // Eigensolver classes and their solve-id lists.
  std::vector<int32_t> eig_ids;
  std::vector<std::pair<int, std::pair<int, int>>> eig_runs;  // (class, (offset, count))
  for (int cls : {16, 32, 64}) {
    const int off = static_cast<int>(eig_ids.size());
    for (int i = 0; i < count; ++i)
      if (eig_class(static_cast<int>(probs[i].n)) == cls) eig_ids.push_back(i);
    const int cnt = static_cast<int>(eig_ids.size()) - off;
    if (cnt > 0) eig_runs.push_back({cls, {off, cnt}});
  }

  // Group items of the reduction launch.
  std::vector<GroupItem> gitems;
  for (int i = 0; i < count; ++i)
    for (int g = 0; g < geo[i].groups; ++g) gitems.push_back(GroupItem{i, g});

  // Control block: descs | items | group items | eig ids | states.
  const size_t off_desc = 0;
  const size_t off_items = al256(off_desc + sizeof(SolveDesc) * count);
  const size_t off_gitems = al256(off_items + sizeof(WorkItem) * items.size());
  const size_t off_ids = al256(off_gitems + sizeof(GroupItem) * gitems.size());
  const size_t off_state = al256(off_ids + sizeof(int32_t) * eig_ids.size());
  const size_t ctrl_bytes = al256(off_state + sizeof(SolveState) * count);
  size_t total = ctrl_bytes;
  std::vector<size_t> base(count);
  for (int i = 0; i < count; ++i) {
    base[i] = total;
    total += big[i].total;
  }

  int dev = 0;
  (void)hipGetLastError();  // launches below report through the per-thread last error
  {
    const hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) {
      set_error("hipGetDevice", ge);
      return RPCA_ERR_DEVICE;
    }
  }
  setup_pool(dev);

  int rc = RPCA_OK;
  char* arena = nullptr;
  std::vector<unsigned char> ctrl_h(ctrl_bytes, 0);
  SolveState* st_h = nullptr;
  std::vector<EvPair> evs;
  bool prof = false;
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    prof = g_prof.on;
  }

  {
    hipError_t ae = hipMallocAsync(reinterpret_cast<void**>(&arena), total, stream);
    if (ae != hipSuccess || arena == nullptr) {
      set_error("hipMallocAsync(workspace)", ae);
      (void)hipGetLastError();
      return RPCA_ERR_NOMEM;
    }
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&st_h), sizeof(SolveState) * count) != hipSuccess) {
    (void)hipFreeAsync(arena, stream);
    return RPCA_ERR_NOMEM;
  }

  {
    SolveDesc* dh = reinterpret_cast<SolveDesc*>(ctrl_h.data() + off_desc);
    SolveState* sd = reinterpret_cast<SolveState*>(arena + off_state);
    for (int i = 0; i < count; ++i) {
      const rpca_problem& p = probs[i];
      char* b = arena + base[i];
      SolveDesc& d = dh[i];
      std::memset(&d, 0, sizeof(d));
      d.X = p.M;
      d.S[0] = b + big[i].S0;
      d.S[1] = b + big[i].S1;
      d.Y[0] = b + big[i].Y0;
      d.Y[1] = b + big[i].Y1;
      d.Lout = p.L;
      d.Sout = p.S;
      d.partials = reinterpret_cast<double*>(b + big[i].part);
      d.gpartials = reinterpret_cast<double*>(b + big[i].gpart);
      d.P = b + big[i].P;
      d.V = reinterpret_cast<double*>(b + big[i].V);
      d.st = sd + i;
#ifdef RPCA_TRACE
      d.wgtrace = reinterpret_cast<int64_t*>(b + big[i].trace);
#endif
      d.m = p.m;
      d.n = static_cast<int32_t>(p.n);
      d.nb = geo[i].nb;
      d.tiles = geo[i].tiles;
      d.tps = geo[i].tps;
      d.slots = geo[i].slots;
      d.groups = geo[i].groups;
      d.pstride = geo[i].pstride;
      d.maxit = p.maxit;
      d.lam_in = p.lambda;
      d.mu_in = p.mu;
      d.tol = p.tol;
    }
    std::memcpy(ctrl_h.data() + off_items, items.data(), sizeof(WorkItem) * items.size());
    std::memcpy(ctrl_h.data() + off_gitems, gitems.data(), sizeof(GroupItem) * gitems.size());
    std::memcpy(ctrl_h.data() + off_ids, eig_ids.data(), sizeof(int32_t) * eig_ids.size());
    // states start at zero (ctrl_h is zero-filled)
  }

  {
    const SolveDesc* descs = reinterpret_cast<const SolveDesc*>(arena + off_desc);
    const WorkItem* items_d = reinterpret_cast<const WorkItem*>(arena + off_items);
    const int32_t* ids_d = reinterpret_cast<const int32_t*>(arena + off_ids);
    const GroupItem* gitems_d = reinterpret_cast<const GroupItem*>(arena + off_gitems);
    const int ngroups = static_cast<int>(gitems.size());
    auto launch_class = [&](const ClassRun& c, int mode) -> hipError_t {
      if (dtype == RPCA_F32)
        return launch_stream_f32(c.nb, mode, c.item_cnt, stream, descs, items_d + c.item_off);
      return launch_stream_f64(c.nb, mode, c.item_cnt, stream, descs, items_d + c.item_off);
    };
    auto ev_begin = [&](int kind, int iter, int cls) {
      if (!prof) return;
      EvPair e;
      e.kind = kind;
      e.iter = iter;
      e.cls = cls;
      (void)hipEventCreate(&e.a);
      (void)hipEventCreate(&e.b);
      (void)hipEventRecord(e.a, stream);
      evs.push_back(e);
    };
    auto ev_end = [&]() {
      if (prof) (void)hipEventRecord(evs.back().b, stream);
    };

    CK(hipMemcpyAsync(arena, ctrl_h.data(), ctrl_bytes, hipMemcpyHostToDevice, stream));
    for (size_t c = 0; c < classes.size(); ++c) {
      ev_begin(0, 0, static_cast<int>(c));
      CK(launch_class(classes[c], kModeInit));
      ev_end();
    }
    CK(launch_reduce(ngroups, stream, descs, gitems_d));

    int maxit_all = 0;
    for (int i = 0; i < count; ++i) maxit_all = std::max(maxit_all, probs[i].maxit);
    int launched = 0;
    int chunk = kChunkFirst;
    bool all_done = false;
    while (!all_done) {
      for (int c = 0; c < chunk; ++c) {
        ++launched;
        for (const auto& er : eig_runs) {
          ev_begin(1, launched, -1);
          CK(launch_eig(dtype == RPCA_F32 ? 1 : 0, er.first, er.second.second, stream, descs,
                        ids_d + er.second.first));
          ev_end();
        }
        for (size_t q = 0; q < classes.size(); ++q) {
          ev_begin(2, launched, static_cast<int>(q));
          CK(launch_class(classes[q], kModeUpdate));
          ev_end();
        }
        CK(launch_reduce(ngroups, stream, descs, gitems_d));
      }
      CK(hipMemcpyAsync(st_h, arena + off_state, sizeof(SolveState) * count,
                        hipMemcpyDeviceToHost, stream));
      CK(hipStreamSynchronize(stream));
      all_done = true;
      for (int i = 0; i < count; ++i) all_done = all_done && st_h[i].done != 0;
      if (!all_done && launched > maxit_all + 1) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "a solve did not stop after %d eigensolve launches (cap %d)", launched,
                      maxit_all);
        rc = RPCA_ERR_DEVICE;  // the device failed to stop a solve by its cap
        goto done;
      }
      chunk = std::min(chunk * 2, kChunkMax);
    }
    for (size_t c = 0; c < classes.size(); ++c) {
      ev_begin(3, 0, static_cast<int>(c));
      CK(launch_class(classes[c], kModeFinalize));
      ev_end();
    }
    CK(hipMemcpyAsync(st_h, arena + off_state, sizeof(SolveState) * count,
                      hipMemcpyDeviceToHost, stream));
    CK(hipStreamSynchronize(stream));

    int worst_neg = 0, any_nc = 0;
    for (int i = 0; i < count; ++i) {
      probs[i].iterations = st_h[i].iter;
      probs[i].status = st_h[i].status;
      probs[i].residual = st_h[i].resid;
      if (st_h[i].status < 0) worst_neg = std::min(worst_neg, st_h[i].status);
      if (st_h[i].status == RPCA_NOT_CONVERGED) any_nc = 1;
    }
    rc = worst_neg < 0 ? worst_neg : (any_nc ? RPCA_NOT_CONVERGED : RPCA_OK);
#ifdef RPCA_TRACE
    trace_report(st_h[0], arena + base[0] + big[0].trace, geo[0].slots, stream);
#endif

    if (prof) {
      double init_ms = 0, eig_ms = 0, upd_ms = 0, fin_ms = 0, upd_bytes = 0;
      int64_t eig_n = 0, upd_n = 0, iters = 0;
      int max_iter = 0;
      for (int i = 0; i < count; ++i) {
        max_iter = std::max(max_iter, st_h[i].iter);
        iters += st_h[i].iter;
      }
      for (auto& e : evs) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e.a, e.b);
        if (e.kind == 0) init_ms += ms;
        else if (e.kind == 3) fin_ms += ms;
        else if (e.kind == 1) {
          if (e.iter <= max_iter) { eig_ms += ms; ++eig_n; }
        } else {
          double bytes = 0;
          for (int s : classes[e.cls].solves) {
            if (st_h[s].iter >= e.iter) {
              const double words = e.iter == 1 ? 3.0 : 5.0;
              bytes += words * static_cast<double>(probs[s].m) * static_cast<double>(probs[s].n) *
                       static_cast<double>(geo[s].es);
            }
          }
          if (bytes > 0) { upd_ms += ms; ++upd_n; upd_bytes += bytes; }
        }
      }
      std::lock_guard<std::mutex> lk(g_prof.mu);
      g_prof.init_ms += init_ms;
      g_prof.eig_ms += eig_ms;
      g_prof.update_ms += upd_ms;
      g_prof.finalize_ms += fin_ms;
      g_prof.eig_launches += eig_n;
      g_prof.update_launches += upd_n;
      g_prof.update_bytes += upd_bytes;
      g_prof.solves += count;
      g_prof.iterations += iters;
    }
  }

done:
  for (auto& e : evs) {
    if (e.a) (void)hipEventDestroy(e.a);
    if (e.b) (void)hipEventDestroy(e.b);
  }
  if (rc == RPCA_ERR_DEVICE) (void)hipGetLastError();
  (void)hipFreeAsync(arena, stream);
  (void)hipStreamSynchronize(stream);
  (void)hipHostFree(st_h);
  return rc;
}

}  // namespace

extern "C" {

int rpca_solve_many(rpca_problem* probs, int32_t count, int32_t dtype, int32_t gram_mode,
                    void* stream) {
  return run_batch(probs, count, dtype, gram_mode, static_cast<hipStream_t>(stream));
}

int rpca_solve_ex(rpca_problem* prob, int32_t dtype, int32_t gram_mode, void* stream) {
  return run_batch(prob, 1, dtype, gram_mode, static_cast<hipStream_t>(stream));
}

static int solve_one(const void* M, int64_t m, int64_t n, double lambda, double mu, double tol,
                     int32_t maxit, void* L, void* S, int32_t* iterations, void* stream,
                     int dtype) {
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
  const int rc = run_batch(&p, 1, dtype, RPCA_GRAM_DEFAULT, static_cast<hipStream_t>(stream));
  if (iterations) *iterations = rc >= 0 ? p.iterations : 0;
  return rc;
}

int rpca_solve_f64(const double* M, int64_t m, int64_t n, double lambda, double mu, double tol,
                   int32_t maxit, double* L, double* S, int32_t* iterations, void* stream) {
  return solve_one(M, m, n, lambda, mu, tol, maxit, L, S, iterations, stream, RPCA_F64);
}

int rpca_solve_f32(const float* M, int64_t m, int64_t n, double lambda, double mu, double tol,
                   int32_t maxit, float* L, float* S, int32_t* iterations, void* stream) {
  return solve_one(M, m, n, lambda, mu, tol, maxit, L, S, iterations, stream, RPCA_F32);
}

size_t rpca_footprint_bytes(int64_t m, int64_t n, int32_t dtype) {
  if (dtype != RPCA_F32 && dtype != RPCA_F64) return 0;
  Geo g;
  if (!geometry(m, n, dtype, g)) return 0;
  const Big b = big_layout(m, n, g);
  return b.total + al256(sizeof(SolveDesc)) + al256(sizeof(SolveState)) +
         al256(sizeof(GroupItem) * g.groups) + al256(sizeof(WorkItem) * g.slots) + 256;
}

const char* rpca_strerror(int code) {
  switch (code) {
    case RPCA_OK: return "converged";
    case RPCA_NOT_CONVERGED: return "iteration cap reached before the stopping test held";
    case RPCA_ERR_ARG: return "invalid argument";
    case RPCA_ERR_NOMEM: return "device memory allocation failed";
    case RPCA_ERR_DEVICE: return "HIP runtime error";
    case RPCA_ERR_NONFINITE: return "non-finite value in the input or the iteration";
    case RPCA_ERR_UNSUPPORTED: return "shape not supported by this build";
    default: return "unknown status";
  }
}

const char* rpca_version(void) { return "rpca_mi355x 0.1"; }

const char* rpca_last_error(void) { return g_last_error; }

void rpca_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = on != 0;
}

int rpca_profile_read(rpca_profile* out, int reset) {
  if (!out) return RPCA_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  out->init_ms = g_prof.init_ms;
  out->eig_ms = g_prof.eig_ms;
  out->update_ms = g_prof.update_ms;
  out->finalize_ms = g_prof.finalize_ms;
  out->eig_launches = g_prof.eig_launches;
  out->update_launches = g_prof.update_launches;
  out->update_bytes = g_prof.update_bytes;
  out->solves = g_prof.solves;
  out->iterations = g_prof.iterations;
  if (reset) {
    g_prof.init_ms = g_prof.eig_ms = g_prof.update_ms = g_prof.finalize_ms = 0;
    g_prof.eig_launches = g_prof.update_launches = g_prof.solves = g_prof.iterations = 0;
    g_prof.update_bytes = 0;
  }
  return RPCA_OK;
}

}  // extern "C"
