// Host runtime of librpca_mi355x: the engine (plans, lanes, enqueue
// helpers) and the solve entry points of the C ABI (include/rpca.h).
//
// A call of rpca_solve_many:
//   * validates every problem and gives each its own device memory (one
//     stream-ordered allocation for the call);
//   * assigns the problems to lanes (streams) balancing their matrix sizes,
//     and builds one plan: solve descriptors, the streaming work items per
//     frame class, the group-reduction items and the eigensolver id lists;
//   * runs the init pass, then chunks of iterations.  A chunk is captured
//     once as a graph (all lanes, forked from and joined into lane 0) and
//     replayed; after each replay one small kernel gathers the solve states
//     and they are copied to pinned host memory.  The next chunk is enqueued
//     before the previous snapshot is inspected, so the host round trip
//     overlaps device work; a solve that has finished makes its later
//     launches exit at once;
//   * runs the finalize pass, reads the states back and frees the memory.
// With kernel timing enabled everything runs on one lane, launched directly
// (no graph) with HIP events around every launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "rpca.h"
#include "common.h"
#include "engine.h"
#include "launch.h"

namespace rpca {

thread_local LaunchEvents t_launch_events;

namespace {

constexpr int kGraphChunk = 16;
constexpr int kDirectChunkFirst = 8;
constexpr int kDirectChunkMax = 64;

size_t al256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

thread_local char g_last_error[512] = "";

// ---------------------------------------------------------------- profiling
struct EvPair {
  hipEvent_t a = nullptr, b = nullptr;
  int kind = 0;   // 0 init, 1 eig, 2 update, 3 finalize
  int iter = 0;   // eig/update: 1-based iteration of the launch
  int lane = 0;
  int cls = -1;   // update: index into the lane's classes
};

struct Profile {
  std::mutex mu;
  bool on = false;
  double init_ms = 0, eig_ms = 0, update_ms = 0, finalize_ms = 0;
  int64_t eig_launches = 0, update_launches = 0, solves = 0, iterations = 0;
  double update_bytes = 0;
};
Profile g_prof;

bool profiling_on() {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  return g_prof.on;
}

thread_local std::vector<EvPair>* t_evs = nullptr;  // set while a profiled run enqueues

void ev_begin(hipStream_t s, int kind, int iter, int lane, int cls) {
  if (!t_evs) return;
  EvPair e;
  e.kind = kind;
  e.iter = iter;
  e.lane = lane;
  e.cls = cls;
  (void)s;
  // timing-only events: no system-scope fence (the run synchronises its
  // stream before the pairs are read), so no cache writeback is timed
  (void)hipEventCreateWithFlags(&e.a, hipEventDisableSystemFence);
  (void)hipEventCreateWithFlags(&e.b, hipEventDisableSystemFence);
  t_evs->push_back(e);
  t_launch_events.start = e.a;  // the next launch times itself into the pair
  t_launch_events.stop = e.b;
}
void ev_end(hipStream_t s) {
  (void)s;
  t_launch_events = LaunchEvents{};
}

}  // namespace

// ------------------------------------------------------------- device pool
namespace {
std::once_flag g_pool_once[64];
}  // namespace

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

bool graphs_disabled() {
  const char* v = std::getenv("RPCA_NO_GRAPH");
  return v && v[0] && v[0] != '0';
}

namespace {

bool overlap(const void* a, const void* b, size_t bytes) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + bytes && y < x + bytes;
}

// `key` is a class key (class_key): frame class, kernel kind and precision.
hipError_t launch_stream(int dtype, int key, int mode, int grid, hipStream_t s, const SolveDesc* d,
                         const WorkItem* it) {
  const int nb = key & 0xff, kind = (key >> 8) & 1, prec = (key >> 9) & 3;
  const bool mt = ((key >> 11) & 1) != 0;
  if (kind == 1)
    return dtype == RPCA_F32 ? launch_wide_f32(nb, mode, prec, grid, s, d, it)
                             : launch_wide_f64(nb, mode, grid, s, d, it);
  return dtype == RPCA_F32 ? launch_stream_f32(nb, mode, mt, grid, s, d, it)
                           : launch_stream_f64(nb, mode, mt, grid, s, d, it);
}

#ifdef RPCA_TRACE
// Trace builds: per-phase eigensolve times and the workgroup timeline of the
// last update pass of the first solve, printed to stderr (10 ns ticks).
void trace_report(const SolveRec& r, hipStream_t stream) {
  std::vector<int64_t> t(static_cast<size_t>(r.geo.slots) * 4);
  if (hipMemcpyAsync(t.data(), r.mem + r.big.trace, t.size() * sizeof(int64_t),
                     hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return;
  const SolveState& st = r.st;
  const double it = st.iter > 0 ? st.iter : 1;
  std::fprintf(stderr,
               "[trace] eig us/iter: reduce+control %.2f warm %.2f jacobi %.2f project %.2f "
               "(sweeps/iter %.2f)\n",
               st.trace[0] * 0.01 / it, st.trace[1] * 0.01 / it, st.trace[2] * 0.01 / it,
               st.trace[3] * 0.01 / it, st.sweeps_total / it);
  int64_t b0 = INT64_MAX, b1 = 0, e1 = 0, e2 = 0;
  double sum_tiles = 0;
  for (int s = 0; s < r.geo.slots; ++s) {
    b0 = std::min(b0, t[s * 4 + 0]);
    b1 = std::max(b1, t[s * 4 + 0]);
    e1 = std::max(e1, t[s * 4 + 1]);
    e2 = std::max(e2, t[s * 4 + 2]);
    sum_tiles += static_cast<double>(t[s * 4 + 1] - t[s * 4 + 0]);
  }
  std::fprintf(stderr,
               "[trace] update us: last WG start %.2f, tiles done %.2f, partials %.2f; "
               "mean WG tile time %.2f\n",
               (b1 - b0) * 0.01, (e1 - b0) * 0.01, (e2 - b0) * 0.01, sum_tiles / r.geo.slots * 0.01);
}
#endif

}  // namespace

// ------------------------------------------------------------------ errors
void set_error(const char* what, hipError_t e) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", what, hipGetErrorString(e),
                static_cast<int>(e));
}
void set_error_text(const char* text) { std::snprintf(g_last_error, sizeof(g_last_error), "%s", text); }

// ---------------------------------------------------------------- geometry
namespace {
// Streaming kernel per FP32 register frame class (index: class value 0..64):
// 0 = register kernel, 1 = MFMA tile kernel.  Classes above 64 frames and the
// split-BF16 mode always use the MFMA tile kernel.  Defaults from timing on
// MI355X: the register kernel up to 32 frames, the tile kernel from 40 (at
// 60 frames the register kernel's FMA chains and partial reductions leave it
// at 2 TB/s against 3.2 TB/s for the tile kernel).
std::atomic<int> g_stream_kernel[kEigMaxN + 1];
struct StreamKernelDefaults {
  StreamKernelDefaults() {
    for (int c = 0; c <= kEigMaxN; ++c) g_stream_kernel[c].store(c >= 40 ? 1 : 0);
  }
} g_stream_kernel_defaults;
}  // namespace

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

// Rows per workgroup of the tile kernel, per tile class nb = 16 (i + 1).
std::atomic<int> g_tile_rows[kEigHugeMaxN / 16];
std::once_flag g_tile_rows_once;
void init_tile_rows() {
  std::call_once(g_tile_rows_once, [] {
    for (int i = 0; i < kEigHugeMaxN / 16; ++i) g_tile_rows[i].store(1024);
  });
}

int tile_rows(int nb) {
  if (nb < 16 || nb > kEigHugeMaxN || nb % 16 != 0) return -1;
  init_tile_rows();
  return g_tile_rows[nb / 16 - 1].load(std::memory_order_relaxed);
}

bool set_tile_rows(int nb, int rows) {
  if (tile_rows(nb) < 0) return false;
  if (rows < kWideRows || rows > 8192 || rows % kWideRows != 0) return false;
  g_tile_rows[nb / 16 - 1].store(rows, std::memory_order_relaxed);
  return true;
}

int stream_kernel_choice(int cls) {
  if (cls < 0 || cls > kEigMaxN) return -1;
  for (int c : kClassesF32)
    if (c == cls) return g_stream_kernel[cls].load(std::memory_order_relaxed);
  return -1;
}

bool set_stream_kernel_choice(int cls, int v) {
  if (stream_kernel_choice(cls) < 0 || (v != 0 && v != 1)) return false;
  g_stream_kernel[cls].store(v, std::memory_order_relaxed);
  return true;
}

// Tiles each workgroup of the register kernel walks, per dtype and register
// class (index: class value 0..64).
std::atomic<int> g_reg_tiles[2][kEigMaxN + 1];
std::once_flag g_reg_tiles_once;
void init_reg_tiles() {
  std::call_once(g_reg_tiles_once, [] {
    // defaults from timing on MI355X (512 x 512 x 20 window): two tiles per
    // workgroup for FP64 up to 20 frames (update pass 39.5 against 41.9 us),
    // one for FP32,
    // whose single-tile kernel keeps a higher occupancy (27.5 against 28.4)
    for (int c = 0; c <= kEigMaxN; ++c) {
      g_reg_tiles[0][c].store(c <= 20 ? 2 : 1);  // the loop leaves 24-32 at one wave per SIMD
      g_reg_tiles[1][c].store(1);
    }
  });
}

int reg_tiles(int dtype, int cls) {
  if (cls < 0 || cls > kEigMaxN || nb_class(cls, dtype) != cls) return -1;
  init_reg_tiles();
  return g_reg_tiles[dtype == RPCA_F32 ? 1 : 0][cls].load(std::memory_order_relaxed);
}

bool set_reg_tiles(int dtype, int cls, int v) {
  if (reg_tiles(dtype, cls) < 0 || v < 1 || v > 16) return false;
  g_reg_tiles[dtype == RPCA_F32 ? 1 : 0][cls].store(v, std::memory_order_relaxed);
  return true;
}

bool geometry(int64_t m, int64_t n, int dtype, int gram_mode, Geo& g) {
  if (m < 1 || n < 1 || n > RPCA_N_MAX) return false;
  if (m >= (int64_t(1) << 30)) return false;  // row offsets are 32-bit byte offsets
  g.es = dtype == RPCA_F32 ? 4 : 8;
  g.prec = gram_mode == RPCA_GRAM_BF16X3 ? 1 : (gram_mode == RPCA_GRAM_BF16X6 ? 2 : 0);
  if (g.prec && dtype != RPCA_F32) return false;
  const int reg = nb_class(n, dtype);
  g.kind = 1;
  if (!g.prec && reg != 0 && (dtype == RPCA_F64 || stream_kernel_choice(reg) == 0)) g.kind = 0;
  if (g.kind == 0) {
    g.nb = reg;
    const int64_t tiles = (m + kTile - 1) / kTile;
    g.tiles = static_cast<int>(tiles);
    // tiles per work item (and per partial slot): the class's knob, capped
    // so that the solve still spreads over at least 256 workgroups where it
    // has 256 tiles to give
    const int64_t cap = std::max<int64_t>(1, tiles / 256);
    const int want = reg_tiles(dtype, reg);
    g.tps = static_cast<int>(std::min<int64_t>(want, cap));
    g.mt = want > 1 ? 1 : 0;
  } else {
    if (n > (dtype == RPCA_F32 ? kEigHugeMaxN : kF64MaxN)) return false;
    g.nb = static_cast<int>((n + 15) / 16 * 16);
    const int64_t tiles = (m + kWideRows - 1) / kWideRows;
    g.tiles = static_cast<int>(tiles);
    // rows per workgroup: the tuning knob of the class (1024 by default, so
    // the O(nb^2) Gram partial stays a few percent of the workgroup's
    // streamed bytes), capped so that the solve spreads over at least 256
    // workgroups (one per CU) where it has 256 rows each to give
    const int64_t cap = std::max<int64_t>(4 * kWideRows, (m / 256) / kWideRows * kWideRows);
    const int rows = static_cast<int>(std::min<int64_t>(tile_rows(g.nb), cap));
    g.tps = (rows + kWideRows - 1) / kWideRows;
  }
  g.slots = (g.tiles + g.tps - 1) / g.tps;
  g.groups = (g.slots + kGroup - 1) / kGroup;
  g.pstride = pstride_for(g.nb);
  return true;
}

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
  b.escratch = o;
  if (n > kEigMaxN) {
    const size_t c = static_cast<size_t>(eig_class(static_cast<int>(n)));
    o += al256(c * c * sizeof(double));
  }
  b.state = o; o += al256(sizeof(SolveState));
  b.trace = o;
#ifdef RPCA_TRACE
  o += al256(static_cast<size_t>(g.slots) * 4 * sizeof(int64_t));
#endif
  b.total = o;
  return b;
}

// --------------------------------------------------------------------- plan
size_t plan_prepare(Plan& plan, const std::vector<SolveRec*>& recs, int nlanes, int dtype) {
  plan.dtype = dtype;
  plan.count = static_cast<int>(recs.size());
  plan.recs = recs;
  plan.lanes.assign(nlanes, LaneRun{});
  for (int i = 0; i < plan.count; ++i) plan.lanes[recs[i]->lane].solves.push_back(i);

  std::vector<WorkItem> items;
  std::vector<GroupItem> gitems;
  std::vector<int32_t> ids;
  for (LaneRun& lr : plan.lanes) {
    std::vector<int> keys;
    for (int i : lr.solves)
      if (std::find(keys.begin(), keys.end(), class_key(recs[i]->geo)) == keys.end())
        keys.push_back(class_key(recs[i]->geo));
    for (int key : keys) {
      const int off = static_cast<int>(items.size());
      for (int i : lr.solves)
        if (class_key(recs[i]->geo) == key)
          for (int q = 0; q < recs[i]->geo.slots; ++q) items.push_back(WorkItem{i, q});
      lr.classes.push_back({key, {off, static_cast<int>(items.size()) - off}});
    }
    for (int cls : {16, 32, 64, kEigWideMaxN, kEigHugeMaxN}) {
      const int off = static_cast<int>(ids.size());
      for (int i : lr.solves)
        if (eig_class(recs[i]->n) == cls) ids.push_back(i);
      const int cnt = static_cast<int>(ids.size()) - off;
      if (cnt > 0) lr.eigs.push_back({cls, {off, cnt}});
    }
    lr.gitem_off = static_cast<int>(gitems.size());
    for (int i : lr.solves)
      for (int g = 0; g < recs[i]->geo.groups; ++g) gitems.push_back(GroupItem{i, g});
    lr.gitem_cnt = static_cast<int>(gitems.size()) - lr.gitem_off;
    // subsets for the extra init stage of the solves with a given start
    for (int key : keys) {
      const int off = static_cast<int>(items.size());
      for (int i : lr.solves)
        if (recs[i]->warm && class_key(recs[i]->geo) == key)
          for (int q = 0; q < recs[i]->geo.slots; ++q) items.push_back(WorkItem{i, q});
      const int cnt = static_cast<int>(items.size()) - off;
      if (cnt > 0) lr.warm_classes.push_back({key, {off, cnt}});
    }
    for (int cls : {16, 32, 64, kEigWideMaxN, kEigHugeMaxN}) {
      const int off = static_cast<int>(ids.size());
      for (int i : lr.solves)
        if (recs[i]->warm && eig_class(recs[i]->n) == cls) ids.push_back(i);
      const int cnt = static_cast<int>(ids.size()) - off;
      if (cnt > 0) lr.warm_eigs.push_back({cls, {off, cnt}});
    }
    lr.warm_gitem_off = static_cast<int>(gitems.size());
    for (int i : lr.solves)
      if (recs[i]->warm)
        for (int g = 0; g < recs[i]->geo.groups; ++g) gitems.push_back(GroupItem{i, g});
    lr.warm_gitem_cnt = static_cast<int>(gitems.size()) - lr.warm_gitem_off;
  }

  const size_t off_desc = 0;
  const size_t off_items = al256(off_desc + sizeof(SolveDesc) * plan.count);
  const size_t off_gitems = al256(off_items + sizeof(WorkItem) * items.size());
  const size_t off_ids = al256(off_gitems + sizeof(GroupItem) * gitems.size());
  const size_t off_gath = al256(off_ids + sizeof(int32_t) * ids.size());
  const size_t bytes = al256(off_gath + sizeof(SolveState) * plan.count);
  plan.host.assign(bytes, 0);
  plan.off_items = off_items;
  plan.off_gitems = off_gitems;
  plan.off_ids = off_ids;
  plan.off_gath = off_gath;

  SolveDesc* dh = reinterpret_cast<SolveDesc*>(plan.host.data() + off_desc);
  for (int i = 0; i < plan.count; ++i) {
    const SolveRec& r = *recs[i];
    char* b = r.mem;
    SolveDesc& d = dh[i];
    std::memset(&d, 0, sizeof(d));
    d.X = r.M;
    d.S[0] = b + r.big.S0;
    d.S[1] = b + r.big.S1;
    d.Y[0] = b + r.big.Y0;
    d.Y[1] = b + r.big.Y1;
    d.Lout = r.L;
    d.Sout = r.S;
    d.Yout = r.Yout;
    d.S0 = r.S0;
    d.Y0 = r.Y0;
    d.warm = r.warm;
    d.partials = reinterpret_cast<double*>(b + r.big.part);
    d.gpartials = reinterpret_cast<double*>(b + r.big.gpart);
    d.P = b + r.big.P;
    d.V = reinterpret_cast<double*>(b + r.big.V);
    d.escratch = r.n > kEigMaxN ? reinterpret_cast<double*>(b + r.big.escratch) : nullptr;
    d.st = reinterpret_cast<SolveState*>(b + r.big.state);
#ifdef RPCA_TRACE
    d.wgtrace = reinterpret_cast<int64_t*>(b + r.big.trace);
#endif
    d.m = r.m;
    d.n = r.n;
    d.nb = r.geo.nb;
    d.tiles = r.geo.tiles;
    d.tps = r.geo.tps;
    d.slots = r.geo.slots;
    d.groups = r.geo.groups;
    d.pstride = r.geo.pstride;
    d.maxit = r.maxit;
    d.lam_in = r.lam;
    d.mu_in = r.mu;
    d.tol = r.tol;
  }
  if (!items.empty())
    std::memcpy(plan.host.data() + off_items, items.data(), sizeof(WorkItem) * items.size());
  if (!gitems.empty())
    std::memcpy(plan.host.data() + off_gitems, gitems.data(), sizeof(GroupItem) * gitems.size());
  if (!ids.empty()) std::memcpy(plan.host.data() + off_ids, ids.data(), sizeof(int32_t) * ids.size());
  return bytes;
}

int plan_upload(Plan& plan, char* ctrl, hipStream_t stream) {
  const hipError_t e = hipMemcpyAsync(ctrl, plan.host.data(), plan.host.size(),
                                      hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) {
    set_error("hipMemcpyAsync(control block)", e);
    return RPCA_ERR_DEVICE;
  }
  plan.descs = reinterpret_cast<SolveDesc*>(ctrl);
  plan.items = reinterpret_cast<WorkItem*>(ctrl + plan.off_items);
  plan.gitems = reinterpret_cast<GroupItem*>(ctrl + plan.off_gitems);
  plan.ids = reinterpret_cast<int32_t*>(ctrl + plan.off_ids);
  plan.gathered = reinterpret_cast<SolveState*>(ctrl + plan.off_gath);
  return RPCA_OK;
}

int plan_build(Plan& plan, const std::vector<SolveRec*>& recs, int nlanes, int dtype,
               hipStream_t stream) {
  const size_t bytes = plan_prepare(plan, recs, nlanes, dtype);
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&plan.ctrl), bytes, stream);
  if (e != hipSuccess || plan.ctrl == nullptr) {
    set_error("hipMallocAsync(control block)", e);
    (void)hipGetLastError();
    plan.ctrl = nullptr;
    return RPCA_ERR_NOMEM;
  }
  return plan_upload(plan, plan.ctrl, stream);
}

void plan_free(Plan& plan, hipStream_t stream) {
  if (plan.ctrl) (void)hipFreeAsync(plan.ctrl, stream);
  plan.ctrl = nullptr;
}

// -------------------------------------------------------------------- lanes
int lanes_create(Lanes& L, int nlanes) {
  L.s.assign(nlanes, nullptr);
  L.join.assign(nlanes, nullptr);
  for (int i = 0; i < nlanes; ++i) {
    hipError_t e = hipStreamCreateWithFlags(&L.s[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&L.join[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      set_error("hipStreamCreateWithFlags/hipEventCreate(lane)", e);
      return RPCA_ERR_DEVICE;
    }
  }
  hipError_t e = hipEventCreateWithFlags(&L.fork, hipEventDisableTiming);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&L.snap[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    set_error("hipEventCreate(lanes)", e);
    return RPCA_ERR_DEVICE;
  }
  return RPCA_OK;
}

int lanes_reserve_pinned(Lanes& L, int count) {
  if (count <= L.pinned_count) return RPCA_OK;
  for (int k = 0; k < 2; ++k) {
    if (L.pinned[k]) (void)hipHostFree(L.pinned[k]);
    L.pinned[k] = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&L.pinned[k]), sizeof(SolveState) * count) != hipSuccess) {
      set_error_text("hipHostMalloc(state snapshots) failed");
      L.pinned_count = 0;
      return RPCA_ERR_NOMEM;
    }
  }
  L.pinned_count = count;
  return RPCA_OK;
}

void lanes_destroy(Lanes& L) {
  for (auto s : L.s)
    if (s) (void)hipStreamSynchronize(s);
  for (auto e : L.join)
    if (e) (void)hipEventDestroy(e);
  for (auto s : L.s)
    if (s) (void)hipStreamDestroy(s);
  if (L.fork) (void)hipEventDestroy(L.fork);
  for (int k = 0; k < 2; ++k) {
    if (L.snap[k]) (void)hipEventDestroy(L.snap[k]);
    if (L.pinned[k]) (void)hipHostFree(L.pinned[k]);
    L.snap[k] = nullptr;
    L.pinned[k] = nullptr;
  }
  L.s.clear();
  L.join.clear();
  L.fork = nullptr;
  L.pinned_count = 0;
}

// ------------------------------------------------------------------ enqueue
#define EQ(expr)                   \
  do {                             \
    const hipError_t e_ = (expr);  \
    if (e_ != hipSuccess) {        \
      set_error(#expr, e_);        \
      return e_;                   \
    }                              \
  } while (0)

hipError_t enqueue_reset_states(const Plan& plan, hipStream_t s) {
  EQ(launch_reset_states(plan.count, s, plan.descs));
  return hipSuccess;
}

// Lanes >= 1 wait for lane 0's work so far (the control block upload).
static hipError_t fork_lanes(const Lanes& L) {
  if (L.s.size() <= 1) return hipSuccess;
  EQ(hipEventRecord(L.fork, L.s[0]));
  for (size_t i = 1; i < L.s.size(); ++i) EQ(hipStreamWaitEvent(L.s[i], L.fork, 0));
  return hipSuccess;
}

hipError_t enqueue_init(const Plan& plan, const Lanes& L) {
  EQ(fork_lanes(L));
  for (size_t l = 0; l < plan.lanes.size(); ++l) {
    const LaneRun& lr = plan.lanes[l];
    hipStream_t s = L.s[l];
    for (size_t c = 0; c < lr.classes.size(); ++c) {
      ev_begin(s, 0, 0, static_cast<int>(l), static_cast<int>(c));
      EQ(launch_stream(plan.dtype, lr.classes[c].first, kModeInit, lr.classes[c].second.second, s,
                       plan.descs, plan.items + lr.classes[c].second.first));
      ev_end(s);
    }
    EQ(launch_reduce(lr.gitem_cnt, s, plan.descs, plan.gitems + lr.gitem_off));
    // solves with a given start: fix mu, then the Gram of A_1 = X - S0 + Y0/mu
    for (const auto& er : lr.warm_eigs) {
      if (er.first > kEigMaxN)
        EQ(launch_eig_wide(plan.dtype == RPCA_F32 ? 1 : 0, er.first, er.second.second, s,
                           plan.descs, plan.ids + er.second.first));
      else
        EQ(launch_eig(plan.dtype == RPCA_F32 ? 1 : 0, er.first, er.second.second, s, plan.descs,
                      plan.ids + er.second.first));
    }
    for (const auto& wc : lr.warm_classes)
      EQ(launch_stream(plan.dtype, wc.first, kModeWarm, wc.second.second, s, plan.descs,
                       plan.items + wc.second.first));
    if (lr.warm_gitem_cnt > 0)
      EQ(launch_reduce(lr.warm_gitem_cnt, s, plan.descs, plan.gitems + lr.warm_gitem_off));
  }
  return hipSuccess;
}

// `first_iter` numbers the launches for kernel timing (1-based).
static hipError_t enqueue_iterations_at(const Plan& plan, const Lanes& L, int iters, int first_iter) {
  for (size_t l = 0; l < plan.lanes.size(); ++l) {
    const LaneRun& lr = plan.lanes[l];
    hipStream_t s = L.s[l];
    for (int k = 0; k < iters; ++k) {
      for (const auto& er : lr.eigs) {
        ev_begin(s, 1, first_iter + k, static_cast<int>(l), -1);
        if (er.first > kEigMaxN)
          EQ(launch_eig_wide(plan.dtype == RPCA_F32 ? 1 : 0, er.first, er.second.second, s,
                             plan.descs, plan.ids + er.second.first));
        else
          EQ(launch_eig(plan.dtype == RPCA_F32 ? 1 : 0, er.first, er.second.second, s, plan.descs,
                        plan.ids + er.second.first));
        ev_end(s);
      }
      for (size_t c = 0; c < lr.classes.size(); ++c) {
        ev_begin(s, 2, first_iter + k, static_cast<int>(l), static_cast<int>(c));
        EQ(launch_stream(plan.dtype, lr.classes[c].first, kModeUpdate, lr.classes[c].second.second,
                         s, plan.descs, plan.items + lr.classes[c].second.first));
        ev_end(s);
      }
      EQ(launch_reduce(lr.gitem_cnt, s, plan.descs, plan.gitems + lr.gitem_off));
    }
  }
  return hipSuccess;
}

hipError_t enqueue_iterations(const Plan& plan, const Lanes& L, int iters) {
  return enqueue_iterations_at(plan, L, iters, 1);
}

hipError_t enqueue_finalize(const Plan& plan, const Lanes& L) {
  for (size_t l = 0; l < plan.lanes.size(); ++l) {
    const LaneRun& lr = plan.lanes[l];
    hipStream_t s = L.s[l];
    for (size_t c = 0; c < lr.classes.size(); ++c) {
      ev_begin(s, 3, 0, static_cast<int>(l), static_cast<int>(c));
      EQ(launch_stream(plan.dtype, lr.classes[c].first, kModeFinalize, lr.classes[c].second.second,
                       s, plan.descs, plan.items + lr.classes[c].second.first));
      ev_end(s);
    }
  }
  return hipSuccess;
}

static hipError_t join_lanes(const Lanes& L) {
  for (size_t i = 1; i < L.s.size(); ++i) {
    EQ(hipEventRecord(L.join[i], L.s[i]));
    EQ(hipStreamWaitEvent(L.s[0], L.join[i], 0));
  }
  return hipSuccess;
}

hipError_t enqueue_snapshot(const Plan& plan, Lanes& L, int slot) {
  EQ(join_lanes(L));
  EQ(launch_gather_states(plan.count, L.s[0], plan.descs, plan.gathered));
  EQ(hipMemcpyAsync(L.pinned[slot], plan.gathered, sizeof(SolveState) * plan.count,
                    hipMemcpyDeviceToHost, L.s[0]));
  EQ(hipEventRecord(L.snap[slot], L.s[0]));
  return hipSuccess;
}

#undef EQ

int make_rec(const rpca_problem& p, int dtype, int gram_mode, SolveRec& r) {
  if (!p.M || !p.L || !p.S || p.m < 1 || p.n < 1 || p.n > RPCA_N_MAX || p.maxit < 1)
    return RPCA_ERR_ARG;
  if (!std::isfinite(p.lambda) || !std::isfinite(p.mu) || std::isnan(p.tol)) return RPCA_ERR_ARG;
  const size_t bytes = static_cast<size_t>(p.m) * static_cast<size_t>(p.n) * (dtype == RPCA_F32 ? 4 : 8);
  // outputs must not overlap each other or any input
  const void* outs[3] = {p.L, p.S, p.Y};
  const void* ins[3] = {p.M, p.S0, p.Y0};
  for (int a = 0; a < 3; ++a) {
    if (!outs[a]) continue;
    for (int b = a + 1; b < 3; ++b)
      if (outs[b] && overlap(outs[a], outs[b], bytes)) return RPCA_ERR_ARG;
    for (int b = 0; b < 3; ++b)
      if (ins[b] && overlap(outs[a], ins[b], bytes)) return RPCA_ERR_ARG;
  }
  if (!geometry(p.m, p.n, dtype, gram_mode, r.geo)) return RPCA_ERR_UNSUPPORTED;
  r.big = big_layout(p.m, p.n, r.geo);
  r.M = p.M;
  r.L = p.L;
  r.S = p.S;
  r.Yout = p.Y;
  r.S0 = p.S0;
  r.Y0 = p.Y0;
  r.warm = (p.S0 || p.Y0) ? 1 : 0;
  r.m = p.m;
  r.n = static_cast<int32_t>(p.n);
  r.lam = p.lambda;
  r.mu = p.mu;
  r.tol = p.tol;
  r.maxit = p.maxit;
  return RPCA_OK;
}

void assign_lanes(std::vector<SolveRec*>& recs, int nlanes) {
  std::vector<int> order(recs.size());
  for (size_t i = 0; i < recs.size(); ++i) order[i] = static_cast<int>(i);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return recs[a]->m * recs[a]->n > recs[b]->m * recs[b]->n;
  });
  std::vector<double> load(nlanes, 0.0);
  for (int i : order) {
    const int l = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    recs[i]->lane = l;
    load[l] += static_cast<double>(recs[i]->m) * recs[i]->n;
  }
}

// ---------------------------------------------------------------- run_batch
namespace {

#define CK(expr)                                  \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) {                       \
      if (!g_last_error[0]) set_error(#expr, e_); \
      rc = RPCA_ERR_DEVICE;                       \
      goto done;                                  \
    }                                             \
  } while (0)

// Streams, events and pinned state buffers for the calls on one device.  A
// call leases an idle set (created when none is idle; creating one costs
// more than a small solve) and gives it back when it returns, after its
// last synchronisation, so a set is never used by two calls at once.  The
// pool holds as many sets as calls ever ran at once on the device, whatever
// the number of host threads that made them; the sets live until the
// process ends.
struct LaneCache {
  Lanes L;
};
std::mutex g_lane_pool_mu;
std::vector<LaneCache*> g_lane_pool[64];

struct LaneLease {
  int dev = -1;
  LaneCache* c = nullptr;
  LaneLease() = default;
  LaneLease(const LaneLease&) = delete;
  LaneLease& operator=(const LaneLease&) = delete;
  ~LaneLease() {
    if (c) {
      std::lock_guard<std::mutex> lk(g_lane_pool_mu);
      g_lane_pool[dev].push_back(c);
    }
  }
};

// Lease a lane set of device `dev` (current) into `lease` and return a view
// of its first `nlanes` lanes with room for `count` solve states in `view`,
// or an error code.
int lease_lanes(int dev, int nlanes, int count, LaneLease& lease, Lanes& view) {
  if (dev < 0 || dev >= 64) return RPCA_ERR_DEVICE;
  LaneCache* c = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_lane_pool_mu);
    if (!g_lane_pool[dev].empty()) {
      c = g_lane_pool[dev].back();
      g_lane_pool[dev].pop_back();
    }
  }
  if (c == nullptr) {
    c = new LaneCache();
    const int rc = lanes_create(c->L, kMaxLanes);
    if (rc != RPCA_OK) {
      lanes_destroy(c->L);
      delete c;
      return rc;
    }
  }
  lease.dev = dev;
  lease.c = c;
  const int rc = lanes_reserve_pinned(c->L, count);
  if (rc != RPCA_OK) return rc;
  view = Lanes{};
  view.s.assign(c->L.s.begin(), c->L.s.begin() + nlanes);
  view.join.assign(c->L.join.begin(), c->L.join.begin() + nlanes);
  view.fork = c->L.fork;
  for (int k = 0; k < 2; ++k) {
    view.pinned[k] = c->L.pinned[k];
    view.snap[k] = c->L.snap[k];
  }
  view.pinned_count = c->L.pinned_count;
  return RPCA_OK;
}

int run_batch(rpca_problem* probs, int count, int dtype, int gram_mode, hipStream_t user) {
  g_last_error[0] = '\0';
  if (count < 1 || probs == nullptr) return RPCA_ERR_ARG;
  if (dtype != RPCA_F32 && dtype != RPCA_F64) return RPCA_ERR_ARG;
  if (gram_mode != RPCA_GRAM_DEFAULT && gram_mode != RPCA_GRAM_BF16X3 &&
      gram_mode != RPCA_GRAM_BF16X6)
    return RPCA_ERR_ARG;
  if (gram_mode != RPCA_GRAM_DEFAULT && dtype != RPCA_F32) return RPCA_ERR_ARG;

  std::vector<SolveRec> recs(count);
  for (int i = 0; i < count; ++i) {
    const int vrc = make_rec(probs[i], dtype, gram_mode, recs[i]);
    if (vrc != RPCA_OK) return vrc;
  }

  // Lanes: balance the matrix sizes, largest first.  Kernel timing runs on
  // one lane so that each launch's event pair brackets that launch alone.
  const bool prof = profiling_on();
  const int nlanes = prof ? 1 : std::min(count, kMaxLanes);

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

  const bool use_graph = !prof && !graphs_disabled();
  int rc = RPCA_OK;
  char* arena = nullptr;
  LaneLease lease;  // returns the lane set when the call returns
  Lanes L;
  Plan plan;
  std::vector<EvPair> evs;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<SolveRec*> ptrs(count);
  int maxit_all = 0;
  for (int i = 0; i < count; ++i) {
    ptrs[i] = &recs[i];
    maxit_all = std::max(maxit_all, recs[i].maxit);
  }
  assign_lanes(ptrs, nlanes);

  rc = lease_lanes(dev, nlanes, count, lease, L);
  if (rc != RPCA_OK) return rc;
  hipStream_t s0 = L.s[0];
  if (prof) t_evs = &evs;

  {
    // inputs are produced on the caller's stream
    hipError_t e = hipStreamSynchronize(user);
    if (e != hipSuccess) {
      set_error("hipStreamSynchronize(caller stream)", e);
      rc = RPCA_ERR_DEVICE;
      goto done;
    }
    size_t total = 0;
    std::vector<size_t> base(count);
    for (int i = 0; i < count; ++i) {
      base[i] = total;
      total += recs[i].big.total;
    }
    e = hipMallocAsync(reinterpret_cast<void**>(&arena), total, s0);
    if (e != hipSuccess || arena == nullptr) {
      set_error("hipMallocAsync(workspace)", e);
      (void)hipGetLastError();
      arena = nullptr;
      rc = RPCA_ERR_NOMEM;
      goto done;
    }
    for (int i = 0; i < count; ++i) recs[i].mem = arena + base[i];
  }
  rc = plan_build(plan, ptrs, nlanes, dtype, s0);
  if (rc != RPCA_OK) goto done;
  CK(enqueue_reset_states(plan, s0));
  CK(enqueue_init(plan, L));
  // The init passes of lanes 1.. run on their own streams; the iteration
  // chunks (a graph launched on lane 0, or direct launches forked from it)
  // must come after them, so join them into lane 0 first.
  CK(join_lanes(L));

  {
    int launched = 0;  // iterations enqueued (eigensolve launches per solve)
    if (use_graph) {
      CK(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
      {
        hipError_t e = fork_lanes(L);
        if (e == hipSuccess) e = enqueue_iterations(plan, L, kGraphChunk);
        if (e == hipSuccess) e = join_lanes(L);
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(s0, &g);
        graph = g;
        CK(e);
        CK(ee);
      }
      CK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    }
    auto run_chunk = [&](int chunk) -> hipError_t {
      hipError_t e;
      if (use_graph) {
        e = hipGraphLaunch(gexec, s0);
      } else {
        e = fork_lanes(L);
        if (e == hipSuccess) e = enqueue_iterations_at(plan, L, chunk, launched + 1);
      }
      launched += chunk;
      return e;
    };
    int chunk = use_graph ? kGraphChunk : kDirectChunkFirst;
    int slot = 0;
    CK(run_chunk(chunk));
    CK(enqueue_snapshot(plan, L, slot));
    for (;;) {
      const int prev = slot;
      slot ^= 1;
      if (!use_graph) chunk = std::min(chunk * 2, kDirectChunkMax);
      const bool all_capped = launched > maxit_all + 1;
      if (!all_capped) {
        CK(run_chunk(chunk));
        CK(enqueue_snapshot(plan, L, slot));
      }
      CK(hipEventSynchronize(L.snap[prev]));
      bool all_done = true;
      for (int i = 0; i < count; ++i) all_done = all_done && L.pinned[prev][i].done != 0;
      if (all_done) break;
      if (all_capped) {
        // snapshot `prev` was taken after every launched iteration
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "a solve did not stop after %d iterations (cap %d)", launched, maxit_all);
        rc = RPCA_ERR_DEVICE;
        goto done;
      }
    }
  }
  CK(enqueue_finalize(plan, L));
  CK(enqueue_snapshot(plan, L, 0));
  CK(hipStreamSynchronize(s0));
  {
    int worst_neg = 0, any_nc = 0;
    for (int i = 0; i < count; ++i) {
      const SolveState& st = L.pinned[0][i];
      recs[i].st = st;
      probs[i].iterations = st.iter;
      probs[i].status = st.status;
      probs[i].residual = st.resid;
      if (st.status < 0) worst_neg = std::min(worst_neg, st.status);
      if (st.status == RPCA_NOT_CONVERGED) any_nc = 1;
    }
    rc = worst_neg < 0 ? worst_neg : (any_nc ? RPCA_NOT_CONVERGED : RPCA_OK);
  }
#ifdef RPCA_TRACE
  trace_report(recs[0], s0);
#endif

  if (prof) {
    double init_ms = 0, eig_ms = 0, upd_ms = 0, fin_ms = 0, upd_bytes = 0;
    int64_t eig_n = 0, upd_n = 0, iters = 0;
    int max_iter = 0;
    for (int i = 0; i < count; ++i) {
      max_iter = std::max(max_iter, recs[i].st.iter);
      iters += recs[i].st.iter;
    }
    for (auto& e : evs) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e.a, e.b);
      if (e.kind == 0) {
        init_ms += ms;
      } else if (e.kind == 3) {
        fin_ms += ms;
      } else if (e.kind == 1) {
        if (e.iter <= max_iter) {
          eig_ms += ms;
          ++eig_n;
        }
      } else {
        const LaneRun& lr = plan.lanes[e.lane];
        const int key = lr.classes[e.cls].first;
        double bytes = 0;
        for (int i : lr.solves) {
          if (class_key(recs[i].geo) == key && recs[i].st.iter >= e.iter) {
            const double words = e.iter == 1 ? 3.0 : 5.0;
            bytes += words * static_cast<double>(recs[i].m) * recs[i].n * recs[i].geo.es;
          }
        }
        if (bytes > 0) {
          upd_ms += ms;
          ++upd_n;
          upd_bytes += bytes;
        }
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

done:
  t_evs = nullptr;
  t_launch_events = LaunchEvents{};
  for (auto& e : evs) {
    if (e.a) (void)hipEventDestroy(e.a);
    if (e.b) (void)hipEventDestroy(e.b);
  }
  if (rc == RPCA_ERR_DEVICE) (void)hipGetLastError();
  for (auto s : L.s)
    if (s) (void)hipStreamSynchronize(s);
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  if (!L.s.empty()) {
    plan_free(plan, L.s[0]);
    if (arena) (void)hipFreeAsync(arena, L.s[0]);
    (void)hipStreamSynchronize(L.s[0]);
  }
  // L is a view of the leased lane set, which the lease gives back (every
  // lane was synchronised above): nothing to destroy
  return rc;
}

#undef CK

}  // namespace

const char* last_error_text() { return g_last_error; }

bool profiling_enabled() { return profiling_on(); }

}  // namespace rpca

using namespace rpca;

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
  if (!geometry(m, n, dtype, RPCA_GRAM_DEFAULT, g)) return 0;
  const Big b = big_layout(m, n, g);
  // plus this solve's share of a control block
  return b.total + al256(sizeof(SolveDesc) + sizeof(SolveState) + sizeof(int32_t)) +
         al256(sizeof(GroupItem) * g.groups) + al256(sizeof(WorkItem) * g.slots);
}

const char* rpca_strerror(int code) {
  switch (code) {
    case RPCA_OK: return "converged";
    case RPCA_NOT_CONVERGED: return "iteration cap reached before the stopping test held";
    case RPCA_ERR_ARG: return "invalid argument";
    case RPCA_ERR_NOMEM: return "device memory allocation failed";
    case RPCA_ERR_DEVICE: return "HIP runtime error";
    case RPCA_ERR_NONFINITE: return "non-finite value in the input or the iteration";
    case RPCA_ERR_UNSUPPORTED: return "shape not supported by the library";
    case RPCA_ERR_TIMEOUT: return "the request's timeout passed before it finished";
    default: return "unknown status";
  }
}

const char* rpca_version(void) { return "rpca_mi355x 0.3"; }

int rpca_tune_set(int32_t knob, int32_t dtype, int32_t cls, int32_t value) {
  if (dtype != RPCA_F32 && dtype != RPCA_F64) return RPCA_ERR_ARG;
  if (knob == RPCA_KNOB_EIG_THREADS) return set_eig_threads(dtype, cls, value) ? RPCA_OK : RPCA_ERR_ARG;
  if (knob == RPCA_KNOB_STREAM_KERNEL) {
    if (dtype != RPCA_F32) return RPCA_ERR_ARG;
    return set_stream_kernel_choice(cls, value) ? RPCA_OK : RPCA_ERR_ARG;
  }
  if (knob == RPCA_KNOB_TILE_ROWS) {
    if (dtype != RPCA_F32) return RPCA_ERR_ARG;
    return set_tile_rows(cls, value) ? RPCA_OK : RPCA_ERR_ARG;
  }
  if (knob == RPCA_KNOB_REG_TILES) return set_reg_tiles(dtype, cls, value) ? RPCA_OK : RPCA_ERR_ARG;
  return RPCA_ERR_ARG;
}

int rpca_tune_get(int32_t knob, int32_t dtype, int32_t cls) {
  if (dtype != RPCA_F32 && dtype != RPCA_F64) return RPCA_ERR_ARG;
  if (knob == RPCA_KNOB_EIG_THREADS) {
    const int v = eig_threads(dtype, cls);
    return v > 0 ? v : RPCA_ERR_ARG;
  }
  if (knob == RPCA_KNOB_STREAM_KERNEL) {
    if (dtype != RPCA_F32) return RPCA_ERR_ARG;
    const int v = stream_kernel_choice(cls);
    return v >= 0 ? v : RPCA_ERR_ARG;
  }
  if (knob == RPCA_KNOB_TILE_ROWS) {
    if (dtype != RPCA_F32) return RPCA_ERR_ARG;
    const int v = tile_rows(cls);
    return v > 0 ? v : RPCA_ERR_ARG;
  }
  if (knob == RPCA_KNOB_REG_TILES) {
    const int v = reg_tiles(dtype, cls);
    return v > 0 ? v : RPCA_ERR_ARG;
  }
  return RPCA_ERR_ARG;
}

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
