// Host-side engine of the library (internal).
//
//   SolveRec  one problem: its parameters, geometry and the device memory that
//             holds its iterate buffers, reduction partials, projector,
//             eigenvectors and state for as long as the solve is active.
//   Plan      the launch tables (descriptors, work items, group items and
//             eigensolver id lists) for a set of active solves, split into
//             lanes: each lane is a stream that runs its own solves' chain
//             [eigensolve -> streaming update -> group reduction], so one
//             lane's eigensolves overlap another lane's streaming passes.
//   Lanes     the streams, events and pinned staging of a run.
//
// rpca_solve_many builds one plan for all its problems and runs it to the
// end; the server builds a plan per quantum from the solves it has admitted.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "rpca.h"
#include "common.h"

namespace rpca {

struct Geo {
  int nb = 0, tiles = 0, tps = 1, slots = 0, groups = 0, pstride = 0;
  int kind = 0;  // streaming kernel: 0 register (thread per row), 1 MFMA tiles
  int prec = 0;  // contraction precision: 0 storage/FP64, 1 BF16x3, 2 BF16x6
  int mt = 0;    // register kernel whose work items walk several tiles
  size_t es = 0;
};

// Launch-class key of a solve: frame class, kernel kind, precision, and for
// the register kernel whether it is the multi-tile variant.
inline int class_key(const Geo& g) { return g.nb | (g.kind << 8) | (g.prec << 9) | (g.mt << 11); }

// Byte offsets of one solve's device memory.
struct Big {
  size_t S0, S1, Y0, Y1, part, gpart, P, V, escratch, state, trace, total;
};

bool geometry(int64_t m, int64_t n, int dtype, int gram_mode, Geo& g);
Big big_layout(int64_t m, int64_t n, const Geo& g);

struct SolveRec {
  const void* M = nullptr;
  void* L = nullptr;
  void* S = nullptr;
  void* Yout = nullptr;        // optional final Y
  const void* S0 = nullptr;    // optional starting S
  const void* Y0 = nullptr;    // optional starting Y
  int warm = 0;                // starts from S0 / Y0
  int64_t m = 0;
  int32_t n = 0;
  double lam = -1.0, mu = -1.0, tol = 0.0;
  int32_t maxit = 1;
  Geo geo;
  Big big{};
  char* mem = nullptr;  // device memory (big.total bytes) or nullptr when not resident
  int lane = 0;
  int64_t tag = 0;
  SolveState st{};      // last state read back
};

struct LaneRun {
  std::vector<std::pair<int, std::pair<int, int>>> classes;  // (class key, (item offset, count))
  std::vector<std::pair<int, std::pair<int, int>>> eigs;     // (class, (id offset, count))
  int gitem_off = 0, gitem_cnt = 0;
  // the same for the lane's solves with a given start (extra init stage)
  std::vector<std::pair<int, std::pair<int, int>>> warm_classes, warm_eigs;
  int warm_gitem_off = 0, warm_gitem_cnt = 0;
  std::vector<int> solves;                                   // plan-local solve indices
};

struct Plan {
  int dtype = RPCA_F32;
  int count = 0;
  std::vector<SolveRec*> recs;
  std::vector<LaneRun> lanes;
  std::vector<unsigned char> host;  // staging copy of the control block
  size_t off_items = 0, off_gitems = 0, off_ids = 0, off_gath = 0;  // byte offsets in it
  char* ctrl = nullptr;             // device control block owned by the plan (plan_build)
  SolveDesc* descs = nullptr;
  WorkItem* items = nullptr;
  GroupItem* gitems = nullptr;
  int32_t* ids = nullptr;
  SolveState* gathered = nullptr;   // k_gather_states output (count states)
};

// Build the control block for `recs` (each rec's lane in [0, nlanes)) and
// upload it on `stream` into a stream-ordered allocation the plan owns.
// Returns a status code.
int plan_build(Plan& plan, const std::vector<SolveRec*>& recs, int nlanes, int dtype,
               hipStream_t stream);
// The two halves of plan_build: fill the host copy of the control block
// (returns its size in bytes), then copy it into device memory `ctrl` of at
// least that size (not owned by the plan) and point the plan's tables there.
size_t plan_prepare(Plan& plan, const std::vector<SolveRec*>& recs, int nlanes, int dtype);
int plan_upload(Plan& plan, char* ctrl, hipStream_t stream);
void plan_free(Plan& plan, hipStream_t stream);

struct Lanes {
  std::vector<hipStream_t> s;
  std::vector<hipEvent_t> join;   // per lane
  hipEvent_t fork = nullptr;
  SolveState* pinned[2] = {nullptr, nullptr};
  hipEvent_t snap[2] = {nullptr, nullptr};
  int pinned_count = 0;
};

int lanes_create(Lanes& L, int nlanes);
void lanes_destroy(Lanes& L);
int lanes_reserve_pinned(Lanes& L, int count);

// Enqueue on the lanes.  Each returns hipSuccess or the failing call's error.
hipError_t enqueue_reset_states(const Plan& plan, hipStream_t s);
hipError_t enqueue_init(const Plan& plan, const Lanes& L);
hipError_t enqueue_iterations(const Plan& plan, const Lanes& L, int iters);
hipError_t enqueue_finalize(const Plan& plan, const Lanes& L);
// Join every lane into lane 0, gather the plan's solve states into pinned
// buffer `slot` and record snap[slot].
hipError_t enqueue_snapshot(const Plan& plan, Lanes& L, int slot);

// Validate one problem and fill its record (parameters, geometry, layout).
// Returns RPCA_OK, RPCA_ERR_ARG or RPCA_ERR_UNSUPPORTED.
int make_rec(const rpca_problem& p, int dtype, int gram_mode, SolveRec& r);
// Spread solves over lanes, balancing m*n, largest first (stable).
void assign_lanes(std::vector<SolveRec*>& recs, int nlanes);
// Memory pool of the device: keep freed blocks cached (set once per device).
void setup_pool(int dev);
bool graphs_disabled();
// Streams a plan's solves are spread over: the hardware queues a process
// gets by default (4).
constexpr int kMaxLanes = 4;
// The server's plans mix solves at every stage of their iterations; six
// streams (two of them sharing hardware queues) keep more eigensolves in
// flight beside the streaming passes there.
constexpr int kServeLanes = 6;

void set_error(const char* what, hipError_t e);
void set_error_text(const char* text);

int nb_class(int64_t n, int dtype);
// FP32 register classes: streaming kernel choice (0 register, 1 MFMA tiles).
int stream_kernel_choice(int cls);
bool set_stream_kernel_choice(int cls, int v);
// tiles per workgroup of the register kernel (-1: no such class)
int reg_tiles(int dtype, int cls);
bool set_reg_tiles(int dtype, int cls, int v);
// rows per workgroup of the tile kernel for tile class nb (-1: no such class)
int tile_rows(int nb);
bool set_tile_rows(int nb, int rows);

}  // namespace rpca
