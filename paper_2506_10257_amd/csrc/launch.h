// Host-side launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_ext.h>

#include "common.h"

namespace rpca {

// Kernel timing: while `start` is set, a solve-path launch on this thread
// records its own start and end timestamps into the pair (the dispatch packet
// carries them, so queue time between launches is not counted).  Null when
// timing is off: then the launch is a plain one.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents t_launch_events;

#define RPCA_LAUNCH(K, G, B, SH, S, ...)                                                      \
  do {                                                                                       \
    if (::rpca::t_launch_events.start)                                                       \
      hipExtLaunchKernelGGL(K, G, B, SH, S, ::rpca::t_launch_events.start,                   \
                            ::rpca::t_launch_events.stop, 0, __VA_ARGS__);                   \
    else                                                                                     \
      hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                                       \
  } while (0)

// Frame classes compiled for the register-resident streaming kernels.  A solve
// with n frames runs on the smallest class >= n.
constexpr int kClassesF32[] = {4, 8, 10, 12, 16, 20, 24, 28, 32, 40, 48, 56, 60, 64};
constexpr int kClassesF64[] = {4, 8, 10, 12, 16, 20, 24, 28, 32};

// kModeWarm: for a solve started from a given S0 / Y0, the Gram of the first
// iterate A_1 = X - S0 + Y0/mu (after mu is fixed), copying S0 and Y0 into the
// iterate buffers that the first update pass reads.
enum StreamMode { kModeInit = 0, kModeUpdate = 1, kModeFinalize = 2, kModeWarm = 3 };

// dtype 0 = FP64, 1 = FP32 (as RPCA_F64 / RPCA_F32).
// mt: the multi-tile register kernel (work items of more than one tile).
hipError_t launch_stream_f32(int nb, int mode, bool mt, int grid, hipStream_t stream,
                             const SolveDesc* descs, const WorkItem* items);
hipError_t launch_stream_f64(int nb, int mode, bool mt, int grid, hipStream_t stream,
                             const SolveDesc* descs, const WorkItem* items);
hipError_t launch_reduce(int grid, hipStream_t stream, const SolveDesc* descs,
                         const GroupItem* items);
hipError_t launch_gather_states(int count, hipStream_t stream, const SolveDesc* descs,
                                SolveState* out);
hipError_t launch_reset_states(int count, hipStream_t stream, const SolveDesc* descs);

// Eigensolver classes 16, 32 and 64: the largest n each handles.  The
// workgroup size of each class (256, 512 or 1024 threads) is a tuning knob.
// ids lists the solves (indices into descs) of the launch.
// Returns 16, 32, 64, kEigWideMaxN or kEigHugeMaxN (0 if n is too large).
int eig_class(int n);
// Classes above 64 frames: the in-place eigensolver, ncls = kEigWideMaxN
// (V in LDS) or kEigHugeMaxN (V in global memory).
hipError_t launch_eig_wide(int dtype, int ncls, int grid, hipStream_t stream,
                           const SolveDesc* descs, const int32_t* ids);
// MFMA streaming kernel.  FP32 storage: nb a multiple of 16 up to 144;
// prec 0 = FP32 rebuild / FP64 Gram, 1 = split-BF16 (3 products) for both,
// 2 = split-BF16 (6 products).  FP64 storage: nb = 48, 64, ..., 128, both
// contractions in FP64.
hipError_t launch_wide_f32(int nb, int mode, int prec, int grid, hipStream_t stream,
                           const SolveDesc* descs, const WorkItem* items);
hipError_t launch_wide_f64(int nb, int mode, int grid, hipStream_t stream, const SolveDesc* descs,
                           const WorkItem* items);
bool eig_threads_valid(int ncls, int nt);
int eig_threads(int dtype, int ncls);
bool set_eig_threads(int dtype, int ncls, int nt);
hipError_t launch_eig(int dtype, int ncls, int grid, hipStream_t stream, const SolveDesc* descs,
                      const int32_t* ids);

}  // namespace rpca
