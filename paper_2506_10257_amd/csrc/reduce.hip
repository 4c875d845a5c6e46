// First level of the fixed-order reduction of the streaming pass's partial
// sums: one workgroup per (solve, group of kGroup slots) adds the group's
// slots in slot order.  The eigensolve kernel adds the group sums in group
// order.  Running it as its own launch (instead of a last-arriving-workgroup
// scheme inside the streaming kernel) keeps device-scope fences, and the L2
// write-backs they imply, out of the streaming pass.
#include "common.h"
#include "launch.h"

namespace rpca {
namespace {

__global__ void __launch_bounds__(kThreads)
k_reduce_groups(const SolveDesc* __restrict__ descs, const GroupItem* __restrict__ items) {
  const GroupItem gi = items[blockIdx.x];
  const SolveDesc& d = descs[gi.solve];
  if (d.st->done) return;
  const int nent = kScalars + gram_blocks((d.n + 3) >> 2) * 16;
  const int lo = gi.group * kGroup;
  const int cnt = min(kGroup, d.slots - lo);
  const double* src = d.partials + static_cast<size_t>(lo) * d.pstride;
  double* dst = d.gpartials + static_cast<size_t>(gi.group) * d.pstride;
  for (int idx = threadIdx.x; idx < nent; idx += kThreads) {
    double v[kGroup];
#pragma unroll
    for (int q = 0; q < kGroup; ++q)
      v[q] = q < cnt ? src[static_cast<size_t>(q) * d.pstride + idx] : 0.0;
    double sum = v[0];
#pragma unroll
    for (int q = 1; q < kGroup; ++q)
      if (q < cnt) sum += v[q];
    dst[idx] = sum;
  }
}

// Copy the state of every solve of a plan to one contiguous array (read back
// by the host with a single copy).
__global__ void __launch_bounds__(64)
k_gather_states(const SolveDesc* __restrict__ descs, int count, SolveState* __restrict__ out) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i < count) out[i] = *descs[i].st;
}

// Zero the state of every solve of a plan (done before its init pass).
__global__ void __launch_bounds__(64)
k_reset_states(const SolveDesc* __restrict__ descs, int count) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i < count) {
    SolveState z{};
    *descs[i].st = z;
  }
}

}  // namespace

hipError_t launch_gather_states(int count, hipStream_t stream, const SolveDesc* descs,
                                SolveState* out) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_states, dim3((count + 63) / 64), dim3(64), 0, stream, descs, count, out);
  return hipGetLastError();
}

hipError_t launch_reset_states(int count, hipStream_t stream, const SolveDesc* descs) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reset_states, dim3((count + 63) / 64), dim3(64), 0, stream, descs, count);
  return hipGetLastError();
}

hipError_t launch_reduce(int grid, hipStream_t stream, const SolveDesc* descs,
                         const GroupItem* items) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_groups, dim3(grid), dim3(kThreads), 0, stream, descs, items);
  return hipGetLastError();
}

}  // namespace rpca
