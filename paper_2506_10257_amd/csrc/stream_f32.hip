// Instantiations of the streaming kernels for float storage (one per frame class).
#include "launch.h"
#include "stream_impl.h"

namespace rpca {

hipError_t launch_stream_f32(int nb, int mode, int grid, hipStream_t stream,
                             const SolveDesc* descs, const WorkItem* items) {
  if (grid <= 0) return hipSuccess;
  const dim3 g(grid), b(kThreads);
  switch (nb) {
#define X(N)                                                                              \
  case N:                                                                                 \
    if (mode == kModeInit)                                                                \
      RPCA_LAUNCH((k_stream<float, N, kModeInit>), g, b, 0, stream, descs, items);       \
    else if (mode == kModeUpdate)                                                         \
      RPCA_LAUNCH((k_stream<float, N, kModeUpdate>), g, b, 0, stream, descs, items);      \
    else if (mode == kModeWarm)                                                           \
      RPCA_LAUNCH((k_stream<float, N, kModeWarm>), g, b, 0, stream, descs, items);     \
    else                                                                                  \
      RPCA_LAUNCH((k_finalize<float, N>), g, b, 0, stream, descs, items);           \
    break;
    X(4) X(8) X(10) X(12) X(16) X(20) X(24) X(28) X(32) X(40) X(48) X(56) X(60) X(64)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rpca
