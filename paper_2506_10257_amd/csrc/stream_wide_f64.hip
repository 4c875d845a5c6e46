// Instantiations of the MFMA streaming kernel for FP64 storage: the frame
// classes above the FP64 register classes, 48 to 128 in steps of 16, with
// both contractions on the f64 matrix cores.
#include "stream_wide_impl.h"

namespace rpca {

hipError_t launch_wide_f64(int nb, int mode, int grid, hipStream_t stream, const SolveDesc* descs,
                           const WorkItem* items) {
  if (grid <= 0) return hipSuccess;
  const dim3 g(grid), b(waves_for(nb) * 64);
#define RPCA_WIDE64(N)                                                                         \
  if (nb == N) {                                                                               \
    if (mode == kModeInit)                                                                     \
      RPCA_LAUNCH((k_wide<double, N, kModeInit, 0>), g, b, 0, stream, descs, items);           \
    else if (mode == kModeWarm)                                                                \
      RPCA_LAUNCH((k_wide<double, N, kModeWarm, 0>), g, b, 0, stream, descs, items);           \
    else if (mode == kModeUpdate)                                                              \
      RPCA_LAUNCH((k_wide<double, N, kModeUpdate, 0>), g, b, 0, stream, descs, items);         \
    else                                                                                       \
      RPCA_LAUNCH((k_wide<double, N, kModeFinalize, 0>), g, b, 0, stream, descs, items);       \
    return hipGetLastError();                                                                  \
  }
  RPCA_WIDE64(48) RPCA_WIDE64(64) RPCA_WIDE64(80) RPCA_WIDE64(96) RPCA_WIDE64(112)
  RPCA_WIDE64(128)
#undef RPCA_WIDE64
  return hipErrorInvalidValue;
}

}  // namespace rpca
