// Instantiations of the MFMA streaming kernel for FP32 storage: frame
// classes 16 to 144 in steps of 16, plain FP32 and both split-BF16 modes.
#include "stream_wide_impl.h"

namespace rpca {

hipError_t launch_wide_f32(int nb, int mode, int prec, int grid, hipStream_t stream,
                           const SolveDesc* descs, const WorkItem* items) {
  if (grid <= 0) return hipSuccess;
  const dim3 g(grid), b(waves_for(nb) * 64);
#define RPCA_WIDE(N, P)                                                                        \
  if (nb == N && prec == P) {                                                                  \
    if (mode == kModeInit)                                                                     \
      RPCA_LAUNCH((k_wide<float, N, kModeInit, P>), g, b, 0, stream, descs, items);            \
    else if (mode == kModeWarm)                                                                \
      RPCA_LAUNCH((k_wide<float, N, kModeWarm, P>), g, b, 0, stream, descs, items);            \
    else if (mode == kModeUpdate)                                                              \
      RPCA_LAUNCH((k_wide<float, N, kModeUpdate, P>), g, b, 0, stream, descs, items);          \
    else                                                                                       \
      RPCA_LAUNCH((k_wide<float, N, kModeFinalize, P>), g, b, 0, stream, descs, items);        \
    return hipGetLastError();                                                                  \
  }
  RPCA_WIDE(16, 0) RPCA_WIDE(32, 0) RPCA_WIDE(48, 0) RPCA_WIDE(64, 0)
  RPCA_WIDE(80, 0) RPCA_WIDE(96, 0) RPCA_WIDE(112, 0) RPCA_WIDE(128, 0) RPCA_WIDE(144, 0)
  RPCA_WIDE(16, 1) RPCA_WIDE(32, 1) RPCA_WIDE(48, 1) RPCA_WIDE(64, 1)
  RPCA_WIDE(80, 1) RPCA_WIDE(96, 1) RPCA_WIDE(112, 1) RPCA_WIDE(128, 1) RPCA_WIDE(144, 1)
  RPCA_WIDE(16, 2) RPCA_WIDE(32, 2) RPCA_WIDE(48, 2) RPCA_WIDE(64, 2)
  RPCA_WIDE(80, 2) RPCA_WIDE(96, 2) RPCA_WIDE(112, 2) RPCA_WIDE(128, 2) RPCA_WIDE(144, 2)
#undef RPCA_WIDE
  return hipErrorInvalidValue;
}

}  // namespace rpca
