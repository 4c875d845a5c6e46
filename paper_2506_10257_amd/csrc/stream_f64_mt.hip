// Instantiations of the register streaming kernels for double storage whose work
// items walk several tiles (RPCA_KNOB_REG_TILES > 1), one per frame class.
#include "launch.h"
#include "stream_impl.h"

namespace rpca {

hipError_t launch_stream_f64_mt(int nb, int mode, int grid, hipStream_t stream,
                                 const SolveDesc* descs, const WorkItem* items) {
  if (grid <= 0) return hipSuccess;
  switch (nb) {
#define X(N) \
  case N:    \
    return launch_stream_class<double, N, true>(mode, grid, stream, descs, items);
    X(4) X(8) X(10) X(12) X(16) X(20) X(24) X(28) X(32)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace rpca
