// Instantiations of the register streaming kernels for double storage, one work
// item per tile (one per frame class); the multi-tile variants are in
// stream_f64_mt.hip.
#include "launch.h"
#include "stream_impl.h"

namespace rpca {

hipError_t launch_stream_f64_mt(int nb, int mode, int grid, hipStream_t stream,
                                 const SolveDesc* descs, const WorkItem* items);

hipError_t launch_stream_f64(int nb, int mode, bool mt, int grid, hipStream_t stream,
                             const SolveDesc* descs, const WorkItem* items) {
  if (grid <= 0) return hipSuccess;
  if (mt) return launch_stream_f64_mt(nb, mode, grid, stream, descs, items);
  switch (nb) {
#define X(N) \
  case N:    \
    return launch_stream_class<double, N, false>(mode, grid, stream, descs, items);
    X(4) X(8) X(10) X(12) X(16) X(20) X(24) X(28) X(32)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace rpca
