// One frame's differentiable step in one call: the statistics pass (Appendix A), the forward
// filter with the MSE seed and the parameter adjoint (Sec. 3.1 eq. path_integral,
// Sec. 5.2-5.3) and the radiance adjoint, enqueued in that order on the caller's stream.
// The kernels, tiles and per-tile partial slots are those of stats_accumulate,
// filter_forward and filter_backward, so every output is bit for bit what those three calls
// give in sequence.
//
// A form that ran the filter on a second stream behind each statistics launch, on the tile
// rows whose windows those launches had completed, measured slower at 1920 x 1080 x 64 spp
// (1.035 ms against 0.949 ms per step on MI355X): every hand-off between the streams left
// a ~6.5 us gap between statistics launches, and the filter's workgroups, sharing the
// compute units with the statistics pass, lengthened each of its launches by ~6 us while
// running 5x slower themselves, so most of the filter's time was not hidden.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace ramlt {

hipError_t launch_step(const ramlt_frame &f, void *ws, hipStream_t st) {
  hipError_t e = launch_stats(&f, nullptr, 1, nullptr, st);
  if (e != hipSuccess) return e;
  e = launch_filter_forward(&f, nullptr, 1, ws, st);
  if (e != hipSuccess) return e;
  return launch_filter_backward(&f, nullptr, 1, ws, st);
}

}  // namespace ramlt
