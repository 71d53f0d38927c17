// Filter kernels with 32 x 16 output tiles (all radii, single frame and batch).
#include "filter_kernels.hpp"

namespace ramlt {
namespace filt {

KindKernels kernels_32x16() { return kind_kernels<Shape32x16>(); }

}  // namespace filt
}  // namespace ramlt
