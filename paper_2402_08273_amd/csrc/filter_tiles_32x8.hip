// Filter kernels with 32 x 8 output tiles (all radii, single frame and batch).
#include "filter_kernels.hpp"

namespace ramlt {
namespace filt {

KindKernels kernels_32x8() { return kind_kernels<Shape32x8>(); }

}  // namespace filt
}  // namespace ramlt
