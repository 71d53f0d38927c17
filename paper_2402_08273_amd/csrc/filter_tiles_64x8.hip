// Filter kernels with 64 x 8 output tiles (all radii, single frame and batch).
#include "filter_kernels.hpp"

namespace ramlt {
namespace filt {

KindKernels kernels_64x8() { return kind_kernels<Shape64x8>(); }

}  // namespace filt
}  // namespace ramlt
