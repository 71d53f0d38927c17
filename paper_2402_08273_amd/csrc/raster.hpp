// Raster map of the screen-space lens chains, shared by the chain step (perturb.hip) and
// the chain reorder (chains.hip), so that both take every pixel decision the same way.
#pragma once

#include <hip/hip_runtime.h>

namespace ramlt {

// Raster position of a primary ray direction of a pinhole camera looking along +z, in
// canonical screen space: sx = 1/2 + (1/2) (x / z) / tx, sy likewise with ty; in the frame
// iff z > 0 and sx, sy in [0, 1). Every operation rounds to nearest on its own (no fused
// multiply-add), so the pixel and every decision taken from it are reproducible one IEEE
// operation at a time.
struct Raster {
  bool inside;
  int ix, iy;
};

__device__ __forceinline__ Raster raster_of(float wx, float wy, float wz, float tx, float ty, int W, int H) {
  // HIP's *_rn helpers are plain operators here: the pragma keeps the compiler from fusing
  // a product into the following sum
#pragma clang fp contract(off)
  const float sx = __fadd_rn(0.5f, __fmul_rn(0.5f, __fdiv_rn(__fdiv_rn(wx, wz), tx)));
  const float sy = __fadd_rn(0.5f, __fmul_rn(0.5f, __fdiv_rn(__fdiv_rn(wy, wz), ty)));
  Raster r;
  r.inside = wz > 0.0f && sx >= 0.0f && sx < 1.0f && sy >= 0.0f && sy < 1.0f;
  r.ix = r.inside ? min((int)__fmul_rn(sx, (float)W), W - 1) : 0;
  r.iy = r.inside ? min((int)__fmul_rn(sy, (float)H), H - 1) : 0;
  return r;
}

}  // namespace ramlt
