// erfc on [0, 6) from cubic Hermite pieces staged in LDS, shared by the
// kernels that evaluate channel averages of the Gaussian line profile
// (optically thin and selectively thin transfer). The pieces are built in
// FP64 by erfc_table_kernel (values and derivatives, -2/sqrt(pi) e^{-x^2},
// at both ends of each piece); 512 pieces of width 6/512 leave an
// interpolation error below 1e-9, under the FP32 rounding of the result.
// Beyond 6, erfc < 3e-17 is taken as zero.
#pragma once

#include "device_util.h"

namespace iris {

constexpr int kErfcN = 512;          // Hermite pieces of erfc on [0, kErfcMax)
constexpr float kErfcMax = 6.f;

// erfc(ax) for ax >= 0 from the staged table.
__device__ __forceinline__ float erfc_tab(const float4* etab, float ax) {
  const float u = ax * ((float)kErfcN / kErfcMax);
  const float fi = fminf(floorf(u), (float)(kErfcN - 1));
  const float s = u - fi;
  const float4 q = etab[(int)fi];
  const float f = fmaf(fmaf(fmaf(q.w, s, q.z), s, q.y), s, q.x);
  return u < (float)kErfcN ? f : 0.f;
}

}  // namespace iris
