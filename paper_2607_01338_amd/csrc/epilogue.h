// Output rows of one sightline, shared by the march kernels: the five
// components in the requested units ("Intensity Versus Temperature") and,
// with velocity subsampling, each channel's composite-Simpson average of its
// marched velocities ("Transfer Solution: Optically Thick Transfer").
#pragma once

#include "device_util.h"

namespace iris {

// `psi` (LDS, one float per marched velocity) times `fs` is the line excess
// [L] in output units (in Rayleigh-Jeans kelvin for Planck brightness
// temperature units). Crj is the continuum [C] in Rayleigh-Jeans kelvin;
// Dout and Bout are [D] and [B] in Rayleigh-Jeans kelvin. The W lanes of the
// sightline's group write; `sl` is the lane within the group. [T] = [C] +
// [L], in intensity space, then converted: a common factor (intensity), or
// the Planck brightness temperature of [T], [C] and [B].
template <int W>
__device__ __forceinline__ void write_outputs(const Folded& c, float* const* out, int64_t pix,
                                              const float* psi, int sl, float fs, float Crj,
                                              double Dout, double Bout) {
  const bool tb = c.units == IRIS_UNITS_TB;
  const float os = c.out_scale, T0 = c.T0;
  auto planck_tb = [T0](float trj) { return trj > 0.f ? T0 / log1pf(T0 / trj) : 0.f; };
  const float Cf = tb ? planck_tb(Crj) : Crj * os;
  const float Df = (float)Dout * os;
  const float Bf = tb ? planck_tb((float)Bout) : (float)Bout * os;
  const int CO = c.n_out;
  float* oT = out[0] ? out[0] + pix * CO : nullptr;
  float* oC = out[1] ? out[1] + pix * CO : nullptr;
  float* oD = out[2] ? out[2] + pix * CO : nullptr;
  float* oL = out[3] ? out[3] + pix * CO : nullptr;
  float* oB = out[4] ? out[4] + pix * CO : nullptr;
  // [T] from the line excess d (already in output units unless tb).
  auto total = [&](float d) { return tb ? planck_tb(Crj + d) : fmaf(Crj, os, d); };
  if (c.simpson_f > 0) {
    // Velocity subsampling: channel k is the composite-Simpson average of
    // the 2f + 1 marched velocities 2fk .. 2f(k+1) (1 4 2 4 ... 4 1 / 6f).
    // The continuum is flat across a channel, so only the excess averages.
    const int f2 = 2 * c.simpson_f;
    const float w1 = 1.f / (3.f * (float)f2), w4 = 4.f * w1, w2 = 2.f * w1;
    for (int k = sl; k < CO; k += W) {
      const float* q = psi + f2 * k;
      float acc = (q[0] + q[f2]) * w1;
      for (int i = 1; i < f2; ++i) acc = fmaf(q[i], (i & 1) ? w4 : w2, acc);
      const float d = acc * fs;
      if (oT) gstore(oT + k, total(d));
      if (oC) gstore(oC + k, Cf);
      if (oD) gstore(oD + k, Df);
      if (oL) gstore(oL + k, d);
      if (oB) gstore(oB + k, Bf);
    }
    return;
  }
  const int C = c.n_chan;
  uintptr_t low = (uintptr_t)C;
#pragma unroll
  for (int j = 0; j < 5; ++j) low |= (uintptr_t)out[j];
  if ((low & 15) == 0 && (C & 3) == 0) {
    // Four channels per lane and 16-byte stores when the rows allow it.
    const float4 c4 = make_float4(Cf, Cf, Cf, Cf);
    const float4 d4 = make_float4(Df, Df, Df, Df);
    const float4 b4 = make_float4(Bf, Bf, Bf, Bf);
    for (int k = 4 * sl; k < C; k += 4 * W) {
      const float4 q = *(const float4*)(psi + k);
      const float4 d = make_float4(q.x * fs, q.y * fs, q.z * fs, q.w * fs);
      if (oT) gstore((float4*)(oT + k), make_float4(total(d.x), total(d.y), total(d.z), total(d.w)));
      if (oC) gstore((float4*)(oC + k), c4);
      if (oD) gstore((float4*)(oD + k), d4);
      if (oL) gstore((float4*)(oL + k), d);
      if (oB) gstore((float4*)(oB + k), b4);
    }
    return;
  }
  for (int k = sl; k < C; k += W) {
    const float d = psi[k] * fs;
    if (oT) gstore(oT + k, total(d));
    if (oC) gstore(oC + k, Cf);
    if (oD) gstore(oD + k, Df);
    if (oL) gstore(oL + k, d);
    if (oB) gstore(oB + k, Bf);
  }
}

}  // namespace iris
