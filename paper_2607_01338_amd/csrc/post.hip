// Post-transfer products of PPV cubes: Gaussian beam convolution over the two
// sky axes (paper, "Beam Convolution") and the l,v mean projection over one
// sky axis (the l,v panels of the paper's figures). Cubes are FP32
// [n1][n2][n_chan], channel fastest.
//
// The beam is separable: one pass along n2 into a workspace, one along n1 into
// the output; both read four channels per lane (16-byte loads) when the rows
// allow it, so that every tap of a wavefront reads whole cache lines and the
// 2R + 1 taps of neighbouring pixels hit in L2. Both passes are bound by HBM:
// each reads and writes the cube once.

#include <hip/hip_runtime.h>

#include <cmath>

#include "device_util.h"
#include "host_common.h"

namespace iris {
namespace {

constexpr int kBeamMaxRadius = 128;

struct BeamArgs {
  const float* in;
  float* out;
  int64_t n1, n2, C;
  int32_t axis;  // 1: along n2 (stride C), 0: along n1 (stride n2 C)
  int32_t R;
  float w[kBeamMaxRadius + 1];  // w[|offset|], unit sum over -R..R
};

template <int V>
__global__ __launch_bounds__(256) void beam_pass_kernel(const BeamArgs a) {
  using T = typename std::conditional<V == 4, float4, float>::type;
  const int64_t nv = a.C / V;
  const int64_t total = a.n1 * a.n2 * nv;
  const int64_t stride = (a.axis == 1 ? a.C : a.n2 * a.C) / V;
  const int64_t n_axis = a.axis == 1 ? a.n2 : a.n1;
  const T* in = (const T*)a.in;
  T* out = (T*)a.out;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / nv;  // pixel index p1 * n2 + p2
    const int64_t pos = a.axis == 1 ? row % a.n2 : row / a.n2;
    const int lo = (int)max((int64_t)-a.R, -pos), hi = (int)min((int64_t)a.R, n_axis - 1 - pos);
    float acc[V] = {};
    for (int j = lo; j <= hi; ++j) {
      const T v = gload(in + e + j * stride);
      const float w = a.w[j < 0 ? -j : j];
      if constexpr (V == 4) {
        acc[0] = fmaf(w, v.x, acc[0]);
        acc[1] = fmaf(w, v.y, acc[1]);
        acc[2] = fmaf(w, v.z, acc[2]);
        acc[3] = fmaf(w, v.w, acc[3]);
      } else {
        acc[0] = fmaf(w, v, acc[0]);
      }
    }
    if constexpr (V == 4)
      gstore(out + e, make_float4(acc[0], acc[1], acc[2], acc[3]));
    else
      gstore(out + e, acc[0]);
  }
}

// Mean over sky axis `axis` of [n1][n2][C]: out [n_other][C], FP64 sums.
template <int V>
__global__ __launch_bounds__(256) void lv_mean_kernel(const float* cube, float* outp, int64_t n1,
                                                      int64_t n2, int64_t C, int axis) {
  using T = typename std::conditional<V == 4, float4, float>::type;
  const int64_t nv = C / V;
  const int64_t n_other = axis == 0 ? n2 : n1;
  const int64_t n_axis = axis == 0 ? n1 : n2;
  const int64_t total = n_other * nv;
  const T* in = (const T*)cube;
  T* out = (T*)outp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = e / nv, k = e % nv;
    // Element (p1, p2, k) sits at (p1 n2 + p2) nv + k.
    const int64_t base = (axis == 0 ? o : o * n2) * nv + k;
    const int64_t step = (axis == 0 ? n2 : 1) * nv;
    double acc[V] = {};
    for (int64_t i = 0; i < n_axis; ++i) {
      const T v = gload(in + base + i * step);
      if constexpr (V == 4) {
        acc[0] += v.x;
        acc[1] += v.y;
        acc[2] += v.z;
        acc[3] += v.w;
      } else {
        acc[0] += v;
      }
    }
    const double s = 1.0 / (double)n_axis;
    if constexpr (V == 4)
      gstore(out + e, make_float4((float)(acc[0] * s), (float)(acc[1] * s), (float)(acc[2] * s),
                                  (float)(acc[3] * s)));
    else
      gstore(out + e, (float)(acc[0] * s));
  }
}

int grid_for(int64_t work) {
  const int64_t b = (work + 255) / 256;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 256 * 64);
}

bool aligned4(const void* p, int64_t C) { return ((uintptr_t)p & 15) == 0 && (C & 3) == 0; }

iris_status check_cube(const float* cube, const float* out, int32_t n1, int32_t n2,
                       int32_t n_chan) {
  if (!cube || !out) return host::fail(IRIS_E_INVALID_ARG, "cube or output is NULL");
  if (n1 < 1 || n2 < 1 || n_chan < 1)
    return host::fail(IRIS_E_INVALID_ARG, "need n1, n2, n_chan >= 1 (got %d, %d, %d)", n1, n2,
                      n_chan);
  return IRIS_OK;
}

}  // namespace
}  // namespace iris

using namespace iris;

extern "C" {

size_t iris_beam_workspace_bytes(int32_t n1, int32_t n2, int32_t n_chan) {
  if (n1 < 1 || n2 < 1 || n_chan < 1) return 0;
  return (size_t)n1 * n2 * n_chan * sizeof(float);
}

iris_status iris_beam_convolve(const float* cube, float* out, int32_t n1, int32_t n2,
                               int32_t n_chan, double fwhm_pix, void* workspace,
                               size_t workspace_bytes, void* stream) {
  host::clear_error();
  iris_status s = check_cube(cube, out, n1, n2, n_chan);
  if (s != IRIS_OK) return s;
  if (!(fwhm_pix > 0.0) || !std::isfinite(fwhm_pix))
    return host::fail(IRIS_E_INVALID_ARG, "fwhm_pix must be > 0");
  const double sigma = fwhm_pix / (2.0 * std::sqrt(2.0 * std::log(2.0)));
  const double rr = std::ceil(4.0 * sigma);
  if (rr > kBeamMaxRadius)
    return host::fail(IRIS_E_UNSUPPORTED, "beam radius %.0f pixels above %d (fwhm_pix %g)", rr,
                      kBeamMaxRadius, fwhm_pix);
  const size_t need = iris_beam_workspace_bytes(n1, n2, n_chan);
  if (!workspace || workspace_bytes < need)
    return host::fail(IRIS_E_WORKSPACE, "beam workspace needs %zu bytes, got %zu", need,
                      workspace_bytes);
  BeamArgs a{};
  a.n1 = n1;
  a.n2 = n2;
  a.C = n_chan;
  a.R = (int32_t)rr;
  double wsum = 0.0, wd[kBeamMaxRadius + 1];
  for (int i = 0; i <= a.R; ++i) {
    wd[i] = std::exp(-(double)i * i / (2.0 * sigma * sigma));
    wsum += i ? 2.0 * wd[i] : wd[i];
  }
  for (int i = 0; i <= a.R; ++i) a.w[i] = (float)(wd[i] / wsum);
  const hipStream_t st = (hipStream_t)stream;
  const bool v4 = aligned4(cube, n_chan) && aligned4(out, n_chan) && aligned4(workspace, n_chan);
  const int V = v4 ? 4 : 1;
  const int blocks = grid_for((int64_t)n1 * n2 * n_chan / V);
  // Along n2 into the workspace, then along n1 into the output.
  a.in = cube;
  a.out = (float*)workspace;
  a.axis = 1;
  if (v4) hipLaunchKernelGGL(beam_pass_kernel<4>, dim3(blocks), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(beam_pass_kernel<1>, dim3(blocks), dim3(256), 0, st, a);
  a.in = (const float*)workspace;
  a.out = out;
  a.axis = 0;
  if (v4) hipLaunchKernelGGL(beam_pass_kernel<4>, dim3(blocks), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(beam_pass_kernel<1>, dim3(blocks), dim3(256), 0, st, a);
  return host::hip_status((int)hipGetLastError(), "beam kernel");
}

iris_status iris_lv_mean(const float* cube, float* out, int32_t n1, int32_t n2, int32_t n_chan,
                         int32_t axis, void* stream) {
  host::clear_error();
  iris_status s = check_cube(cube, out, n1, n2, n_chan);
  if (s != IRIS_OK) return s;
  if (axis != 0 && axis != 1) return host::fail(IRIS_E_INVALID_ARG, "axis must be 0 or 1");
  const int64_t n_other = axis == 0 ? n2 : n1;
  const bool v4 = aligned4(cube, n_chan) && aligned4(out, n_chan);
  const hipStream_t st = (hipStream_t)stream;
  if (v4)
    hipLaunchKernelGGL(lv_mean_kernel<4>, dim3(grid_for(n_other * n_chan / 4)), dim3(256), 0, st,
                       cube, out, (int64_t)n1, (int64_t)n2, (int64_t)n_chan, (int)axis);
  else
    hipLaunchKernelGGL(lv_mean_kernel<1>, dim3(grid_for(n_other * n_chan)), dim3(256), 0, st,
                       cube, out, (int64_t)n1, (int64_t)n2, (int64_t)n_chan, (int)axis);
  return host::hip_status((int)hipGetLastError(), "l,v mean kernel");
}

}  // extern "C"
