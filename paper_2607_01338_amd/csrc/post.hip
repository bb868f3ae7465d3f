// Post-transfer products of PPV cubes: Gaussian beam convolution over the two
// sky axes (paper, "Beam Convolution") and the l,v mean projection over one
// sky axis (the l,v panels of the paper's figures). Cubes are FP32
// [n1][n2][n_chan], channel fastest.
//
// The beam is separable: one pass along n2 into a workspace, one along n1 into
// the output. A lane computes a run of four consecutive positions along the
// pass axis for four channels (16-byte accesses when the rows allow it), so
// that the 2R + 1 taps of the run share 4 + 2R loads; each XCD takes a
// contiguous range of the work, so that rows re-read by neighbouring runs hit
// in its L2. Both passes are bound by HBM: each reads and writes the cube once.

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

// Positions along the pass axis handled by one lane: the 2R + 1 taps of
// kBeamRun consecutive outputs share kBeamRun + 2R loads.
constexpr int kBeamRun = 4;

template <int V>
__global__ __launch_bounds__(256) void beam_pass_kernel(const BeamArgs a) {
  using T = typename std::conditional<V == 4, float4, float>::type;
  const int64_t nv = a.C / V;
  const int64_t n_axis = a.axis == 1 ? a.n2 : a.n1;
  const int64_t n_runs = (n_axis + kBeamRun - 1) / kBeamRun;
  const int64_t n_other = a.axis == 1 ? a.n1 : a.n2;
  const int64_t total = n_other * n_runs * nv;
  const int64_t stride = (a.axis == 1 ? a.C : a.n2 * a.C) / V;
  const T* in = (const T*)a.in;
  T* out = (T*)a.out;
  // One run of outputs per lane, columns fastest; each XCD takes a contiguous
  // range of the work, so that the rows a tap re-reads were loaded into the
  // same L2.
  const int64_t e = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t col = e % nv, t = e / nv;
  const int64_t run = t % n_runs, other = t / n_runs;
  const int64_t pos0 = run * kBeamRun;
  // Element (p1, p2, col) sits at (p1 n2 + p2) nv + col.
  const int64_t e0 = (a.axis == 1 ? other * a.n2 + pos0 : pos0 * a.n2 + other) * nv + col;
  const int jlo = (int)max((int64_t)-a.R, -pos0);
  const int jhi = (int)min((int64_t)(kBeamRun - 1 + a.R), n_axis - 1 - pos0);
  float acc[kBeamRun][V] = {};
  for (int j = jlo; j <= jhi; ++j) {
    const T v = gload(in + e0 + j * stride);
#pragma unroll
    for (int m = 0; m < kBeamRun; ++m) {
      const int d = j - m < 0 ? m - j : j - m;
      if (d <= a.R) {
        const float w = a.w[d];
        if constexpr (V == 4) {
          acc[m][0] = fmaf(w, v.x, acc[m][0]);
          acc[m][1] = fmaf(w, v.y, acc[m][1]);
          acc[m][2] = fmaf(w, v.z, acc[m][2]);
          acc[m][3] = fmaf(w, v.w, acc[m][3]);
        } else {
          acc[m][0] = fmaf(w, v, acc[m][0]);
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < kBeamRun; ++m) {
    if (pos0 + m < n_axis) {
      if constexpr (V == 4)
        gstore(out + e0 + m * stride, make_float4(acc[m][0], acc[m][1], acc[m][2], acc[m][3]));
      else
        gstore(out + e0 + m * stride, acc[m][0]);
    }
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
  // Work items of a pass: the other axis x runs of kBeamRun positions x columns.
  auto blocks_for = [&](int64_t n_axis, int64_t n_other) {
    return ((n_axis + kBeamRun - 1) / kBeamRun * n_other * (n_chan / V) + 255) / 256;
  };
  const int64_t b2 = blocks_for(n2, n1), b1 = blocks_for(n1, n2);
  if (std::max(b1, b2) > 0x7FFFFFFF)
    return host::fail(IRIS_E_UNSUPPORTED, "cube too large for one launch");
  // Along n2 into the workspace, then along n1 into the output.
  a.in = cube;
  a.out = (float*)workspace;
  a.axis = 1;
  if (v4) hipLaunchKernelGGL(beam_pass_kernel<4>, dim3((int)b2), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(beam_pass_kernel<1>, dim3((int)b2), dim3(256), 0, st, a);
  a.in = (const float*)workspace;
  a.out = out;
  a.axis = 0;
  if (v4) hipLaunchKernelGGL(beam_pass_kernel<4>, dim3((int)b1), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(beam_pass_kernel<1>, dim3((int)b1), dim3(256), 0, st, a);
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
