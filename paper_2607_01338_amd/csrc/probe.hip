// Issue-rate probes behind the roofline figures: independent chains of the
// hardware base-2 exponential (v_exp_f32) and of FP32 FMAs, eight per lane,
// over a grid that fills the device. Diagnostics only: not on the synthesis
// path.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "host_common.h"

namespace iris {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeIters = 4096;

__global__ __launch_bounds__(256) void probe_exp_kernel(float* out) {
  float x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = threadIdx.x * 1e-3f + 0.1f * j;
  for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = __builtin_amdgcn_exp2f(-x[j]);  // negation is free
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void probe_fma_kernel(float* out, float a) {
  float x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = threadIdx.x * 1e-3f + 0.1f * j;
  for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = fmaf(x[j], a, 0.5f);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace
}  // namespace iris

using namespace iris::host;

extern "C" iris_status iris_probe_issue_rates(double* exp_per_s, double* fma_per_s) {
  clear_error();
  if (!exp_per_s || !fma_per_s) return fail(IRIS_E_INVALID_ARG, "output pointer is NULL");
  int dev = 0, n_cu = 0;
  iris_status s;
  if ((s = hip_status(hipGetDevice(&dev), "hipGetDevice")) != IRIS_OK) return s;
  if ((s = hip_status(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev),
                      "hipDeviceGetAttribute")) != IRIS_OK)
    return s;
  const int blocks = n_cu * 16;
  float* out = nullptr;
  if ((s = hip_status(hipMalloc(&out, (size_t)blocks * iris::kProbeThreads * sizeof(float)),
                      "hipMalloc (probe)")) != IRIS_OK)
    return s;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  s = hip_status(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
  if (s == IRIS_OK) s = hip_status(hipEventCreate(&e0), "hipEventCreate");
  if (s == IRIS_OK) s = hip_status(hipEventCreate(&e1), "hipEventCreate");
  const double ops = (double)blocks * iris::kProbeThreads * iris::kProbeIters * 8;
  double best[2] = {0.0, 0.0};
  for (int which = 0; which < 2 && s == IRIS_OK; ++which) {
    for (int rep = 0; rep < 4 && s == IRIS_OK; ++rep) {  // the first run warms up
      s = hip_status(hipEventRecord(e0, st), "hipEventRecord");
      if (s != IRIS_OK) break;
      if (which == 0)
        hipLaunchKernelGGL(iris::probe_exp_kernel, dim3(blocks), dim3(iris::kProbeThreads), 0, st,
                           out);
      else
        hipLaunchKernelGGL(iris::probe_fma_kernel, dim3(blocks), dim3(iris::kProbeThreads), 0,
                           st, out, 0.999f);
      s = hip_status(hipGetLastError(), "probe kernel");
      if (s == IRIS_OK) s = hip_status(hipEventRecord(e1, st), "hipEventRecord");
      if (s == IRIS_OK) s = hip_status(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      if (s == IRIS_OK) s = hip_status(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      if (s == IRIS_OK && rep > 0 && ms > 0.f) best[which] = std::max(best[which], ops / (ms * 1e-3));
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  (void)hipFree(out);
  if (s == IRIS_OK) {
    *exp_per_s = best[0];
    *fma_per_s = best[1];
  }
  return s;
}
