// Input scan for values the march cannot use (an optional check before a
// synthesis): non-finite values in any field, kinetic or dust temperatures
// not above zero, negative abundances. One pass over every field, a count
// per workgroup reduced in LDS and added to one device counter.

#include <hip/hip_runtime.h>

#include "device_util.h"
#include "host_common.h"

using namespace iris::host;

namespace iris {
namespace {

struct ScanParams {
  const void* f[5];
  int64_t n;
  int n_fields;
  unsigned long long* count;
};

template <typename FT>
__device__ __forceinline__ bool bad_value(const FT* p, int64_t i, int field) {
  const float v = to_f32(gload(p + i));
  if (!(fabsf(v) <= 3.0e38f)) return true;         // NaN or infinite (or FP32-overflowing)
  if ((field == 1 || field == 4) && !(v > 0.f)) return true;  // T_kin, T_dust > 0
  if (field == 3 && v < 0.f) return true;          // X >= 0
  return false;
}

template <typename FT>
__global__ __launch_bounds__(256) void scan_kernel(const ScanParams P) {
  __shared__ unsigned int part[256];
  unsigned int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int fld = 0; fld < P.n_fields; ++fld) {
    const FT* p = (const FT*)P.f[fld];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += stride)
      bad += bad_value(p, i, fld) ? 1u : 0u;
  }
  part[threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && part[0]) atomicAdd(P.count, (unsigned long long)part[0]);
}

template <typename FT>
void launch_scan(const ScanParams& P, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((P.n + 255) / 256, 4096);
  hipLaunchKernelGGL(scan_kernel<FT>, dim3((unsigned)blocks), dim3(256), 0, st, P);
}

}  // namespace
}  // namespace iris

extern "C" {

iris_status iris_rt_check_fields(const iris_fields* fields, void* scratch, size_t scratch_bytes,
                                 void* stream, int64_t* bad) {
  clear_error();
  Geo g;
  iris_status s = check_fields(fields, &g);
  if (s != IRIS_OK) return s;
  if (!bad) return fail(IRIS_E_INVALID_ARG, "bad-count pointer is NULL");
  if (!scratch || scratch_bytes < 8)
    return fail(IRIS_E_WORKSPACE, "the scan needs 8 bytes of device scratch");
  iris::ScanParams P{};
  const void* src[5] = {fields->ln_nh2, fields->t_kin, fields->v_los, fields->x_tracer,
                        fields->t_dust};
  for (int i = 0; i < 5; ++i) P.f[i] = src[i];
  P.n = g.n_cells;
  P.n_fields = g.n_fields;
  P.count = (unsigned long long*)scratch;
  const hipStream_t st = (hipStream_t)stream;
  unsigned long long zero = 0;
  int e = (int)hipMemcpyAsync(scratch, &zero, 8, hipMemcpyHostToDevice, st);
  if (e) return hip_status(e, "scan counter reset");
  switch (fields->dtype) {
    case IRIS_F64: iris::launch_scan<double>(P, st); break;
    case IRIS_F32: iris::launch_scan<float>(P, st); break;
    case IRIS_BF16: iris::launch_scan<iris::bf16_t>(P, st); break;
    case IRIS_F16: iris::launch_scan<_Float16>(P, st); break;
  }
  e = (int)hipGetLastError();
  if (e) return hip_status(e, "scan kernel");
  unsigned long long n = 0;
  e = (int)hipMemcpyAsync(&n, scratch, 8, hipMemcpyDeviceToHost, st);
  if (!e) e = (int)hipStreamSynchronize(st);
  if (e) return hip_status(e, "scan count");
  *bad = (int64_t)n;
  if (n) return fail(IRIS_E_NONFINITE, "%llu field values are non-finite or out of range", n);
  return IRIS_OK;
}

}  // extern "C"
