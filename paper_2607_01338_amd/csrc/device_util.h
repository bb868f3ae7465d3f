// Device helpers for the gfx950 kernels: field loads, wavefront scans and
// lane broadcasts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "iris_internal.h"

namespace iris {

constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kLn2 = 0.69314718055994530942f;
constexpr float kSqrtLog2e = 1.20112240878644981f;  // sqrt(log2(e))

// Hardware base-2 exponential (v_exp_f32).
__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

// Loads and stores of device memory through global-address-space pointers.
// Pointers read from memory (a plan's per-cube parameters) are generic, and
// generic (flat) accesses also count against the LDS wait counter, which
// would tie every LDS wait of the march to the outstanding field loads.
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
typedef float gv4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 gload(const float4* p) {
  const gv4f v = *(const __attribute__((address_space(1))) gv4f*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstore(float4* p, float4 x) {
  const gv4f v = {x.x, x.y, x.z, x.w};
  *(__attribute__((address_space(1))) gv4f*)p = v;
}
typedef float gv2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 gload(const float2* p) {
  const gv2f v = *(const __attribute__((address_space(1))) gv2f*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ bf16_t gload(const bf16_t* p) {
  bf16_t r;
  r.bits = gload((const uint16_t*)p);
  return r;
}

// 1 - e^{-x} for x >= 0 with a relative error of a few ulp: the Taylor
// series to x^6 below 1/4 (truncation x^6/7! relative), 1 - 2^{-x log2 e}
// above, where no cancellation occurs.
__device__ __forceinline__ float one_minus_exp_neg_small(float x) {  // 0 <= x < 1/4
  float q = fmaf(-x, 1.f / 720.f, 1.f / 120.f);
  q = fmaf(-x, q, 1.f / 24.f);
  q = fmaf(-x, q, 1.f / 6.f);
  q = fmaf(-x, q, 0.5f);
  q = fmaf(-x, q, 1.f);
  return x * q;
}
__device__ __forceinline__ float one_minus_exp_neg(float x) {
  const float big = 1.f - ex2(-x * kLog2e);
  return x < 0.25f ? one_minus_exp_neg_small(x) : big;
}

// Tile of workgroup b in a grid of nb: workgroups are dispatched to the 8
// XCDs round-robin (b mod 8), so giving each XCD a contiguous range of tiles
// keeps neighbouring sightlines, which share cache lines of the native field
// layout, on one L2. A bijection of [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  constexpr int kXcds = 8;
  const int q = nb / kXcds, r = nb % kXcds, x = b % kXcds;
  return x * q + min(x, r) + b / kXcds;
}

// Work claiming of a persistent launch over kSlices queue slices (workgroup
// b serves slice b mod kSlices, whose XCD it runs on).
//  * With `rounds` set (a launch that runs alone with every workgroup
//    resident) a slice of n items gives per * (n / per) of them out in static
//    rounds: wavefront rank r takes r, r + per, ... (per = the slice's
//    wavefronts; items are sorted by cost, so round-robin shares are even).
//    No atomics, so no bursts of them when every item costs the same.
//  * The rest of the slice (all of it without `rounds`) is claimed one atomic
//    per item, first by the slice's own wavefronts, then by any wavefront
//    whose slice is done.
// Every wavefront ends after at most kSlices failed claims. Requires
// gridDim.x to be a multiple of kSlices; `counter` (kSlices heads) is zero at
// launch.
struct ItemClaim {
  int x0, rank, per, round, tried;
  bool rounds;
  __device__ __forceinline__ ItemClaim(int waves_per_block, int wave, bool static_rounds) {
    x0 = (int)(blockIdx.x % kSlices);
    per = (int)(gridDim.x / kSlices) * waves_per_block;
    rank = (int)(blockIdx.x / kSlices) * waves_per_block + wave;
    round = 0;
    tried = 0;
    rounds = static_rounds;
  }
  __device__ __forceinline__ int static_items(int n) const { return rounds ? per * (n / per) : 0; }
  // Next item index, or -1 when every slice is drained.
  __device__ __forceinline__ int next(const int32_t* begin, int* counter) {
    if (per * round < static_items(begin[x0 + 1] - begin[x0]))
      return begin[x0] + rank + per * round++;
    while (tried < kSlices) {
      const int x = (x0 + tried) % kSlices;
      const int n = begin[x + 1] - begin[x];
      const int tail = n - static_items(n);
      int k = tail;
      if (tail > 0 && (threadIdx.x & 63) == 0) k = atomicAdd(&counter[x], 1);
      k = __builtin_amdgcn_readfirstlane(k);
      if (k < tail) return begin[x] + (n - tail) + k;
      ++tried;
    }
    return -1;
  }
};

// Stored element -> float / double.
__device__ __forceinline__ float to_f32(float x) { return x; }
__device__ __forceinline__ float to_f32(double x) { return (float)x; }
__device__ __forceinline__ float to_f32(_Float16 x) { return (float)x; }
__device__ __forceinline__ float to_f32(bf16_t x) {
  return __uint_as_float((uint32_t)x.bits << 16);
}
__device__ __forceinline__ double to_f64(float x) { return (double)x; }
__device__ __forceinline__ double to_f64(double x) { return x; }
__device__ __forceinline__ double to_f64(_Float16 x) { return (double)(float)x; }
__device__ __forceinline__ double to_f64(bf16_t x) { return (double)to_f32(x); }

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ double wave_scan_incl(double x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double y = __shfl_up(x, (unsigned)d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// DPP lane moves (GCN/CDNA encodings): row_shr:n shifts within rows of 16
// lanes, row_bcast:15 / row_bcast:31 broadcast the last lane of a row / of
// the lower half into the following rows, wave_shr:1 shifts the whole wave.
// Lanes whose source is outside the pattern receive 0.
constexpr int kDppRowShr = 0x110;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
constexpr int kDppWaveShr1 = 0x138;

template <int Ctrl, int RowMask>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), Ctrl, RowMask, 0xF, false));
}

// Inclusive prefix sum within aligned groups of W = 16, 32 or 64 lanes, FP32,
// on DPP moves only (no LDS round trips): four row shifts give the scan
// inside each row of 16, then row broadcasts carry row totals upward.
template <int W>
__device__ __forceinline__ float group_scan_dpp(float x) {
  static_assert(W == 16 || W == 32 || W == 64, "group width");
  x += dpp_f32<kDppRowShr + 1, 0xF>(x);
  x += dpp_f32<kDppRowShr + 2, 0xF>(x);
  x += dpp_f32<kDppRowShr + 4, 0xF>(x);
  x += dpp_f32<kDppRowShr + 8, 0xF>(x);
  if (W >= 32) x += dpp_f32<kDppRowBcast15, 0xA>(x);
  if (W == 64) x += dpp_f32<kDppRowBcast31, 0xC>(x);
  return x;
}

// Sum over the 64 lanes, FP32, as a wave-uniform value: the DPP scan leaves
// the total in lane 63. All 64 lanes must be active.
__device__ __forceinline__ float wave_sum_dpp(float x) {
  x = group_scan_dpp<64>(x);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Sum within aligned groups of W = 16, 32 or 64 lanes, FP32, result in every
// lane of the group: a cyclic butterfly of row rotations inside each row of
// 16 (DPP), then a lane swizzle across the two rows of a 32-lane half, then
// the two halves for W = 64.
constexpr int kDppRowRor = 0x120;
template <int W>
__device__ __forceinline__ float group_allsum(float x) {
  static_assert(W == 16 || W == 32 || W == 64, "group width");
  x += dpp_f32<kDppRowRor + 8, 0xF>(x);
  x += dpp_f32<kDppRowRor + 4, 0xF>(x);
  x += dpp_f32<kDppRowRor + 2, 0xF>(x);
  x += dpp_f32<kDppRowRor + 1, 0xF>(x);
  if (W >= 32) {
    // Bit-mask swizzle inside 32 lanes: and 0x1F, or 0, xor 0x10.
    x += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x401F));
  }
  if (W == 64) {
    const int xi = __float_as_int(x);
    x = __int_as_float(__builtin_amdgcn_readlane(xi, 0)) +
        __int_as_float(__builtin_amdgcn_readlane(xi, 32));
  }
  return x;
}

// Largest of a group-uniform value over the G groups of W lanes (wave-uniform).
template <int G>
__device__ __forceinline__ int groups_max(int x) {
  int m = __builtin_amdgcn_readlane(x, 0);
#pragma unroll
  for (int g = 1; g < G; ++g) m = max(m, __builtin_amdgcn_readlane(x, g * (64 / G)));
  return m;
}

// Inclusive prefix sum within aligned groups of W lanes, FP64, on DPP moves of
// the two halves of each value (no LDS round trips).
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, Ctrl, RowMask, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), Ctrl, RowMask, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
template <int W>
__device__ __forceinline__ double group_scan_dpp(double x) {
  static_assert(W == 16 || W == 32 || W == 64, "group width");
  x += dpp_f64<kDppRowShr + 1, 0xF>(x);
  x += dpp_f64<kDppRowShr + 2, 0xF>(x);
  x += dpp_f64<kDppRowShr + 4, 0xF>(x);
  x += dpp_f64<kDppRowShr + 8, 0xF>(x);
  if (W >= 32) x += dpp_f64<kDppRowBcast15, 0xA>(x);
  if (W == 64) x += dpp_f64<kDppRowBcast31, 0xC>(x);
  return x;
}

// FP64 DPP move whose lanes without a source keep `old`.
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_f64_keep(double x, double old) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint64_t o = (uint64_t)__double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)u, Ctrl, RowMask,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(u >> 32),
                                             Ctrl, RowMask, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Inclusive scan of affine maps x -> M x + C (applied in lane order) within
// aligned groups of W lanes, with an additive companion S, FP64 on DPP moves.
// Lane j ends with the composition of the maps of lanes 0..j of its group.
template <int W>
__device__ __forceinline__ void group_scan_affine(double& M, double& C, double& S) {
  static_assert(W == 16 || W == 32 || W == 64, "group width");
  auto step = [&](auto ctrl_tag, auto mask_tag) {
    constexpr int kc = decltype(ctrl_tag)::value, km = decltype(mask_tag)::value;
    const double Mp = dpp_f64_keep<kc, km>(M, 1.0);
    const double Cp = dpp_f64_keep<kc, km>(C, 0.0);
    const double Sp = dpp_f64_keep<kc, km>(S, 0.0);
    C = fma(M, Cp, C);
    M = M * Mp;
    S = S + Sp;
  };
  using I = int;
  step(std::integral_constant<I, kDppRowShr + 1>{}, std::integral_constant<I, 0xF>{});
  step(std::integral_constant<I, kDppRowShr + 2>{}, std::integral_constant<I, 0xF>{});
  step(std::integral_constant<I, kDppRowShr + 4>{}, std::integral_constant<I, 0xF>{});
  step(std::integral_constant<I, kDppRowShr + 8>{}, std::integral_constant<I, 0xF>{});
  if (W >= 32) step(std::integral_constant<I, kDppRowBcast15>{}, std::integral_constant<I, 0xA>{});
  if (W == 64) step(std::integral_constant<I, kDppRowBcast31>{}, std::integral_constant<I, 0xC>{});
}

// Inclusive running maximum within aligned groups of W lanes, FP64, on DPP
// moves (lanes without a source keep their own value).
template <int W>
__device__ __forceinline__ double group_scan_max(double x) {
  static_assert(W == 16 || W == 32 || W == 64, "group width");
  x = fmax(x, dpp_f64_keep<kDppRowShr + 1, 0xF>(x, x));
  x = fmax(x, dpp_f64_keep<kDppRowShr + 2, 0xF>(x, x));
  x = fmax(x, dpp_f64_keep<kDppRowShr + 4, 0xF>(x, x));
  x = fmax(x, dpp_f64_keep<kDppRowShr + 8, 0xF>(x, x));
  if (W >= 32) x = fmax(x, dpp_f64_keep<kDppRowBcast15, 0xA>(x, x));
  if (W == 64) x = fmax(x, dpp_f64_keep<kDppRowBcast31, 0xC>(x, x));
  return x;
}

// Value of lane - 1 (0 in lane 0), across the whole wave.
__device__ __forceinline__ float lane_up1(float x) { return dpp_f32<kDppWaveShr1, 0xF>(x); }

// Inclusive prefix sum within aligned groups of W lanes (W a power of two).
template <int W, typename T>
__device__ __forceinline__ T group_scan_incl(T x, int sl) {
#pragma unroll
  for (int d = 1; d < W; d <<= 1) {
    const T y = __shfl_up(x, (unsigned)d, W);
    if (sl >= d) x += y;
  }
  return x;
}

// Sum within aligned groups of W lanes (result in every lane of the group).
template <int W, typename T>
__device__ __forceinline__ T group_sum(T x) {
#pragma unroll
  for (int d = W / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Maximum within aligned groups of W lanes, taken across groups: lanes that
// hold the same index inside their group get the max over all groups.
template <int W>
__device__ __forceinline__ int cross_group_max(int x) {
#pragma unroll
  for (int d = W; d < 64; d <<= 1) x = max(x, __shfl_xor(x, d, 64));
  return x;
}
template <int W>
__device__ __forceinline__ int cross_group_min(int x) {
#pragma unroll
  for (int d = W; d < 64; d <<= 1) x = min(x, __shfl_xor(x, d, 64));
  return x;
}

// Sum over the 64 lanes (result in every lane).
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Value of lane i (wave-uniform i) broadcast to the whole wavefront.
__device__ __forceinline__ float bcast(float x, int i) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), i));
}
__device__ __forceinline__ int bcast(int x, int i) { return __builtin_amdgcn_readlane(x, i); }
__device__ __forceinline__ double bcast(double x, int i) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, i);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), i);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Keeps the compiler from moving LDS accesses of one wavefront across this
// point (lanes read channel state written by other lanes).
__device__ __forceinline__ void wave_order() { __builtin_amdgcn_wave_barrier(); }

}  // namespace iris
