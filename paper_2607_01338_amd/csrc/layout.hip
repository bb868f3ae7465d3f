// Field ingest: native [nx][ny][nz] fields -> sightline-major [n_pix][n_los].
//
// For a sightline axis other than the fastest one this is a batched 2-D
// transpose, src[b][rows][cols] -> dst[b][cols][rows]:
//   axis 1: b = x, rows = y, cols = z  (pixel = x*nz + z, position = y)
//   axis 0: b = 1, rows = x, cols = y*nz + z  (pixel = y*nz + z, position = x)
// Tiles of 64x64 elements go through LDS so that both the read along `cols`
// and the write along `rows` are coalesced. Pure data movement: the output is
// a bit-exact permutation of the input.

#include <hip/hip_runtime.h>

#include "iris_internal.h"

namespace iris {

// One 64x64 tile of batch b: src [rows][cols] -> dst [cols][rows].
template <typename E>
__device__ __forceinline__ void transpose_tile(const void* srcv, void* dstv, int64_t rows,
                                               int64_t cols, int64_t b, int64_t r0, int64_t c0,
                                               E (*tile)[65]) {
  const int tx = threadIdx.x & 63;
  const int ty = threadIdx.x >> 6;  // 0..3
  const E* src = (const E*)srcv + b * rows * cols;
  E* dst = (E*)dstv + b * rows * cols;
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t gr = r0 + r, gc = c0 + tx;
    if (gr < rows && gc < cols) tile[r][tx] = src[gr * cols + gc];
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t gc = c0 + cc, gr = r0 + tx;
    if (gr < rows && gc < cols) dst[gc * rows + gr] = tile[tx][cc];
  }
}

template <typename E>
__global__ __launch_bounds__(256) void transpose_kernel(const LayoutParams P) {
  __shared__ E tile[64][65];
  for (int fi = 0; fi < P.n_fields; ++fi)
    transpose_tile<E>(P.src[fi], P.dst[fi], P.rows, P.cols, blockIdx.z, (int64_t)blockIdx.y * 64,
                      (int64_t)blockIdx.x * 64, tile);
}

// Many transposes (one job per cube, all its fields) in a single launch:
// block i handles global tile i; its job is found by binary search over the
// jobs' first tiles.
__global__ __launch_bounds__(256) void batched_transpose_kernel(const TransposeJob* jobs,
                                                                int n_jobs) {
  __shared__ uint64_t tile_mem[64 * 65];
  int lo = 0, hi = n_jobs - 1;
  const int64_t bid = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (jobs[mid].tile_begin <= bid) lo = mid;
    else hi = mid - 1;
  }
  const TransposeJob& J = jobs[lo];
  int64_t t = bid - J.tile_begin;
  const int64_t per_b = (int64_t)J.tiles_r * J.tiles_c;
  const int64_t b = t / per_b;
  t -= b * per_b;
  const int64_t r0 = (t / J.tiles_c) * 64, c0 = (t % J.tiles_c) * 64;
  for (int fi = 0; fi < J.n_fields; ++fi) {
    switch (J.elem) {
      case 2:
        transpose_tile<uint16_t>(J.src[fi], J.dst[fi], J.rows, J.cols, b, r0, c0,
                                 (uint16_t(*)[65])tile_mem);
        break;
      case 4:
        transpose_tile<uint32_t>(J.src[fi], J.dst[fi], J.rows, J.cols, b, r0, c0,
                                 (uint32_t(*)[65])tile_mem);
        break;
      default:
        transpose_tile<uint64_t>(J.src[fi], J.dst[fi], J.rows, J.cols, b, r0, c0,
                                 (uint64_t(*)[65])tile_mem);
        break;
    }
  }
}

// Zero a few ints (work-queue heads) with vector stores: a kernel node
// rather than a memset node inside captured graphs.
__global__ void zero_ints_kernel(int* p, int n) {
  for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) p[i] = 0;
}

int launch_batched_layout(const TransposeJob* jobs, int n_jobs, int64_t n_tiles, void* stream) {
  hipLaunchKernelGGL(batched_transpose_kernel, dim3((unsigned)n_tiles), dim3(256), 0,
                     (hipStream_t)stream, jobs, n_jobs);
  return (int)hipGetLastError();
}

int launch_zero_ints(int* p, int n, void* stream) {
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, p, n);
  return (int)hipGetLastError();
}

int launch_layout(const LayoutParams& p, void* stream) {
  const dim3 grid((unsigned)((p.cols + 63) / 64), (unsigned)((p.rows + 63) / 64),
                  (unsigned)p.batch);
  const dim3 block(256);
  switch (p.elem) {
    case 2:
      hipLaunchKernelGGL(transpose_kernel<uint16_t>, grid, block, 0, (hipStream_t)stream, p);
      break;
    case 4:
      hipLaunchKernelGGL(transpose_kernel<uint32_t>, grid, block, 0, (hipStream_t)stream, p);
      break;
    case 8:
      hipLaunchKernelGGL(transpose_kernel<uint64_t>, grid, block, 0, (hipStream_t)stream, p);
      break;
    default:
      return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

}  // namespace iris
