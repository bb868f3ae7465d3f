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

template <typename E>
__global__ __launch_bounds__(256) void transpose_kernel(const LayoutParams P) {
  __shared__ E tile[64][65];
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  const int64_t r0 = (int64_t)blockIdx.y * 64;
  const int64_t b = blockIdx.z;
  const int tx = threadIdx.x & 63;
  const int ty = threadIdx.x >> 6;  // 0..3
  for (int fi = 0; fi < P.n_fields; ++fi) {
    const E* src = (const E*)P.src[fi] + b * P.rows * P.cols;
    E* dst = (E*)P.dst[fi] + b * P.rows * P.cols;
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
      const int64_t gr = r0 + r, gc = c0 + tx;
      if (gr < P.rows && gc < P.cols) tile[r][tx] = src[gr * P.cols + gc];
    }
    __syncthreads();
    for (int cc = ty; cc < 64; cc += 4) {
      const int64_t gc = c0 + cc, gr = r0 + tx;
      if (gr < P.rows && gc < P.cols) dst[gc * P.rows + gr] = tile[tx][cc];
    }
  }
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
