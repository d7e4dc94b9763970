// Peak keys -> per-row peaks. A key is (float bits of a power << 32) |
// (0xFFFFFFFF - p); the largest key of a row is its largest power, ties going
// to the lowest plane index p.
#include <algorithm>

#include "jerk_internal.h"

namespace jerk {
namespace {

__global__ void peaks_reduce_kernel(const uint64_t* __restrict__ keys, int32_t rows, int64_t per_row, int64_t ld,
                                    jerk_peak* __restrict__ out) {
  const int32_t row = blockIdx.x;
  if (row >= rows) return;
  uint64_t best = 0;
  for (int64_t i = threadIdx.x; i < per_row; i += blockDim.x) {
    const uint64_t k = keys[row * ld + i];
    best = k > best ? k : best;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint64_t o = __shfl_xor(best, off, 64);
    best = o > best ? o : best;
  }
  __shared__ uint64_t red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) best = red[w] > best ? red[w] : best;
    best = red[0] > best ? red[0] : best;
    jerk_peak pk;
    pk.power = __uint_as_float((uint32_t)(best >> 32));
    pk.p = 0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFu);
    out[row] = pk;
  }
}

__global__ void fill_u64_kernel(uint64_t* __restrict__ dst, int64_t n, uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = v;
}

}  // namespace

void fill_u64(uint64_t* dst, int64_t n, uint64_t v, hipStream_t stream) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, dst, n, v);
  JERK_HIP_CHECK(hipGetLastError());
}

void peaks_reduce(const uint64_t* keys, int32_t rows, int64_t per_row, int64_t ld, jerk_peak* out,
                  hipStream_t stream) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(peaks_reduce_kernel, dim3((unsigned)rows), dim3(256), 0, stream, keys, rows, per_row, ld, out);
  JERK_HIP_CHECK(hipGetLastError());
}

}  // namespace jerk
