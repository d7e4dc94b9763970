// Candidate selection over a plane slab (paper, section "Results": the search
// is timed with the mean and standard deviation of the plane and a peak finder
// that keeps only peaks above a user threshold).
//
// Row statistics: population mean and standard deviation per row, one read of
// the row. Each thread folds 8 values at a time: their sum in FP64 is exact for
// FP32 inputs, so the group mean and the group's sum of squared deviations are
// formed directly, and groups are merged with the pairwise update of Chan,
// Golub and LeVeque (1979). A constant row therefore gets a standard deviation
// of exactly 0. Chunks of a row are merged in a fixed order, so the result does
// not depend on scheduling.
//
// Candidates: a point is kept when its power, widened to FP64, is strictly above
// mean + k * sigma of its row, it is strictly greater than its left neighbour
// and not less than its right one (row ends have no neighbour on that side).
// Each wave appends its hits with one atomic add on the shared counter.
#include "jerk_internal.h"

namespace jerk {
namespace {

constexpr int kStatThreads = 256;
constexpr int kStatPerThread = 8;
constexpr int64_t kStatTile = kStatThreads * kStatPerThread;  // 2048 points
constexpr int kPeakThreads = 256;
constexpr int kPeakPerThread = 4;
constexpr int64_t kPeakTile = kPeakThreads * kPeakPerThread;  // 1024 points
constexpr int kMaxGridY = 65535;

struct Moments {
  double n, m, m2;  // count, mean, sum of squared deviations from the mean
};

__device__ __forceinline__ Moments merge(Moments a, Moments b) {
  const double n = a.n + b.n;
  if (b.n == 0.0) return a;
  if (a.n == 0.0) return b;
  const double d = b.m - a.m;
  const double fb = b.n / n;
  Moments r;
  r.n = n;
  r.m = a.m + d * fb;
  r.m2 = (a.m2 + b.m2) + d * d * a.n * fb;
  return r;
}

__device__ __forceinline__ Moments shfl_xor_moments(Moments v, int off) {
  Moments o;
  o.n = __shfl_xor(v.n, off, 64);
  o.m = __shfl_xor(v.m, off, 64);
  o.m2 = __shfl_xor(v.m2, off, 64);
  return o;
}

// grid (chunks, min(rows, 65535)); chunk c of a row covers [c * span, (c + 1) * span).
__global__ void __launch_bounds__(kStatThreads) row_moments_kernel(const float* __restrict__ plane, int64_t ld,
                                                                   int32_t rows, int64_t n_r, int64_t span,
                                                                   Moments* __restrict__ part) {
  const int32_t chunks = (int32_t)gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * span;
  const int64_t hi = lo + span < n_r ? lo + span : n_r;
  __shared__ Moments red[kStatThreads / 64];
  for (int32_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const float* src = plane + (int64_t)row * ld;
    Moments acc{0.0, 0.0, 0.0};
    for (int64_t base = lo; base < hi; base += kStatTile) {
      float v[kStatPerThread];
      int cnt = 0;
      double sum = 0.0;
#pragma unroll
      for (int j = 0; j < kStatPerThread; ++j) {
        const int64_t p = base + j * kStatThreads + threadIdx.x;
        v[j] = 0.0f;
        if (p < hi) {
          v[j] = src[p];
          sum += (double)v[j];
          ++cnt;
        }
      }
      if (cnt > 0) {
        Moments g;
        g.n = (double)cnt;
        g.m = sum / g.n;
        g.m2 = 0.0;
#pragma unroll
        for (int j = 0; j < kStatPerThread; ++j) {
          if (j * kStatThreads + threadIdx.x + base < hi) {
            const double e = (double)v[j] - g.m;
            g.m2 = fma(e, e, g.m2);
          }
        }
        acc = merge(acc, g);
      }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const Moments o = shfl_xor_moments(acc, off);
      // lower lane first, so lane 0 always merges in index order
      acc = (threadIdx.x & off) ? merge(o, acc) : merge(acc, o);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      Moments r = red[0];
      for (int w = 1; w < kStatThreads / 64; ++w) r = merge(r, red[w]);
      part[(int64_t)row * chunks + blockIdx.x] = r;
    }
    __syncthreads();
  }
}

__global__ void row_stats_finish_kernel(const Moments* __restrict__ part, int32_t rows, int32_t chunks,
                                        double* __restrict__ stats) {
  const int32_t row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  Moments r = part[(int64_t)row * chunks];
  for (int32_t c = 1; c < chunks; ++c) r = merge(r, part[(int64_t)row * chunks + c]);
  stats[2 * (int64_t)row] = r.m;
  stats[2 * (int64_t)row + 1] = r.n > 0.0 ? sqrt(r.m2 / r.n) : 0.0;
}

// grid (ceil(n_r / 1024), min(rows, 65535)). Thread i of a block takes points
// base + j * 256 + i, j = 0..3, so every load is coalesced; neighbours come from
// the adjacent lanes, the wave's edge lanes read theirs.
__global__ void __launch_bounds__(kPeakThreads) find_candidates_kernel(
    const float* __restrict__ plane, int64_t ld, int32_t rows, int64_t n_r, const double* __restrict__ stats,
    double k_sigma, const int32_t* __restrict__ row_template, int32_t t_base, jerk_candidate* __restrict__ out,
    int64_t capacity, unsigned long long* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int32_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const float* src = plane + (int64_t)row * ld;
    const double mu = stats[2 * (int64_t)row];
    const double sd = stats[2 * (int64_t)row + 1];
    const double thr = mu + k_sigma * sd;
    const uint32_t t = row_template ? (uint32_t)row_template[row] : (uint32_t)(t_base + row);
#pragma unroll
    for (int j = 0; j < kPeakPerThread; ++j) {
      const int64_t p = (int64_t)blockIdx.x * kPeakTile + j * kPeakThreads + threadIdx.x;
      const bool in = p < n_r;
      const float v = in ? src[p] : 0.0f;
      float left = __shfl_up(v, 1, 64);
      float right = __shfl_down(v, 1, 64);
      if (lane == 0 && in && p > 0) left = src[p - 1];
      if (lane == 63 && p + 1 < n_r) right = src[p + 1];
      const bool hit = in && (p == 0 || v > left) && (p + 1 == n_r || v >= right) && (double)v > thr;
      const uint64_t mask = __ballot(hit);
      if (mask == 0ull) continue;
      const int leader = __ffsll((unsigned long long)mask) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(mask));
      base = __shfl(base, leader, 64);
      if (hit) {
        const unsigned long long idx = base + (unsigned long long)__popcll(mask & below);
        if (idx < (unsigned long long)capacity) {
          jerk_candidate c;
          c.t = t;
          c.p = (uint32_t)p;
          c.power = v;
          c.sigma = (float)(((double)v - mu) / sd);
          out[idx] = c;
        }
      }
    }
  }
}

int32_t stat_chunks(int32_t rows, int64_t n_r) {
  if (rows <= 0 || n_r <= 0) return 0;
  const int64_t tiles = (n_r + kStatTile - 1) / kStatTile;
  int64_t c = (4096 + rows - 1) / rows;
  if (c > tiles) c = tiles;
  if (c > 4096) c = 4096;
  return (int32_t)(c < 1 ? 1 : c);
}

}  // namespace

size_t stats_workspace_bytes(int32_t rows, int64_t n_r) {
  return (size_t)(rows > 0 ? rows : 0) * (size_t)stat_chunks(rows, n_r) * sizeof(Moments);
}

void plane_stats(const float* plane, int64_t ld, int32_t rows, int64_t n_r, double* stats, void* ws,
                 size_t ws_bytes, hipStream_t stream) {
  if (rows <= 0 || n_r <= 0) return;
  require(ws_bytes >= stats_workspace_bytes(rows, n_r), JERK_ENOMEM, "statistics workspace too small");
  const int32_t chunks = stat_chunks(rows, n_r);
  const int64_t tiles = (n_r + kStatTile - 1) / kStatTile;
  const int64_t span = (tiles + chunks - 1) / chunks * kStatTile;
  const dim3 grid((unsigned)chunks, (unsigned)(rows < kMaxGridY ? rows : kMaxGridY));
  hipLaunchKernelGGL(row_moments_kernel, grid, dim3(kStatThreads), 0, stream, plane, ld, rows, n_r, span,
                     static_cast<Moments*>(ws));
  JERK_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(row_stats_finish_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, stream,
                     static_cast<const Moments*>(ws), rows, chunks, stats);
  JERK_HIP_CHECK(hipGetLastError());
}

void find_candidates(const float* plane, int64_t ld, int32_t rows, int64_t n_r, const double* stats,
                     double k_sigma, const int32_t* row_template, int32_t t_base, jerk_candidate* out,
                     int64_t capacity, unsigned long long* count, hipStream_t stream) {
  if (rows <= 0 || n_r <= 0) return;
  const int64_t bx = (n_r + kPeakTile - 1) / kPeakTile;
  const dim3 grid((unsigned)bx, (unsigned)(rows < kMaxGridY ? rows : kMaxGridY));
  hipLaunchKernelGGL(find_candidates_kernel, grid, dim3(kPeakThreads), 0, stream, plane, ld, rows, n_r, stats,
                     k_sigma, row_template, t_base, out, capacity, count);
  JERK_HIP_CHECK(hipGetLastError());
}

}  // namespace jerk
