// Incoherent harmonic summing over a full (r, z, w) power plane.
//
// The h-th harmonic of a signal with fundamental (r, zbar, w) sits at
// (h r, h zbar, h w). When the zbar lattice contains 0 (zmax a multiple of dz)
// every harmonic of a lattice point is a lattice point: fundamental
// (i, j, p) reads template (i0 + h (i - i0), J + h (j - J)) at plane index h p,
// i0 the index of zbar = 0. Each output is the FP32 sum over h = 1..H in that
// order. Rows of the output are the fundamentals whose H harmonics all lie on
// the plane, in w-major lattice order.
//
// One workgroup covers 1024 consecutive outputs of one fundamental row; lane i
// takes outputs base + k * 256 + i, so harmonic h reads its row at stride h:
// for h = 1 every load is coalesced, for larger h each cache line serves
// 32 / h lanes (the lines' other words belong to no output of this row, so the
// bytes moved are those of the lines touched, not 4 per read). The plane is read at most once per (fundamental, harmonic) pair
// that maps onto it, and the harmonic-summed plane is at most 1/H of the
// plane's width and ~1/H^2 of its rows.
#include <cmath>

#include "jerk_internal.h"

namespace jerk {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int64_t kTile = kThreads * kPerThread;
constexpr int kMaxGridY = 65535;
constexpr int kChunk = 8;

__global__ void __launch_bounds__(kThreads) harmonic_sum_kernel(const float* __restrict__ plane, int64_t ld,
                                                                int32_t n_z, int32_t i0, int32_t J, int32_t n_zf,
                                                                int32_t n_wf, int32_t n_harm, int64_t n_pf,
                                                                float* __restrict__ out, int64_t out_ld) {
  const int32_t rows = n_zf * n_wf;
  for (int32_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const int32_t di = row % n_zf - n_zf / 2;
    const int32_t dj = row / n_zf - n_wf / 2;
    // harmonics in chunks of kChunk: every load of a chunk (all outputs of the thread) is issued
    // before the first add, so a thread keeps kPerThread x kChunk reads in flight; the adds still
    // run in h order
    float s[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) s[k] = 0.0f;
    for (int32_t h0 = 1; h0 <= n_harm; h0 += kChunk) {
      float v[kPerThread][kChunk];
#pragma unroll
      for (int q = 0; q < kChunk; ++q) {
        const int32_t h = h0 + q;
        const int32_t hr = h <= n_harm ? h : n_harm;  // rows past the last harmonic are not read
        const int64_t t = (int64_t)(J + hr * dj) * n_z + (i0 + hr * di);
        const float* __restrict__ rowp = plane + t * ld;
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
          const int64_t p = (int64_t)blockIdx.x * kTile + k * kThreads + threadIdx.x;
          v[k][q] = (h <= n_harm && p < n_pf) ? rowp[(int64_t)h * p] : 0.0f;
        }
      }
#pragma unroll
      for (int q = 0; q < kChunk; ++q)
#pragma unroll
        for (int k = 0; k < kPerThread; ++k)
          if (h0 + q <= n_harm) s[k] += v[k][q];
    }
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int64_t p = (int64_t)blockIdx.x * kTile + k * kThreads + threadIdx.x;
      if (p < n_pf) __builtin_nontemporal_store(s[k], &out[(int64_t)row * out_ld + p]);
    }
  }
}

}  // namespace

HarmonicShape harmonic_shape(const Plan& p, int64_t n_r, int32_t n_harm) {
  const double q = p.desc.zmax / p.desc.dz;
  require(std::fabs(q - std::nearbyint(q)) <= 1e-9, JERK_EUNSUPPORTED,
          "harmonic sums need zmax to be a multiple of dz (zbar = 0 on the lattice)");
  require(n_harm >= 1 && n_harm <= 64, JERK_EINVAL, "n_harm must be in [1, 64]");
  require(n_r >= 1, JERK_EINVAL, "n_r must be >= 1");
  HarmonicShape s;
  s.i0 = (int32_t)std::nearbyint(q);
  require(2 * s.i0 + 1 == p.n_z, JERK_EINTERNAL, "zbar lattice is not symmetric about 0");
  s.n_zf = 2 * (s.i0 / n_harm) + 1;
  s.n_wf = 2 * (p.J / n_harm) + 1;
  s.n_pf = (n_r - 1) / n_harm + 1;
  return s;
}

void harmonic_sum(const Plan& p, const float* plane, int64_t ld, int64_t n_r, int32_t n_harm, float* out,
                  int64_t out_ld, hipStream_t stream) {
  const HarmonicShape s = harmonic_shape(p, n_r, n_harm);
  require(ld >= n_r && out_ld >= s.n_pf, JERK_EINVAL, "need ld >= n_r and out_ld >= the fundamentals per row");
  const int32_t rows = s.n_zf * s.n_wf;
  const dim3 grid((unsigned)((s.n_pf + kTile - 1) / kTile), (unsigned)(rows < kMaxGridY ? rows : kMaxGridY));
  hipLaunchKernelGGL(harmonic_sum_kernel, grid, dim3(kThreads), 0, stream, plane, ld, p.n_z, s.i0, p.J, s.n_zf,
                     s.n_wf, n_harm, s.n_pf, out, out_ld);
  JERK_HIP_CHECK(hipGetLastError());
}

}  // namespace jerk
