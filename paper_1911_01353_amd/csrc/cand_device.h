// Device helpers of candidate selection shared by the fused FFT epilogue and
// the selection kernels.
#pragma once

#include "jerk_internal.h"

namespace jerk {

// Lane data movement within a 64-lane wave (DPP). CTRL: 0xB1 quad_perm [1,0,3,2],
// 0x4E quad_perm [2,3,0,1], 0x124 / 0x128 rotate by 4 / 8 within rows of 16,
// 0x138 lane i reads lane i - 1, 0x130 lane i reads lane i + 1. Lanes without a
// source keep `old`.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float old, float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes of a wave, the same value in every lane. Each row of 16
// lanes is summed as pairs, then quads, then groups of 8 and 16; the four row
// sums are taken from lanes 0, 16, 32, 48 and added in that order, so the
// result does not depend on anything but the inputs.
__device__ __forceinline__ double wave_sum_f64(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  x += dpp_f64<0x124>(x);
  x += dpp_f64<0x128>(x);
  return ((readlane_f64(x, 0) + readlane_f64(x, 16)) + readlane_f64(x, 32)) + readlane_f64(x, 48);
}

// Appends the candidates of the lanes with `hit` set to out (one atomic per wave).
// Entered by every lane of the wave.
__device__ __forceinline__ void emit_candidates(bool hit, uint32_t t, uint32_t p, float power, double mean,
                                                double sigma, jerk_candidate* __restrict__ out, int64_t capacity,
                                                unsigned long long* __restrict__ count) {
  const uint64_t mask = __ballot(hit);
  if (mask == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(mask));
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(base & 0xffffffffull), leader);
  const int hi = __builtin_amdgcn_readlane((int)(base >> 32), leader);
  base = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
  if (hit) {
    const unsigned long long i = base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull));
    if (i < (unsigned long long)capacity) {
      jerk_candidate c;
      c.t = t;
      c.p = p;
      c.power = power;
      c.sigma = (float)(((double)power - mean) / sigma);
      out[i] = c;
    }
  }
}

}  // namespace jerk
