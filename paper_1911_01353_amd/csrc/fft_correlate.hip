// Fused overlap-save correlation on gfx950: segment FFT -> x template spectrum ->
// inverse FFT -> |.|^2 -> strip the overlap -> plane, with the segment held in
// registers and LDS for the whole template loop (paper, Figure 1 and section
// "Implementation": overlap-and-save with an on-chip FFT so segments do not
// round-trip device memory).
//
// Segment s of a width group with K taps covers bins
//   [s U - (K/2 - 1), s U - (K/2 - 1) + S),   U = S - K + 1,
// and its circular correlation with the K taps at lags m < U equals the plane
// outputs k0 = s U + m (no wrap-around there). Bins outside [0, nbins) are 0.
//
// FFT: self-sorting (Stockham) radix passes. A pass of radix R over sub-DFTs
// of length L reads element b + r S/R (b < S/R is the butterfly, r < R), scales
// it by W_{LR}^{r (b mod L)}, takes a radix-R DFT in registers and writes
// output k to (b - b mod L) R + b mod L + L k. After the last forward pass
// thread b holds frequencies b + k S/R_last in natural order, which is exactly
// what the first inverse pass (same radix, L = 1) reads, so the spectrum
// stays in registers between the forward transform, the template multiply and
// the inverse transform. One workgroup handles one segment and a block of
// templates; the forward FFT of the segment is done once per workgroup.
#include "jerk_internal.h"

namespace jerk {
namespace {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}

// cos / sin of 2 pi m / 16, m = 0..7
__device__ constexpr float kC16[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                                      0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
__device__ constexpr float kS16[8] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                                      1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f};

// v * W_R^k with W_R = exp(-+2 pi i / R) (minus for the forward transform).
template <int R, bool INV>
__device__ __forceinline__ float2 twiddle_const(int k, float2 v) {
  const int m = k * (16 / R);  // angle 2 pi m / 16
  if (m == 0) return v;
  if (m == 4) return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
  if (m == 2) {
    const float c = 0.70710678118654752f;
    return INV ? make_float2(c * (v.x - v.y), c * (v.x + v.y)) : make_float2(c * (v.x + v.y), c * (v.y - v.x));
  }
  if (m == 6) {
    const float c = 0.70710678118654752f;
    return INV ? make_float2(-c * (v.x + v.y), c * (v.x - v.y)) : make_float2(c * (v.y - v.x), -c * (v.x + v.y));
  }
  const float c = kC16[m], s = INV ? kS16[m] : -kS16[m];
  return make_float2(fmaf(v.x, c, -v.y * s), fmaf(v.x, s, v.y * c));
}

// In-register DFT of size R (power of two <= 16) by radix-2 decimation in time.
template <int R, bool INV>
struct Dft {
  __device__ __forceinline__ static void run(float2* x) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    Dft<R / 2, INV>::run(e);
    Dft<R / 2, INV>::run(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const float2 t = twiddle_const<R, INV>(k, o[k]);
      x[k] = cadd(e[k], t);
      x[k + R / 2] = csub(e[k], t);
    }
  }
};
template <bool INV>
struct Dft<1, INV> {
  __device__ __forceinline__ static void run(float2*) {}
};

// Padded LDS index: one spare float2 every 16 keeps the strided pass writes
// on distinct banks.
__device__ __forceinline__ int lds_idx(int i) { return i + (i >> 4); }

// One Stockham pass. The thread owns butterflies b = tid + m * TPB, m < E / R.
// tw: table of exp(-2 pi i k / S), k < S.
template <int S, int E, int R, int L, bool INV, bool FROM_LDS, bool TO_LDS>
__device__ __forceinline__ void stockham_pass(float2 (&v)[E], float2* lds, const float2* __restrict__ tw,
                                              int tid) {
  constexpr int TPB = S / E;
  constexpr int M = E / R;
  if constexpr (FROM_LDS) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int b = tid + m * TPB;
#pragma unroll
      for (int r = 0; r < R; ++r) v[m * R + r] = lds[lds_idx(b + r * (S / R))];
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int b = tid + m * TPB;
    if constexpr (L > 1) {
      const int j = b % L;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tw[(r * j * (S / (L * R))) & (S - 1)];
        v[m * R + r] = INV ? cmulc(v[m * R + r], w) : cmul(v[m * R + r], w);
      }
    }
    Dft<R, INV>::run(&v[m * R]);
  }
  if constexpr (TO_LDS) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int b = tid + m * TPB;
      const int j = b % L;
#pragma unroll
      for (int k = 0; k < R; ++k) lds[lds_idx((b - j) * R + j + L * k)] = v[m * R + k];
    }
    __syncthreads();
  }
}

template <int S, int E, int R1, int R2, int R3>
__global__ void __launch_bounds__(S / E) fft_correlate_kernel(FftArgs a, const float2* __restrict__ tw) {
  constexpr int TPB = S / E;
  static_assert(R1 * R2 * R3 == S, "radices must multiply to S");
  __shared__ float2 lds[S + S / 16];
  const int tid = threadIdx.x;
  const int K = a.taps;
  const int U = S - K + 1;
  const int64_t n_seg = (a.nbins + U - 1) / U;
  const int64_t blk = blockIdx.x;
  const int64_t seg = blk % n_seg;
  const int tb = (int)(blk / n_seg);
  const int64_t base = seg * U - (K / 2 - 1);

  // ---- forward FFT of the segment (radices R1, R2, R3) ----
  float2 v[E];
  {
    constexpr int M = E / R1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int b = tid + m * TPB;
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int64_t k = base + b + r * (S / R1);
        v[m * R1 + r] = (k >= 0 && k < a.nbins) ? a.spec[k] : make_float2(0.f, 0.f);
      }
    }
  }
  stockham_pass<S, E, R1, 1, false, false, true>(v, lds, tw, tid);
  stockham_pass<S, E, R2, R1, false, true, true>(v, lds, tw, tid);
  stockham_pass<S, E, R3, R1 * R2, false, true, false>(v, lds, tw, tid);
  float2 F[E];
#pragma unroll
  for (int e = 0; e < E; ++e) F[e] = v[e];

  // ---- template loop ----
  const int m0 = a.m_begin + tb * a.tpb;
  const int m1 = min(m0 + a.tpb, a.m_end);
  for (int mm = m0; mm < m1; ++mm) {
    const int t = a.members[mm];
    float* row = a.plane + (int64_t)(t - a.t_begin) * a.ld;
    float P0[E];
#pragma unroll
    for (int phase = 0; phase < 2; ++phase) {
      const float2* H = a.bank_fft + ((int64_t)mm * 2 + phase) * S;
      {
        constexpr int M = E / R3;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const int b = tid + m * TPB;
#pragma unroll
          for (int k = 0; k < R3; ++k) v[m * R3 + k] = cmul(F[m * R3 + k], H[b + k * (S / R3)]);
        }
      }
      stockham_pass<S, E, R3, 1, true, false, true>(v, lds, tw, tid);
      stockham_pass<S, E, R2, R3, true, true, true>(v, lds, tw, tid);
      stockham_pass<S, E, R1, R3 * R2, true, true, false>(v, lds, tw, tid);
      // thread holds lag b + k S/R1 in v[m R1 + k]
      if (phase == 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) P0[e] = fmaf(v[e].x, v[e].x, v[e].y * v[e].y);
      } else {
        constexpr int M = E / R1;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const int b = tid + m * TPB;
#pragma unroll
          for (int k = 0; k < R1; ++k) {
            const int lag = b + k * (S / R1);
            const int64_t k0 = seg * U + lag;
            if (lag < U && k0 < a.nbins) {
              const float2 vv = v[m * R1 + k];
              const float p1 = fmaf(vv.x, vv.x, vv.y * vv.y);
              *reinterpret_cast<float2*>(row + 2 * k0) = make_float2(P0[m * R1 + k], p1);
            }
          }
        }
      }
    }
  }
}

}  // namespace

void fft_correlate_launch(const FftArgs& a, const float2* twiddles, hipStream_t stream) {
  const int n_members = a.m_end - a.m_begin;
  if (n_members <= 0 || a.nbins <= 0) return;
  const int U = a.seg_len - a.taps + 1;
  require(U >= 1, JERK_EINTERNAL, "segment shorter than the template");
  const int64_t n_seg = (a.nbins + U - 1) / U;
  const int64_t n_tb = (n_members + a.tpb - 1) / a.tpb;
  const int64_t blocks = n_seg * n_tb;
  require(blocks < (1ll << 31), JERK_EINVAL, "search too large for one launch; split the template range");
  switch (a.seg_len) {
    case 4096:
      hipLaunchKernelGGL((fft_correlate_kernel<4096, 16, 16, 16, 16>), dim3((unsigned)blocks), dim3(256), 0,
                         stream, a, twiddles);
      break;
    case 2048:
      hipLaunchKernelGGL((fft_correlate_kernel<2048, 16, 8, 16, 16>), dim3((unsigned)blocks), dim3(128), 0,
                         stream, a, twiddles);
      break;
    case 1024:
      hipLaunchKernelGGL((fft_correlate_kernel<1024, 16, 4, 16, 16>), dim3((unsigned)blocks), dim3(64), 0,
                         stream, a, twiddles);
      break;
    case 512:
      hipLaunchKernelGGL((fft_correlate_kernel<512, 8, 8, 8, 8>), dim3((unsigned)blocks), dim3(64), 0, stream,
                         a, twiddles);
      break;
    default:
      throw Error(JERK_EINTERNAL, "unsupported segment length");
  }
  JERK_HIP_CHECK(hipGetLastError());
}

}  // namespace jerk
