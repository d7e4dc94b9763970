// Spectrum preparation on the GPU: N real float32 samples -> N/2 complex64
// bins, DC zeroed and scaled to unit mean power above DC (the search's input
// contract), with every step in FP64.
//
// The N real samples are read as M = N/2 complex points z[m] = x[2m] + i x[2m+1].
// Their length-M DFT Z comes from self-sorting Stockham passes in global memory
// (radix 16, then one radix 2/4/8 pass for the rest of log2 M). A pass with
// sub-transform length L and radix R reads in[b + r M/R], r < R, multiplies by
// the twiddle w_{LR}^{r j} (j = b mod L) and writes the R-point DFT to
// out[j + L (r' + R q)], b = j + L q: after the last pass the result is in
// natural order. Twiddles come from sincospi in FP64; the R-point DFTs are
// radix-2 butterflies, so a constant input gives exact zeros above DC (as a
// butterfly FFT in FP64 on the host does) rather than rounding noise that the
// normalisation would then blow up.
//
// The real spectrum follows from E[k] = (Z[k] + conj Z[M-k]) / 2 (even samples),
// O[k] = (Z[k] - conj Z[M-k]) / (2i) (odd samples) and X[k] = E[k] + e^{-2 pi i k / N} O[k],
// k < M. The power sum above DC is reduced in a fixed order (per-block trees,
// then one block), so the result does not depend on scheduling.
#include "jerk_internal.h"

namespace jerk {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 unit(double turns_times_two) {  // exp(i pi t)
  double s, c;
  sincospi(turns_times_two, &s, &c);
  return make_double2(c, s);
}

// In-register FP64 DFT of size R by radix-2 decimation in time.
template <int R>
struct DftD {
  __device__ __forceinline__ static void run(double2* x) {
    double2 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    DftD<R / 2>::run(e);
    DftD<R / 2>::run(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const double2 t = k == 0 ? o[k] : cmul(o[k], unit(-2.0 * (double)k / (double)R));
      x[k] = make_double2(e[k].x + t.x, e[k].y + t.y);
      x[k + R / 2] = make_double2(e[k].x - t.x, e[k].y - t.y);
    }
  }
};
template <>
struct DftD<1> {
  __device__ __forceinline__ static void run(double2*) {}
};

template <int R, bool FROM_REAL>
__global__ void __launch_bounds__(kThreads) stockham_pass_fp64(const void* __restrict__ in_v,
                                                               double2* __restrict__ out, int64_t M, int64_t L) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t stride = M / R;
  if (b >= stride) return;
  const int64_t j = b % L;
  double2 a[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = b + r * stride;
    if constexpr (FROM_REAL) {
      const float2 v = static_cast<const float2*>(in_v)[i];
      a[r] = make_double2((double)v.x, (double)v.y);
    } else {
      a[r] = static_cast<const double2*>(in_v)[i];
    }
    if (r > 0 && L > 1) a[r] = cmul(a[r], unit(-2.0 * (double)(r * j) / (double)(L * R)));
  }
  DftD<R>::run(a);
  const int64_t q = b / L;
#pragma unroll
  for (int rr = 0; rr < R; ++rr) out[j + L * (rr + (int64_t)R * q)] = a[rr];
}

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// X[k] for k < M (X[0] = 0) and the per-block sum of |X[k]|^2.
__global__ void __launch_bounds__(kThreads) real_split_kernel(const double2* __restrict__ Z, int64_t M,
                                                              double2* __restrict__ X, double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double p = 0.0;
  if (k < M) {
    double2 x = make_double2(0.0, 0.0);
    if (k > 0) {
      const double2 zk = Z[k];
      const double2 zc = Z[M - k];
      const double2 e = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y - zc.y));
      // (zk - conj zc) / (2i) = ((zk.y + zc.y) - i (zk.x - zc.x)) / 2
      const double2 o = make_double2(0.5 * (zk.y + zc.y), -0.5 * (zk.x - zc.x));
      const double2 t = cmul(o, unit(-(double)k / (double)M));  // exp(-2 pi i k / N), N = 2M
      x = make_double2(e.x + t.x, e.y + t.y);
      p = x.x * x.x + x.y * x.y;
    }
    X[k] = x;
  }
  const double s = block_sum(p, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// One block: scale = 1 / sqrt(mean power above DC), or 0 when that power is 0.
__global__ void __launch_bounds__(kThreads) power_scale_kernel(const double* __restrict__ part, int64_t nparts,
                                                               int64_t M, double* __restrict__ scale) {
  __shared__ double red[kThreads / 64];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += kThreads) v += part[i];
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) {
    const double mean = s / (double)(M - 1);
    scale[0] = mean > 0.0 ? 1.0 / sqrt(mean) : 0.0;
  }
}

__global__ void __launch_bounds__(kThreads) scale_round_kernel(const double2* __restrict__ X, int64_t M,
                                                               const double* __restrict__ scale,
                                                               float2* __restrict__ spec) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= M) return;
  const double s = scale[0];
  const double2 x = X[k];
  spec[k] = make_float2((float)(x.x * s), (float)(x.y * s));
}

struct WsLayout {
  size_t a, b, part, scale, total;
  int64_t blocks;
};

WsLayout ws_layout(int64_t M) {
  WsLayout w{};
  w.blocks = (M + kThreads - 1) / kThreads;
  w.a = 0;
  w.b = align_up((size_t)M * sizeof(double2));
  w.part = w.b + align_up((size_t)M * sizeof(double2));
  w.scale = w.part + align_up((size_t)w.blocks * sizeof(double));
  w.total = w.scale + kAlign;
  return w;
}

template <int R>
void launch_pass(bool from_real, const void* in, double2* out, int64_t M, int64_t L, hipStream_t stream) {
  const int64_t threads = M / R;
  const dim3 grid((unsigned)((threads + kThreads - 1) / kThreads));
  if (from_real)
    hipLaunchKernelGGL((stockham_pass_fp64<R, true>), grid, dim3(kThreads), 0, stream, in, out, M, L);
  else
    hipLaunchKernelGGL((stockham_pass_fp64<R, false>), grid, dim3(kThreads), 0, stream, in, out, M, L);
  JERK_HIP_CHECK(hipGetLastError());
}

}  // namespace

size_t spectrum_workspace_bytes(int64_t n_samples) { return ws_layout(n_samples / 2).total; }

void spectrum_prepare(const float* series, int64_t n_samples, float2* spec, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
  const int64_t M = n_samples / 2;
  const WsLayout w = ws_layout(M);
  require(ws_bytes >= w.total, JERK_ENOMEM, "spectrum workspace too small");
  char* base = static_cast<char*>(ws);
  double2* buf[2] = {reinterpret_cast<double2*>(base + w.a), reinterpret_cast<double2*>(base + w.b)};
  double* part = reinterpret_cast<double*>(base + w.part);
  double* scale = reinterpret_cast<double*>(base + w.scale);
  const void* in = series;
  bool from_real = true;
  int cur = 0;
  int64_t L = 1;
  while (L < M) {
    const int64_t rest = M / L;
    const int R = rest >= 16 ? 16 : (int)rest;
    switch (R) {
      case 16: launch_pass<16>(from_real, in, buf[cur], M, L, stream); break;
      case 8: launch_pass<8>(from_real, in, buf[cur], M, L, stream); break;
      case 4: launch_pass<4>(from_real, in, buf[cur], M, L, stream); break;
      default: launch_pass<2>(from_real, in, buf[cur], M, L, stream); break;
    }
    in = buf[cur];
    from_real = false;
    cur ^= 1;
    L *= R;
  }
  // M = 1 cannot occur (n_samples >= 4), so at least one pass ran and `in` holds Z.
  double2* X = buf[cur];
  const dim3 grid((unsigned)w.blocks);
  hipLaunchKernelGGL(real_split_kernel, grid, dim3(kThreads), 0, stream, static_cast<const double2*>(in), M, X,
                     part);
  JERK_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(power_scale_kernel, dim3(1), dim3(kThreads), 0, stream, part, w.blocks, M, scale);
  JERK_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(scale_round_kernel, grid, dim3(kThreads), 0, stream, X, M, scale, spec);
  JERK_HIP_CHECK(hipGetLastError());
}

}  // namespace jerk
