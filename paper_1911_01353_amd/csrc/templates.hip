// Template bank generation on the GPU, in FP64.
//
// Each tap is the response of a tone with constant fdot and fddot (paper,
// section "Implementation": one filter per (z, w)), evaluated as
//   T(qbar; zbar, w) = R(qbar - zbar/2 + w/12; zbar - w/2, w),
//   R(q; z, w)       = integral_0^1 exp(2 pi i (q u + z u^2/2 + w u^3/6)) du,
// by composite 16-point Gauss-Legendre quadrature with one panel per phase
// cycle (plus one): the phase derivative is at most |q| + |z| + |w|/2 cycles
// per unit u, so each panel spans at most one cycle, where a 16-node rule is
// exact to FP64 rounding.
//
// The FP64 taps are kept in the bank; the path-specific banks are derived
// from them:
//   FFT path  - spectra H[f] = (1/S) sum_j c_j exp(+2 pi i f j / S), f < S,
//               so that IFFT(FFT(segment) * H) is the circular correlation of
//               the segment with the taps (the overlap-save identity).
//   MFMA path - tap fragments (gemm_correlate.hip).
#include <cmath>

#include "jerk_internal.h"

namespace jerk {
namespace {

struct GlRule {
  double x[16];
  double w[16];
};

struct TapGen {
  double zmax, dz, dw;
  int32_t n_z, J;
  int32_t taps;        // K_g
  int32_t n_members;
  const int32_t* members;
  double2* out;        // [n][2][taps]
  int32_t margin;
};

__device__ inline double2 response_r(double q, double z, double w, const GlRule& gl) {
  // Panels: at most one phase cycle each.
  const double cycles = fabs(q) + fabs(z) + 0.5 * fabs(w);
  const int32_t panels = (int32_t)ceil(cycles) + 1;
  const double hw = 0.5 / panels;  // half panel width
  const double z2 = 0.5 * z, w6 = w / 6.0;
  double re = 0.0, im = 0.0;
  for (int32_t p = 0; p < panels; ++p) {
    const double mid = (2 * p + 1) * hw;
    double pre = 0.0, pim = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double u = mid + hw * gl.x[k];
      double ph = u * (q + u * (z2 + u * w6));  // cycles
      ph -= rint(ph);
      double s, c;
      sincospi(2.0 * ph, &s, &c);
      pre = fma(gl.w[k], c, pre);
      pim = fma(gl.w[k], s, pim);
    }
    re += pre;
    im += pim;
  }
  return make_double2(re * hw, im * hw);
}

__global__ void gen_taps_kernel(TapGen a, GlRule gl) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)a.n_members * 2 * a.taps;
  if (idx >= total) return;
  const int32_t j = (int32_t)(idx % a.taps);
  const int32_t phase = (int32_t)((idx / a.taps) % 2);
  const int32_t m = (int32_t)(idx / (2 * (int64_t)a.taps));
  const int32_t t = a.members[m];
  const double zb = -a.zmax + (t % a.n_z) * a.dz;
  const double w = (t / a.n_z - a.J) * a.dw;
  const int32_t h = (int32_t)ceil(fabs(zb) * 0.5 + fabs(w) / 12.0) + a.margin;
  const int32_t hg = a.taps / 2;
  double2 c = make_double2(0.0, 0.0);
  if (j >= hg - h && j < hg + h) {
    // tap j multiplies bin k0 - hg + 1 + j: offset qbar = hg - 1 - j + phase/2
    const double qbar = (double)(hg - 1 - j) + 0.5 * phase;
    const double2 r = response_r(qbar - 0.5 * zb + w / 12.0, zb - 0.5 * w, w, gl);
    c = make_double2(r.x, -r.y);  // conjugated: the correlation multiplies conj(T)
  }
  a.out[idx] = c;
}

struct SpecGen {
  const double2* taps;  // [n][2][K]
  float2* out;          // [n][2][S]
  int32_t n_members, K, S;
};

// H[f] = (1/S) sum_j c_j exp(+2 pi i f j / S) for one (member, phase) per y-block row.
__global__ void gen_fft_spectra_kernel(SpecGen a) {
  const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t row = blockIdx.y;  // member * 2 + phase
  if (f >= a.S) return;
  const double2* c = a.taps + (int64_t)row * a.K;
  double re = 0.0, im = 0.0;
  for (int32_t j = 0; j < a.K; ++j) {
    const double2 cj = c[j];
    if (cj.x == 0.0 && cj.y == 0.0) continue;
    const int64_t e = ((int64_t)f * j) % a.S;
    double s, co;
    sincospi(2.0 * (double)e / (double)a.S, &s, &co);
    re += cj.x * co - cj.y * s;
    im += cj.x * s + cj.y * co;
  }
  const double inv = 1.0 / (double)a.S;
  a.out[(int64_t)row * a.S + f] = make_float2((float)(re * inv), (float)(im * inv));
}

// exp(-2 pi i k / n), k < n, from FP64 and rounded once to complex64.
__global__ void gen_twiddles_kernel(float2* out, int32_t n) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s, c;
  sincospi(-2.0 * (double)k / (double)n, &s, &c);
  out[k] = make_float2((float)c, (float)s);
}

}  // namespace

void gen_twiddles(float2* out, int32_t n, hipStream_t stream) {
  hipLaunchKernelGGL(gen_twiddles_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, out, n);
  JERK_HIP_CHECK(hipGetLastError());
}

void gemm_bank_build(const Plan& p, const Group& g, const double2* taps, void* out, hipStream_t stream);

void taps_launch(const Plan& p, int32_t taps, const int32_t* d_members, int32_t n, double2* out, hipStream_t stream) {
  if (n <= 0) return;
  GlRule gl;
  for (int k = 0; k < 16; ++k) {
    gl.x[k] = p.gl_x[k];
    gl.w[k] = p.gl_w[k];
  }
  TapGen a{p.desc.zmax, p.desc.dz, p.desc.dw, p.n_z, p.J, taps, n, d_members, out, p.desc.margin_bins};
  const int64_t total = (int64_t)n * 2 * taps;
  hipLaunchKernelGGL(gen_taps_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, a, gl);
  JERK_HIP_CHECK(hipGetLastError());
}

void fft_spectra_launch(const double2* taps, int32_t n, int32_t K, int32_t S, float2* out, hipStream_t stream) {
  if (n <= 0) return;
  SpecGen s{taps, out, n, K, S};
  dim3 grid((unsigned)((S + 255) / 256), (unsigned)(2 * n));
  hipLaunchKernelGGL(gen_fft_spectra_kernel, grid, dim3(256), 0, stream, s);
  JERK_HIP_CHECK(hipGetLastError());
}

void bank_build(Plan& p, void* d_bank, hipStream_t stream) {
  if (!p.pinned_members) {
    void* h = nullptr;
    JERK_HIP_CHECK(hipHostMalloc(&h, sizeof(int32_t) * (size_t)p.T, hipHostMallocDefault));
    p.pinned_members = static_cast<int32_t*>(h);
    int32_t k = 0;
    for (const auto& g : p.groups)
      for (int32_t t : g.members) p.pinned_members[k++] = t;
  }
  char* bank = static_cast<char*>(d_bank);
  JERK_HIP_CHECK(hipMemcpyAsync(bank + p.off_members, p.pinned_members, sizeof(int32_t) * (size_t)p.T,
                                hipMemcpyHostToDevice, stream));
  for (int i = 0; i < 4; ++i) gen_twiddles(reinterpret_cast<float2*>(bank + p.off_tw[i]), 512 << i, stream);
  templates_build(p, d_bank, stream);
}

void templates_build(const Plan& p, void* d_bank, hipStream_t stream) {
  char* bank = static_cast<char*>(d_bank);
  GlRule gl;
  for (int k = 0; k < 16; ++k) {
    gl.x[k] = p.gl_x[k];
    gl.w[k] = p.gl_w[k];
  }
  const int32_t* d_members = reinterpret_cast<const int32_t*>(bank + p.off_members);
  for (const Group& g : p.groups) {
    const int32_t n = (int32_t)g.members.size();
    if (n == 0) continue;
    double2* taps = reinterpret_cast<double2*>(bank + g.off_taps);
    TapGen a{p.desc.zmax, p.desc.dz, p.desc.dw, p.n_z, p.J, g.taps, n, d_members + g.first_member,
             taps, p.desc.margin_bins};
    const int64_t total = (int64_t)n * 2 * g.taps;
    const int threads = 256;
    const int64_t blocks = (total + threads - 1) / threads;
    hipLaunchKernelGGL(gen_taps_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, a, gl);
    JERK_HIP_CHECK(hipGetLastError());
    if (g.path == JERK_PATH_FFT_FP32) {
      SpecGen s{taps, reinterpret_cast<float2*>(bank + g.off_fft), n, g.taps, g.seg_len};
      dim3 grid((unsigned)((g.seg_len + 255) / 256), (unsigned)(2 * n));
      hipLaunchKernelGGL(gen_fft_spectra_kernel, grid, dim3(256), 0, stream, s);
      JERK_HIP_CHECK(hipGetLastError());
    } else {
      gemm_bank_build(p, g, taps, bank + g.off_gemm, stream);
    }
  }
}

}  // namespace jerk
