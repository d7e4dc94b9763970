// Direct correlation of a spectrum with a width group's templates as a dense
// real GEMM on the gfx950 matrix cores (v_mfma_f32_32x32x16_{bf16,f16}).
//
// For outputs k0 (columns) and template components (rows), the contraction runs
// over the group's K taps, real-expanded to 2K:
//   Yr = sum_j Xr[k0-h+1+j] br_j - Xi[k0-h+1+j] bi_j
//   Yi = sum_j Xr[k0-h+1+j] bi_j + Xi[k0-h+1+j] br_j          (h = K/2)
// with b_j = conj(T(h - 1 - j + phase/2)) the template's taps. The spectrum
// operand is a Hankel matrix B[kk][n] = X[base + n + kk]; it is never formed:
// a window of the spectrum sits in LDS and each lane reads 8 consecutive
// values of it. Eight copies of the window, shifted by 0..7 elements, make
// every such read a 16-byte-aligned ds_read_b128 (the shift a lane needs is
// fixed by its column).
//
// Split-BF16: X = X_hi + X_lo and A = A_hi + A_lo with bf16 parts; the
// product keeps A_hi X_hi + A_hi X_lo + A_lo X_hi (FP32 accumulation), a
// relative error of a few 2^-17. FP16: one product in FP16 (2^-11).
//
// Row layout of the tap operand (32 rows per block of 8 templates): row i is
// template i/4 of the block, component i%4 = (Yr phase 0, Yi phase 0,
// Yr phase 1, Yi phase 1). In the 32x32 accumulator, lane l holds column l%32
// and, in registers 4q..4q+3, the four components of template 2q + l/32, so
// each lane forms both phases' powers in place and stores them as one float2.
#include "jerk_internal.h"

namespace jerk {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kWaves = 4;          // waves per workgroup
constexpr int kColTiles = 4;       // 32-column tiles per window
constexpr int kWin = 32 * kColTiles;  // outputs per window
constexpr int kKsChunk = 4;        // k-steps of tap fragments held in registers at once

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f16_bits(float x) {
  _Float16 h = (_Float16)x;
  return __builtin_bit_cast(uint16_t, h);
}

// Window stride (elements) of one shifted copy: 64 m + 8, so that the eight
// copies start 16 bytes apart modulo 128 bytes (distinct LDS banks for the
// eight lanes of a ds_read_b128 group).
__host__ __device__ constexpr int win_stride(int taps) { return ((kWin + taps + 8 + 63) / 64) * 64 + 8; }

template <bool SPLIT>
__host__ __device__ constexpr int n_parts() { return SPLIT ? 4 : 2; }  // (r_hi, i_hi, r_lo, i_lo) or (r, i)

// Workgroup: kWaves waves, wave wv owns row blocks rb0 + wv*RB .. + RB-1 (8
// templates each) and every column of the window.
template <int RB, bool SPLIT>
__global__ void __launch_bounds__(64 * kWaves) gemm_correlate_kernel(GemmArgs a, int64_t windows_per_wg,
                                                                      int64_t n_colchunks) {
  extern __shared__ uint16_t lds[];  // [parts][8 shifts][stride]
  const int K = a.taps;
  const int hg = K / 2;
  const int KS = 2 * K / 16;        // k-steps of the real-expanded contraction
  const int ksr = K / 16;           // k-steps over the real parts
  const int stride = win_stride(K);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t cc = blockIdx.x % n_colchunks;
  const int tblk = (int)(blockIdx.x / n_colchunks);
  const int n_members = a.m_end - a.m_begin;
  const int rb_first = (tblk * kWaves + wv) * RB;  // row block index within [m_begin, m_end) / 8
  constexpr int P = SPLIT ? 2 : 1;  // parts of the tap operand

  const uint16_t* frag = static_cast<const uint16_t*>(a.bank_gemm);
  // Fragment (rb, ks, part) of the group: 64 lanes x 8 values.
  auto frag_ptr = [&](int rb_global, int ks, int part) {
    return frag + ((((int64_t)rb_global * KS + ks) * P + part) * 64 + lane) * 8;
  };
  const int rb_base_global = a.m_begin / 8;  // m_begin is a multiple of 8

  for (int64_t wi = 0; wi < windows_per_wg; ++wi) {
    const int64_t win = cc * windows_per_wg + wi;
    const int64_t col0 = win * kWin;  // first output k0 of the window
    if (col0 >= a.nbins) break;
    // ---- fill the LDS window: position x holds bin col0 - hg + 1 + x + shift ----
    const int64_t bin0 = col0 - hg + 1;
    const int npos = kWin + K + 8;
    for (int x = threadIdx.x; x < npos; x += 64 * kWaves) {
      const int64_t bin = bin0 + x;
      float2 v = make_float2(0.f, 0.f);
      if (bin >= 0 && bin < a.nbins) v = a.spec[bin];
      uint16_t parts[4];
      if constexpr (SPLIT) {
        parts[0] = bf16_rne(v.x);
        parts[1] = bf16_rne(v.y);
        parts[2] = bf16_rne(v.x - bf16_to_f32(parts[0]));
        parts[3] = bf16_rne(v.y - bf16_to_f32(parts[1]));
      } else {
        parts[0] = f16_bits(v.x);
        parts[1] = f16_bits(v.y);
      }
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int xs = x - s;  // copy s holds element xs + s at index xs
        if (xs >= 0 && xs < stride) {
#pragma unroll
          for (int pp = 0; pp < n_parts<SPLIT>(); ++pp) lds[(pp * 8 + s) * stride + xs] = parts[pp];
        }
      }
    }
    __syncthreads();

    f32x16 acc[RB][kColTiles];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int c = 0; c < kColTiles; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[r][c][v] = 0.f;

    const int col = lane & 31;
    const int shift = col & 7;
    const int khalf = (lane >> 5) * 8;
    for (int ks0 = 0; ks0 < KS; ks0 += kKsChunk) {
      // tap fragments of this chunk
      uint4 afr[RB][kKsChunk][P];
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < kKsChunk; ++q)
#pragma unroll
          for (int pp = 0; pp < P; ++pp) {
            const int ks = ks0 + q;
            if (ks < KS) afr[r][q][pp] = *reinterpret_cast<const uint4*>(frag_ptr(rb_base_global + rb_first + r, ks, pp));
            else afr[r][q][pp] = make_uint4(0, 0, 0, 0);
          }
#pragma unroll
      for (int q = 0; q < kKsChunk; ++q) {
        const int ks = ks0 + q;
        if (ks >= KS) break;
        const bool imag = ks >= ksr;
        const int koff = (imag ? ks - ksr : ks) * 16 + khalf;  // tap offset of this lane's 8 values
#pragma unroll
        for (int c = 0; c < kColTiles; ++c) {
          const int x = c * 32 + col + koff;  // window position of the first value
          const int xa = x - shift;            // aligned index in copy 'shift'
          const int p_hi = imag ? 1 : 0;
          const uint4 bhi = *reinterpret_cast<const uint4*>(&lds[(p_hi * 8 + shift) * stride + xa]);
          if constexpr (SPLIT) {
            const uint4 blo = *reinterpret_cast<const uint4*>(&lds[((p_hi + 2) * 8 + shift) * stride + xa]);
#pragma unroll
            for (int r = 0; r < RB; ++r) {
              acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, afr[r][q][0]),
                                                                 __builtin_bit_cast(bf16x8, bhi), acc[r][c], 0, 0, 0);
              acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, afr[r][q][0]),
                                                                 __builtin_bit_cast(bf16x8, blo), acc[r][c], 0, 0, 0);
              acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, afr[r][q][1]),
                                                                 __builtin_bit_cast(bf16x8, bhi), acc[r][c], 0, 0, 0);
            }
          } else {
#pragma unroll
            for (int r = 0; r < RB; ++r)
              acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, afr[r][q][0]),
                                                                __builtin_bit_cast(f16x8, bhi), acc[r][c], 0, 0, 0);
          }
        }
      }
    }
    // ---- epilogue: |Y|^2 for both phases, one float2 per (template, k0) ----
#pragma unroll
    for (int r = 0; r < RB; ++r) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m_local = (rb_first + r) * 8 + 2 * q + (lane >> 5);
        if (m_local >= n_members) continue;
        const int t = a.members[a.m_begin + m_local];
        if (t < a.t_begin || t >= a.t_end) continue;
        float* row = a.plane + (int64_t)(t - a.t_begin) * a.ld;
#pragma unroll
        for (int c = 0; c < kColTiles; ++c) {
          const int64_t k0 = col0 + c * 32 + col;
          if (k0 < a.nbins) {
            const f32x16& z = acc[r][c];
            const float p0 = fmaf(z[4 * q], z[4 * q], z[4 * q + 1] * z[4 * q + 1]);
            const float p1 = fmaf(z[4 * q + 2], z[4 * q + 2], z[4 * q + 3] * z[4 * q + 3]);
            *reinterpret_cast<float2*>(row + 2 * k0) = make_float2(p0, p1);
          }
        }
      }
    }
    __syncthreads();  // LDS is refilled for the next window
  }
}

// Converts FP64 taps [n][2][K] into tap-operand fragments [rb][ks][part][lane][8].
__global__ void gemm_frag_kernel(const double2* __restrict__ taps, uint16_t* __restrict__ out, int n, int K,
                                 int split, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int P = split ? 2 : 1;
  const int KS = 2 * K / 16;
  const int e = (int)(idx % 8);
  const int lane = (int)((idx / 8) % 64);
  const int part = (int)((idx / 512) % P);
  const int ks = (int)((idx / (512 * P)) % KS);
  const int64_t rb = idx / (512 * (int64_t)P * KS);
  const int i = lane & 31;
  const int m = (int)(rb * 8 + i / 4);
  const int comp = i % 4;
  const int phase = comp / 2;
  const bool im_row = (comp & 1) != 0;
  const int kk = ks * 16 + (lane >> 5) * 8 + e;
  double val = 0.0;
  if (m < n) {
    const bool re_col = kk < K;
    const int j = re_col ? kk : kk - K;
    const double2 b = taps[((int64_t)m * 2 + phase) * K + j];
    // Yr row: [ br | -bi ], Yi row: [ bi | br ]
    val = im_row ? (re_col ? b.y : b.x) : (re_col ? b.x : -b.y);
  }
  uint16_t bits;
  if (split) {
    const float hi_f = (float)val;  // nearest float, then nearest bf16 of it
    uint32_t u = __float_as_uint(hi_f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    const uint16_t hi = (uint16_t)(u >> 16);
    if (part == 0) {
      bits = hi;
    } else {
      const double rem = val - (double)__uint_as_float((uint32_t)hi << 16);
      uint32_t v = __float_as_uint((float)rem);
      v += 0x7FFFu + ((v >> 16) & 1u);
      bits = (uint16_t)(v >> 16);
    }
  } else {
    _Float16 h = (_Float16)(float)val;
    bits = __builtin_bit_cast(uint16_t, h);
  }
  out[idx] = bits;
}

}  // namespace

size_t gemm_bank_bytes(int32_t n_members, int32_t taps, int32_t path) {
  const size_t P = path == JERK_PATH_GEMM_FP16 ? 1 : 2;
  const size_t n_rb = ((size_t)n_members + 7) / 8 + 2 * kWaves;  // padded: a workgroup may read past the end
  return n_rb * (2 * (size_t)taps / 16) * P * 64 * 8 * sizeof(uint16_t);
}

void gemm_bank_build(const Plan& p, const Group& g, const double2* taps, void* out, hipStream_t stream) {
  (void)p;
  const int n = (int)g.members.size();
  const int split = g.path == JERK_PATH_GEMM_FP16 ? 0 : 1;
  const int64_t total = (int64_t)(g.gemm_bytes / sizeof(uint16_t));
  const int threads = 256;
  hipLaunchKernelGGL(gemm_frag_kernel, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, stream,
                     taps, static_cast<uint16_t*>(out), n, g.taps, split, total);
  JERK_HIP_CHECK(hipGetLastError());
}

void gemm_correlate_launch(const GemmArgs& a, hipStream_t stream) {
  const int n_members = a.m_end - a.m_begin;
  if (n_members <= 0 || a.nbins <= 0) return;
  require(a.m_begin % 8 == 0, JERK_EINTERNAL, "GEMM member range must start on a block of 8");
  require(a.taps % 16 == 0 && a.taps >= 16 && a.taps <= 512, JERK_EINTERNAL, "GEMM taps out of range");
  const bool split = a.path != JERK_PATH_GEMM_FP16;
  const int stride = win_stride(a.taps);
  const size_t lds_bytes = (size_t)n_parts<true>() * 8 * stride * sizeof(uint16_t);
  const size_t lds_use = split ? lds_bytes : lds_bytes / 2;
  const int64_t n_win = (a.nbins + kWin - 1) / kWin;
  // RB = 2 row blocks per wave for narrow groups (fewer tap-fragment loads per MFMA), 1 otherwise.
  const int RB = n_members > 8 * kWaves ? 2 : 1;
  const int64_t templates_per_wg = (int64_t)8 * kWaves * RB;
  const int64_t n_tblk = (n_members + templates_per_wg - 1) / templates_per_wg;
  // Enough workgroups to fill the chip several times over; each walks consecutive windows.
  int64_t windows_per_wg = 1;
  while (n_tblk * ((n_win + windows_per_wg - 1) / windows_per_wg) > 8192 && windows_per_wg < 64) windows_per_wg *= 2;
  const int64_t n_colchunks = (n_win + windows_per_wg - 1) / windows_per_wg;
  const int64_t blocks = n_tblk * n_colchunks;
  require(blocks < (1ll << 31), JERK_EINVAL, "search too large for one launch");
  dim3 grid((unsigned)blocks), block(64 * kWaves);
  if (split) {
    if (RB == 2)
      hipLaunchKernelGGL((gemm_correlate_kernel<2, true>), grid, block, lds_use, stream, a, windows_per_wg, n_colchunks);
    else
      hipLaunchKernelGGL((gemm_correlate_kernel<1, true>), grid, block, lds_use, stream, a, windows_per_wg, n_colchunks);
  } else {
    if (RB == 2)
      hipLaunchKernelGGL((gemm_correlate_kernel<2, false>), grid, block, lds_use, stream, a, windows_per_wg, n_colchunks);
    else
      hipLaunchKernelGGL((gemm_correlate_kernel<1, false>), grid, block, lds_use, stream, a, windows_per_wg, n_colchunks);
  }
  JERK_HIP_CHECK(hipGetLastError());
}

}  // namespace jerk
