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
// values of it. Two copies of the window, the second shifted by one element,
// make every such read four aligned 32-bit words (which copy a lane reads is
// fixed by the parity of its column).
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
#include <algorithm>

#include "jerk_internal.h"

namespace jerk {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f2v __attribute__((ext_vector_type(2)));

constexpr int kFragKsPad = 8;  // spare row blocks at the end of a group's fragments (see gemm_bank_bytes)

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

// Largest 32-bit value of the 32-lane half of a wave that holds `lane` (lanes 0-31 and 32-63
// separately), the same in every lane of that half: rows of 16 lanes by DPP (pairs, quads,
// rotations by 4 and 8), then each half's two row maxima from lanes 0, 16 (32, 48). Entered by
// every lane.
__device__ __forceinline__ uint32_t half_wave_max_u32(uint32_t x, int lane) {
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xF, 0xF, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false));
  const uint32_t a = max((uint32_t)__builtin_amdgcn_readlane((int)x, 0), (uint32_t)__builtin_amdgcn_readlane((int)x, 16));
  const uint32_t b = max((uint32_t)__builtin_amdgcn_readlane((int)x, 32), (uint32_t)__builtin_amdgcn_readlane((int)x, 48));
  return lane < 32 ? a : b;
}

// LDS window of one wave: for each part (re_hi, im_hi, re_lo, im_lo; FP16: re, im)
// two copies of the window, copy s holding element x + s at element index x, so
// that any 8 consecutive elements starting at x are 4 aligned 32-bit words of
// copy (x mod 2). Copy stride in words is 32 m + 16: the two copies of a part
// start 16 banks apart.
__host__ __device__ constexpr int win_words(int cols, int taps) {
  return ((cols + taps + 8) / 2 + 15) / 32 * 32 + 16;
}

template <int CT>
__host__ __device__ constexpr int window_cols() { return 32 * CT; }

// NW = 1: one wave per workgroup. The wave owns RB row blocks (8 templates each)
// of the group and a run of consecutive windows of 32*CT outputs. Tap fragments
// for up to KC k-steps stay in registers; the spectrum window is double-buffered
// in LDS and the next window's loads are issued before the current window's MFMAs.
// NW > 1 (resident split-BF16, RB = 1): NW waves share one row block, each with
// its own run of windows; the block's tap fragments are copied once into LDS and
// read from there at every k-step instead of being held in 64+ registers per wave,
// which leaves room for a third wave per SIMD.
// LDS words of a row block's resident split-BF16 tap fragments: kc slots x hi/lo x 64 lanes x uint4
__host__ __device__ constexpr int lds_a_words(int kc) { return kc * 2 * 64 * 4; }

template <int RB, int CT, int KC, int MAXLD, bool SPLIT, bool RESIDENT, bool KEYS, int KT, int NW = 1>
__device__ __forceinline__ void gemm_tile(const GemmArgs& a, int64_t windows_per_wg, int64_t n_colchunks, int64_t blk,
                                          uint32_t* lds32) {
  static_assert(NW == 1 || (RB == 1 && SPLIT && RESIDENT), "several waves per workgroup: resident split-BF16 only");
  constexpr int P = SPLIT ? 2 : 1;        // parts of each operand (hi, lo)
  constexpr int NPART = 2 * P;            // LDS part arrays (re/im x hi/lo)
  constexpr int COLS = window_cols<CT>();
  const int K = KT > 0 ? KT : a.taps;  // KT > 0: the tap count is a compile-time constant
  const int hg = K / 2;
  const int KS = 2 * K / 16;   // k-steps of the real-expanded contraction
  const int ksr = K / 16;      // k-steps over the real parts
  const int WW = win_words(COLS, K);
  const int buf_words = NPART * 2 * WW;
  const int lane = threadIdx.x & 63;
  const int wave = NW > 1 ? (int)(threadIdx.x >> 6) : 0;
  const int64_t ncg = (n_colchunks + NW - 1) / NW;  // column-chunk groups (one chunk per wave)
  const int64_t cc = (blk % ncg) * NW + wave;
  const int tblk = (int)(blk / ncg);
  // NW > 1: the row block's tap fragments [slot][part][lane] (uint4) first, then each wave's
  // window buffers
  uint4* const lds_a = reinterpret_cast<uint4*>(lds32);
  if constexpr (NW > 1) lds32 += lds_a_words(KC) + wave * 2 * (2 * P * 2 * win_words(COLS, K));
  const int n_members = a.m_end - a.m_begin;
  const int rb0 = a.m_begin / 8 + tblk * RB;  // first row block (group-relative)
  const uint16_t* __restrict__ frag = static_cast<const uint16_t*>(a.bank_gemm);
  auto frag_ptr = [&](int rb, int ks, int part) {
    return reinterpret_cast<const uint4*>(frag + ((((int64_t)rb * KS + ks) * P + part) * 64 + lane) * 8);
  };

  const int64_t win_first = cc * windows_per_wg;
  const int64_t n_win_total = (a.nbins + COLS - 1) / COLS;
  const int64_t win_last = min(win_first + windows_per_wg, n_win_total);
  if constexpr (NW > 1) {
    // every wave copies its share of the fragments before any wave may leave
    constexpr int NI_ = KC / 4 > 0 ? KC / 4 : 1;
    for (int e = threadIdx.x; e < KC * P * 64; e += 64 * NW) {
      const int slot = e / (P * 64), pp = (e / 64) % P, ln = e % 64;
      const int part = slot / (2 * NI_), parity = (slot / NI_) % 2, i = slot % NI_;
      const int ksp = parity + 2 * i;
      const int rbg = a.m_begin / 8 + tblk;
      lds_a[e] = ksp < ksr ? *reinterpret_cast<const uint4*>(frag + ((((int64_t)rbg * KS + part * ksr + ksp) * P + pp) * 64 + ln) * 8)
                           : make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
  }
  if (win_first >= win_last) return;
  const int npos = COLS + K + 8;            // window elements (with alignment slack), <= 64 * MAXLD

  // Loads of one window into registers (lane x covers positions lane + 64 i).
  float2 pre[MAXLD];
  auto load_window = [&](int64_t win) {
    const int64_t bin0 = win * COLS - hg + 1;
#pragma unroll
    for (int i = 0; i < MAXLD; ++i) {
      const int x = lane + 64 * i;
      const int64_t bin = bin0 + x;
      pre[i] = (x < npos && bin >= 0 && bin < a.nbins) ? a.spec[bin] : make_float2(0.f, 0.f);
    }
  };
  // Split and store a loaded window into LDS buffer `buf`.
  auto store_window = [&](int buf) {
    uint16_t* l16 = reinterpret_cast<uint16_t*>(lds32 + buf * buf_words);
#pragma unroll
    for (int i = 0; i < MAXLD; ++i) {
      const int x = lane + 64 * i;
      if (x < npos) {
        uint16_t parts[4];
        if constexpr (SPLIT) {
          parts[0] = bf16_rne(pre[i].x);
          parts[1] = bf16_rne(pre[i].y);
          parts[2] = bf16_rne(pre[i].x - bf16_to_f32(parts[0]));
          parts[3] = bf16_rne(pre[i].y - bf16_to_f32(parts[1]));
        } else {
          parts[0] = f16_bits(pre[i].x);
          parts[1] = f16_bits(pre[i].y);
        }
#pragma unroll
        for (int pp = 0; pp < NPART; ++pp) {
          // copy 0: element x at index x; copy 1: element x at index x - 1
          l16[(pp * 2 + 0) * 2 * WW + x] = parts[pp];
          if (x >= 1) l16[(pp * 2 + 1) * 2 * WW + x - 1] = parts[pp];
        }
      }
    }
  };

  // Tap fragments stay resident across windows when the group fits in KC
  // k-steps (RESIDENT: the host guarantees KS <= KC).
  uint4 afr[RB][KC][P];
  auto load_frags = [&](int ks0) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < KC; ++q)
#pragma unroll
        for (int pp = 0; pp < P; ++pp)
          afr[r][q][pp] = (ks0 + q < KS) ? *frag_ptr(rb0 + r, ks0 + q, pp) : make_uint4(0, 0, 0, 0);
  };
  // Split-BF16 resident fragments are kept in the order the main loop visits
  // k-steps: slot (part * 2 + parity) * NI + i holds k-step part * ksr + parity + 2 i.
  // (FP16 keeps k-step order: its 32 resident slots leave no room for the
  // fragment ring below.)
  constexpr bool REUSE = RESIDENT && SPLIT;
  constexpr int NI = KC / 4 > 0 ? KC / 4 : 1;
  if constexpr (!REUSE && RESIDENT) load_frags(0);
  if constexpr (REUSE && NW == 1) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int slot = 0; slot < KC; ++slot) {
        const int part = slot / (2 * NI), parity = (slot / NI) % 2, i = slot % NI;
        const int ksp = parity + 2 * i;
#pragma unroll
        for (int pp = 0; pp < P; ++pp)
          afr[r][slot][pp] = ksp < ksr ? *frag_ptr(rb0 + r, part * ksr + ksp, pp) : make_uint4(0, 0, 0, 0);
      }
  }

  const int col = lane & 31;
  const int shift = col & 1;
  const int khalf = (lane >> 5) * 8;

  // The spectrum operand of column tile c at k-step ks' (within a part) starts
  // at window element 32 c + 16 ks' + col + khalf = 16 d + col + khalf with
  // d = 2 c + ks': fragments depend on d only (Hankel structure).
  auto load_b = [&](const uint32_t* lb, int part, int d, uint4& h, uint4& l) {
    const int x = d * 16 + col + khalf;  // first element of this lane's 8
    const int w0 = (x - shift) >> 1;     // word index in copy `shift`
    const uint32_t* ph = lb + (part * 2 + shift) * WW + w0;
    h = make_uint4(ph[0], ph[1], ph[2], ph[3]);
    if constexpr (SPLIT) {
      const uint32_t* pl = lb + ((part + 2) * 2 + shift) * WW + w0;
      l = make_uint4(pl[0], pl[1], pl[2], pl[3]);
    }
  };
  // The products of one k-step (tap fragments afr[.][q]), ordered so that
  // consecutive MFMAs update different accumulators.
  auto products_with = [&](const uint4 (&A)[RB][KC][P], int q, const uint4 (&bhi)[CT], const uint4 (&blo)[CT],
                           f32x16 (&acc)[RB][CT]) {
    if constexpr (SPLIT) {
#pragma unroll
      for (int prod = 0; prod < 3; ++prod)
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int c = 0; c < CT; ++c) {
            const uint4 av = prod == 2 ? A[r][q][1] : A[r][q][0];
            const uint4 bv = prod == 1 ? blo[c] : bhi[c];
            acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                               __builtin_bit_cast(bf16x8, bv), acc[r][c], 0, 0, 0);
          }
    } else {
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, A[r][q][0]),
                                                            __builtin_bit_cast(f16x8, bhi[c]), acc[r][c], 0, 0, 0);
    }
  };
  auto products = [&](int q, const uint4 (&bhi)[CT], const uint4 (&blo)[CT], f32x16 (&acc)[RB][CT]) {
    if constexpr (NW > 1) {
      // this k-step's hi and lo tap fragments from LDS (slot q)
      uint4 A1[RB][KC][P];
#pragma unroll
      for (int pp = 0; pp < P; ++pp) A1[0][0][pp] = lds_a[(q * P + pp) * 64 + lane];
      products_with(A1, 0, bhi, blo, acc);
    } else {
      products_with(afr, q, bhi, blo, acc);
    }
  };

  // Peak of each of this lane's rows (template 2q + lane/32 of each row block) over all its
  // windows: the best power's bits and 0xFFFFFFFF - p of its plane index (0: no point yet).
  // Points come in increasing p, so only a strictly larger power replaces the best and equal
  // powers keep the lowest index, the order of the 64-bit key (bits << 32 | 0xFFFFFFFF - p).
  uint32_t bhi_k[KEYS ? RB : 1][4], blo_k[KEYS ? RB : 1][4];
#pragma unroll
  for (int r = 0; r < (KEYS ? RB : 1); ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) bhi_k[r][q] = blo_k[r][q] = 0u;

  // Output row of each of this lane's templates (2q + lane/32 of each row
  // block), -1 when it is outside the requested range; fixed for all windows.
  int64_t orow_of[RB][4];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m_local = (tblk * RB + r) * 8 + 2 * q + (lane >> 5);
      int64_t orow = -1;
      if (m_local < n_members) {
        const int t = a.members[a.m_begin + m_local];
        const int64_t o =
            a.row_by_member ? (int64_t)(a.m_begin + m_local - a.row_base) : (int64_t)(t - a.t_begin);
        // o < 0: below the requested member range (same block of 8)
        if (t >= a.t_begin && t < a.t_end && o >= 0) orow = o;
      }
      orow_of[r][q] = orow;
    }

  // Wait here for the loop-invariant loads above (resident tap fragments, member
  // rows). Otherwise the first use inside the window loop waits on the vector
  // memory counter, which by then also counts the previous window's plane
  // stores and the next window's loads, and every window stalls on them.
  // 0x0F70: vmcnt 0, expcnt and lgkmcnt unconstrained.
  __builtin_amdgcn_s_waitcnt(0x0F70);

  // The window buffers of a wave are its own: with NW > 1 only the compiler has to keep the LDS
  // stores and loads in order (a wave's LDS instructions execute in issue order).
  auto window_sync = [&]() {
    if constexpr (NW > 1) asm volatile("" ::: "memory");
    else __syncthreads();
  };
  load_window(win_first);
  store_window(0);
  window_sync();
  for (int64_t win = win_first; win < win_last; ++win) {
    const int buf = (int)((win - win_first) & 1);
    if (win + 1 < win_last) load_window(win + 1);  // in flight during the MFMAs
    const uint32_t* lb = lds32 + buf * buf_words;

    f32x16 acc[RB][CT];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[r][c][v] = 0.f;

    if constexpr (REUSE) {
      // k-steps of each part in two interleaved runs (even, then odd ks'):
      // stepping ks' by 2 moves every column tile's fragment to the next tile's,
      // so each step reads one new fragment from LDS instead of CT.
#pragma unroll
      for (int part = 0; part < 2; ++part)
#pragma unroll
        for (int parity = 0; parity < 2; ++parity) {
          if (parity >= ksr) continue;
          uint4 bhi[CT], blo[CT];
#pragma unroll
          for (int c = 0; c < CT; ++c) load_b(lb, part, parity + 2 * c, bhi[c], blo[c]);
#pragma unroll
          for (int i = 0; i < NI; ++i) {
            const int ksp = parity + 2 * i;
            if (ksp >= ksr) break;
            products((part * 2 + parity) * NI + i, bhi, blo, acc);
            if (ksp + 2 < ksr) {
#pragma unroll
              for (int c = 0; c + 1 < CT; ++c) {
                bhi[c] = bhi[c + 1];
                blo[c] = blo[c + 1];
              }
              load_b(lb, part, ksp + 2 + 2 * (CT - 1), bhi[CT - 1], blo[CT - 1]);
            }
          }
        }
    } else {
      // one chunk of KC k-steps: its tap fragments (streamed), then its products
      auto chunk = [&](int ks0) {
        if constexpr (!RESIDENT) load_frags(ks0);
#pragma unroll
        for (int q = 0; q < KC; ++q) {
          const int ks = ks0 + q;
          if (ks >= KS) break;
          const int part = ks >= ksr ? 1 : 0;
          uint4 bhi[CT], blo[CT];
#pragma unroll
          for (int c = 0; c < CT; ++c) load_b(lb, part, ks - part * ksr + 2 * c, bhi[c], blo[c]);
          products(q, bhi, blo, acc);
        }
      };
      if constexpr (KT > 0 && !RESIDENT && KT <= (KEYS ? 160 : 192)) {
        // Two chunk buffers: the next chunk's tap fragments load while this
        // chunk's MFMAs run (the tap count is a compile-time constant, so the
        // buffer of every chunk is fixed). Wider groups would spill.
        constexpr int KST = 2 * KT / 16;
        constexpr int NCH = (KST + KC - 1) / KC;
        uint4 abuf[2][RB][KC][P];
        auto load_into = [&](uint4 (&A)[RB][KC][P], int ks0) {
#pragma unroll
          for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int q = 0; q < KC; ++q)
#pragma unroll
              for (int pp = 0; pp < P; ++pp)
                A[r][q][pp] = (ks0 + q < KST) ? *frag_ptr(rb0 + r, ks0 + q, pp) : make_uint4(0, 0, 0, 0);
        };
        load_into(abuf[0], 0);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          if (ch + 1 < NCH) {
            load_into(abuf[(ch + 1) & 1], (ch + 1) * KC);
            // keep the loads here: the scheduler would otherwise sink each one to
            // just before its MFMA, leaving its latency exposed
            __builtin_amdgcn_sched_barrier(0);
          }
#pragma unroll
          for (int q = 0; q < KC; ++q) {
            const int ks = ch * KC + q;
            if (ks >= KST) break;
            const int part = ks >= ksr ? 1 : 0;
            uint4 bhi[CT], blo[CT];
#pragma unroll
            for (int c = 0; c < CT; ++c) load_b(lb, part, ks - part * ksr + 2 * c, bhi[c], blo[c]);
            products_with(abuf[ch & 1], q, bhi, blo, acc);
          }
        }
      } else if constexpr (KT > 0) {
#pragma unroll
        for (int ks0 = 0; ks0 < 2 * KT / 16; ks0 += KC) chunk(ks0);
      } else {
        for (int ks0 = 0; ks0 < KS; ks0 += KC) chunk(ks0);
      }
    }
    // ---- epilogue: |Y|^2 for both phases, one float2 per (template, k0) ----
    const int64_t col0 = win * COLS;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t orow = orow_of[r][q];
        if (orow < 0) continue;
        float2* __restrict__ row = a.plane ? reinterpret_cast<float2*>(a.plane + orow * a.ld) + col0 : nullptr;
        const int lim = (int)min((int64_t)COLS, a.nbins - col0);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const int j = c * 32 + col;
          if (j < lim) {
            const f32x16& z = acc[r][c];
            const float p0 = fmaf(z[4 * q], z[4 * q], z[4 * q + 1] * z[4 * q + 1]);
            const float p1 = fmaf(z[4 * q + 2], z[4 * q + 2], z[4 * q + 3] * z[4 * q + 3]);
            // written once, never read here: non-temporal, as on the FFT path
            if (row) __builtin_nontemporal_store(f2v{p0, p1}, reinterpret_cast<f2v*>(row) + j);
            if constexpr (KEYS) {
              const uint32_t lo0 = 0xFFFFFFFFu - 2u * (uint32_t)(col0 + j);  // p < 2^32 (nbins < 2^31)
              const uint32_t u0 = __float_as_uint(p0), u1 = __float_as_uint(p1);
              if (u0 > bhi_k[r][q] || blo_k[r][q] == 0u) {
                bhi_k[r][q] = u0;
                blo_k[r][q] = lo0;
              }
              if (u1 > bhi_k[r][q]) {
                bhi_k[r][q] = u1;
                blo_k[r][q] = lo0 - 1u;
              }
            }
          }
        }
      }
    }
    if (win + 1 < win_last) store_window(buf ^ 1);
    window_sync();
  }
  if constexpr (KEYS) {
    // combine the 32 lanes of each row (lanes l and l + 32 hold different templates)
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // high words first, then the low words of the lanes holding the largest high word
        const uint32_t mh = half_wave_max_u32(bhi_k[r][q], lane);
        const uint32_t ml = half_wave_max_u32(bhi_k[r][q] == mh ? blo_k[r][q] : 0u, lane);
        const uint64_t k = ((uint64_t)mh << 32) | ml;
        if ((lane & 31) == 0 && orow_of[r][q] >= 0)
          atomicMax(reinterpret_cast<unsigned long long*>(a.row_max + orow_of[r][q]), (unsigned long long)k);
      }
  }
}

template <int RB, int CT, int KC, int MAXLD, bool SPLIT, bool RESIDENT, bool KEYS, int KT>
__global__ void __launch_bounds__(64, 2) gemm_correlate_kernel(GemmArgs a, int64_t windows_per_wg, int64_t n_colchunks) {
  extern __shared__ uint32_t lds32[];
  gemm_tile<RB, CT, KC, MAXLD, SPLIT, RESIDENT, KEYS, KT>(a, windows_per_wg, n_colchunks, blockIdx.x, lds32);
}

// NW waves per workgroup sharing one row block's tap fragments in LDS (resident split-BF16).
template <int CT, int KC, int MAXLD, bool KEYS, int KT, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3)))
gemm_correlate_mw_kernel(GemmArgs a, int64_t windows_per_wg, int64_t n_colchunks) {
  extern __shared__ uint32_t lds32[];
  gemm_tile<1, CT, KC, MAXLD, true, true, KEYS, KT, NW>(a, windows_per_wg, n_colchunks, blockIdx.x, lds32);
}

// Several narrow width groups in one launch (split-BF16 with at most 64 taps, or FP16 with
// at most 256): workgroup i belongs to the job whose block range holds it and runs that
// job's kernel body (one per tap count), so a small search is one launch instead of one per
// group. The job table travels in the kernel arguments.
constexpr int kGemmMultiJobs = 8;
struct GemmMulti {
  GemmArgs job[kGemmMultiJobs];
  int64_t windows_per_wg[kGemmMultiJobs];
  int64_t n_colchunks[kGemmMultiJobs];
  int64_t block_begin[kGemmMultiJobs + 1];
  int32_t n;
};

template <bool SPLIT, bool KEYS>
__global__ void __launch_bounds__(64, 2) gemm_multi_kernel(GemmMulti m) {
  extern __shared__ uint32_t lds32[];
  const int64_t blk = blockIdx.x;
  int j = 0;
  while (j + 1 < m.n && blk >= m.block_begin[j + 1]) ++j;
  const GemmArgs& a = m.job[j];
  const int64_t local = blk - m.block_begin[j];
  if constexpr (SPLIT) {
    switch (a.taps) {
      case 16: gemm_tile<1, 4, 4, 4, true, true, KEYS, 16>(a, m.windows_per_wg[j], m.n_colchunks[j], local, lds32); break;
      case 32: gemm_tile<1, 4, 4, 4, true, true, KEYS, 32>(a, m.windows_per_wg[j], m.n_colchunks[j], local, lds32); break;
      case 48: gemm_tile<1, 4, 8, 4, true, true, KEYS, 48>(a, m.windows_per_wg[j], m.n_colchunks[j], local, lds32); break;
      default: gemm_tile<1, 4, 8, 4, true, true, KEYS, 64>(a, m.windows_per_wg[j], m.n_colchunks[j], local, lds32); break;
    }
  } else {
    gemm_tile<1, 2, 32, 6, false, true, KEYS, 0>(a, m.windows_per_wg[j], m.n_colchunks[j], local, lds32);
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
  // padded: the last workgroup of a member range may read up to kFragKsPad row blocks past the end
  const size_t n_rb = ((size_t)n_members + 7) / 8 + kFragKsPad;
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

namespace {

struct GemmGrid {
  int64_t windows_per_wg, n_colchunks, blocks;
};

// Workgroups of one job: RB row blocks of 8 templates each by runs of consecutive windows of
// 32 CT outputs, about 16384 workgroups (16 one-wave workgroups per SIMD over the launch) or
// fewer: narrow groups have few row blocks, and 4096 left them at 2-3 waves per SIMD for the
// whole launch (the 48-tap group of the 2^22-bin search: 6.1e11 -> 7.1e11 points/s).
GemmGrid gemm_grid(const GemmArgs& a, int RB, int CT) {
  const int n_members = a.m_end - a.m_begin;
  const int cols = 32 * CT;
  const int64_t n_win = (a.nbins + cols - 1) / cols;
  const int64_t n_tblk = (n_members + 8 * RB - 1) / (8 * RB);
  int64_t wpw = 1;
  while (n_tblk * ((n_win + wpw - 1) / wpw) > 16384 && wpw < 256) wpw *= 2;
  const int64_t ncc = (n_win + wpw - 1) / wpw;
  return {wpw, ncc, n_tblk * ncc};
}

template <int RB, int CT, int KC, int MAXLD, bool SPLIT, bool RESIDENT, bool KEYS, int KT = 0>
void launch_cfg(const GemmArgs& a, hipStream_t stream) {
  require(KT == 0 || a.taps == KT, JERK_EINTERNAL, "GEMM kernel built for another tap count");
  constexpr int COLS = window_cols<CT>();
  const GemmGrid gg = gemm_grid(a, RB, CT);
  const int64_t windows_per_wg = gg.windows_per_wg, n_colchunks = gg.n_colchunks, blocks = gg.blocks;
  require(blocks < (1ll << 31), JERK_EINVAL, "search too large for one launch");
  require(COLS + a.taps + 8 <= 64 * MAXLD, JERK_EINTERNAL, "GEMM window larger than the per-lane load budget");
  require(!RESIDENT || 2 * a.taps / 16 <= KC, JERK_EINTERNAL, "resident tap fragments exceed the register budget");
  const size_t lds = (size_t)2 * (SPLIT ? 4 : 2) * 2 * win_words(COLS, a.taps) * sizeof(uint32_t);
  hipLaunchKernelGGL((gemm_correlate_kernel<RB, CT, KC, MAXLD, SPLIT, RESIDENT, KEYS, KT>), dim3((unsigned)blocks), dim3(64), lds, stream, a,
                     windows_per_wg, n_colchunks);
}

}  // namespace

// Split-BF16 groups of up to 128 taps: one kernel per tap count, so the k-step
// runs unroll completely and the fragment ring lives in fixed registers. Up to
// 96 taps a wave covers 4 column tiles (128 outputs) per window.
// Split-BF16 groups of more than 128 taps, tap fragments streamed in chunks of
// 8 k-steps. Up to 240 taps one kernel per tap count, so the chunk loop unrolls
// and the fragment loads can be issued early.
template <bool KEYS>
void launch_split_streamed(const GemmArgs& a, hipStream_t stream) {
  // chunks of 4 k-steps where the two chunk buffers fit in registers, else 8
  constexpr bool K = KEYS;
  switch (a.taps) {
    case 144: launch_cfg<1, 2, 4, 6, true, false, K, 144>(a, stream); break;
    case 160: launch_cfg<1, 2, 4, 6, true, false, K, 160>(a, stream); break;
    case 176: launch_cfg<1, 2, K ? 8 : 4, 6, true, false, K, 176>(a, stream); break;
    case 192: launch_cfg<1, 2, K ? 8 : 4, 6, true, false, K, 192>(a, stream); break;
    case 208: launch_cfg<1, 2, 8, 6, true, false, K, 208>(a, stream); break;
    case 224: launch_cfg<1, 2, 8, 6, true, false, K, 224>(a, stream); break;
    case 240: launch_cfg<1, 2, 8, 6, true, false, K, 240>(a, stream); break;
    // wider: the generic streamed kernels (fully unrolled, these would spill)
    default:
      if (a.taps <= 256) launch_cfg<1, 2, 8, 6, true, false, KEYS>(a, stream);
      else launch_cfg<1, 2, 8, 10, true, false, KEYS>(a, stream);
      break;
  }
}

// NW waves per workgroup (gemm_correlate_mw_kernel): workgroups of one row block by NW column
// chunks, the tap fragments in LDS.
template <int CT, int KC, int MAXLD, bool KEYS, int KT, int NW>
void launch_cfg_mw(const GemmArgs& a, hipStream_t stream) {
  require(a.taps == KT, JERK_EINTERNAL, "GEMM kernel built for another tap count");
  constexpr int COLS = window_cols<CT>();
  const GemmGrid gg = gemm_grid(a, 1, CT);
  const int64_t n_tblk = gg.blocks / gg.n_colchunks;
  const int64_t blocks = n_tblk * ((gg.n_colchunks + NW - 1) / NW);
  require(blocks < (1ll << 31), JERK_EINVAL, "search too large for one launch");
  require(COLS + a.taps + 8 <= 64 * MAXLD, JERK_EINTERNAL, "GEMM window larger than the per-lane load budget");
  require(2 * a.taps / 16 <= KC, JERK_EINTERNAL, "resident tap fragments exceed the slots");
  const size_t lds = (size_t)(lds_a_words(KC) + NW * 2 * (2 * 2 * 2 * win_words(COLS, a.taps))) * sizeof(uint32_t);
  hipLaunchKernelGGL((gemm_correlate_mw_kernel<CT, KC, MAXLD, KEYS, KT, NW>), dim3((unsigned)blocks), dim3(64 * NW), lds,
                     stream, a, gg.windows_per_wg, gg.n_colchunks);
}

template <bool KEYS>
void launch_split_resident(const GemmArgs& a, hipStream_t stream) {
  switch (a.taps) {
    case 16: launch_cfg<1, 4, 4, 4, true, true, KEYS, 16>(a, stream); break;
    case 32: launch_cfg<1, 4, 4, 4, true, true, KEYS, 32>(a, stream); break;
    // plane launches: four waves per workgroup sharing the tap fragments in LDS (3 waves per SIMD
    // instead of 2); peak-key launches keep one wave (their keys would spill)
    case 48:
      if constexpr (KEYS) launch_cfg<1, 4, 8, 4, true, true, KEYS, 48>(a, stream);
      else launch_cfg_mw<4, 8, 4, KEYS, 48, 4>(a, stream);
      break;
    case 64:
      if constexpr (KEYS) launch_cfg<1, 4, 8, 4, true, true, KEYS, 64>(a, stream);
      else launch_cfg_mw<4, 8, 4, KEYS, 64, 4>(a, stream);
      break;
    case 80:
      if constexpr (KEYS) launch_cfg<1, 4, 12, 4, true, true, KEYS, 80>(a, stream);
      else launch_cfg_mw<4, 12, 4, KEYS, 80, 4>(a, stream);
      break;
    case 96: launch_cfg<1, 4, 12, 4, true, true, KEYS, 96>(a, stream); break;
    case 112: launch_cfg<1, 2, 16, 4, true, true, KEYS, 112>(a, stream); break;
    default: launch_cfg<1, 2, 16, 4, true, true, KEYS, 128>(a, stream); break;
  }
}

bool gemm_multi_eligible(const GemmArgs& a) {
  return a.path == JERK_PATH_GEMM_FP16 ? a.taps <= 256 : a.taps <= 64;
}

// One launch for jobs[0..n) (2 <= n <= 8), all eligible, all split-BF16 or all FP16, all with
// or all without peak keys, each m_begin a multiple of 8.
void gemm_correlate_multi_launch(const GemmArgs* jobs, int n, hipStream_t stream) {
  require(n >= 1 && n <= kGemmMultiJobs, JERK_EINTERNAL, "bad GEMM job count");
  const bool split = jobs[0].path != JERK_PATH_GEMM_FP16;
  const bool keys = jobs[0].row_max != nullptr;
  GemmMulti m{};
  m.n = n;
  size_t lds = 0;
  int64_t total = 0;
  for (int i = 0; i < n; ++i) {
    const GemmArgs& a = jobs[i];
    require((a.path != JERK_PATH_GEMM_FP16) == split && (a.row_max != nullptr) == keys && gemm_multi_eligible(a),
            JERK_EINTERNAL, "GEMM jobs of one launch must share path and key mode");
    require(a.m_begin % 8 == 0 && a.taps % 16 == 0 && a.taps >= 16, JERK_EINTERNAL, "bad GEMM job");
    const int ct = split ? 4 : 2;
    const GemmGrid gg = gemm_grid(a, 1, ct);
    m.job[i] = a;
    m.windows_per_wg[i] = gg.windows_per_wg;
    m.n_colchunks[i] = gg.n_colchunks;
    m.block_begin[i] = total;
    total += a.m_end > a.m_begin && a.nbins > 0 ? gg.blocks : 0;
    lds = std::max(lds, (size_t)2 * (split ? 4 : 2) * 2 * win_words(32 * ct, a.taps) * sizeof(uint32_t));
  }
  m.block_begin[n] = total;
  if (total == 0) return;
  require(total < (1ll << 31), JERK_EINVAL, "search too large for one launch");
  if (split) {
    if (keys) hipLaunchKernelGGL((gemm_multi_kernel<true, true>), dim3((unsigned)total), dim3(64), lds, stream, m);
    else hipLaunchKernelGGL((gemm_multi_kernel<true, false>), dim3((unsigned)total), dim3(64), lds, stream, m);
  } else {
    if (keys) hipLaunchKernelGGL((gemm_multi_kernel<false, true>), dim3((unsigned)total), dim3(64), lds, stream, m);
    else hipLaunchKernelGGL((gemm_multi_kernel<false, false>), dim3((unsigned)total), dim3(64), lds, stream, m);
  }
  JERK_HIP_CHECK(hipGetLastError());
}

void gemm_correlate_launch(const GemmArgs& a, hipStream_t stream) {
  const int n_members = a.m_end - a.m_begin;
  if (n_members <= 0 || a.nbins <= 0) return;
  require(a.m_begin % 8 == 0, JERK_EINTERNAL, "GEMM member range must start on a block of 8");
  require(a.taps % 16 == 0 && a.taps >= 16 && a.taps <= 512, JERK_EINTERNAL, "GEMM taps out of range");
  const bool split = a.path != JERK_PATH_GEMM_FP16;
  // One row block (8 templates) per wave; the tap fragments of up to 128 taps
  // (split) or 256 taps (FP16) stay in registers across windows.
  // window = 64 outputs + taps + 8 slack elements, loaded 64 per lane-step
  if (a.row_max) {
    // peak-key launches keep one row block per wave (room for the per-row keys)
    if (split) {
      if (a.taps <= 128) launch_split_resident<true>(a, stream);
      else launch_split_streamed<true>(a, stream);
    } else {
      if (a.taps <= 256) launch_cfg<1, 2, 32, 6, false, true, true>(a, stream);
      else launch_cfg<1, 2, 16, 10, false, false, true>(a, stream);
    }
  } else if (split) {
    if (a.taps <= 128) launch_split_resident<false>(a, stream);
    else launch_split_streamed<false>(a, stream);
  } else {
    if (a.taps <= 256) launch_cfg<1, 2, 32, 6, false, true, false>(a, stream);
    else launch_cfg<1, 2, 16, 10, false, false, false>(a, stream);
  }
  JERK_HIP_CHECK(hipGetLastError());
}

}  // namespace jerk
