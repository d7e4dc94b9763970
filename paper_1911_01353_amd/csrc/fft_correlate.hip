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
#include <algorithm>

#include "cand_device.h"
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

// Global-memory views for a job's pointers. A pointer read from a device-side
// job table (batched launches) may point anywhere as far as the compiler knows,
// so it emits flat accesses: 64-bit per-lane addresses, and waits that also
// cover LDS traffic. Through these views the accesses stay global loads and
// stores. Kernels that take the job as a kernel argument need no view (the
// compiler knows such pointers are global).
typedef float f2vec __attribute__((ext_vector_type(2)));
using gcf2_ptr = __attribute__((address_space(1))) const f2vec*;
using gf2_ptr = __attribute__((address_space(1))) f2vec*;
using gci32_ptr = __attribute__((address_space(1))) const int32_t*;
__device__ __forceinline__ float2 gload(gcf2_ptr p) {
  const f2vec q = *p;
  return make_float2(q.x, q.y);
}

// cos / sin of 2 pi m / 16, m = 0..7
__device__ constexpr float kC16[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                                      0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
__device__ constexpr float kS16[8] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                                      1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f};

// Radix-2 butterfly with a constant twiddle W = W_R^k = exp(-+2 pi i k / R)
// (minus for the forward transform): x = e + W o, y = e - W o. General
// twiddles use fused multiply-adds and y = 2e - x, six instructions instead of
// eight; multiplications by 1 and -+i are free.
template <int R, bool INV>
__device__ __forceinline__ void butterfly(int k, float2 e, float2 o, float2& x, float2& y) {
  const int m = k * (16 / R);  // angle 2 pi m / 16
  if (m == 0) {
    x = cadd(e, o);
    y = csub(e, o);
    return;
  }
  if (m == 4) {  // W = -i (forward) or +i (inverse)
    const float2 t = INV ? make_float2(-o.y, o.x) : make_float2(o.y, -o.x);
    x = cadd(e, t);
    y = csub(e, t);
    return;
  }
  float2 r;
  if (m == 2 || m == 6) {
    // W = (+-1 -+ i) / sqrt(2): W o = c (u, v) with u, v sums of o's parts
    const float c = 0.70710678118654752f;
    float u, v;
    if (m == 2) {
      u = INV ? o.x - o.y : o.x + o.y;
      v = INV ? o.x + o.y : o.y - o.x;
    } else {
      u = INV ? -(o.x + o.y) : o.y - o.x;
      v = INV ? o.x - o.y : -(o.x + o.y);
    }
    r = make_float2(fmaf(c, u, e.x), fmaf(c, v, e.y));
  } else {
    const float c = kC16[m], sn = INV ? kS16[m] : -kS16[m];
    r = make_float2(fmaf(c, o.x, fmaf(-sn, o.y, e.x)), fmaf(sn, o.x, fmaf(c, o.y, e.y)));
  }
  x = r;
  y = make_float2(fmaf(2.0f, e.x, -r.x), fmaf(2.0f, e.y, -r.y));
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
    for (int k = 0; k < R / 2; ++k) butterfly<R, INV>(k, e[k], o[k], x[k], x[k + R / 2]);
  }
};
template <bool INV>
struct Dft<1, INV> {
  __device__ __forceinline__ static void run(float2*) {}
};

// LDS slot of element i of an exchange written by a pass of span LW. On gfx950 a wave's float2
// stores go 16 lanes per cycle over 32 four-byte banks and its float2 loads 32 lanes per cycle
// over 64 banks (the rates that reproduce the SQ_LDS_BANK_CONFLICT shares measured with one
// padding for all exchanges: 40% of LDS cycles at S = 512, 25% with 16 elements per thread).
// Each exchange gets its own padding, all of the form i + c (i >> s), so that every lane's
// addresses stay one base plus per-element constants (no address registers): one spare float2
// per 16 for LW = 1 (its loads still meet two-way conflicts, which no such padding avoids), LW
// spare per 8 LW for LW = 2, 4, 8, none from LW = 16 on. Checked exhaustively on the host against
// that model for every kernel variant: a template's inverse transforms spend 10-14% of their LDS
// cycles in conflicts instead of 25-40%.
constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }
template <int LW>
__device__ __forceinline__ int lds_slot(int i) {
  if constexpr (LW == 1)
    return i + (i >> 4);
  else if constexpr (LW >= 16)
    return i;
  else
    return i + LW * (i >> (ilog2c(LW) + 3));
}
// LDS float2 slots of a segment of S points under every padding above.
template <int S>
constexpr int lds_slots() { return S + S / 8; }

// One Stockham pass. The thread owns butterflies b = tid + m * TPB, m < E / R.
// tw: table of exp(-2 pi i k / S), k < S. RP: radix of the pass that wrote the
// LDS exchange this pass reads (FROM_LDS), whose span was L / RP.
template <int S, int E, int R, int L, bool INV, bool FROM_LDS, bool TO_LDS, int RP = 1>
__device__ __forceinline__ void stockham_pass(float2 (&v)[E], float2* lds, const float2* __restrict__ tw,
                                              int tid) {
  constexpr int TPB = S / E;
  constexpr int M = E / R;
  if constexpr (FROM_LDS) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int b = tid + m * TPB;
#pragma unroll
      for (int r = 0; r < R; ++r) v[m * R + r] = lds[lds_slot<L / RP>(b + r * (S / R))];
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
      for (int k = 0; k < R; ++k) lds[lds_slot<L>((b - j) * R + j + L * k)] = v[m * R + k];
    }
    __syncthreads();
  }
}

// Largest 32-bit value of the 64 lanes of a wave, the same in every lane: rows of 16 lanes by
// DPP (pairs, quads, rotations by 4 and 8), then the four row maxima from lanes 0, 16, 32, 48.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xF, 0xF, false));
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false));
  const uint32_t a = max((uint32_t)__builtin_amdgcn_readlane((int)x, 0), (uint32_t)__builtin_amdgcn_readlane((int)x, 16));
  const uint32_t b = max((uint32_t)__builtin_amdgcn_readlane((int)x, 32), (uint32_t)__builtin_amdgcn_readlane((int)x, 48));
  return max(a, b);
}

// Largest key of the lanes of a workgroup (TPB threads); returned to every thread. Within a
// wave the high words (power bits) are reduced first, then the low words of the lanes that
// hold the largest high word. Entered by every lane.
template <int TPB>
__device__ __forceinline__ uint64_t block_max_key(uint64_t k, uint64_t* red) {
  const uint32_t hi = (uint32_t)(k >> 32);
  const uint32_t mh = wave_max_u32(hi);
  const uint32_t ml = wave_max_u32(hi == mh ? (uint32_t)k : 0u);
  k = ((uint64_t)mh << 32) | ml;
  if constexpr (TPB > 64) {
    static_assert(TPB <= 512, "reduction buffer holds 8 waves");
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = k;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) k = red[w] > k ? red[w] : k;
    __syncthreads();
  }
  return k;
}

// Reduction key of a power at plane index p: larger power wins, then lower p.
__device__ __forceinline__ uint64_t peak_key(float power, int64_t p) {
  return ((uint64_t)__float_as_uint(power) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)p);
}

// Candidate epilogue of one template row of a tile (paper, section "Results":
// statistics of the plane and a peak finder with a user threshold, here without
// writing the plane). P0[e] and P1[e] are the powers at plane points
// p = 2 (seg U + lag) + phase of lag = tid + TPB c, the register of column c
// being e = (c mod M) R1 + c / M (M = E / R1). A point is a peak when it is
// strictly above its left neighbour and not below its right one. The left
// neighbour of phase 0 at a lag is phase 1 at the lag before, the right one of
// phase 1 is phase 0 at the next lag: one lane over, across a wave boundary from
// the neighbouring wave, and across a column boundary from the last (first)
// thread of the previous (next) column. The segment's first point (phase 0 at
// lag 0) and last point (phase 1 at its last lag) have a neighbour in another
// segment and are decided later from the stored edge powers.
//   Mode 1 (speculative): writes the row's sum and sum of squares over the
//   segment (FP64, fixed order), the edge powers, and stages the interior peaks
//   above ca.pre in the tile's own run of ca.cap_tile slots (counted in LDS, so
//   no device-wide atomics, and none at all when the workgroup is one wave);
//   hits past the run go to the shared pool (one atomic per wave and template),
//   and a hit that finds the pool full marks its row in ca.ovf.
// The wave finds its peaks of all columns first and reserves their slots once.
//   Mode 2 (exact): appends the interior peaks above the row's final threshold
//   to the candidate list.
template <int S, int E, int R1, int CAND>
__device__ __forceinline__ void cand_epilogue(const CandArgs& ca, const FftJob& j, int64_t seg, int U, int lag_lim,
                                              int64_t row, int64_t row0, int t, const float (&P0)[E],
                                              const float (&P1)[E], float* xch, double2* wsum, uint32_t* n_hit,
                                              int tid) {
  constexpr int TPB = S / E;
  constexpr int M = E / R1;
  constexpr int W = TPB / 64;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t slot = row * j.n_seg + seg;
  double s = 0.0, q = 0.0;
  if constexpr (CAND == 1) {
#pragma unroll
    for (int c = 0; c < E; ++c) {
      const int e = (c % M) * R1 + c / M;
      if (tid + TPB * c < lag_lim) {
        const double a = (double)P0[e], b = (double)P1[e];
        s += a;
        s += b;
        q = fma(a, a, q);
        q = fma(b, b, q);
      }
    }
    s = wave_sum_f64(s);
    q = wave_sum_f64(q);
  }
  float* xl = xch;          // [W][E]: P1 of lane 63 of each wave (W > 1)
  float* xr = xch + W * E;  // [W][E]: P0 of lane 0 of each wave
  if constexpr (W > 1) {
    if (lane == 63) {
#pragma unroll
      for (int c = 0; c < E; ++c) xl[wave * E + c] = P1[(c % M) * R1 + c / M];
    }
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < E; ++c) xr[wave * E + c] = P0[(c % M) * R1 + c / M];
      if constexpr (CAND == 1) wsum[wave] = make_double2(s, q);
    }
    __syncthreads();
    if constexpr (CAND == 1) {
      if (tid == 0) {
        s = wsum[0].x;
        q = wsum[0].y;
#pragma unroll
        for (int w = 1; w < W; ++w) {
          s += wsum[w].x;
          q += wsum[w].y;
        }
      }
    }
  }
  // P1 one lag left of lane 0's lag in column c, and P0 one lag right of lane 63's
  auto fill_left = [&](int c) -> float {
    if constexpr (W == 1)
      return c > 0 ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(P1[((c - 1) % M) * R1 + (c - 1) / M]), 63))
                   : 0.0f;
    else
      return wave > 0 ? xl[(wave - 1) * E + c] : (c > 0 ? xl[(W - 1) * E + c - 1] : 0.0f);
  };
  auto fill_right = [&](int c) -> float {
    if constexpr (W == 1)
      return c + 1 < E
                 ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(P0[((c + 1) % M) * R1 + (c + 1) / M]), 0))
                 : 0.0f;
    else
      return wave + 1 < W ? xr[(wave + 1) * E + c] : (c + 1 < E ? xr[c + 1] : 0.0f);
  };
  double thr, mean = 0.0, sigma = 0.0;
  if constexpr (CAND == 1) {
    thr = ca.pre;
    if (tid == 0) {
      ca.part[slot] = make_double2(s, q);
      ca.edge[2 * slot] = make_float2(P0[0], P1[0]);
    }
    const int last = lag_lim - 1;
    if (tid == last % TPB) {
      const int cl = last / TPB;
#pragma unroll
      for (int c = 0; c < E; ++c) {
        const int e = (c % M) * R1 + c / M;
        if (c == cl) ca.edge[2 * slot + 1] = make_float2(P0[e], P1[e]);
      }
    }
  } else {
    const CandRowStat st = ca.rs[row];
    thr = st.thr;
    mean = st.mean;
    sigma = st.sigma;
  }
  // For a float x, (double) x > thr exactly when x > thr rounded down to a float.
  const float thr_f = __double2float_rd(thr);
  const int64_t pbase = 2 * (seg * U);
  // Bit c of hits: this lane's column c holds a peak; of ph1: that peak is the phase-1 point
  // (never both points: a phase-0 peak needs P0 >= P1, a phase-1 peak P1 > P0).
  uint32_t hits = 0u, ph1 = 0u;
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int e = (c % M) * R1 + c / M;
    const float a = P0[e], b = P1[e];
    // Wave-uniform: most columns of a wave hold no point above the level (about four in five at
    // the usual level), and they need no neighbours.
    if (__ballot(fmaxf(a, b) > thr_f) == 0ull) continue;
    const float left = dpp_f32<0x138>(fill_left(c), b);   // lane i reads P1 of lane i - 1
    const float right = dpp_f32<0x130>(fill_right(c), a);  // lane i reads P0 of lane i + 1
    const int lag = tid + TPB * c;
    const bool h0 = lag > 0 && lag < lag_lim && a > left && a >= b && a > thr_f;
    const bool h1 = lag + 1 < lag_lim && b > a && b >= right && b > thr_f;
    hits |= (uint32_t)(h0 || h1) << c;
    ph1 |= (uint32_t)h1 << c;
  }
  // The wave's total and this lane's exclusive prefix of the per-lane counts, from one ballot
  // per bit of the count.
  const uint32_t cnt = (uint32_t)__popc(hits);
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t total = 0u, prefix = 0u;
#pragma unroll
  for (int bit = 0; (1 << bit) <= E; ++bit) {
    const uint64_t m = __ballot((cnt >> bit) & 1u);
    total += (uint32_t)__popcll(m) << bit;
    prefix += (uint32_t)__popcll(m & below) << bit;
  }
  if (total == 0u) return;  // wave-uniform
  // one reservation for all the wave's peaks of this template; lane order, then column order
  if constexpr (CAND == 1) {
    uint32_t base;
    if constexpr (W == 1) {
      base = *n_hit;  // the workgroup is this wave: the running count is a register
      *n_hit = base + total;
    } else {
      uint32_t b0 = 0;
      if (lane == 0) b0 = atomicAdd(n_hit, total);
      base = (uint32_t)__builtin_amdgcn_readlane((int)b0, 0);
    }
    const uint32_t cap = (uint32_t)ca.cap_tile;
    const uint32_t first = base > cap ? base : cap;  // slot index of the first hit beyond the tile's run
    unsigned long long pb = 0;
    if (base + total > cap) {  // wave-uniform: the excess goes to the pool
      unsigned long long p0 = 0;
      if (lane == 0) p0 = atomicAdd(ca.pool_count, (unsigned long long)(base + total - first));
      const int lo = __builtin_amdgcn_readlane((int)(unsigned)(p0 & 0xffffffffull), 0);
      const int hi = __builtin_amdgcn_readlane((int)(p0 >> 32), 0);
      pb = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
    }
    uint32_t i = base + prefix;
#pragma unroll
    for (int c = 0; c < E; ++c) {
      if ((hits >> c) & 1u) {
        const int e = (c % M) * R1 + c / M;
        const bool h1 = (ph1 >> c) & 1u;
        const uint32_t poff = (uint32_t)(2 * (tid + TPB * c) + (h1 ? 1 : 0));
        const float pw = h1 ? P1[e] : P0[e];
        if (i < cap) {
          ca.hits[(int64_t)blockIdx.x * cap + i] = CandHit{((uint32_t)(row - row0) << 16) | poff, pw};
        } else {
          const unsigned long long qq = pb + (i - first);
          if (qq < (unsigned long long)ca.pool_cap)
            ca.pool[qq] = CandPoolHit{(uint32_t)row, (uint32_t)pbase + poff, pw, 0u};
          else
            ca.ovf[row] = 1;
        }
        ++i;
      }
    }
  } else {
    unsigned long long g0 = 0;
    if (lane == 0) g0 = atomicAdd(ca.count, (unsigned long long)total);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(g0 & 0xffffffffull), 0);
    const int hi = __builtin_amdgcn_readlane((int)(g0 >> 32), 0);
    unsigned long long i = (((unsigned long long)(unsigned)hi << 32) | (unsigned)lo) + prefix;
#pragma unroll
    for (int c = 0; c < E; ++c) {
      if ((hits >> c) & 1u) {
        const int e = (c % M) * R1 + c / M;
        const bool h1 = (ph1 >> c) & 1u;
        if (i < (unsigned long long)ca.capacity) {
          jerk_candidate cd;
          cd.t = (uint32_t)t;
          cd.p = (uint32_t)pbase + (uint32_t)(2 * (tid + TPB * c) + (h1 ? 1 : 0));
          cd.power = h1 ? P1[e] : P0[e];
          cd.sigma = (float)(((double)cd.power - mean) / sigma);
          ca.out[i] = cd;
        }
        ++i;
      }
    }
  }
}

// One tile: segment `seg` of job `j` against members [m0, m1) of its member
// list. CAND = 0 writes the plane rows and/or the per-(row, segment) peak
// keys; CAND = 1 and 2 write neither and run the candidate epilogue instead
// (cand_epilogue). Radices R1..R4 (R4 = 1: three passes) run forward in that
// order and inverse in the reverse order. TABLE: the job was read from a
// device-side job table (its accesses go through the global views).
template <int S, int E, int R1, int R2, int R3, int R4, bool KEYS, int CAND = 0, bool TABLE = false>
__device__ __forceinline__ void fft_tile(const FftJob& j, int64_t seg, int m0, int m1, float2* lds, uint64_t* red,
                                         const float2* __restrict__ tw, const CandArgs* ca = nullptr,
                                         float* xch = nullptr, double2* wsum = nullptr, uint32_t* n_hit = nullptr) {
  constexpr int TPB = S / E;
  constexpr bool P4 = R4 > 1;
  constexpr int RL = P4 ? R4 : R3;  // last forward radix = first inverse radix
  const int tid = threadIdx.x;
  const int K = j.taps;
  const int U = S - K + 1;
  const int64_t base = seg * U - (K / 2 - 1);

  // ---- forward FFT of the segment ----
  float2 v[E];
  {
    constexpr int M = E / R1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int b = tid + m * TPB;
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int64_t k = base + b + r * (S / R1);
        v[m * R1 + r] = (k >= 0 && k < j.nbins) ? (TABLE ? gload((gcf2_ptr)j.spec + k) : j.spec[k]) : make_float2(0.f, 0.f);
      }
    }
  }
  stockham_pass<S, E, R1, 1, false, false, true>(v, lds, tw, tid);
  stockham_pass<S, E, R2, R1, false, true, true, R1>(v, lds, tw, tid);
  if constexpr (P4) {
    stockham_pass<S, E, R3, R1 * R2, false, true, true, R2>(v, lds, tw, tid);
    stockham_pass<S, E, R4, R1 * R2 * R3, false, true, false, R3>(v, lds, tw, tid);
  } else {
    stockham_pass<S, E, R3, R1 * R2, false, true, false, R2>(v, lds, tw, tid);
  }
  float2 F[E];
#pragma unroll
  for (int e = 0; e < E; ++e) F[e] = v[e];

  // ---- template loop ----
  // lags kept by this segment: lag < U and k0 = seg U + lag < nbins
  const int lag_lim = (int)min((int64_t)U, j.nbins - seg * U);
  for (int mm = m0; mm < m1; ++mm) {
    const int t = TABLE ? ((gci32_ptr)j.members)[mm] : j.members[mm];
    const int64_t row = j.row_by_member ? (int64_t)(mm - j.row_base) : (int64_t)(t - j.t_begin);
    float P0[E];
#pragma unroll
    for (int phase = 0; phase < 2; ++phase) {
      const float2* __restrict__ H = j.bank_fft + ((int64_t)mm * 2 + phase) * S;
      const gcf2_ptr Hg = (gcf2_ptr)j.bank_fft + ((int64_t)mm * 2 + phase) * S;  // TABLE
      {
        constexpr int M = E / RL;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const unsigned b = tid + m * TPB;
#pragma unroll
          for (int k = 0; k < RL; ++k) v[m * RL + k] = cmul(F[m * RL + k], TABLE ? gload(Hg + b + k * (S / RL)) : H[b + k * (S / RL)]);
        }
      }
      if constexpr (P4) {
        stockham_pass<S, E, R4, 1, true, false, true>(v, lds, tw, tid);
        stockham_pass<S, E, R3, R4, true, true, true, R4>(v, lds, tw, tid);
        stockham_pass<S, E, R2, R4 * R3, true, true, true, R3>(v, lds, tw, tid);
        stockham_pass<S, E, R1, R4 * R3 * R2, true, true, false, R2>(v, lds, tw, tid);
      } else {
        stockham_pass<S, E, R3, 1, true, false, true>(v, lds, tw, tid);
        stockham_pass<S, E, R2, R3, true, true, true, R3>(v, lds, tw, tid);
        stockham_pass<S, E, R1, R3 * R2, true, true, false, R2>(v, lds, tw, tid);
      }
      // thread holds lag b + k S/R1 in v[m R1 + k]
      if (phase == 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) P0[e] = fmaf(v[e].x, v[e].x, v[e].y * v[e].y);
      } else if constexpr (CAND > 0) {
        float P1[E];
#pragma unroll
        for (int e = 0; e < E; ++e) P1[e] = fmaf(v[e].x, v[e].x, v[e].y * v[e].y);
        cand_epilogue<S, E, R1, CAND>(*ca, j, seg, U, lag_lim, row, (int64_t)(m0 - j.row_base), t, P0, P1, xch,
                                      wsum, n_hit, tid);
      } else {
        constexpr int M = E / R1;
        // KEYS: this lane's best power bits and 2c + phase of the column c holding it; columns
        // are visited in increasing lag order and only a strictly larger power replaces the
        // best, so equal powers keep the lowest plane index (the order of peak_key)
        [[maybe_unused]] uint32_t bb = 0;
        [[maybe_unused]] int bc = -1;
        // uniform row base; lanes add 32-bit offsets (through a global view: the job may come from
        // a device-side table)
        const bool out2 = j.plane != nullptr;
        const gf2_ptr out2g = j.plane ? (gf2_ptr)(j.plane + row * j.ld) + seg * U : nullptr;
#pragma unroll
        for (int i = 0; i < E; ++i) {
          // column c holds lag tid + c TPB in v[(c mod M) R1 + c / M]; KEYS visits the columns
          // in order, the plane alone in register order
          const int e = KEYS ? (i % M) * R1 + i / M : i;
          const int c = KEYS ? i : i / R1 + (i % R1) * M;
          const int lag = tid + c * TPB;
          if (lag < lag_lim) {
            const float2 vv = v[e];
            const float p0 = P0[e];
            const float p1 = fmaf(vv.x, vv.x, vv.y * vv.y);
            // plane points are written once and never read here: non-temporal stores keep
            // them from displacing the template spectra and segments in the caches
            if (out2) __builtin_nontemporal_store(f2vec{p0, p1}, &out2g[(unsigned)lag]);
            if constexpr (KEYS) {
              const uint32_t u0 = __float_as_uint(p0), u1 = __float_as_uint(p1);
              if (c == 0 || u0 > bb) {
                bb = u0;
                bc = 2 * c;
              }
              if (u1 > bb) {
                bb = u1;
                bc = 2 * c + 1;
              }
            }
          }
        }
        [[maybe_unused]] uint64_t best = 0;
        if constexpr (KEYS) {
          if (bc >= 0) {
            const int64_t p = 2 * (seg * U + tid) + (int64_t)(bc >> 1) * (2 * TPB) + (bc & 1);
            best = peak_key(__uint_as_float(bb), p);
          }
          best = block_max_key<TPB>(best, red);
          if (tid == 0) {
            if (j.rmax_ld == 0) atomicMax(reinterpret_cast<unsigned long long*>(j.row_max + row), (unsigned long long)best);
            else j.row_max[row * j.rmax_ld + seg] = best;
          }
        }
      }
    }
  }
  // per-segment keys: the last segment's tile also clears its rows' keys past this group's
  // segment count, so a row holds no stale keys from an earlier spectrum (after the template
  // loop, where it costs no registers of the FFTs)
  if constexpr (KEYS && CAND == 0) {
    if (j.rmax_ld != 0 && seg == j.n_seg - 1) {
      for (int mm = m0; mm < m1; ++mm) {
        const int t = TABLE ? ((gci32_ptr)j.members)[mm] : j.members[mm];
        const int64_t row = j.row_by_member ? (int64_t)(mm - j.row_base) : (int64_t)(t - j.t_begin);
        for (int64_t q = j.n_seg + tid; q < j.rmax_ld; q += TPB) j.row_max[row * j.rmax_ld + q] = 0;
      }
    }
  }
}

// One job, one workgroup per tile: blockIdx = tb * n_seg + seg. KEYS: write
// peak keys (j.row_max) as well as (or instead of) the plane.
template <int S, int E, int R1, int R2, int R3, int R4, bool KEYS>
__global__ void __launch_bounds__(S / E) fft_correlate_kernel(FftJob j, const float2* __restrict__ tw) {
  static_assert(R1 * R2 * R3 * R4 == S, "radices must multiply to S");
  __shared__ float2 lds[lds_slots<S>()];
  __shared__ uint64_t red[8];
  const int64_t blk = blockIdx.x;
  const int m0 = j.m_begin + (int)(blk / j.n_seg) * j.tpb;
  fft_tile<S, E, R1, R2, R3, R4, KEYS>(j, blk % j.n_seg, m0, min(m0 + j.tpb, j.m_end), lds, red, tw);
}

// Persistent launch over a job table: every workgroup takes tiles from a
// device counter until all tiles of all jobs are done (every workgroup
// reaches the exit test). Tile i belongs to the job whose [tile_begin,
// next tile_begin) holds it; within a job, tile = tb * n_seg + seg.
template <int S, int E, int R1, int R2, int R3, int R4, bool KEYS>
__global__ void __launch_bounds__(S / E) fft_persistent_kernel(const FftJob* __restrict__ jobs,
                                                               BatchHeader* __restrict__ hdr,
                                                               const float2* __restrict__ tw) {
  __shared__ float2 lds[lds_slots<S>()];
  __shared__ uint64_t red[8];
  __shared__ int64_t s_tile;
  const int64_t total = hdr->total_tiles;
  const int n_jobs = hdr->n_jobs;
  for (;;) {
    if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(&hdr->counter, 1ull);
    __syncthreads();
    const int64_t tile = s_tile;
    __syncthreads();
    if (tile >= total) break;
    int lo = 0, hi = n_jobs - 1;  // last job with tile_begin <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].tile_begin <= tile) lo = mid;
      else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);  // uniform: the job's fields go to scalar registers
    const FftJob& j = jobs[lo];
    const int64_t local = tile - j.tile_begin;
    // An opaque copy of the twiddle pointer per tile: otherwise the compiler
    // hoists the twiddle loads out of the tile loop and keeps them live across
    // tiles, which costs more registers (and waves) than reloading them. The
    // copy is made in the global address space so that the loads stay global.
    __attribute__((address_space(1))) const float2* twg = (__attribute__((address_space(1))) const float2*)tw;
    asm volatile("" : "+s"(twg));
    const float2* twt = (const float2*)twg;
    const int m0 = j.m_begin + (int)(local / j.n_seg) * j.tpb;
    fft_tile<S, E, R1, R2, R3, R4, KEYS, 0, true>(j, local % j.n_seg, m0, min(m0 + j.tpb, j.m_end), lds, red, twt);
  }
}

// One launch over a job table, one workgroup per tile (grid = total tiles):
// workgroup i takes tile i, the hardware dispatcher balancing the load.
template <int S, int E, int R1, int R2, int R3, int R4, bool KEYS>
__global__ void __launch_bounds__(S / E) fft_multi_kernel(const FftJob* __restrict__ jobs,
                                                          const BatchHeader* __restrict__ hdr,
                                                          const float2* __restrict__ tw) {
  __shared__ float2 lds[lds_slots<S>()];
  __shared__ uint64_t red[8];
  const int64_t tile = blockIdx.x;
  const int n_jobs = hdr->n_jobs;
  int lo = 0, hi = n_jobs - 1;  // last job with tile_begin <= tile
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const FftJob& j = jobs[lo];
  const int64_t local = tile - j.tile_begin;
  const int m0 = j.m_begin + (int)(local / j.n_seg) * j.tpb;
  fft_tile<S, E, R1, R2, R3, R4, KEYS, 0, true>(j, local % j.n_seg, m0, min(m0 + j.tpb, j.m_end), lds, red, tw);
}

// Several jobs of one variant in one flat launch, the job table travelling in the kernel
// arguments: workgroup i takes tile i of the job whose tile range holds it.
struct FftArgJobs {
  FftJob job[kFftArgJobs];
  int32_t n;
};

template <int S, int E, int R1, int R2, int R3, int R4, bool KEYS>
__global__ void __launch_bounds__(S / E) fft_args_kernel(FftArgJobs m, const float2* __restrict__ tw) {
  __shared__ float2 lds[lds_slots<S>()];
  __shared__ uint64_t red[8];
  const int64_t tile = blockIdx.x;
  int k = 0;
  while (k + 1 < m.n && tile >= m.job[k + 1].tile_begin) ++k;
  const FftJob& j = m.job[k];
  const int64_t local = tile - j.tile_begin;
  const int m0 = j.m_begin + (int)(local / j.n_seg) * j.tpb;
  fft_tile<S, E, R1, R2, R3, R4, KEYS, 0, true>(j, local % j.n_seg, m0, min(m0 + j.tpb, j.m_end), lds, red, tw);
}

// Candidate passes over one width-group job (cand_epilogue). Mode 1: one
// workgroup per tile (template block, segment), as fft_correlate_kernel. Mode 2:
// the flagged rows, one template per tile, the grid striding over (flagged row,
// segment) tiles; with no flagged row every workgroup exits at once.
template <int S, int E, int R1, int R2, int R3, int R4, int CAND>
__global__ void __launch_bounds__(S / E) fft_cand_kernel(FftJob j, const float2* __restrict__ tw, CandArgs ca) {
  constexpr int W = S / E / 64;
  __shared__ float2 lds[lds_slots<S>()];
  __shared__ uint64_t red[8];
  __shared__ float xch[2 * W * E];
  __shared__ double2 wsum[W];
  __shared__ uint32_t n_hit_lds;  // hits of the tile, counted by every wave (W > 1)
  if constexpr (CAND == 1) {
    uint32_t n_hit_reg = 0u;  // hits of the tile when the workgroup is one wave
    if (threadIdx.x == 0) n_hit_lds = 0u;  // the forward transform's barriers order this before any use
    const int64_t blk = blockIdx.x;
    const int m0 = j.m_begin + (int)(blk / j.n_seg) * j.tpb;
    fft_tile<S, E, R1, R2, R3, R4, false, 1>(j, blk % j.n_seg, m0, min(m0 + j.tpb, j.m_end), lds, red, tw, &ca, xch,
                                             wsum, W == 1 ? &n_hit_reg : &n_hit_lds);
    if constexpr (W == 1) {
      if (threadIdx.x == 0) ca.tile_hits[blk] = n_hit_reg;
    } else {
      __syncthreads();
      if (threadIdx.x == 0) ca.tile_hits[blk] = n_hit_lds;
    }
  } else {
    const int64_t tiles = (int64_t)*ca.n_flagged * j.n_seg;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
      const int m0 = j.m_begin + ca.flagged[tile / j.n_seg];
      fft_tile<S, E, R1, R2, R3, R4, false, 2>(j, tile % j.n_seg, m0, m0 + 1, lds, red, tw, &ca, xch, wsum);
    }
  }
}

__global__ void batch_reset_kernel(BatchHeader* hdr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) hdr->counter = 0ull;
}

}  // namespace

int64_t fft_job_tiles(FftJob& j, int32_t seg_len) {
  const int U = seg_len - j.taps + 1;
  require(U >= 1, JERK_EINTERNAL, "segment shorter than the template");
  j.n_seg = (j.nbins + U - 1) / U;
  const int64_t n_tb = (j.m_end - j.m_begin + j.tpb - 1) / j.tpb;
  return j.n_seg * n_tb;
}

// Kernel variants: segment length x elements per thread (16: three radix-16
// passes where possible; 8: radix-8 passes, one more LDS exchange, about half
// the registers and twice the waves per SIMD).
#define JERK_FFT_VARIANTS(X)              \
  X(512, 8, 8, 8, 8, 1)                   \
  X(1024, 16, 4, 16, 16, 1)               \
  X(1024, 8, 2, 8, 8, 8)                  \
  X(2048, 16, 8, 16, 16, 1)               \
  X(2048, 8, 4, 8, 8, 8)                  \
  X(4096, 16, 16, 16, 16, 1)              \
  X(4096, 8, 8, 8, 8, 8)

bool fft_variant_supported(int32_t seg_len, int32_t ept) {
#define X(S, E, A, B, C, D) \
  if (seg_len == S && ept == E) return true;
  JERK_FFT_VARIANTS(X)
#undef X
  return false;
}

void fft_correlate_launch(FftJob j, int32_t seg_len, int32_t ept, const float2* twiddles, hipStream_t stream) {
  if (j.m_end <= j.m_begin || j.nbins <= 0) return;
  const int64_t blocks = fft_job_tiles(j, seg_len);
  require(blocks < (1ll << 31), JERK_EINVAL, "search too large for one launch; split the template range");
  const bool keys = j.row_max != nullptr;
#define X(S, E, A, B, C, D)                                                                                       \
  if (seg_len == S && ept == E) {                                                                                 \
    if (keys)                                                                                                     \
      hipLaunchKernelGGL((fft_correlate_kernel<S, E, A, B, C, D, true>), dim3((unsigned)blocks), dim3(S / E), 0,  \
                         stream, j, twiddles);                                                                    \
    else                                                                                                          \
      hipLaunchKernelGGL((fft_correlate_kernel<S, E, A, B, C, D, false>), dim3((unsigned)blocks), dim3(S / E), 0, \
                         stream, j, twiddles);                                                                    \
    JERK_HIP_CHECK(hipGetLastError());                                                                            \
    return;                                                                                                       \
  }
  JERK_FFT_VARIANTS(X)
#undef X
  throw Error(JERK_EINTERNAL, "unsupported FFT kernel variant");
}

void fft_cand_launch(FftJob j, int32_t seg_len, int32_t ept, const float2* twiddles, const CandArgs& ca, int mode,
                     hipStream_t stream) {
  if (j.m_end <= j.m_begin || j.nbins <= 0) return;
  require(j.plane == nullptr && j.row_max == nullptr && j.row_by_member && j.row_base == j.m_begin, JERK_EINTERNAL,
          "candidate passes take a group job without plane or keys");
  const int64_t tiles = fft_job_tiles(j, seg_len);
  require(tiles < (1ll << 31), JERK_EINVAL, "search too large for one launch; split the template range");
  int dev = 0, cus = 0, per_cu = 0;
  if (mode == 2) {
    JERK_HIP_CHECK(hipGetDevice(&dev));
    JERK_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  const int64_t row_tiles = (int64_t)(j.m_end - j.m_begin) * j.n_seg;
#define X(S, E, A, B, C, D)                                                                                      \
  if (seg_len == S && ept == E) {                                                                                \
    if (mode == 1) {                                                                                             \
      hipLaunchKernelGGL((fft_cand_kernel<S, E, A, B, C, D, 1>), dim3((unsigned)tiles), dim3(S / E), 0, stream, j, \
                         twiddles, ca);                                                                          \
    } else {                                                                                                     \
      JERK_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(                                               \
          &per_cu, reinterpret_cast<const void*>(fft_cand_kernel<S, E, A, B, C, D, 2>), S / E, 0));              \
      const int64_t grid = std::min<int64_t>(row_tiles, (int64_t)std::max(1, cus) * std::max(1, per_cu));       \
      hipLaunchKernelGGL((fft_cand_kernel<S, E, A, B, C, D, 2>), dim3((unsigned)grid), dim3(S / E), 0, stream, j, \
                         twiddles, ca);                                                                          \
    }                                                                                                            \
    JERK_HIP_CHECK(hipGetLastError());                                                                           \
    return;                                                                                                      \
  }
  JERK_FFT_VARIANTS(X)
#undef X
  throw Error(JERK_EINTERNAL, "unsupported FFT kernel variant");
}

int32_t fft_persistent_grid(int32_t seg_len, int32_t ept) {
  int dev = 0, cus = 0, per_cu = 0, per_cu_k = 0;
  JERK_HIP_CHECK(hipGetDevice(&dev));
  JERK_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
#define X(S, E, A, B, C, D)                                                                                 \
  if (seg_len == S && ept == E) {                                                                           \
    JERK_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(                                            \
        &per_cu, reinterpret_cast<const void*>(fft_persistent_kernel<S, E, A, B, C, D, false>), S / E, 0)); \
    JERK_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(                                            \
        &per_cu_k, reinterpret_cast<const void*>(fft_persistent_kernel<S, E, A, B, C, D, true>), S / E, 0)); \
  }
  JERK_FFT_VARIANTS(X)
#undef X
  per_cu = std::max(per_cu, per_cu_k);
  require(per_cu > 0, JERK_EINTERNAL, "unsupported FFT kernel variant");
  return std::max(1, cus) * per_cu;
}

void fft_persistent_launch(const FftJob* d_jobs, BatchHeader* d_hdr, int32_t seg_len, int32_t ept, bool keys,
                           const float2* twiddles, int32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, stream, d_hdr);
#define X(S, E, A, B, C, D)                                                                                       \
  if (seg_len == S && ept == E) {                                                                                 \
    if (keys)                                                                                                     \
      hipLaunchKernelGGL((fft_persistent_kernel<S, E, A, B, C, D, true>), dim3(grid), dim3(S / E), 0, stream,     \
                         d_jobs, d_hdr, twiddles);                                                                \
    else                                                                                                          \
      hipLaunchKernelGGL((fft_persistent_kernel<S, E, A, B, C, D, false>), dim3(grid), dim3(S / E), 0, stream,    \
                         d_jobs, d_hdr, twiddles);                                                                \
    JERK_HIP_CHECK(hipGetLastError());                                                                            \
    return;                                                                                                       \
  }
  JERK_FFT_VARIANTS(X)
#undef X
  throw Error(JERK_EINTERNAL, "unsupported FFT kernel variant");
}

void fft_args_launch(FftJob* jobs, int n, int32_t seg_len, int32_t ept, bool keys, const float2* twiddles,
                     hipStream_t stream) {
  require(n >= 1 && n <= kFftArgJobs, JERK_EINTERNAL, "fft_args_launch takes 1..8 jobs");
  FftArgJobs m{};
  int64_t total = 0;
  for (int k = 0; k < n; ++k) {
    m.job[k] = jobs[k];
    m.job[k].tile_begin = total;
    total += fft_job_tiles(m.job[k], seg_len);
    require((m.job[k].row_max != nullptr) == keys, JERK_EINTERNAL, "every job of one launch keys or none does");
  }
  m.n = n;
  if (total == 0) return;
  require(total < (int64_t(1) << 31), JERK_EINVAL, "search too large for one launch; split the template range");
#define X(S, E, A, B, C, D)                                                                                       \
  if (seg_len == S && ept == E) {                                                                                 \
    if (keys)                                                                                                     \
      hipLaunchKernelGGL((fft_args_kernel<S, E, A, B, C, D, true>), dim3((unsigned)total), dim3(S / E), 0, stream, \
                         m, twiddles);                                                                            \
    else                                                                                                          \
      hipLaunchKernelGGL((fft_args_kernel<S, E, A, B, C, D, false>), dim3((unsigned)total), dim3(S / E), 0,       \
                         stream, m, twiddles);                                                                    \
    JERK_HIP_CHECK(hipGetLastError());                                                                            \
    return;                                                                                                       \
  }
  JERK_FFT_VARIANTS(X)
#undef X
  throw Error(JERK_EINTERNAL, "unsupported FFT kernel variant");
}

void fft_multi_launch(const FftJob* d_jobs, const BatchHeader* d_hdr, int64_t total, int32_t seg_len, int32_t ept,
                      bool keys, const float2* twiddles, hipStream_t stream) {
  require(total >= 1 && total < (int64_t(1) << 31), JERK_EINVAL, "batch too large for one flat launch");
#define X(S, E, A, B, C, D)                                                                                       \
  if (seg_len == S && ept == E) {                                                                                 \
    if (keys)                                                                                                     \
      hipLaunchKernelGGL((fft_multi_kernel<S, E, A, B, C, D, true>), dim3((unsigned)total), dim3(S / E), 0,       \
                         stream, d_jobs, d_hdr, twiddles);                                                        \
    else                                                                                                          \
      hipLaunchKernelGGL((fft_multi_kernel<S, E, A, B, C, D, false>), dim3((unsigned)total), dim3(S / E), 0,      \
                         stream, d_jobs, d_hdr, twiddles);                                                        \
    JERK_HIP_CHECK(hipGetLastError());                                                                            \
    return;                                                                                                       \
  }
  JERK_FFT_VARIANTS(X)
#undef X
  throw Error(JERK_EINTERNAL, "unsupported FFT kernel variant");
}

}  // namespace jerk
