// Candidate selection over a plane slab (paper, section "Results": the search
// is timed with the mean and standard deviation of the plane and a peak finder
// that keeps only peaks above a user threshold).
//
// Row statistics: population mean and standard deviation per row, one read of
// the row. Each thread folds 16 values at a time: the group mean is their FP64
// sum over 16 and the group's squared deviations are formed directly; groups
// are merged with the pairwise update of Chan, Golub and LeVeque (1979). A constant row therefore gets a standard deviation
// of exactly 0. Chunks of a row are merged in a fixed order, so the result does
// not depend on scheduling.
//
// Candidates: a point is kept when its power, widened to FP64, is strictly above
// mean + k * sigma of its row, it is strictly greater than its left neighbour
// and not less than its right one (row ends have no neighbour on that side).
// Hits are staged in LDS per workgroup and appended with one atomic add on the
// shared counter per flush.
#include <algorithm>

#include "cand_device.h"
#include "jerk_internal.h"

namespace jerk {
namespace {

constexpr int kStatThreads = 256;
constexpr int kStatPerThread = 16;                            // four float4 per thread
constexpr int64_t kStatTile = kStatThreads * kStatPerThread;  // 4096 points
constexpr int kPeakThreads = 256;
constexpr int kPeakPerThread = 4;
constexpr int64_t kPeakTile = kPeakThreads * kPeakPerThread;  // 1024 points
constexpr int kPeakTilesPerBlock = 32;                        // a block scans 32768 points of a row
constexpr int kStage = 2048;                                  // LDS candidate staging slots
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
// VEC: rows are 16-byte aligned (plane aligned, ld a multiple of 4), so a thread's
// 16 values of a tile are four coalesced float4 loads; otherwise 16 scalar loads.
template <bool VEC>
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
      bool ok[kStatPerThread];
#pragma unroll
      for (int q = 0; q < kStatPerThread / 4; ++q) {
        // element e = 4 (q * 256 + tid) + c of the tile
        const int64_t p0 = base + 4 * ((int64_t)q * kStatThreads + threadIdx.x);
        if (VEC && p0 + 3 < hi) {
          const float4 f = *reinterpret_cast<const float4*>(src + p0);
          v[4 * q + 0] = f.x;
          v[4 * q + 1] = f.y;
          v[4 * q + 2] = f.z;
          v[4 * q + 3] = f.w;
#pragma unroll
          for (int c = 0; c < 4; ++c) ok[4 * q + c] = true;
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            ok[4 * q + c] = p0 + c < hi;
            v[4 * q + c] = ok[4 * q + c] ? src[p0 + c] : 0.0f;
          }
        }
      }
      int cnt = 0;
      double sum = 0.0;
#pragma unroll
      for (int e = 0; e < kStatPerThread; ++e) {
        if (ok[e]) {
          sum += (double)v[e];
          ++cnt;
        }
      }
      if (cnt > 0) {
        Moments g;
        g.n = (double)cnt;
        g.m = cnt == kStatPerThread ? sum * (1.0 / kStatPerThread) : sum / g.n;
        g.m2 = 0.0;
#pragma unroll
        for (int e = 0; e < kStatPerThread; ++e) {
          if (ok[e]) {
            const double d = (double)v[e] - g.m;
            g.m2 = fma(d, d, g.m2);
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

// grid (ceil(n_r / 32768), min(rows, 65535)). A block scans 32 tiles of 1024
// points of a row, two tiles per step. In a tile, thread i takes the 4
// consecutive points 4 i .. 4 i + 3 (one float4 load when rows are 16-byte
// aligned) and reads their outer neighbours directly (cache hits), so no lane
// exchange is needed. Hits are staged in LDS as (p, power) and flushed with one
// atomic add on the shared counter per flush: two tiles hold at most 1024 peaks
// (peaks are never adjacent), so the stage is flushed whenever fewer than 1024
// of its slots are free.
struct Staged {
  uint32_t p;
  float power;
};

template <bool VEC>
__global__ void __launch_bounds__(kPeakThreads) find_candidates_kernel(
    const float* __restrict__ plane, int64_t ld, int32_t rows, int64_t n_r, const double* __restrict__ stats,
    double k_sigma, const int32_t* __restrict__ row_template, int32_t t_base, jerk_candidate* __restrict__ out,
    int64_t capacity, unsigned long long* __restrict__ count) {
  __shared__ Staged stage[kStage];
  __shared__ int n_stage;
  __shared__ unsigned long long s_base;
  const int lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1ull;
  if (threadIdx.x == 0) n_stage = 0;
  __syncthreads();
  double mu = 0.0, sd = 0.0;
  uint32_t t = 0;
  // Entered by all threads together. Every read of n_stage that decides a
  // branch sits between two barriers, so all waves take the same branch.
  auto flush = [&]() {
    __syncthreads();  // every hit of the block is in the stage
    const int n = n_stage;
    __syncthreads();  // every thread has read n before it changes
    if (n == 0) return;
    if (threadIdx.x == 0) s_base = atomicAdd(count, (unsigned long long)n);
    __syncthreads();
    const unsigned long long b = s_base;
    for (int i = threadIdx.x; i < n; i += kPeakThreads) {
      if (b + (unsigned long long)i < (unsigned long long)capacity) {
        const Staged e = stage[i];
        jerk_candidate c;
        c.t = t;
        c.p = e.p;
        c.power = e.power;
        c.sigma = (float)(((double)e.power - mu) / sd);
        out[b + i] = c;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) n_stage = 0;
    __syncthreads();
  };
  for (int32_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const float* src = plane + (int64_t)row * ld;
    mu = stats[2 * (int64_t)row];
    sd = stats[2 * (int64_t)row + 1];
    const double thr = mu + k_sigma * sd;
    t = row_template ? (uint32_t)row_template[row] : (uint32_t)(t_base + row);
    for (int tile = 0; tile < kPeakTilesPerBlock; tile += 2) {
      const int64_t base = ((int64_t)blockIdx.x * kPeakTilesPerBlock + tile) * kPeakTile;
      if (base >= n_r) break;  // uniform
      float v[2][4], nb[2][2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int64_t p0 = base + u * kPeakTile + 4 * threadIdx.x;
        if (VEC && p0 + 3 < n_r) {
          const float4 f = *reinterpret_cast<const float4*>(src + p0);
          v[u][0] = f.x;
          v[u][1] = f.y;
          v[u][2] = f.z;
          v[u][3] = f.w;
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) v[u][c] = p0 + c < n_r ? src[p0 + c] : 0.0f;
        }
        nb[u][0] = p0 > 0 && p0 - 1 < n_r ? src[p0 - 1] : 0.0f;
        nb[u][1] = p0 + 4 < n_r ? src[p0 + 4] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int64_t p0 = base + u * kPeakTile + 4 * threadIdx.x;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t p = p0 + c;
          const float x = v[u][c];
          const float left = c == 0 ? nb[u][0] : v[u][c - 1];
          const float right = c == 3 ? nb[u][1] : v[u][c + 1];
          const bool hit = p < n_r && (p == 0 || x > left) && (p + 1 == n_r || x >= right) && (double)x > thr;
          const uint64_t mask = __ballot(hit);
          if (mask == 0ull) continue;
          const int leader = __ffsll((unsigned long long)mask) - 1;
          int slot = 0;
          if (lane == leader) slot = atomicAdd(&n_stage, __popcll(mask));
          slot = __builtin_amdgcn_readlane(slot, leader);  // leader is wave-uniform
          if (hit) stage[slot + __popcll(mask & below)] = Staged{(uint32_t)p, x};
        }
      }
      __syncthreads();
      const bool full = n_stage > kStage - (int)kPeakTile;
      __syncthreads();
      if (full) flush();
    }
    flush();
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

// ---- steps of the fused search with candidate selection --------------------
// (the FFT passes are in fft_correlate.hip). Rows are members of one width
// group; the per-(row, segment) partial sums cover 2 lim points, lim =
// min(U, nbins - s U) lags of segment s.

__global__ void __launch_bounds__(256) cand_reset_kernel(int32_t* __restrict__ ovf, int32_t rows,
                                                         uint32_t* __restrict__ n_flagged,
                                                         unsigned long long* __restrict__ pool_count) {
  for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < rows; i += gridDim.x * 256) ovf[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *n_flagged = 0u;
    *pool_count = 0ull;
  }
}

// One wave per row: lane l merges a contiguous run of the row's segments, then
// the lanes are merged in index order. A row is flagged for the exact pass when
// its threshold lies below the speculative level or when one of its staged hits
// found no room (tile slots and pool full).
__global__ void __launch_bounds__(256) cand_finish_kernel(const double2* __restrict__ part, int32_t rows,
                                                          int64_t n_seg, int32_t U, int64_t nbins,
                                                          const int32_t* __restrict__ ovf, double k_sigma, double pre,
                                                          const int32_t* __restrict__ members, int32_t t_begin,
                                                          double* __restrict__ stats_out, CandRowStat* __restrict__ rs,
                                                          int32_t* __restrict__ flagged, uint32_t* __restrict__ n_flagged) {
  const int lane = threadIdx.x & 63;
  const int32_t row = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6);
  if (row >= rows) return;  // whole waves
  const int64_t run = (n_seg + 63) / 64;
  const int64_t s0 = lane * run;
  const int64_t s1 = s0 + run < n_seg ? s0 + run : n_seg;
  Moments acc{0.0, 0.0, 0.0};
  for (int64_t sg = s0; sg < s1; ++sg) {
    const double2 v = part[(int64_t)row * n_seg + sg];
    const int64_t lim = nbins - sg * U < U ? nbins - sg * U : U;
    Moments g;
    g.n = 2.0 * (double)lim;
    g.m = v.x / g.n;
    g.m2 = fmax(0.0, v.y - v.x * g.m);
    acc = merge(acc, g);
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const Moments o = shfl_xor_moments(acc, off);
    acc = (lane & off) ? merge(o, acc) : merge(acc, o);
  }
  if (lane == 0) {
    CandRowStat st;
    st.mean = acc.m;
    st.sigma = acc.n > 0.0 ? sqrt(acc.m2 / acc.n) : 0.0;
    st.thr = st.mean + k_sigma * st.sigma;
    st.flag = (ovf[row] != 0 || st.thr < pre) ? 1 : 0;
    st.pad = 0;
    rs[row] = st;
    if (stats_out) {
      const int64_t o = 2 * (int64_t)(members[row] - t_begin);
      stats_out[o] = st.mean;
      stats_out[o + 1] = st.sigma;
    }
    if (st.flag) flagged[atomicAdd(n_flagged, 1u)] = row;
  }
}

// Staged hits of rows that are not flagged and lie above their row's threshold:
// first the tiles' slots, a thread per tile looping over its hits (the loop bound
// is the block's largest count, so every thread reaches the barriers), then the
// pool. Kept candidates are gathered in LDS and appended with one atomic add on
// the shared counter per flush: a step adds at most 256, so the stage is flushed
// once fewer than 256 of its slots are free.
constexpr int kFilterStage = 2048;

__global__ void __launch_bounds__(256) cand_filter_kernel(const CandHit* __restrict__ hits,
                                                          const uint32_t* __restrict__ tile_hits, int32_t tiles,
                                                          int32_t cap_tile, int32_t n_seg, int32_t tpb, int32_t U,
                                                          const CandPoolHit* __restrict__ pool,
                                                          const unsigned long long* __restrict__ pool_count,
                                                          int64_t pool_cap, const CandRowStat* __restrict__ rs,
                                                          const int32_t* __restrict__ members,
                                                          jerk_candidate* __restrict__ out, int64_t capacity,
                                                          unsigned long long* __restrict__ count) {
  __shared__ jerk_candidate stage[kFilterStage];
  __shared__ int n_stage;
  __shared__ unsigned long long s_base;
  __shared__ int32_t s_most[4];
  const int lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1ull;
  if (threadIdx.x == 0) n_stage = 0;
  __syncthreads();
  // Entered by all threads together; reads of n_stage that decide a branch sit between barriers.
  auto flush = [&]() {
    __syncthreads();
    const int n = n_stage;
    __syncthreads();
    if (n == 0) return;
    if (threadIdx.x == 0) s_base = atomicAdd(count, (unsigned long long)n);
    __syncthreads();
    const unsigned long long b = s_base;
    for (int i = threadIdx.x; i < n; i += 256)
      if (b + (unsigned long long)i < (unsigned long long)capacity) out[b + i] = stage[i];
    __syncthreads();
    if (threadIdx.x == 0) n_stage = 0;
    __syncthreads();
  };
  auto push = [&](bool keep, const jerk_candidate& c) {
    const uint64_t mask = __ballot(keep);
    if (mask == 0ull) return;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int slot = 0;
    if (lane == leader) slot = atomicAdd(&n_stage, __popcll(mask));
    slot = __builtin_amdgcn_readlane(slot, leader);
    if (keep) stage[slot + __popcll(mask & below)] = c;
  };
  auto step_done = [&]() {
    __syncthreads();
    const bool full = n_stage > kFilterStage - 256;
    __syncthreads();
    if (full) flush();
  };
  for (int32_t base = blockIdx.x * 256; base < tiles; base += gridDim.x * 256) {
    const int32_t tile = base + (int32_t)threadIdx.x;
    int32_t cnt = 0, row0 = 0;
    uint32_t p0 = 0u;
    if (tile < tiles) {
      const uint32_t c = tile_hits[tile];
      cnt = c < (uint32_t)cap_tile ? (int32_t)c : cap_tile;
      row0 = (tile / n_seg) * tpb;
      p0 = 2u * (uint32_t)(tile % n_seg) * (uint32_t)U;
    }
    int32_t most = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t o = __shfl_xor(most, off, 64);
      most = o > most ? o : most;
    }
    if (lane == 0) s_most[threadIdx.x >> 6] = most;
    __syncthreads();
    most = max(max(s_most[0], s_most[1]), max(s_most[2], s_most[3]));
    __syncthreads();
    for (int32_t k = 0; k < most; ++k) {
      bool keep = false;
      jerk_candidate cd{0u, 0u, 0.0f, 0.0f};
      if (k < cnt) {
        const CandHit h = hits[(int64_t)tile * cap_tile + k];
        const int32_t row = row0 + (int32_t)(h.code >> 16);
        const CandRowStat st = rs[row];
        keep = !st.flag && (double)h.power > st.thr;
        if (keep) {
          cd.t = (uint32_t)members[row];
          cd.p = p0 + (h.code & 0xFFFFu);
          cd.power = h.power;
          cd.sigma = (float)(((double)h.power - st.mean) / st.sigma);
        }
      }
      push(keep, cd);
      step_done();
    }
  }
  const unsigned long long pc = *pool_count;
  const int64_t np = pc < (unsigned long long)pool_cap ? (int64_t)pc : pool_cap;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < np; base += (int64_t)gridDim.x * 256) {
    const int64_t i = base + threadIdx.x;
    bool keep = false;
    jerk_candidate cd{0u, 0u, 0.0f, 0.0f};
    if (i < np) {
      const CandPoolHit h = pool[i];
      const CandRowStat st = rs[h.row];
      keep = !st.flag && (double)h.power > st.thr;
      if (keep) {
        cd.t = (uint32_t)members[h.row];
        cd.p = h.p;
        cd.power = h.power;
        cd.sigma = (float)(((double)h.power - st.mean) / st.sigma);
      }
    }
    push(keep, cd);
    step_done();
  }
  flush();
}

// The first and last point of every (row, segment), whose neighbours lie in the
// adjacent segments. edge[2 i] = (P0, P1) at lag 0, edge[2 i + 1] = (P0, P1) at
// the last lag, i = row n_seg + segment. Grid (segment blocks, rows).
__global__ void __launch_bounds__(256) cand_edges_kernel(const float2* __restrict__ edge, int32_t rows, int64_t n_seg,
                                                         int32_t U, int64_t nbins, const CandRowStat* __restrict__ rs,
                                                         const int32_t* __restrict__ members,
                                                         jerk_candidate* __restrict__ out, int64_t capacity,
                                                         unsigned long long* __restrict__ count) {
  for (int32_t r = blockIdx.y; r < rows; r += gridDim.y) {
    const CandRowStat st = rs[r];
    const uint32_t t = (uint32_t)members[r];
    const float2* row_edge = edge + 2 * (int64_t)r * n_seg;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n_seg; base += (int64_t)gridDim.x * 256) {
      const int64_t sg = base + threadIdx.x;
      bool h0 = false, h1 = false;
      float a0 = 0.0f, b1 = 0.0f;
      uint32_t p0 = 0u, p1 = 0u;
      if (sg < n_seg) {
        const float2 first = row_edge[2 * sg], last = row_edge[2 * sg + 1];
        const int64_t lim = nbins - sg * U < U ? nbins - sg * U : U;
        a0 = first.x;
        b1 = last.y;
        p0 = (uint32_t)(2 * (sg * U));
        p1 = (uint32_t)(2 * (sg * U + lim - 1) + 1);
        const bool left_ok = sg == 0 || a0 > row_edge[2 * (sg - 1) + 1].y;
        h0 = left_ok && a0 >= first.y && (double)a0 > st.thr;
        const bool right_ok = sg + 1 == n_seg || b1 >= row_edge[2 * (sg + 1)].x;
        h1 = b1 > last.x && right_ok && (double)b1 > st.thr;
      }
      emit_candidates(h0, t, p0, a0, st.mean, st.sigma, out, capacity, count);
      emit_candidates(h1, t, p1, b1, st.mean, st.sigma, out, capacity, count);
    }
  }
}

__global__ void __launch_bounds__(256) scatter_row_stats_kernel(const double* __restrict__ stats, int32_t rows,
                                                                const int32_t* __restrict__ members, int32_t t_begin,
                                                                double* __restrict__ out) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= rows) return;
  const int64_t o = 2 * (int64_t)(members[i] - t_begin);
  out[o] = stats[2 * (int64_t)i];
  out[o + 1] = stats[2 * (int64_t)i + 1];
}

}  // namespace

void scatter_row_stats(const double* stats, int32_t rows, const int32_t* d_members, int32_t t_begin, double* out,
                       hipStream_t stream) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(scatter_row_stats_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, stream, stats,
                     rows, d_members, t_begin, out);
  JERK_HIP_CHECK(hipGetLastError());
}

void cand_reset(int32_t* ovf, int32_t rows, uint32_t* n_flagged, unsigned long long* pool_count, hipStream_t stream) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(1024, ((int64_t)rows + 255) / 256));
  hipLaunchKernelGGL(cand_reset_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, ovf, rows, n_flagged,
                     pool_count);
  JERK_HIP_CHECK(hipGetLastError());
}

void cand_finish(const double2* part, int32_t rows, int64_t n_seg, int32_t U, int64_t nbins, const int32_t* ovf,
                 double k_sigma, double pre, const int32_t* d_members, int32_t t_begin, double* stats_out,
                 CandRowStat* rs, int32_t* flagged, uint32_t* n_flagged, hipStream_t stream) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(cand_finish_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, stream, part, rows, n_seg,
                     U, nbins, ovf, k_sigma, pre, d_members, t_begin, stats_out, rs, flagged, n_flagged);
  JERK_HIP_CHECK(hipGetLastError());
}

void cand_filter(const CandHit* hits, const uint32_t* tile_hits, int32_t tiles, int32_t cap_tile, int32_t n_seg,
                 int32_t tpb, int32_t U, const CandPoolHit* pool, const unsigned long long* pool_count,
                 int64_t pool_cap, const CandRowStat* rs, const int32_t* d_members, jerk_candidate* out,
                 int64_t capacity, unsigned long long* count, hipStream_t stream) {
  if (tiles <= 0) return;
  const int64_t blocks = std::min<int64_t>(4096, ((int64_t)tiles + 255) / 256);
  hipLaunchKernelGGL(cand_filter_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, hits, tile_hits, tiles,
                     cap_tile, n_seg, tpb, U, pool, pool_count, pool_cap, rs, d_members, out, capacity, count);
  JERK_HIP_CHECK(hipGetLastError());
}

void cand_edges(const float2* edge, int32_t rows, int64_t n_seg, int32_t U, int64_t nbins, const CandRowStat* rs,
                const int32_t* d_members, jerk_candidate* out, int64_t capacity, unsigned long long* count,
                hipStream_t stream) {
  if (rows <= 0 || n_seg <= 0) return;
  const int64_t bx = std::min<int64_t>(64, (n_seg + 255) / 256);
  const dim3 grid((unsigned)bx, (unsigned)(rows < kMaxGridY ? rows : kMaxGridY));
  hipLaunchKernelGGL(cand_edges_kernel, grid, dim3(256), 0, stream, edge, rows, n_seg, U, nbins, rs, d_members, out,
                     capacity, count);
  JERK_HIP_CHECK(hipGetLastError());
}

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
  const bool vec = (reinterpret_cast<uintptr_t>(plane) & 15u) == 0 && ld % 4 == 0;
  if (vec)
    hipLaunchKernelGGL(row_moments_kernel<true>, grid, dim3(kStatThreads), 0, stream, plane, ld, rows, n_r, span,
                       static_cast<Moments*>(ws));
  else
    hipLaunchKernelGGL(row_moments_kernel<false>, grid, dim3(kStatThreads), 0, stream, plane, ld, rows, n_r, span,
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
  const int64_t span = kPeakTile * kPeakTilesPerBlock;
  const int64_t bx = (n_r + span - 1) / span;
  const dim3 grid((unsigned)bx, (unsigned)(rows < kMaxGridY ? rows : kMaxGridY));
  const bool vec = (reinterpret_cast<uintptr_t>(plane) & 15u) == 0 && ld % 4 == 0;
  if (vec)
    hipLaunchKernelGGL(find_candidates_kernel<true>, grid, dim3(kPeakThreads), 0, stream, plane, ld, rows, n_r,
                       stats, k_sigma, row_template, t_base, out, capacity, count);
  else
    hipLaunchKernelGGL(find_candidates_kernel<false>, grid, dim3(kPeakThreads), 0, stream, plane, ld, rows, n_r,
                       stats, k_sigma, row_template, t_base, out, capacity, count);
  JERK_HIP_CHECK(hipGetLastError());
}

}  // namespace jerk
