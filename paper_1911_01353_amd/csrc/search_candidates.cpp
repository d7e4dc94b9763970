// Matched filter and candidate selection in one pass (paper, section "Results":
// the search is timed together with the mean and standard deviation of the plane
// and a peak finder with a user threshold), without writing the plane.
//
// The threshold of a row, mean + k sigma, is known only once the whole row has
// been computed, so each width group takes these steps on the stream:
//   1. speculative FFT pass: per (row, segment) FP64 sum and sum of squares of
//      the powers, the powers at both ends of the segment, and every interior
//      peak above a level `pre` staged in its tile's own run of slots or, past
//      those, in a shared pool;
//   2. finish: row mean, sigma, threshold; a row is flagged when its threshold
//      lies below `pre` (its staged hits may miss candidates) or when one of its
//      hits found no room (tile slots and pool full);
//   3. filter: staged hits of unflagged rows above their row's threshold;
//   4. edges: the first and last point of every (row, segment);
//   5. exact FFT pass over the flagged rows only, with their final thresholds.
// Width groups on an MFMA path have no FFT bank; their rows go through plane
// slabs of at most 2^30 bytes in the workspace instead: search, row statistics,
// peak finder (the two-step path, whose result this call equals).
// Every step is exact: with pre below every row's threshold (e.g. about (1 + k)
// times the mean power of a noise row, scaled down a little) step 5 has no work,
// and with any other pre the flagged rows are recomputed. The result equals the
// plane written by jerk_search followed by jerk_plane_stats and
// jerk_find_candidates, up to the rounding of the FP64 statistics.
//
// Staging slots per tile (tpb templates x 2U points): the caller's number, or
// by default 2 exp(-pre) of the tile's points plus 16, the expected share of
// points above pre on a spectrum of unit mean power being exp(-pre). Never more
// than tpb U, the most peaks a tile can hold (peaks are never adjacent). Tiles
// with more hits (a strong signal leaks high powers into the r range around it
// in every template) spill into a shared pool of half the slots (plus 2^16 with
// the default slot count); only a hit that finds the pool full flags its row.
#include <algorithm>
#include <cmath>

#include "jerk_internal.h"

namespace jerk {
namespace {

struct CandLayout {
  size_t part = 0, edge = 0, rs = 0, flagged = 0, n_flagged = 0, ovf = 0, tile_hits = 0, hits = 0, pool = 0,
         slab = 0, slab_stats = 0, slab_ws = 0, total = 0;
  int64_t pool_cap = 0;
  int32_t slab_rows = 0;  // rows per plane slab of an MFMA-path group
  int64_t slab_ld = 0;
};

// Rows of an MFMA-path group searched per plane slab: a multiple of 8 (a row
// block of the MFMA kernel), at most 2^30 bytes of plane but never fewer than 8.
int32_t slab_rows_for(int64_t nbins) {
  const int64_t ld = (2 * nbins + 3) / 4 * 4;
  const int64_t r = ((int64_t(1) << 30) / (ld * 4)) / 8 * 8;
  return (int32_t)std::max<int64_t>(8, std::min<int64_t>(r, 1 << 20));
}

void group_range(const Group& g, int32_t t_begin, int32_t t_end, int32_t* lo, int32_t* hi) {
  *lo = (int32_t)(std::lower_bound(g.members.begin(), g.members.end(), t_begin) - g.members.begin());
  *hi = (int32_t)(std::lower_bound(g.members.begin(), g.members.end(), t_end) - g.members.begin());
}

int64_t group_segments(const Group& g, int64_t nbins) {
  const int64_t U = g.seg_len - g.taps + 1;
  return (nbins + U - 1) / U;
}

int64_t group_tiles(const Group& g, int32_t rows, int64_t nbins) {
  return (int64_t)((rows + g.tpb - 1) / g.tpb) * group_segments(g, nbins);
}

int32_t group_cap(const Group& g, double pre, int64_t staged) {
  const int64_t U = g.seg_len - g.taps + 1;
  const int64_t most = (int64_t)g.tpb * U;
  int64_t cap = staged;
  if (cap <= 0) {
    const double pts = 2.0 * (double)g.tpb * (double)U;
    cap = (int64_t)std::ceil(2.0 * pts * std::exp(-std::max(0.0, pre))) + 16;
  }
  return (int32_t)std::min(cap, most);
}

CandLayout cand_layout(const Plan& p, int64_t nbins, int32_t t_begin, int32_t t_end, double pre, int64_t staged) {
  int64_t max_rs = 0, max_rows = 0, max_tiles = 0, max_slots = 0, max_slab = 0;
  const int32_t sr = slab_rows_for(nbins);
  for (const Group& g : p.groups) {
    int32_t lo, hi;
    group_range(g, t_begin, t_end, &lo, &hi);
    if (lo >= hi) continue;
    if (g.path != JERK_PATH_FFT_FP32) {
      max_slab = std::max<int64_t>(max_slab, std::min<int64_t>(sr, hi - lo));
      continue;
    }
    max_rows = std::max<int64_t>(max_rows, hi - lo);
    max_rs = std::max<int64_t>(max_rs, (int64_t)(hi - lo) * group_segments(g, nbins));
    const int64_t tiles = group_tiles(g, hi - lo, nbins);
    max_tiles = std::max(max_tiles, tiles);
    max_slots = std::max(max_slots, tiles * group_cap(g, pre, staged));
  }
  CandLayout L;
  L.part = 0;
  L.edge = L.part + align_up((size_t)max_rs * sizeof(double2));
  L.rs = L.edge + align_up((size_t)max_rs * 2 * sizeof(float2));
  L.flagged = L.rs + align_up((size_t)max_rows * sizeof(CandRowStat));
  L.n_flagged = L.flagged + align_up((size_t)max_rows * sizeof(int32_t));
  L.ovf = L.n_flagged + kAlign;
  L.tile_hits = L.ovf + align_up((size_t)max_rows * sizeof(int32_t));
  L.hits = L.tile_hits + align_up((size_t)max_tiles * sizeof(uint32_t));
  L.pool = L.hits + align_up((size_t)max_slots * sizeof(CandHit));
  L.pool_cap = max_slots / 2 + (staged > 0 ? 0 : (int64_t(1) << 16));
  L.slab_rows = (int32_t)max_slab;
  L.slab_ld = (2 * nbins + 3) / 4 * 4;
  L.slab = L.pool + align_up((size_t)L.pool_cap * sizeof(CandPoolHit));
  L.slab_stats = L.slab + align_up((size_t)max_slab * (size_t)L.slab_ld * sizeof(float));
  L.slab_ws = L.slab_stats + align_up((size_t)max_slab * 2 * sizeof(double));
  // statistics workspace for every slab size used: full slabs and each group's last one
  // (the size is not monotonic in the row count)
  size_t stats_ws = 0;
  if (max_slab > 0) {
    stats_ws = stats_workspace_bytes((int32_t)max_slab, 2 * nbins);
    for (const Group& g : p.groups) {
      int32_t lo, hi;
      group_range(g, t_begin, t_end, &lo, &hi);
      if (lo >= hi || g.path == JERK_PATH_FFT_FP32) continue;
      const int32_t last = (hi - lo) % (int32_t)max_slab;
      if (last > 0) stats_ws = std::max(stats_ws, stats_workspace_bytes(last, 2 * nbins));
    }
  }
  L.total = L.slab_ws + align_up(stats_ws);
  return L;
}

}  // namespace

size_t search_candidates_workspace_bytes(const Plan& p, int64_t nbins, int32_t t_begin, int32_t t_end, double pre,
                                         int64_t staged) {
  return cand_layout(p, nbins, t_begin, t_end, pre, staged).total;
}

// Every check of one search before anything of it is queued.
void search_candidates_check(const Plan& p, int64_t nbins, int32_t t_begin, int32_t t_end, double pre, int64_t staged,
                             size_t ws_bytes) {
  for (const Group& g : p.groups) {
    int32_t lo, hi;
    group_range(g, t_begin, t_end, &lo, &hi);
    if (lo >= hi || g.path != JERK_PATH_FFT_FP32) continue;
    const int64_t U = g.seg_len - g.taps + 1;
    require(g.tpb <= 65535 && 2 * U <= 65536, JERK_EINTERNAL, "tile too large for the hit encoding");
    require(group_tiles(g, hi - lo, nbins) < (int64_t(1) << 31) && group_segments(g, nbins) < (int64_t(1) << 31),
            JERK_EINVAL, "search too large for one launch; split the template range");
  }
  require(ws_bytes >= cand_layout(p, nbins, t_begin, t_end, pre, staged).total, JERK_ENOMEM,
          "search-candidates workspace too small");
}

void search_candidates(const Plan& p, const void* d_bank, const void* d_spec, int64_t nbins, int32_t t_begin,
                       int32_t t_end, double k_sigma, double pre, double* d_stats, jerk_candidate* d_out,
                       int64_t capacity, unsigned long long* d_count, int64_t staged, void* d_ws, size_t ws_bytes,
                       hipStream_t stream) {
  search_candidates_check(p, nbins, t_begin, t_end, pre, staged, ws_bytes);
  const CandLayout L = cand_layout(p, nbins, t_begin, t_end, pre, staged);
  char* ws = static_cast<char*>(d_ws);
  double2* part = reinterpret_cast<double2*>(ws + L.part);
  float2* edge = reinterpret_cast<float2*>(ws + L.edge);
  CandRowStat* rs = reinterpret_cast<CandRowStat*>(ws + L.rs);
  int32_t* flagged = reinterpret_cast<int32_t*>(ws + L.flagged);
  uint32_t* n_flagged = reinterpret_cast<uint32_t*>(ws + L.n_flagged);
  int32_t* ovf = reinterpret_cast<int32_t*>(ws + L.ovf);
  uint32_t* tile_hits = reinterpret_cast<uint32_t*>(ws + L.tile_hits);
  CandHit* hits = reinterpret_cast<CandHit*>(ws + L.hits);
  CandPoolHit* pool = reinterpret_cast<CandPoolHit*>(ws + L.pool);
  unsigned long long* pool_count = reinterpret_cast<unsigned long long*>(ws + L.n_flagged + 64);
  const char* bank = static_cast<const char*>(d_bank);
  const int32_t* members = reinterpret_cast<const int32_t*>(bank + p.off_members);
  float* slab = reinterpret_cast<float*>(ws + L.slab);
  double* slab_stats = reinterpret_cast<double*>(ws + L.slab_stats);
  void* slab_ws = ws + L.slab_ws;
  const size_t slab_ws_bytes = L.total - L.slab_ws;
  for (int32_t gi = 0; gi < (int32_t)p.groups.size(); ++gi) {
    const Group& g = p.groups[gi];
    int32_t lo, hi;
    group_range(g, t_begin, t_end, &lo, &hi);
    if (lo >= hi) continue;
    if (g.path != JERK_PATH_FFT_FP32) {
      const int32_t* gm = members + g.first_member;
      for (int32_t m0 = lo; m0 < hi; m0 += L.slab_rows) {
        const int32_t m1 = std::min(hi, m0 + L.slab_rows);
        search_members_enqueue(p, d_bank, d_spec, nbins, slab, L.slab_ld, gi, m0, m1, stream);
        plane_stats(slab, L.slab_ld, m1 - m0, 2 * nbins, slab_stats, slab_ws, slab_ws_bytes, stream);
        find_candidates(slab, L.slab_ld, m1 - m0, 2 * nbins, slab_stats, k_sigma, gm + m0, 0, d_out, capacity, d_count,
                        stream);
        if (d_stats) scatter_row_stats(slab_stats, m1 - m0, gm + m0, t_begin, d_stats, stream);
      }
      continue;
    }
    FftJob j{};
    j.spec = static_cast<const float2*>(d_spec);
    j.nbins = nbins;
    j.bank_fft = reinterpret_cast<const float2*>(bank + g.off_fft);
    j.members = members + g.first_member;
    j.m_begin = lo;
    j.m_end = hi;
    j.t_begin = t_begin;
    j.row_by_member = 1;
    j.row_base = lo;
    j.taps = g.taps;
    j.tpb = g.tpb;
    const int32_t U = g.seg_len - g.taps + 1;
    const int64_t n_seg = group_segments(g, nbins);
    const int32_t rows = hi - lo;
    const int32_t* row_t = j.members + lo;  // template of row r
    const float2* tw = reinterpret_cast<const float2*>(bank + p.off_tw[tw_slot(g.seg_len)]);
    const int32_t cap = group_cap(g, pre, staged);
    const int64_t tiles = group_tiles(g, rows, nbins);
    CandArgs ca{};
    ca.pre = pre;
    ca.part = part;
    ca.edge = edge;
    ca.hits = hits;
    ca.tile_hits = tile_hits;
    ca.pool = pool;
    ca.pool_count = pool_count;
    ca.pool_cap = L.pool_cap;
    ca.ovf = ovf;
    ca.cap_tile = cap;
    ca.rs = rs;
    ca.flagged = flagged;
    ca.n_flagged = n_flagged;
    ca.out = d_out;
    ca.capacity = capacity;
    ca.count = d_count;
    cand_reset(ovf, rows, n_flagged, pool_count, stream);
    fft_cand_launch(j, g.seg_len, g.ept, tw, ca, 1, stream);
    cand_finish(part, rows, n_seg, U, nbins, ovf, k_sigma, pre, row_t, t_begin, d_stats, rs, flagged, n_flagged,
                stream);
    cand_filter(hits, tile_hits, (int32_t)tiles, cap, (int32_t)n_seg, g.tpb, U, pool, pool_count, L.pool_cap, rs,
                row_t, d_out, capacity, d_count, stream);
    cand_edges(edge, rows, n_seg, U, nbins, rs, row_t, d_out, capacity, d_count, stream);
    fft_cand_launch(j, g.seg_len, g.ept, tw, ca, 2, stream);
  }
}

// Many spectra, one after the other on the stream in one workspace (each search's steps
// finish reading the workspace before the next search's first step writes it: stream order).
size_t batch_search_candidates_workspace_bytes(const Plan& p, const jerk_batch_cand_item* items, int32_t count,
                                               int32_t t_begin, int32_t t_end, double pre, int64_t staged) {
  size_t most = 0;
  for (int32_t i = 0; i < count; ++i)
    most = std::max(most, cand_layout(p, items[i].nbins, t_begin, t_end, pre, staged).total);
  return most;
}

void batch_search_candidates(const Plan& p, const void* d_bank, const jerk_batch_cand_item* items, int32_t count,
                             int32_t t_begin, int32_t t_end, double k_sigma, double pre, int64_t staged, void* d_ws,
                             size_t ws_bytes, hipStream_t stream) {
  for (int32_t i = 0; i < count; ++i)
    search_candidates_check(p, items[i].nbins, t_begin, t_end, pre, staged, ws_bytes);
  for (int32_t i = 0; i < count; ++i) {
    const jerk_batch_cand_item& it = items[i];
    search_candidates(p, d_bank, it.spec, it.nbins, t_begin, t_end, k_sigma, pre, it.stats, it.out, it.capacity,
                      it.count, staged, d_ws, ws_bytes, stream);
  }
}

}  // namespace jerk
