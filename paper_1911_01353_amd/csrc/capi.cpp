// C ABI entry points: argument checks, status codes and per-thread error text.
// No C++ exception crosses this boundary.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "jerk_internal.h"

namespace jerk {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

template <class F>
int32_t guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return JERK_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return JERK_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = std::string("internal error: ") + e.what();
    return JERK_EINTERNAL;
  } catch (...) {
    g_last_error = "internal error";
    return JERK_EINTERNAL;
  }
}

void gen_twiddles(float2* out, int32_t n, hipStream_t stream);
// reduce.hip: n copies of v (a kernel, so that the call may be captured in a graph)
void fill_u64(uint64_t* dst, int64_t n, uint64_t v, hipStream_t stream);
// search_candidates.cpp: many spectra through the search with candidate selection
size_t batch_search_candidates_workspace_bytes(const Plan& p, const jerk_batch_cand_item* items, int32_t count,
                                               int32_t t_begin, int32_t t_end, double pre, int64_t staged);
void batch_search_candidates(const Plan& p, const void* d_bank, const jerk_batch_cand_item* items, int32_t count,
                             int32_t t_begin, int32_t t_end, double k_sigma, double pre, int64_t staged, void* d_ws,
                             size_t ws_bytes, hipStream_t stream);
// gemm_correlate.hip: several narrow MFMA-path groups in one launch (up to 8 jobs)
bool gemm_multi_eligible(const GemmArgs& a);
void gemm_correlate_multi_launch(const GemmArgs* jobs, int n, hipStream_t stream);

// Member sub-range [lo, hi) of group g whose templates lie in [t_begin, t_end).
static void member_range(const Group& g, int32_t t_begin, int32_t t_end, int32_t* lo, int32_t* hi) {
  *lo = (int32_t)(std::lower_bound(g.members.begin(), g.members.end(), t_begin) - g.members.begin());
  *hi = (int32_t)(std::lower_bound(g.members.begin(), g.members.end(), t_end) - g.members.begin());
}

// Plane rows [t_begin, t_end) of groups [g_begin, g_end) into d_plane and/or, when row_max is
// set, one peak key per row (row t - t_begin, combined with atomicMax; cleared by the caller).
void search_enqueue(const Plan& p, const void* d_bank, const void* d_spec, int64_t nbins, float* d_plane,
                    int64_t ld, int32_t t_begin, int32_t t_end, int32_t g_begin, int32_t g_end,
                    hipStream_t stream, uint64_t* row_max = nullptr) {
  const char* bank = static_cast<const char*>(d_bank);
  const int32_t* members = reinterpret_cast<const int32_t*>(bank + p.off_members);
  // launch limits of every group before any launch, so an error queues nothing
  for (int32_t gi = g_begin; gi < g_end; ++gi) {
    const Group& g = p.groups[gi];
    int32_t lo, hi;
    member_range(g, t_begin, t_end, &lo, &hi);
    if (lo >= hi || g.path != JERK_PATH_FFT_FP32) continue;
    const int64_t U = g.seg_len - g.taps + 1;
    const int64_t tiles = (nbins + U - 1) / U * ((hi - lo + g.tpb - 1) / g.tpb);
    require(tiles < (1ll << 31), JERK_EINVAL, "search too large for one launch; split the template range");
  }
  // narrow MFMA-path groups of one kind (split-BF16 or FP16) go out together in one launch
  GemmArgs pending[8];
  int n_pending = 0;
  auto flush = [&]() {
    if (n_pending == 1) gemm_correlate_launch(pending[0], stream);
    else if (n_pending > 1) gemm_correlate_multi_launch(pending, n_pending, stream);
    n_pending = 0;
  };
  // FFT-path groups of one kernel variant (segment length, elements per thread) go out
  // together too, up to kFftArgJobs per launch: one launch and one tail instead of one per group
  FftJob fpend[kFftArgJobs];
  int n_fpend = 0, f_seg = 0, f_ept = 0;
  int64_t f_tiles = 0;  // tiles of the pending jobs (one launch stays below 2^31 workgroups)
  const float2* f_tw = nullptr;
  auto fflush = [&]() {
    if (n_fpend == 1) fft_correlate_launch(fpend[0], f_seg, f_ept, f_tw, stream);
    else if (n_fpend > 1) fft_args_launch(fpend, n_fpend, f_seg, f_ept, row_max != nullptr, f_tw, stream);
    n_fpend = 0;
    f_tiles = 0;
  };
  for (int32_t gi = g_begin; gi < g_end; ++gi) {
    const Group& g = p.groups[gi];
    int32_t lo, hi;
    member_range(g, t_begin, t_end, &lo, &hi);
    if (lo >= hi) continue;
    if (g.path == JERK_PATH_FFT_FP32) {
      FftJob j{};
      j.spec = static_cast<const float2*>(d_spec);
      j.nbins = nbins;
      j.bank_fft = reinterpret_cast<const float2*>(bank + g.off_fft);
      j.members = members + g.first_member;
      j.m_begin = lo;
      j.m_end = hi;
      j.t_begin = t_begin;
      j.plane = d_plane;
      j.ld = ld;
      j.taps = g.taps;
      j.tpb = g.tpb;
      j.row_max = row_max;
      j.rmax_ld = 0;
      const int64_t U = g.seg_len - g.taps + 1;
      const int64_t tiles = (nbins + U - 1) / U * ((hi - lo + g.tpb - 1) / g.tpb);
      if (n_fpend > 0 && (f_seg != g.seg_len || f_ept != g.ept || f_tiles + tiles >= (1ll << 31))) fflush();
      f_tiles += tiles;
      f_seg = g.seg_len;
      f_ept = g.ept;
      f_tw = reinterpret_cast<const float2*>(bank + p.off_tw[tw_slot(g.seg_len)]);
      fpend[n_fpend++] = j;
      if (n_fpend == kFftArgJobs) fflush();
    } else {
      GemmArgs a{};
      a.spec = static_cast<const float2*>(d_spec);
      a.nbins = nbins;
      a.bank_gemm = bank + g.off_gemm;
      a.members = members + g.first_member;
      a.m_begin = lo / 8 * 8;
      a.m_end = hi;
      a.t_begin = t_begin;
      a.t_end = t_end;
      a.plane = d_plane;
      a.ld = ld;
      a.taps = g.taps;
      a.path = g.path;
      a.row_max = row_max;
      if (gemm_multi_eligible(a)) {
        if (n_pending > 0 && pending[0].path != a.path) flush();
        pending[n_pending++] = a;
        if (n_pending == 8) flush();
      } else {
        gemm_correlate_launch(a, stream);
      }
    }
  }
  flush();
  fflush();
}

// Rows [m_begin, m_end) of group g's member list, output row = member - m_begin.
void search_members_enqueue(const Plan& p, const void* d_bank, const void* d_spec, int64_t nbins, float* d_plane,
                            int64_t ld, int32_t gi, int32_t m_begin, int32_t m_end, hipStream_t stream) {
  const char* bank = static_cast<const char*>(d_bank);
  const int32_t* members = reinterpret_cast<const int32_t*>(bank + p.off_members);
  const Group& g = p.groups[gi];
  if (g.path == JERK_PATH_FFT_FP32) {
    FftJob j{};
    j.spec = static_cast<const float2*>(d_spec);
    j.nbins = nbins;
    j.bank_fft = reinterpret_cast<const float2*>(bank + g.off_fft);
    j.members = members + g.first_member;
    j.m_begin = m_begin;
    j.m_end = m_end;
    j.row_by_member = 1;
    j.row_base = m_begin;
    j.plane = d_plane;
    j.ld = ld;
    j.taps = g.taps;
    j.tpb = g.tpb;
    fft_correlate_launch(j, g.seg_len, g.ept, reinterpret_cast<const float2*>(bank + p.off_tw[tw_slot(g.seg_len)]),
                         stream);
  } else {
    GemmArgs a{};
    a.spec = static_cast<const float2*>(d_spec);
    a.nbins = nbins;
    a.bank_gemm = bank + g.off_gemm;
    a.members = members + g.first_member;
    a.m_begin = m_begin / 8 * 8;
    a.m_end = m_end;
    a.t_begin = 0;
    a.t_end = p.T;
    a.row_by_member = 1;
    a.row_base = m_begin;
    a.plane = d_plane;
    a.ld = ld;
    a.taps = g.taps;
    a.path = g.path;
    // members below m_begin (in the first block of 8) are computed but not written (row < 0)
    gemm_correlate_launch(a, stream);
  }
}

}  // namespace jerk

using jerk::Error;
using jerk::guarded;
using jerk::require;

extern "C" {

const char* jerk_status_str(int32_t s) {
  switch (s) {
    case JERK_OK: return "JERK_OK";
    case JERK_EINVAL: return "JERK_EINVAL";
    case JERK_ENOMEM: return "JERK_ENOMEM";
    case JERK_EAGAIN: return "JERK_EAGAIN";
    case JERK_EPENDING: return "JERK_EPENDING";
    case JERK_EHIP: return "JERK_EHIP";
    case JERK_EUNSUPPORTED: return "JERK_EUNSUPPORTED";
    case JERK_EINTERNAL: return "JERK_EINTERNAL";
    case JERK_ECANCELED: return "JERK_ECANCELED";
    default: return "JERK_UNKNOWN";
  }
}

const char* jerk_last_error(void) { return jerk::g_last_error.c_str(); }

const char* jerk_version(void) { return "jerk-mi355x 1.0 gfx950"; }

int32_t jerk_stream_check(hipStream_t stream) {
  int32_t pending = 0;
  const int32_t st = guarded([&] {
    const hipError_t e = hipStreamQuery(stream);
    if (e == hipErrorNotReady) {
      pending = 1;
      return;
    }
    JERK_HIP_CHECK(e);
  });
  return st == JERK_OK && pending ? JERK_EPENDING : st;
}

int32_t jerk_plan_create(const jerk_plan_desc* desc, jerk_plan** out) {
  return guarded([&] {
    require(desc != nullptr && out != nullptr, JERK_EINVAL, "desc and out must not be NULL");
    *out = nullptr;
    jerk_plan* p = new jerk_plan();
    try {
      jerk::plan_build(p->p, *desc);
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
  });
}

int32_t jerk_plan_destroy(jerk_plan* plan) {
  return guarded([&] {
    if (!plan) return;
    if (plan->p.pinned_members) (void)hipHostFree(plan->p.pinned_members);
    jerk::batch_ctx_free(plan->p.batch);
    delete plan;
  });
}

int32_t jerk_plan_info(const jerk_plan* plan, jerk_plan_info_t* out) {
  return guarded([&] {
    require(plan && out, JERK_EINVAL, "plan and out must not be NULL");
    const jerk::Plan& p = plan->p;
    std::memset(out, 0, sizeof(*out));
    out->n_z = p.n_z;
    out->n_w = p.n_w;
    out->n_templates = p.T;
    out->n_groups = (int32_t)p.groups.size();
    out->nbins = p.desc.nbins;
    out->n_r = 2 * p.desc.nbins;
    out->max_taps = p.max_taps;
    out->path = p.desc.path;
    out->bank_bytes = p.bank_bytes;
    out->workspace_bytes = 0;
    out->plane_row_bytes = (size_t)(2 * p.desc.nbins) * sizeof(float);
    out->taps_offset = p.groups.empty() ? 0 : p.groups[0].off_taps;
  });
}

int32_t jerk_plan_group(const jerk_plan* plan, int32_t g, jerk_group_info_t* out) {
  return guarded([&] {
    require(plan && out, JERK_EINVAL, "plan and out must not be NULL");
    require(g >= 0 && g < (int32_t)plan->p.groups.size(), JERK_EINVAL, "group index out of range");
    const jerk::Group& G = plan->p.groups[g];
    std::memset(out, 0, sizeof(*out));
    out->taps = G.taps;
    out->seg_len = G.seg_len;
    out->templates_per_block = G.tpb;
    out->path = G.path;
    out->n_members = (int32_t)G.members.size();
    out->first_member = G.first_member;
    out->taps_offset = G.off_taps;
    out->fft_ept = G.ept;
  });
}

int32_t jerk_plan_template(const jerk_plan* plan, int32_t t, double* zbar, double* w, int32_t* half_width,
                           int32_t* group, int32_t* slot) {
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    require(t >= 0 && t < plan->p.T, JERK_EINVAL, "template index out of range");
    const jerk::Plan& p = plan->p;
    if (zbar) *zbar = p.zbar[t];
    if (w) *w = p.w[t];
    if (half_width) *half_width = p.half[t];
    if (group) *group = p.group_of[t];
    if (slot) *slot = p.slot[t];
  });
}

int32_t jerk_plan_members(const jerk_plan* plan, int32_t* out, int32_t count) {
  return guarded([&] {
    require(plan && out, JERK_EINVAL, "plan and out must not be NULL");
    require(count >= plan->p.T, JERK_ENOMEM, "output holds fewer than n_templates entries");
    int32_t k = 0;
    for (const auto& g : plan->p.groups)
      for (int32_t t : g.members) out[k++] = t;
  });
}

int32_t jerk_plan_set_group(jerk_plan* plan, int32_t g, int32_t seg_len, int32_t templates_per_block,
                            int32_t path, int32_t fft_ept) {
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    jerk::Plan& p = plan->p;
    require(g >= 0 && g < (int32_t)p.groups.size(), JERK_EINVAL, "group index out of range");
    jerk::Group& G = p.groups[g];
    require(jerk::seg_len_supported(seg_len) && seg_len >= 2 * G.taps, JERK_EINVAL,
            "seg_len must be 512..4096 (power of two) and at least twice the group's taps");
    require(templates_per_block >= 1 && templates_per_block <= 64, JERK_EINVAL,
            "templates_per_block must be in [1, 64]");
    require(path == JERK_PATH_FFT_FP32 || path == JERK_PATH_GEMM_SPLIT_BF16 || path == JERK_PATH_GEMM_FP16,
            JERK_EINVAL, "group path must be FFT_FP32, GEMM_SPLIT_BF16 or GEMM_FP16");
    require(path == JERK_PATH_FFT_FP32 || G.taps <= 512, JERK_EUNSUPPORTED,
            "MFMA paths support templates up to 512 taps");
    if (fft_ept == 0) fft_ept = seg_len == 512 ? 8 : 16;
    require(jerk::fft_variant_supported(seg_len, fft_ept), JERK_EINVAL,
            "no FFT kernel variant with this segment length and elements per thread");
    G.seg_len = seg_len;
    G.tpb = templates_per_block;
    G.path = path;
    G.ept = fft_ept;
    jerk::plan_layout(p);
  });
}

int32_t jerk_templates_build(jerk_plan* plan, void* d_bank, size_t bank_bytes, hipStream_t stream) {
  return guarded([&] {
    require(plan != nullptr && d_bank != nullptr, JERK_EINVAL, "plan and d_bank must not be NULL");
    jerk::Plan& p = plan->p;
    require(bank_bytes >= p.bank_bytes, JERK_ENOMEM, "bank buffer smaller than bank_bytes");
    require(reinterpret_cast<uintptr_t>(d_bank) % 256 == 0, JERK_EINVAL, "bank must be 256-byte aligned");
    jerk::bank_build(p, d_bank, stream);
  });
}

int32_t jerk_search(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins, float* d_plane,
                    int64_t ld, int32_t t_begin, int32_t t_end, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  (void)d_ws;
  (void)ws_bytes;
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    const jerk::Plan& p = plan->p;
    require(0 <= t_begin && t_begin <= t_end && t_end <= p.T, JERK_EINVAL, "template range outside [0, n_templates]");
    if (t_begin == t_end) return;  // empty range: nothing to do, pointers unused
    require(d_bank && d_spec && d_plane, JERK_EINVAL, "bank, spectrum and plane must not be NULL");
    require(nbins >= 1, JERK_EINVAL, "nbins must be >= 1");
    require(ld >= 2 * nbins, JERK_EINVAL, "ld must be >= 2 * nbins");
    require(ld % 2 == 0, JERK_EINVAL, "ld must be even (phase pairs are stored as float2)");
    require(reinterpret_cast<uintptr_t>(d_plane) % 8 == 0 && reinterpret_cast<uintptr_t>(d_spec) % 8 == 0,
            JERK_EINVAL, "spectrum and plane must be 8-byte aligned");
    require(0 <= t_begin && t_begin <= t_end && t_end <= p.T, JERK_EINVAL, "template range outside [0, n_templates]");
    jerk::search_enqueue(p, d_bank, d_spec, nbins, d_plane, ld, t_begin, t_end, 0, (int32_t)p.groups.size(), stream);
  });
}

int32_t jerk_search_group(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                          float* d_plane, int64_t ld, int32_t t_begin, int32_t t_end, int32_t g,
                          hipStream_t stream) {
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    const jerk::Plan& p = plan->p;
    require(0 <= t_begin && t_begin <= t_end && t_end <= p.T, JERK_EINVAL, "template range outside [0, n_templates]");
    require(g >= 0 && g < (int32_t)p.groups.size(), JERK_EINVAL, "group index out of range");
    if (t_begin == t_end) return;
    require(d_bank && d_spec && d_plane, JERK_EINVAL, "bank, spectrum and plane must not be NULL");
    require(nbins >= 1, JERK_EINVAL, "nbins must be >= 1");
    require(ld >= 2 * nbins && ld % 2 == 0, JERK_EINVAL, "ld must be even and >= 2 * nbins");
    require(reinterpret_cast<uintptr_t>(d_plane) % 8 == 0 && reinterpret_cast<uintptr_t>(d_spec) % 8 == 0,
            JERK_EINVAL, "spectrum and plane must be 8-byte aligned");
    require(0 <= t_begin && t_begin <= t_end && t_end <= p.T, JERK_EINVAL, "template range outside [0, n_templates]");
    require(g >= 0 && g < (int32_t)p.groups.size(), JERK_EINVAL, "group index out of range");
    jerk::search_enqueue(p, d_bank, d_spec, nbins, d_plane, ld, t_begin, t_end, g, g + 1, stream);
  });
}

size_t jerk_batch_workspace_bytes(const jerk_plan* plan, int32_t count) {
  if (!plan || count < 0) return 0;
  return jerk::batch_workspace_bytes(plan->p, count);
}

int64_t jerk_batch_keys_per_row(const jerk_plan* plan, int64_t nbins) {
  if (!plan || nbins < 1) return 0;
  return jerk::batch_keys_per_row(plan->p, nbins);
}

int32_t jerk_batch_search(jerk_plan* plan, const void* d_bank, const jerk_batch_item* items, int32_t count,
                          int32_t t_begin, int32_t t_end, void* d_ws, size_t ws_bytes, uint32_t flags,
                          hipStream_t stream) {
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    jerk::batch_search(plan->p, d_bank, items, count, t_begin, t_end, d_ws, ws_bytes, flags, stream);
  });
}

int32_t jerk_peaks_reduce(const uint64_t* d_keys, int32_t rows, int64_t keys_per_row, int64_t keys_ld,
                          jerk_peak* d_out, hipStream_t stream) {
  return guarded([&] {
    require(rows >= 0 && keys_per_row >= 1 && keys_ld >= keys_per_row, JERK_EINVAL, "bad key layout");
    if (rows == 0) return;
    require(d_keys && d_out, JERK_EINVAL, "keys and output must not be NULL");
    jerk::peaks_reduce(d_keys, rows, keys_per_row, keys_ld, d_out, stream);
  });
}

int32_t jerk_harmonic_shape(const jerk_plan* plan, int64_t n_r, int32_t n_harm, int32_t* n_zf, int32_t* n_wf,
                            int64_t* n_pf) {
  return guarded([&] {
    require(plan && n_zf && n_wf && n_pf, JERK_EINVAL, "plan and outputs must not be NULL");
    const jerk::HarmonicShape s = jerk::harmonic_shape(plan->p, n_r, n_harm);
    *n_zf = s.n_zf;
    *n_wf = s.n_wf;
    *n_pf = s.n_pf;
  });
}

int32_t jerk_harmonic_sum(const jerk_plan* plan, const float* d_plane, int64_t ld, int64_t n_r, int32_t n_harm,
                          float* d_out, int64_t out_ld, hipStream_t stream) {
  return guarded([&] {
    require(plan && d_plane && d_out, JERK_EINVAL, "plan, plane and output must not be NULL");
    jerk::harmonic_sum(plan->p, d_plane, ld, n_r, n_harm, d_out, out_ld, stream);
  });
}

static bool spectrum_length_ok(int64_t n) { return n >= 4 && n <= (int64_t(1) << 30) && (n & (n - 1)) == 0; }

size_t jerk_spectrum_workspace_bytes(int64_t n_samples) {
  if (!spectrum_length_ok(n_samples)) return 0;
  return jerk::spectrum_workspace_bytes(n_samples);
}

int32_t jerk_spectrum_prepare(const float* d_series, int64_t n_samples, void* d_spec, void* d_ws,
                              size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    require(n_samples >= 4 && n_samples <= (int64_t(1) << 30), JERK_EINVAL, "n_samples must be in [4, 2^30]");
    require(spectrum_length_ok(n_samples), JERK_EUNSUPPORTED, "n_samples must be a power of two");
    require(d_series && d_spec && d_ws, JERK_EINVAL, "series, spectrum and workspace must not be NULL");
    require((reinterpret_cast<uintptr_t>(d_series) & 7u) == 0 && (reinterpret_cast<uintptr_t>(d_spec) & 7u) == 0 &&
                (reinterpret_cast<uintptr_t>(d_ws) & 15u) == 0,
            JERK_EINVAL, "series and spectrum must be 8-byte aligned, the workspace 16-byte aligned");
    jerk::spectrum_prepare(d_series, n_samples, static_cast<float2*>(d_spec), d_ws, ws_bytes, stream);
  });
}

size_t jerk_stats_workspace_bytes(int32_t rows, int64_t n_r) {
  if (rows < 0 || n_r < 0) return 0;
  return jerk::stats_workspace_bytes(rows, n_r);
}

int32_t jerk_plane_stats(const float* d_plane, int64_t ld, int32_t rows, int64_t n_r, double* d_stats,
                         void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    require(rows >= 0 && n_r >= 0 && ld >= n_r, JERK_EINVAL, "need rows >= 0, n_r >= 0 and ld >= n_r");
    if (rows == 0 || n_r == 0) return;
    require(d_plane && d_stats && d_ws, JERK_EINVAL, "plane, stats and workspace must not be NULL");
    jerk::plane_stats(d_plane, ld, rows, n_r, d_stats, d_ws, ws_bytes, stream);
  });
}

int32_t jerk_find_candidates(const float* d_plane, int64_t ld, int32_t rows, int64_t n_r, const double* d_stats,
                             double k_sigma, const int32_t* d_row_template, int32_t t_base,
                             jerk_candidate* d_out, int64_t capacity, unsigned long long* d_count,
                             hipStream_t stream) {
  return guarded([&] {
    require(rows >= 0 && n_r >= 0 && ld >= n_r, JERK_EINVAL, "need rows >= 0, n_r >= 0 and ld >= n_r");
    require(n_r < (int64_t(1) << 32), JERK_EINVAL, "n_r must be < 2^32");
    require(std::isfinite(k_sigma), JERK_EINVAL, "k_sigma must be finite");
    require(capacity >= 0, JERK_EINVAL, "capacity must be >= 0");
    if (rows == 0 || n_r == 0) return;
    require(d_plane && d_stats && d_count, JERK_EINVAL, "plane, stats and count must not be NULL");
    require(d_out || capacity == 0, JERK_EINVAL, "output must not be NULL when capacity > 0");
    require(d_row_template || (t_base >= 0 && (int64_t)t_base + rows - 1 <= INT32_MAX), JERK_EINVAL,
            "t_base must be >= 0 and t_base + rows - 1 must fit int32");
    jerk::find_candidates(d_plane, ld, rows, n_r, d_stats, k_sigma, d_row_template, t_base, d_out, capacity,
                          d_count, stream);
  });
}

size_t jerk_search_peaks_workspace_bytes(const jerk_plan* plan, int32_t t_begin, int32_t t_end) {
  if (!plan || t_begin < 0 || t_end < t_begin || t_end > plan->p.T) return 0;
  return (size_t)(t_end - t_begin) * sizeof(uint64_t);
}

int32_t jerk_search_peaks(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                          int32_t t_begin, int32_t t_end, jerk_peak* d_out, void* d_ws, size_t ws_bytes,
                          hipStream_t stream) {
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    const jerk::Plan& p = plan->p;
    require(0 <= t_begin && t_begin <= t_end && t_end <= p.T, JERK_EINVAL, "template range outside [0, n_templates]");
    if (t_begin == t_end) return;
    require(d_bank && d_spec && d_out && d_ws, JERK_EINVAL, "bank, spectrum, output and workspace must not be NULL");
    require(nbins >= 1 && nbins < (int64_t(1) << 31), JERK_EINVAL, "nbins must be in [1, 2^31)");
    require(reinterpret_cast<uintptr_t>(d_spec) % 8 == 0 && reinterpret_cast<uintptr_t>(d_ws) % 8 == 0, JERK_EINVAL,
            "spectrum and workspace must be 8-byte aligned");
    const int32_t rows = t_end - t_begin;
    require(ws_bytes >= (size_t)rows * sizeof(uint64_t), JERK_ENOMEM, "peak workspace too small");
    uint64_t* keys = static_cast<uint64_t*>(d_ws);
    jerk::fill_u64(keys, rows, 0ull, stream);
    jerk::search_enqueue(p, d_bank, d_spec, nbins, nullptr, 2 * nbins, t_begin, t_end, 0, (int32_t)p.groups.size(),
                         stream, keys);
    jerk::peaks_reduce(keys, rows, 1, 1, d_out, stream);
  });
}

namespace {
// Key workspace of jerk_search_peaks_noalloc: one copy per GPU, found by symbol lookup.
constexpr int kMaxDevices = 64;
static __device__ __align__(256) uint64_t scratch[JERK_NOALLOC_MAX_ROWS];
std::mutex g_scratch_mu;
uint64_t* g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up once per device).
uint64_t* scratch_on_current_device() {
  int dev = 0;
  JERK_HIP_CHECK(hipGetDevice(&dev));
  require(dev >= 0 && dev < kMaxDevices, JERK_EUNSUPPORTED, "device index beyond the no-allocation table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* ptr = nullptr;
    JERK_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    require(ptr != nullptr, JERK_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch[dev] = static_cast<uint64_t*>(ptr);
  }
  return g_scratch[dev];
}
}  // namespace

int32_t jerk_search_peaks_noalloc(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                                  int32_t t_begin, int32_t t_end, jerk_peak* d_out, hipStream_t stream) {
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    const jerk::Plan& p = plan->p;
    require(0 <= t_begin && t_begin <= t_end && t_end <= p.T, JERK_EINVAL, "template range outside [0, n_templates]");
    if (t_begin == t_end) return;
    require(d_bank && d_spec && d_out, JERK_EINVAL, "bank, spectrum and output must not be NULL");
    require(nbins >= 1 && nbins < (int64_t(1) << 31), JERK_EINVAL, "nbins must be in [1, 2^31)");
    require(reinterpret_cast<uintptr_t>(d_spec) % 8 == 0, JERK_EINVAL, "spectrum must be 8-byte aligned");
    const int32_t rows = t_end - t_begin;
    require(rows <= JERK_NOALLOC_MAX_ROWS, JERK_EINVAL,
            "t_end - t_begin exceeds JERK_NOALLOC_MAX_ROWS (32768): split the template range");
    uint64_t* keys = scratch_on_current_device();  // never the array's name: a host-side stand-in
    jerk::fill_u64(keys, rows, 0ull, stream);
    jerk::search_enqueue(p, d_bank, d_spec, nbins, nullptr, 2 * nbins, t_begin, t_end, 0, (int32_t)p.groups.size(),
                         stream, keys);
    jerk::peaks_reduce(keys, rows, 1, 1, d_out, stream);
  });
}

size_t jerk_batch_search_candidates_workspace_bytes(const jerk_plan* plan, const jerk_batch_cand_item* items,
                                                    int32_t count, int32_t t_begin, int32_t t_end, double pre_level,
                                                    int64_t staged) {
  if (!plan || (!items && count > 0) || count < 0 || staged < 0 || !std::isfinite(pre_level) || t_begin < 0 ||
      t_end < t_begin || t_end > plan->p.T)
    return 0;
  for (int32_t i = 0; i < count; ++i)
    if (items[i].nbins < 1 || items[i].nbins >= (int64_t(1) << 31)) return 0;
  return jerk::batch_search_candidates_workspace_bytes(plan->p, items, count, t_begin, t_end, pre_level, staged);
}

int32_t jerk_batch_search_candidates(const jerk_plan* plan, const void* d_bank, const jerk_batch_cand_item* items,
                                     int32_t count, int32_t t_begin, int32_t t_end, double k_sigma, double pre_level,
                                     int64_t staged, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    require(count >= 0 && (items || count == 0), JERK_EINVAL, "items must not be NULL when count > 0");
    require(t_begin >= 0 && t_begin <= t_end && t_end <= plan->p.T, JERK_EINVAL, "bad template range");
    require(std::isfinite(k_sigma) && std::isfinite(pre_level), JERK_EINVAL, "k_sigma and pre_level must be finite");
    require(staged >= 0, JERK_EINVAL, "staged must be >= 0");
    if (count == 0 || t_begin == t_end) return;
    require(d_bank && d_ws, JERK_EINVAL, "bank and workspace must not be NULL");
    for (int32_t i = 0; i < count; ++i) {
      const jerk_batch_cand_item& it = items[i];
      require(it.nbins >= 1 && it.nbins < (int64_t(1) << 31), JERK_EINVAL, "item nbins must be in [1, 2^31)");
      require(it.spec && it.count && it.capacity >= 0 && (it.out || it.capacity == 0), JERK_EINVAL,
              "item spectrum, count and (with capacity > 0) output must not be NULL");
    }
    jerk::batch_search_candidates(plan->p, d_bank, items, count, t_begin, t_end, k_sigma, pre_level, staged, d_ws,
                                  ws_bytes, stream);
  });
}

size_t jerk_search_candidates_workspace_bytes(const jerk_plan* plan, int64_t nbins, int32_t t_begin, int32_t t_end,
                                              double pre_level, int64_t staged) {
  if (!plan || nbins < 1 || nbins >= (int64_t(1) << 31) || staged < 0 || !std::isfinite(pre_level) || t_begin < 0 ||
      t_end < t_begin || t_end > plan->p.T)
    return 0;
  return jerk::search_candidates_workspace_bytes(plan->p, nbins, t_begin, t_end, pre_level, staged);
}

int32_t jerk_search_candidates(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                               int32_t t_begin, int32_t t_end, double k_sigma, double pre_level, int64_t staged,
                               double* d_stats, jerk_candidate* d_out, int64_t capacity,
                               unsigned long long* d_count, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    require(t_begin >= 0 && t_begin <= t_end && t_end <= plan->p.T, JERK_EINVAL, "bad template range");
    require(nbins >= 1 && nbins < (int64_t(1) << 31), JERK_EINVAL, "nbins must be in [1, 2^31)");
    require(std::isfinite(k_sigma) && std::isfinite(pre_level), JERK_EINVAL, "k_sigma and pre_level must be finite");
    require(staged >= 0 && capacity >= 0, JERK_EINVAL, "staged and capacity must be >= 0");
    if (t_begin == t_end) return;
    require(d_bank && d_spec && d_count && d_ws, JERK_EINVAL, "bank, spectrum, count and workspace must not be NULL");
    require(d_out || capacity == 0, JERK_EINVAL, "output must not be NULL when capacity > 0");
    jerk::search_candidates(plan->p, d_bank, d_spec, nbins, t_begin, t_end, k_sigma, pre_level, d_stats, d_out,
                            capacity, d_count, staged, d_ws, ws_bytes, stream);
  });
}

size_t jerk_autotune_scratch_bytes(const jerk_plan* plan, int64_t nbins) {
  if (!plan || nbins < 1) return 0;
  return jerk::autotune_scratch_bytes(plan->p, nbins);
}

int32_t jerk_plan_autotune(jerk_plan* plan, const void* d_spec, int64_t nbins, void* d_scratch, size_t scratch_bytes,
                           uint32_t flags, hipStream_t stream) {
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    jerk::autotune(plan->p, d_spec, nbins, d_scratch, scratch_bytes, flags, stream);
  });
}

int32_t jerk_serve_create(const jerk_serve_desc* desc, void* d_arena, size_t arena_bytes, jerk_server** out) {
  return guarded([&] {
    require(desc != nullptr && out != nullptr, JERK_EINVAL, "desc and out must not be NULL");
    *out = nullptr;
    jerk::serve_create(*desc, d_arena, arena_bytes, out);
  });
}

int32_t jerk_serve_submit(jerk_server* srv, const jerk_request* req, uint64_t* ticket) {
  return guarded([&] {
    require(srv && req && ticket, JERK_EINVAL, "server, request and ticket must not be NULL");
    jerk::serve_submit(*srv, *req, ticket);
  });
}

int32_t jerk_serve_poll(jerk_server* srv, uint64_t ticket, jerk_result* out) {
  int32_t rc = JERK_OK;
  const int32_t st = guarded([&] {
    require(srv && out, JERK_EINVAL, "server and out must not be NULL");
    rc = jerk::serve_poll(*srv, ticket, out, 0.0);
  });
  return st != JERK_OK ? st : rc;
}

int32_t jerk_serve_wait(jerk_server* srv, uint64_t ticket, jerk_result* out, double timeout_s) {
  int32_t rc = JERK_OK;
  const int32_t st = guarded([&] {
    require(srv && out, JERK_EINVAL, "server and out must not be NULL");
    rc = jerk::serve_poll(*srv, ticket, out, timeout_s);
  });
  return st != JERK_OK ? st : rc;
}

int32_t jerk_serve_stats_get(jerk_server* srv, jerk_serve_stats* out) {
  return guarded([&] {
    require(srv && out, JERK_EINVAL, "server and out must not be NULL");
    jerk::serve_stats(*srv, out);
  });
}

int32_t jerk_serve_inject_failure(jerk_server* srv, int32_t op, int64_t n) {
  return guarded([&] {
    require(srv != nullptr, JERK_EINVAL, "server must not be NULL");
    jerk::serve_inject(*srv, op, n);
  });
}

int32_t jerk_serve_destroy(jerk_server* srv) {
  return guarded([&] {
    if (srv) jerk::serve_destroy(srv);
  });
}

int32_t jerk_search_members(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                            float* d_plane, int64_t ld, int32_t g, int32_t m_begin, int32_t m_end, hipStream_t stream) {
  return guarded([&] {
    require(plan != nullptr, JERK_EINVAL, "plan must not be NULL");
    const jerk::Plan& p = plan->p;
    require(g >= 0 && g < (int32_t)p.groups.size(), JERK_EINVAL, "group index out of range");
    const int32_t n = (int32_t)p.groups[g].members.size();
    require(0 <= m_begin && m_begin <= m_end && m_end <= n, JERK_EINVAL, "member range outside the group");
    if (m_begin == m_end) return;
    require(d_bank && d_spec && d_plane, JERK_EINVAL, "bank, spectrum and plane must not be NULL");
    require(nbins >= 1, JERK_EINVAL, "nbins must be >= 1");
    require(ld >= 2 * nbins && ld % 2 == 0, JERK_EINVAL, "ld must be even and >= 2 * nbins");
    require(reinterpret_cast<uintptr_t>(d_plane) % 8 == 0 && reinterpret_cast<uintptr_t>(d_spec) % 8 == 0,
            JERK_EINVAL, "spectrum and plane must be 8-byte aligned");
    jerk::search_members_enqueue(p, d_bank, d_spec, nbins, d_plane, ld, g, m_begin, m_end, stream);
  });
}

}  // extern "C"
