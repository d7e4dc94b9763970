// Internal declarations shared by the library's translation units.
#pragma once

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/jerk.h"

namespace jerk {

// Error carried to the C ABI boundary, where it becomes a status code.
struct Error : std::runtime_error {
  int32_t status;
  Error(int32_t s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

inline void require(bool ok, int32_t status, const std::string& msg) {
  if (!ok) throw Error(status, msg);
}

#define JERK_HIP_CHECK(expr)                                                              \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::jerk::Error(JERK_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// Per-width-group data. All templates of a group use K = taps (zero-padded
// beyond their own 2 h_t window) and one FFT segment length.
struct Group {
  int32_t taps = 0;        // K_g (multiple of the tap quantum)
  int32_t seg_len = 0;     // S_g
  int32_t ept = 16;        // FFT kernel variant: complex elements per thread (8 or 16)
  int32_t tpb = 8;         // templates per workgroup (FFT path)
  int32_t path = JERK_PATH_FFT_FP32;
  std::vector<int32_t> members;  // template indices, ascending
  int32_t first_member = 0;      // offset in the concatenated member table
  // bank byte offsets
  size_t off_taps = 0;   // complex128 [n][2][taps]
  size_t off_fft = 0;    // complex64 [n][2][seg_len]    (FFT path)
  size_t off_gemm = 0;   // tap fragments                (MFMA paths)
  size_t gemm_bytes = 0;
};

// Host state of batched launches of one plan (staging buffer, capture stream, graph).
struct BatchCtx;
void batch_ctx_free(BatchCtx* c);

struct Plan {
  jerk_plan_desc desc{};
  int32_t n_z = 0, n_w = 0, J = 0, T = 0;
  std::vector<double> zbar, w;
  std::vector<int32_t> half;      // h_t
  std::vector<int32_t> group_of;  // t -> g
  std::vector<int32_t> slot;      // t -> index in group
  std::vector<Group> groups;
  size_t off_members = 0;         // int32 [T] member table (group by group)
  size_t off_tw[4] = {0, 0, 0, 0}; // complex64 exp(-2 pi i k / S), S = 512 << i
  int32_t* pinned_members = nullptr;  // host copy (pinned) uploaded by templates_build
  size_t bank_bytes = 0;
  int32_t max_taps = 0;
  // Gauss-Legendre rule on [-1, 1] used by the template generator.
  double gl_x[16], gl_w[16];
  BatchCtx* batch = nullptr;
};

// plan.cpp
void plan_build(Plan& p, const jerk_plan_desc& d);
void plan_layout(Plan& p);  // recompute bank offsets after a group change
inline int tw_slot(int32_t seg_len) { return seg_len == 512 ? 0 : seg_len == 1024 ? 1 : seg_len == 2048 ? 2 : 3; }
bool seg_len_supported(int32_t s);

// templates.hip
void templates_build(const Plan& p, void* d_bank, hipStream_t stream);
// Member table + twiddle tables + templates_build (what jerk_templates_build enqueues).
void bank_build(Plan& p, void* d_bank, hipStream_t stream);
// FP64 taps [n][2][taps] of templates d_members[0..n) (K = taps, zero outside each template's window).
void taps_launch(const Plan& p, int32_t taps, const int32_t* d_members, int32_t n, double2* out, hipStream_t stream);
// FFT-path spectra [n][2][S] of FP64 taps [n][2][K].
void fft_spectra_launch(const double2* taps, int32_t n, int32_t K, int32_t S, float2* out, hipStream_t stream);
void gen_twiddles(float2* out, int32_t n, hipStream_t stream);
void gemm_bank_build(const Plan& p, const Group& g, const double2* taps, void* out, hipStream_t stream);

// fft_correlate.hip. One FFT-path job: one spectrum, one width group, the
// group's member range [m_begin, m_end), every segment.
struct FftJob {
  const float2* spec;
  int64_t nbins;
  const float2* bank_fft;     // group's spectra, member 0 phase 0
  const int32_t* members;     // group's member list (device)
  int32_t m_begin, m_end;     // members to process
  int32_t t_begin;            // output row of template t is t - t_begin ...
  int32_t row_by_member;      // ... or, when set, mm - row_base for group member mm
  int32_t row_base;
  int32_t taps, tpb;
  float* plane;               // plane rows (row stride ld floats), or null
  int64_t ld;
  uint64_t* row_max;          // peak keys [row][segment] (row stride rmax_ld), or null;
  int64_t rmax_ld;            // rmax_ld == 0: one key per row, combined with atomicMax
  int64_t n_seg;              // set by fft_job_tiles
  int64_t tile_begin;         // first tile of the job in a persistent launch
};
// Header of a persistent launch's work list (device memory).
struct BatchHeader {
  int64_t total_tiles;
  unsigned long long counter;
  int32_t n_jobs;
  int32_t pad;
};
// Candidate selection fused into the FFT path (search_candidates.cpp). Rows are the
// members [lo, hi) of one width group's member list, row r = member lo + r.
struct CandRowStat {
  double mean, sigma, thr;  // thr = mean + k sigma
  int32_t flag;             // the row is recomputed by the exact pass
  int32_t pad;
};
struct CandHit {   // a staged hit of the speculative pass, in its tile's run of slots
  uint32_t code;   // (row - first row of the tile's template block) << 16 | (p - 2 seg U)
  float power;
};
struct CandPoolHit {  // a staged hit beyond its tile's slots
  uint32_t row, p;
  float power;
  uint32_t pad;
};
struct CandArgs {
  // speculative pass (mode 1); tile i = template block * n_seg + segment
  double pre;                     // interior peaks above this level are staged
  double2* part;                  // [rows][n_seg] (sum, sum of squares) of the row's powers in the segment
  float2* edge;                   // [rows][n_seg][2] (P0, P1) at lag 0 and at the segment's last lag
  CandHit* hits;                  // [tiles][cap_tile]
  uint32_t* tile_hits;            // [tiles] hits found (also those beyond cap_tile)
  CandPoolHit* pool;              // hits beyond their tile's slots, pool_count of them (shared, atomic)
  unsigned long long* pool_count;
  int64_t pool_cap;
  int32_t* ovf;                   // [rows] set when a hit of the row found no room in the pool either
  int32_t cap_tile;
  // exact pass (mode 2) and the final list
  const CandRowStat* rs;          // [rows]
  const int32_t* flagged;         // rows to recompute, n_flagged of them
  const uint32_t* n_flagged;
  jerk_candidate* out;
  int64_t capacity;
  unsigned long long* count;
};
// Speculative pass (mode 1) over a group job (plane and row_max null, row_by_member set,
// row_base = m_begin); exact pass (mode 2) over the flagged rows of the same job.
void fft_cand_launch(FftJob j, int32_t seg_len, int32_t ept, const float2* twiddles, const CandArgs& ca, int mode,
                     hipStream_t stream);
// candidates.hip: the steps between and after the FFT passes.
void cand_reset(int32_t* ovf, int32_t rows, uint32_t* n_flagged, unsigned long long* pool_count, hipStream_t stream);
void cand_finish(const double2* part, int32_t rows, int64_t n_seg, int32_t U, int64_t nbins, const int32_t* ovf,
                 double k_sigma, double pre, const int32_t* d_members, int32_t t_begin, double* stats_out,
                 CandRowStat* rs, int32_t* flagged, uint32_t* n_flagged, hipStream_t stream);
void cand_filter(const CandHit* hits, const uint32_t* tile_hits, int32_t tiles, int32_t cap_tile, int32_t n_seg,
                 int32_t tpb, int32_t U, const CandPoolHit* pool, const unsigned long long* pool_count,
                 int64_t pool_cap, const CandRowStat* rs, const int32_t* d_members, jerk_candidate* out,
                 int64_t capacity, unsigned long long* count, hipStream_t stream);
void cand_edges(const float2* edge, int32_t rows, int64_t n_seg, int32_t U, int64_t nbins, const CandRowStat* rs,
                const int32_t* d_members, jerk_candidate* out, int64_t capacity, unsigned long long* count,
                hipStream_t stream);
// (row mean, sigma) of slab rows [rows][2] to out[2 (members[i] - t_begin)]
void scatter_row_stats(const double* stats, int32_t rows, const int32_t* d_members, int32_t t_begin, double* out,
                       hipStream_t stream);
// capi.cpp: rows [m_begin, m_end) of group gi's member list into d_plane (row = member - m_begin)
void search_members_enqueue(const Plan& p, const void* d_bank, const void* d_spec, int64_t nbins, float* d_plane,
                            int64_t ld, int32_t gi, int32_t m_begin, int32_t m_end, hipStream_t stream);
// search_candidates.cpp
size_t search_candidates_workspace_bytes(const Plan& p, int64_t nbins, int32_t t_begin, int32_t t_end, double pre,
                                         int64_t staged);
void search_candidates(const Plan& p, const void* d_bank, const void* d_spec, int64_t nbins, int32_t t_begin,
                       int32_t t_end, double k_sigma, double pre, double* d_stats, jerk_candidate* d_out,
                       int64_t capacity, unsigned long long* d_count, int64_t staged, void* d_ws, size_t ws_bytes,
                       hipStream_t stream);

// Sets j.n_seg and returns the job's tile count (segments x template blocks).
int64_t fft_job_tiles(FftJob& j, int32_t seg_len);
// twiddles: exp(-2 pi i k / seg_len), k < seg_len (complex64, device).
// ept: complex elements per thread of the kernel variant (8 or 16).
bool fft_variant_supported(int32_t seg_len, int32_t ept);
void fft_correlate_launch(FftJob j, int32_t seg_len, int32_t ept, const float2* twiddles, hipStream_t stream);
// keys: the jobs write peak keys (every job's row_max set) - selects the kernel instantiation.
// One flat launch over a job table: grid = total tiles, workgroup i takes tile i.
void fft_multi_launch(const FftJob* d_jobs, const BatchHeader* d_hdr, int64_t total, int32_t seg_len, int32_t ept,
                      bool keys, const float2* twiddles, hipStream_t stream);
// Up to kFftArgJobs jobs of one kernel variant in one flat launch, the job table in the kernel
// arguments (no device buffer): every job's keys flag must match `keys`.
constexpr int kFftArgJobs = 8;
void fft_args_launch(FftJob* jobs, int n, int32_t seg_len, int32_t ept, bool keys, const float2* twiddles,
                     hipStream_t stream);
void fft_persistent_launch(const FftJob* d_jobs, BatchHeader* d_hdr, int32_t seg_len, int32_t ept, bool keys,
                           const float2* twiddles, int32_t grid, hipStream_t stream);
// Workgroups of the persistent kernel that fit on the current device at once.
int32_t fft_persistent_grid(int32_t seg_len, int32_t ept);

// gemm_correlate.hip
struct GemmArgs {
  const float2* spec;
  int64_t nbins;
  const void* bank_gemm;      // group's fragments
  const int32_t* members;
  int32_t m_begin, m_end;     // m_begin a multiple of 8 (a fragment row block)
  int32_t t_begin, t_end;     // only templates in [t_begin, t_end) are written
  float* plane;
  int64_t ld;
  int32_t taps;
  int32_t path;               // JERK_PATH_GEMM_SPLIT_BF16 or JERK_PATH_GEMM_FP16
  uint64_t* row_max;          // one peak key per row (atomicMax), or null; plane may then be null
  int32_t row_by_member;      // output row is (member index - row_base) instead of t - t_begin
  int32_t row_base;
};
void gemm_correlate_launch(const GemmArgs& a, hipStream_t stream);
size_t gemm_bank_bytes(int32_t n_members, int32_t taps, int32_t path);

// batch.cpp
size_t batch_workspace_bytes(const Plan& p, int32_t count);
int64_t batch_keys_per_row(const Plan& p, int64_t nbins);
void batch_search(Plan& p, const void* d_bank, const jerk_batch_item* items, int32_t count, int32_t t_begin,
                  int32_t t_end, void* d_ws, size_t ws_bytes, uint32_t flags, hipStream_t stream);

// tune.cpp
size_t autotune_scratch_bytes(const Plan& p, int64_t nbins);
void autotune(Plan& p, const void* d_spec, int64_t nbins, void* d_scratch, size_t scratch_bytes, uint32_t flags,
              hipStream_t stream);

// serve.cpp
void serve_create(const jerk_serve_desc& d, void* d_arena, size_t arena_bytes, jerk_server** out);
void serve_submit(jerk_server& s, const jerk_request& r, uint64_t* ticket);
int32_t serve_poll(jerk_server& s, uint64_t ticket, jerk_result* out, double timeout_s);
void serve_stats(jerk_server& s, jerk_serve_stats* out);
void serve_inject(jerk_server& s, int32_t op, int64_t n);
void serve_destroy(jerk_server* s);

// reduce.hip
// harmonics.hip
struct HarmonicShape {
  int32_t i0 = 0, n_zf = 0, n_wf = 0;
  int64_t n_pf = 0;
};
HarmonicShape harmonic_shape(const Plan& p, int64_t n_r, int32_t n_harm);
void harmonic_sum(const Plan& p, const float* plane, int64_t ld, int64_t n_r, int32_t n_harm, float* out,
                  int64_t out_ld, hipStream_t stream);
size_t spectrum_workspace_bytes(int64_t n_samples);
void spectrum_prepare(const float* series, int64_t n_samples, float2* spec, void* ws, size_t ws_bytes,
                      hipStream_t stream);
size_t stats_workspace_bytes(int32_t rows, int64_t n_r);
void plane_stats(const float* plane, int64_t ld, int32_t rows, int64_t n_r, double* stats, void* ws,
                 size_t ws_bytes, hipStream_t stream);
void find_candidates(const float* plane, int64_t ld, int32_t rows, int64_t n_r, const double* stats,
                     double k_sigma, const int32_t* row_template, int32_t t_base, jerk_candidate* out,
                     int64_t capacity, unsigned long long* count, hipStream_t stream);
void peaks_reduce(const uint64_t* keys, int32_t rows, int64_t per_row, int64_t ld, jerk_peak* out,
                  hipStream_t stream);

// Error-reporting state of the C ABI.
void set_last_error(const std::string& msg);

}  // namespace jerk

struct jerk_plan {
  jerk::Plan p;
};
