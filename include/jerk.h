/*
 * jerk.h - C ABI of the MI355X (gfx950) Fourier-domain "jerk" search matched filter.
 *
 * The library correlates a complex spectrum with a bank of response templates,
 * one per (zbar, w) pair of a lattice, and writes the (r, z, w) power plane
 * (Adamek, Novotny, Dimoudi, Armour, arXiv:1911.01353, section
 * "Implementation": each filter fits the Fourier response for a given first
 * frequency derivative z = fdot T^2 and second frequency derivative
 * w = fddot T^3; Figure 1: the correlation is evaluated by overlap-and-save).
 *
 * Definitions used by every entry point
 * -------------------------------------
 *  Spectrum      X[k], k = 0..nbins-1, complex64 interleaved (re, im) float pairs,
 *                in device memory. X[k] is taken as 0 outside [0, nbins).
 *  Lattice       zbar_i = -zmax + i dz, i < n_z = floor(2 zmax / dz) + 1;
 *                w_j = (j - J) dw, j < n_w = 2J + 1, J = floor(wmax / dw);
 *                template t = j * n_z + i (w-major).
 *  Response      T(qbar; zbar, w) = R(qbar - zbar/2 + w/12; zbar - w/2, w),
 *                R(q; z, w) = integral_0^1 exp(2 pi i (q u + z u^2/2 + w u^3/6)) du
 *                (zbar, rbar are observation averages of fdot and frequency).
 *  Half-width    h_t = ceil(|zbar|/2 + |w|/12) + margin_bins; 2 h_t taps.
 *  Plane         for p = 2 k0 + phase (r = p / 2), p in [0, 2 nbins):
 *                P[t][p] = | sum_{k=k0-h_t+1}^{k0+h_t} X[k] conj(T(k0 + phase/2 - k)) |^2
 *                stored as float32, row t at plane + (t - t_begin) * ld.
 *
 * Conventions
 * -----------
 *  - Every function returns an int32 status: JERK_OK (0) or a negative code.
 *    Arguments are checked before any work is queued; on error nothing is queued
 *    and jerk_last_error() (per thread) describes the problem.
 *  - The caller owns all device memory and streams. The library never allocates
 *    device memory on the search path; it states the sizes it needs
 *    (jerk_plan_info) and works in caller buffers. Work is queued on the caller's
 *    stream and returns before it completes; buffers must stay valid until the
 *    stream work ends. Device faults surface at the caller's next synchronisation.
 *  - Plan and server objects are opaque host handles, freed by *_destroy.
 */
#ifndef JERK_H
#define JERK_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define JERK_OK 0
#define JERK_EINVAL (-1)       /* an argument is invalid                         */
#define JERK_ENOMEM (-2)       /* a caller buffer is too small / never fits      */
#define JERK_EAGAIN (-3)       /* queue full, retry later                        */
#define JERK_EPENDING (-4)     /* request not finished yet                       */
#define JERK_EHIP (-5)         /* a HIP runtime call failed                      */
#define JERK_EUNSUPPORTED (-6) /* valid but not supported by this build          */
#define JERK_EINTERNAL (-7)    /* library bug                                    */
#define JERK_ECANCELED (-8)    /* request dropped (server destroyed before it ran) */

/* ---- correlation paths ------------------------------------------------- */
#define JERK_PATH_FFT_FP32 0       /* fused overlap-save FFT, FP32                  */
#define JERK_PATH_GEMM_SPLIT_BF16 1 /* direct correlation on MFMA, split-BF16 hi+lo  */
#define JERK_PATH_GEMM_FP16 2      /* direct correlation on MFMA, FP16              */
#define JERK_PATH_AUTO 3           /* per width group: the faster of FFT / split-BF16 */

/* Human-readable name of a status code (static string). */
const char* jerk_status_str(int32_t status);
/* Last error message of the calling thread (valid until its next library call). */
const char* jerk_last_error(void);
/* Library version string, e.g. "jerk-mi355x 1.0 gfx950". */
const char* jerk_version(void);
/* State of the work queued on `stream` so far, without blocking: JERK_OK when it has all
 * finished without error, JERK_EPENDING while some of it still runs, JERK_EHIP (text in
 * jerk_last_error) when the device reported an error. Asynchronous kernel faults of the other
 * entry points surface here or at the caller's next synchronisation. */
int32_t jerk_stream_check(hipStream_t stream);

/* ---- plans -------------------------------------------------------------- */
typedef struct jerk_plan jerk_plan;

typedef struct jerk_plan_desc {
  int64_t nbins;               /* spectrum length the plan is sized for, >= 1          */
  double zmax, wmax;           /* lattice extents (>= 0)                               */
  double dz, dw;               /* lattice steps (> 0; dw may be 0 only if wmax == 0)   */
  int32_t numbetween;          /* outputs per bin: must be 2 (half-bin r spacing)      */
  int32_t margin_bins;         /* half-width margin M (0..256), usually 16             */
  int32_t path;                /* JERK_PATH_*                                          */
  int32_t seg_len;             /* FFT segment length (512, 1024, 2048, 4096) or 0       */
  int32_t templates_per_block; /* FFT path templates per workgroup (1..64), or 0: per group the
                                  largest of 64, 32, 16, 8 whose launch over the whole group
                                  has 4096 workgroups at nbins, else 4                      */
  int32_t tap_quantum;         /* width-group granularity in taps (16..512, mult of 16) or 0 */
  uint32_t flags;              /* reserved, must be 0                                  */
} jerk_plan_desc;

typedef struct jerk_plan_info_t {
  int32_t n_z, n_w, n_templates, n_groups;
  int64_t nbins;          /* as in the descriptor                                    */
  int64_t n_r;            /* outputs per row = 2 * nbins                              */
  int32_t max_taps;       /* largest 2 h_t                                            */
  int32_t path;           /* path of the descriptor                                  */
  size_t bank_bytes;      /* device bytes of the template bank                       */
  size_t workspace_bytes; /* device workspace jerk_search needs (may be 0)           */
  size_t plane_row_bytes; /* 4 * n_r                                                 */
  size_t taps_offset;     /* byte offset in the bank of the FP64 taps (see group info) */
} jerk_plan_info_t;

typedef struct jerk_group_info_t {
  int32_t taps;                /* K_g: taps of every template of the group (even)        */
  int32_t seg_len;             /* FFT segment length S_g                                */
  int32_t templates_per_block; /* FFT path templates per workgroup                      */
  int32_t path;                /* resolved path (FFT_FP32, GEMM_SPLIT_BF16 or GEMM_FP16) */
  int32_t n_members;           /* templates in the group                                */
  int32_t first_member;        /* index of its first entry in jerk_plan_members order   */
  int32_t fft_ept;             /* FFT kernel variant: complex elements per thread (8 or 16) */
  int32_t reserved;
  size_t taps_offset;          /* bank byte offset of the group's FP64 taps:
                                  complex128 [n_members][2 phases][taps], tap j multiplies
                                  bin k0 - taps/2 + 1 + j; taps outside the template's own
                                  2 h_t window are 0                                     */
} jerk_group_info_t;

/* Builds the lattice, half-widths, width groups and bank layout. Host only.
 * EINVAL for an invalid descriptor (non-positive steps, numbetween != 2, ...). */
int32_t jerk_plan_create(const jerk_plan_desc* desc, jerk_plan** out);
int32_t jerk_plan_destroy(jerk_plan* plan);
int32_t jerk_plan_info(const jerk_plan* plan, jerk_plan_info_t* out);
int32_t jerk_plan_group(const jerk_plan* plan, int32_t g, jerk_group_info_t* out);
/* Parameters of template t: zbar, w, half-width h_t, width group and slot in it. */
int32_t jerk_plan_template(const jerk_plan* plan, int32_t t, double* zbar, double* w,
                           int32_t* half_width, int32_t* group, int32_t* slot);
/* Template indices of all groups, group by group (n_templates int32, host memory). */
int32_t jerk_plan_members(const jerk_plan* plan, int32_t* out, int32_t count);
/* Overrides one group's FFT segment length, templates per block, path and FFT kernel variant
 * (fft_ept: complex elements per thread, 8 or 16; 0 = default) before jerk_templates_build
 * (used by the autotuner). Changes bank_bytes; EINVAL if out of range. */
int32_t jerk_plan_set_group(jerk_plan* plan, int32_t g, int32_t seg_len,
                            int32_t templates_per_block, int32_t path, int32_t fft_ept);

/* ---- autotuner -------------------------------------------------------------- */
#define JERK_TUNE_UNIFORM 1u /* one FFT segment length for all groups (for jerk_batch_search) */

/* Device scratch bytes jerk_plan_autotune needs for a probe spectrum of nbins bins. */
size_t jerk_autotune_scratch_bytes(const jerk_plan* plan, int64_t nbins);
/* For every width group, times the candidate kernels on up to 64 of the group's templates over
 * the first min(nbins, 2^22) bins of d_spec (a probe plane of up to 2 GiB in d_scratch, larger
 * than the device's caches, so the ranking holds for full-size searches): the FFT path with
 * segment lengths 512..4096 (at least twice the group width) and 8, 16, 32 or 64 templates
 * per workgroup (also 4 for groups whose whole launch would give fewer than 4 waves per SIMD),
 * and for JERK_PATH_AUTO plans also the split-BF16 MFMA path. Keeps the fastest per output
 * point (JERK_TUNE_UNIFORM: FFT only, one segment length minimising the estimated total). Call
 * before jerk_templates_build; bank_bytes may change. Synchronous (waits on stream). Choices
 * are cached per process by (device, group width and size, bins, probe size, candidate set).
 * Plans with a fixed MFMA path are left unchanged. */
int32_t jerk_plan_autotune(jerk_plan* plan, const void* d_spec, int64_t nbins, void* d_scratch,
                           size_t scratch_bytes, uint32_t flags, hipStream_t stream);

/* ---- template bank (FP64 generation on the GPU) -------------------------- */
/* Generates every template's taps in FP64 by composite Gauss-Legendre quadrature of R
 * (16 nodes per panel, at most one phase cycle per panel) and derives the bank of each
 * group's path: FP32 segment spectra for the FFT path, BF16 hi/lo or FP16 tap
 * fragments for the MFMA path. d_bank: device buffer of at least bank_bytes.
 * Asynchronous on stream. ENOMEM if bank_bytes is too small. */
int32_t jerk_templates_build(jerk_plan* plan, void* d_bank, size_t bank_bytes, hipStream_t stream);

/* ---- search ----------------------------------------------------------------- */
/* Writes plane rows [t_begin, t_end) (all 2 nbins outputs each) of the spectrum d_spec
 * (nbins complex64 values, any nbins >= 1) into d_plane, row t at d_plane + (t - t_begin) * ld,
 * ld >= 2 nbins floats. Uses the bank built by jerk_templates_build for this plan.
 * d_ws: workspace of at least workspace_bytes (may be NULL when that is 0).
 * Asynchronous on stream. EINVAL for a bad range or stride. An empty range (t_begin == t_end)
 * queues nothing and ignores the pointers. */
int32_t jerk_search(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                    float* d_plane, int64_t ld, int32_t t_begin, int32_t t_end, void* d_ws,
                    size_t ws_bytes, hipStream_t stream);

/* As jerk_search, restricted to the templates of width group g (one kernel launch). Lets a
 * caller time or schedule the groups separately; the union over all groups equals jerk_search. */
int32_t jerk_search_group(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                          float* d_plane, int64_t ld, int32_t t_begin, int32_t t_end, int32_t g,
                          hipStream_t stream);

/* As jerk_search_group for members [m_begin, m_end) of group g's member list (jerk_plan_members
 * order), with output row (member - m_begin): d_plane + (member - m_begin) * ld. Lets a caller cut
 * the plane into slabs of whole width groups, so every launch works on full template blocks. */
int32_t jerk_search_members(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                            float* d_plane, int64_t ld, int32_t g, int32_t m_begin, int32_t m_end,
                            hipStream_t stream);

/* ---- batched search: many spectra, one persistent launch -------------------- */
typedef struct jerk_batch_item {
  const void* spec;  /* device complex64 spectrum [nbins]                                 */
  int64_t nbins;     /* >= 1; items may have different lengths                          */
  float* plane;      /* device plane rows [t_begin, t_end) x 2 nbins (row stride ld), or NULL */
  int64_t ld;        /* even, >= 2 nbins when plane is set                              */
  uint64_t* peaks;   /* device peak keys [t_end - t_begin][keys_ld], or NULL (see below); either
                        every item of a batch has one or none has                          */
  int64_t keys_ld;   /* >= jerk_batch_keys_per_row(plan, nbins) when peaks is set. Every
                        key of a searched row [0, keys_ld) is written (keys past a width
                        group's own segment count are set to 0), so the buffer needs no
                        clearing between calls                                          */
} jerk_batch_item;

#define JERK_BATCH_GRAPH 1u      /* capture the launch in a hipGraph on first use and replay it     */
#define JERK_BATCH_FLAT 2u       /* one flat launch: a workgroup per tile, the hardware dispatcher
                                    balancing the load (the default; the flag only states it)      */
#define JERK_BATCH_PERSISTENT 4u /* one persistent launch instead: a full-device grid whose
                                    workgroups take tiles from a device counter until none is left;
                                    same results bit for bit, slower (its tile loop costs registers
                                    and so waves per SIMD)                                         */

/* Workspace bytes jerk_batch_search needs for up to `count` items. */
size_t jerk_batch_workspace_bytes(const jerk_plan* plan, int32_t count);
/* Peak keys written per plane row for a spectrum of nbins bins (one per FFT segment). A key
 * is (float bits of the power << 32) | (0xFFFFFFFF - p): the largest key of a row is its
 * peak power, ties going to the lowest r index p (jerk_peaks_reduce turns keys into peaks). */
int64_t jerk_batch_keys_per_row(const jerk_plan* plan, int64_t nbins);
/* Searches rows [t_begin, t_end) of every item in ONE kernel launch over a job table of
 * (spectrum, width group, template block, segment) tiles: by default a flat launch (one
 * workgroup per tile), with JERK_BATCH_PERSISTENT a persistent kernel whose workgroups take
 * tiles from a device counter until all are done. All width groups must be on the FFT path
 * with one segment length.
 * Results equal jerk_search's bit for bit. With JERK_BATCH_GRAPH the launch is captured in
 * a hipGraph the first time (per plan, workspace and device) and replayed afterwards; the
 * job table is rewritten before every replay. Overlapping calls on one plan serialise on
 * its staging buffer. Asynchronous on stream. */
int32_t jerk_batch_search(jerk_plan* plan, const void* d_bank, const jerk_batch_item* items, int32_t count,
                          int32_t t_begin, int32_t t_end, void* d_ws, size_t ws_bytes, uint32_t flags,
                          hipStream_t stream);

/* Peak of one plane row: its largest power and that power's plane index p (r = p / 2). */
typedef struct jerk_peak {
  float power;
  uint32_t p;
} jerk_peak;

/* Per-row peaks of rows [t_begin, t_end) without writing the plane: d_out[t - t_begin] holds the
 * largest power of row t and its plane index p (the lowest p among equal powers), what a row
 * argmax of jerk_search's plane gives, on any path (the FFT and MFMA epilogues keep one key per
 * row). d_ws: device workspace of jerk_search_peaks_workspace_bytes bytes (8 per row), 8-byte
 * aligned. Enqueues kernels only (no memset), so the call may be captured in a graph.
 * EINVAL for a bad range, nbins outside [1, 2^31), NULL or misaligned pointers; ENOMEM for a
 * short workspace. Asynchronous on stream. */
size_t jerk_search_peaks_workspace_bytes(const jerk_plan* plan, int32_t t_begin, int32_t t_end);
int32_t jerk_search_peaks(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                          int32_t t_begin, int32_t t_end, jerk_peak* d_out, void* d_ws, size_t ws_bytes,
                          hipStream_t stream);

/* For callers that cannot allocate device memory (code under graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): jerk_search_peaks with its key workspace in a
 * fixed library-owned device array of JERK_NOALLOC_MAX_ROWS keys (8 bytes each, 256 KiB on
 * every GPU the library runs on, held until the process ends) instead of a caller buffer.
 * Allocates nothing: no hipMalloc, hipFree or allocating library call; the first call on a
 * device looks up that device's copy of the array. The keys are cleared by a kernel at the
 * start of every call. Results equal jerk_search_peaks's bit for bit. EINVAL when
 * t_end - t_begin exceeds JERK_NOALLOC_MAX_ROWS (split the range into several calls), and
 * as jerk_search_peaks otherwise. Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads) race, and the caller must serialise them.
 * Asynchronous on stream. */
#define JERK_NOALLOC_MAX_ROWS 32768
int32_t jerk_search_peaks_noalloc(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                                  int32_t t_begin, int32_t t_end, jerk_peak* d_out, hipStream_t stream);

/* Reduces peak keys [rows][keys_ld] (first keys_per_row of each row) to one jerk_peak per row.
 * Rows whose keys were all left 0 report power 0 and p = 0xFFFFFFFF. Asynchronous on stream. */
int32_t jerk_peaks_reduce(const uint64_t* d_keys, int32_t rows, int64_t keys_per_row, int64_t keys_ld,
                          jerk_peak* d_out, hipStream_t stream);

/* ---- harmonic summing ------------------------------------------------------------
 * The stage after matched filtering (paper, section "Results": the harmonic sum improves
 * the sensitivity of Fourier searches and costs at least as much as the filtering; the
 * paper gives no definition). The h-th harmonic of a signal with fundamental (r, zbar, w)
 * lies at (h r, h zbar, h w); with zmax a multiple of dz every harmonic of a lattice point
 * is a lattice point, and S_H(r, zbar, w) = sum_{h=1}^{H} P(h r, h zbar, h w) (FP32 sum,
 * h ascending). Fundamentals are kept when all H harmonics lie on the plane:
 * |zbar| <= floor(zmax / dz / H) dz, |w| <= floor(J / H) dw and H p <= n_r - 1. */

/* Shape of S_H for a plane of n_r points per row: n_zf x n_wf fundamental templates (rows
 * ordered like the plan's lattice, w-major, zbar and w centred on 0) of n_pf points each.
 * EUNSUPPORTED when zmax is not a multiple of dz; EINVAL unless 1 <= n_harm <= 64, n_r >= 1. */
int32_t jerk_harmonic_shape(const jerk_plan* plan, int64_t n_r, int32_t n_harm, int32_t* n_zf, int32_t* n_wf,
                            int64_t* n_pf);
/* S_H of a full plane d_plane (device; every template of the plan, row t at t * ld, n_r
 * points per row, e.g. jerk_search over [0, T)) into d_out (device; row f at f * out_ld,
 * n_pf points). EINVAL for NULL pointers, ld < n_r or out_ld < n_pf. Asynchronous on stream. */
int32_t jerk_harmonic_sum(const jerk_plan* plan, const float* d_plane, int64_t ld, int64_t n_r, int32_t n_harm,
                          float* d_out, int64_t out_ld, hipStream_t stream);

/* ---- spectrum preparation --------------------------------------------------------
 * The search's input from a real time series (paper, section "Introduction": periodicity
 * searches work on the Fourier transform of the series), in FP64 on the device: the DFT
 * X[k] = sum_j x[j] exp(-2 pi i j k / N) of the N float32 samples, bins 0 .. N/2 - 1 kept
 * (Nyquist dropped), X[0] set to 0, scaled by 1 / sqrt(mean over 1 <= k < N/2 of |X[k]|^2)
 * (no scaling when that mean is 0), rounded once to complex64. */

/* Device workspace bytes jerk_spectrum_prepare needs for n_samples samples (0 if invalid). */
size_t jerk_spectrum_workspace_bytes(int64_t n_samples);
/* d_series: n_samples float32 samples (device, 8-byte aligned); n_samples a power of two,
 * 4 <= n_samples <= 2^30. d_spec: n_samples / 2 complex64 bins (device, interleaved re, im).
 * d_ws: caller device workspace of jerk_spectrum_workspace_bytes(n_samples) bytes.
 * EINVAL for a NULL or misaligned pointer, EUNSUPPORTED for a length that is not a power of
 * two, ENOMEM for a short workspace. Asynchronous on stream. */
int32_t jerk_spectrum_prepare(const float* d_series, int64_t n_samples, void* d_spec, void* d_ws,
                              size_t ws_bytes, hipStream_t stream);

/* ---- candidate selection ------------------------------------------------------
 * Paper, section "Results": the timed search includes the mean and standard deviation of
 * the plane and a peak finder that keeps only peaks above a user threshold. Both work on
 * plane slabs already in device memory: rows of n_r float powers with row stride ld. */

/* A candidate: template t, plane index p (r = p / 2), its power and significance
 * (power - mean) / sigma of its row. */
typedef struct jerk_candidate {
  uint32_t t;
  uint32_t p;
  float power;
  float sigma;
} jerk_candidate;

/* Device workspace bytes jerk_plane_stats needs for `rows` rows of n_r points (0 if empty). */
size_t jerk_stats_workspace_bytes(int32_t rows, int64_t n_r);
/* Per-row population mean and standard deviation (divisor n_r) of a plane slab, accumulated in
 * FP64, into d_stats[rows][2] = {mean, sigma} (device). One read of the slab; the result does
 * not depend on scheduling, and a constant row gets sigma = 0 exactly. d_ws: caller device
 * workspace of jerk_stats_workspace_bytes(rows, n_r) bytes. rows = 0 or n_r = 0 is a no-op.
 * EINVAL for a NULL pointer or ld < n_r; ENOMEM for a short workspace. Asynchronous on stream. */
int32_t jerk_plane_stats(const float* d_plane, int64_t ld, int32_t rows, int64_t n_r, double* d_stats,
                         void* d_ws, size_t ws_bytes, hipStream_t stream);
/* Appends the candidates of a plane slab to d_out: points whose power, widened to FP64, is
 * strictly above mean + k_sigma * sigma of its row (d_stats as written by jerk_plane_stats)
 * and that are peaks along r: strictly greater than the left neighbour and not less than the
 * right one, the row's ends having no neighbour on that side. Row i is template
 * d_row_template[i] (device int32 array) or, when that is NULL, t_base + i. *d_count (device)
 * is incremented by the number of candidates found; a candidate whose slot index is
 * >= capacity is counted but not stored, so several slabs can share one list and a count
 * above capacity reports overflow. The caller clears *d_count before the first slab. The
 * order of the list is unspecified. n_r must be < 2^32. EINVAL for a NULL pointer, ld < n_r
 * or a non-finite k_sigma. Asynchronous on stream. */
int32_t jerk_find_candidates(const float* d_plane, int64_t ld, int32_t rows, int64_t n_r, const double* d_stats,
                             double k_sigma, const int32_t* d_row_template, int32_t t_base,
                             jerk_candidate* d_out, int64_t capacity, unsigned long long* d_count,
                             hipStream_t stream);

/* ---- search with candidate selection, no plane ---------------------------------
 * The matched filter of jerk_search and the selection of jerk_plane_stats +
 * jerk_find_candidates in one call that never writes the plane (the paper times the
 * filter together with this selection, section "Results"). Rows [t_begin, t_end).
 * Width groups on an MFMA path (no FFT bank) go through plane slabs of at most 2^30 bytes
 * inside the workspace: search, jerk_plane_stats, jerk_find_candidates. The rest:
 *
 * The threshold mean + k_sigma * sigma of a row is known only after the whole row, so the
 * call runs per width group: a speculative pass that accumulates each row's sum and sum
 * of squares (FP64) and stages the peaks above pre_level in a run of slots per tile
 * (tile = FFT segment x template block), a tile's excess going to a shared pool of half
 * the slots; row statistics; the staged peaks above their row's threshold; the points at
 * segment ends; and an exact pass that recomputes the rows whose threshold lies below
 * pre_level or that lost a staged peak to a full pool.
 * The candidates are therefore the same for any pre_level and `staged`; those two only
 * set the cost. A good pre_level sits a little below the lowest row threshold expected:
 * for a spectrum normalised to unit mean power the noise powers are close to exponential
 * with mean and sigma near 1, so thresholds lie near 1 + k_sigma and e.g.
 * 0.9 (1 + k_sigma) leaves the exact pass idle.
 *
 * staged: slots per tile; 0 = 2 exp(-pre_level) of the tile's points + 16 (the expected
 * share above pre_level on a unit-mean-power spectrum is exp(-pre_level)) and 2^16 more
 * pool entries.
 * d_stats: (mean, sigma) of row t at d_stats[2 (t - t_begin)] (device, FP64), or NULL.
 * Candidates are appended to d_out as by jerk_find_candidates (t = template index, count
 * in *d_count, which the caller clears first; order unspecified; capacity overflow counted).
 * EINVAL for a bad range, nbins outside [1, 2^31), non-finite k_sigma or pre_level, a
 * negative staged or capacity, or NULL pointers; ENOMEM for a workspace smaller than
 * jerk_search_candidates_workspace_bytes (0 for invalid arguments). Asynchronous on stream. */
size_t jerk_search_candidates_workspace_bytes(const jerk_plan* plan, int64_t nbins, int32_t t_begin, int32_t t_end,
                                              double pre_level, int64_t staged);
int32_t jerk_search_candidates(const jerk_plan* plan, const void* d_bank, const void* d_spec, int64_t nbins,
                               int32_t t_begin, int32_t t_end, double k_sigma, double pre_level, int64_t staged,
                               double* d_stats, jerk_candidate* d_out, int64_t capacity,
                               unsigned long long* d_count, void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Many spectra (e.g. de-dispersion trials) through jerk_search_candidates in one call, one after
 * the other on the stream, sharing one workspace; each item has its own candidate list. Every item
 * is checked before anything is queued. d_ws: at least jerk_batch_search_candidates_workspace_bytes
 * (the largest single-search workspace over the items). Asynchronous on stream. */
typedef struct jerk_batch_cand_item {
  const void* spec;            /* device complex64 spectrum [nbins]                               */
  int64_t nbins;               /* in [1, 2^31)                                                    */
  jerk_candidate* out;         /* device candidate list of this spectrum                          */
  int64_t capacity;            /* records out holds                                               */
  unsigned long long* count;   /* device count of this spectrum's candidates; cleared by the caller */
  double* stats;               /* device (mean, sigma) per row [t_end - t_begin][2], or NULL       */
} jerk_batch_cand_item;

size_t jerk_batch_search_candidates_workspace_bytes(const jerk_plan* plan, const jerk_batch_cand_item* items,
                                                    int32_t count, int32_t t_begin, int32_t t_end, double pre_level,
                                                    int64_t staged);
int32_t jerk_batch_search_candidates(const jerk_plan* plan, const void* d_bank, const jerk_batch_cand_item* items,
                                     int32_t count, int32_t t_begin, int32_t t_end, double k_sigma, double pre_level,
                                     int64_t staged, void* d_ws, size_t ws_bytes, hipStream_t stream);

/* ---- serving: continuous batching of search requests ----------------------- */
typedef struct jerk_server jerk_server;

#define JERK_SERVE_DRYRUN 1u /* host-only scheduler test mode: no device calls, tiles finish at once */

typedef struct jerk_serve_desc {
  int32_t max_active;       /* requests admitted to the device at once (>= 1)                      */
  int32_t queue_capacity;   /* submitted, not yet admitted (>= 1); submit returns EAGAIN when full */
  int64_t tiles_per_launch; /* scheduling quantum: FFT tiles per launch over all requests (0 = auto) */
  int32_t seg_len;          /* FFT segment length of serving plans (0 = per-group default)          */
  int32_t slots;            /* launches in flight at once, each on its own stream (1..8, 0 = 3)     */
  uint32_t flags;           /* JERK_SERVE_* */
  int32_t reserved;
} jerk_serve_desc;

/* One entry of a request's global top-k: the k templates whose row peaks are strongest, in
 * descending power (ties to the lower t), each with its row peak's plane index p (r = p / 2).
 * One entry per template, so k strong templates are reported rather than k neighbouring points
 * of one peak. */
typedef struct jerk_top {
  int32_t t;
  uint32_t p;
  float power;
  int32_t reserved;
} jerk_top;

typedef struct jerk_request {
  const void* spec;        /* device complex64 spectrum [nbins]; caller-owned, valid until done  */
  int64_t nbins;
  double zmax, wmax, dz, dw; /* lattice (margin 16 bins, two outputs per bin)                   */
  int32_t path;            /* JERK_PATH_FFT_FP32 or JERK_PATH_GEMM_SPLIT_BF16                     */
  int32_t peaks_capacity;  /* entries of `peaks`                                                  */
  float* plane;            /* optional device buffer for the plane, rows t x 2 nbins at stride ld */
  int64_t ld;
  jerk_peak* peaks;        /* optional host array: per-template peaks, filled on completion       */
  jerk_top* top;           /* optional host array: the request's global top-k, filled on completion */
  int32_t top_capacity;    /* k: entries of `top` (0 with top = NULL)                             */
  int32_t reserved;
} jerk_request;

typedef struct jerk_result {
  int32_t status;          /* JERK_OK or the error that ended the request                        */
  int32_t n_templates;
  float best_power;        /* global peak: largest power, ties to the lowest (t, p)              */
  int32_t best_t;
  uint32_t best_p;         /* r index of the peak (r = p / 2)                                    */
  int32_t top_count;       /* entries written to the request's `top` array                       */
  uint64_t points;         /* plane points searched (2 nbins x n_templates)                      */
  double t_submit, t_admit, t_first_launch, t_done; /* seconds on the server's steady clock    */
} jerk_result;

typedef struct jerk_serve_stats {
  uint64_t submitted, completed, failed, launches, bank_builds, bank_evictions;
  int32_t queued, active;
  size_t arena_used, arena_bytes;
  uint64_t shared_launches;  /* launches that carried work units of two or more requests           */
  int32_t max_in_flight;     /* most requests with work on the device at one time                  */
  int32_t reserved;
} jerk_serve_stats;

/* Creates a server whose scheduler thread runs requests on the current device. d_arena
 * (caller device memory, 256-byte aligned) holds the template-bank cache, per-request
 * peak buffers and launch tables; requests are admitted while their footprint fits. */
int32_t jerk_serve_create(const jerk_serve_desc* desc, void* d_arena, size_t arena_bytes, jerk_server** out);
/* Queues a request without blocking. EAGAIN: queue full; ENOMEM: can never fit the arena;
 * EINVAL: bad request. Requests that arrive while others run are admitted as slots and
 * arena memory free up; their tiles are interleaved with the running requests' tiles in the
 * same launches (round-robin), and each result is independent of the mix. */
int32_t jerk_serve_submit(jerk_server* srv, const jerk_request* req, uint64_t* ticket);
/* EPENDING until the request is done, then JERK_OK with *out filled (out->status says how it ended). */
int32_t jerk_serve_poll(jerk_server* srv, uint64_t ticket, jerk_result* out);
/* As poll, blocking up to timeout_s seconds (< 0: no limit). */
int32_t jerk_serve_wait(jerk_server* srv, uint64_t ticket, jerk_result* out, double timeout_s);
int32_t jerk_serve_stats_get(jerk_server* srv, jerk_serve_stats* out);
/* Test hooks: op 1 fails the n-th launch from now (counting from 1), op 2 the n-th bank build;
 * the requests involved end with JERK_EHIP and the others continue; n = 0 disarms. op 3 holds
 * admission while n != 0 (queued requests stay queued) and releases it with n = 0. op 4 makes
 * the next n completion queries of launch slots report a device error, as a sticky device
 * fault would (n = 0 disarms): every request with work in flight then ends with JERK_EHIP, the
 * slots are released and the server keeps running (later requests are served once the error
 * clears). */
int32_t jerk_serve_inject_failure(jerk_server* srv, int32_t op, int64_t n);
/* Stops the scheduler after the work on the device finishes; queued requests end JERK_ECANCELED. */
int32_t jerk_serve_destroy(jerk_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* JERK_H */
