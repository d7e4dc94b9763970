/*
 * A plain C caller of the library (no Python, no torch): a plan, the template bank, the plane
 * search and the search with fused candidate selection, in device buffers and a stream of its
 * own. Reads a complex64 spectrum from a file; writes the FP32 plane and the candidate records.
 *
 *   jerk_demo SPECTRUM NBINS ZMAX WMAX PLANE_OUT CANDIDATES_OUT
 *
 * Lattice steps dz = 2, dw = 20, FFT path; candidates at k = 3 sigma with the speculative level
 * 0.9 (1 + k). Output files: PLANE_OUT = float32 [T][2 NBINS]; CANDIDATES_OUT = int64 count,
 * then that many jerk_candidate records. Exit status 0 on success.
 */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "jerk.h"

#define CHECK_HIP(x)                                                     \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) {                                              \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
      return 2;                                                          \
    }                                                                    \
  } while (0)
#define CHECK_JERK(x)                                                                  \
  do {                                                                                 \
    int32_t s_ = (x);                                                                  \
    if (s_ != JERK_OK) {                                                               \
      fprintf(stderr, "%s: %s (%s)\n", #x, jerk_status_str(s_), jerk_last_error());    \
      return 3;                                                                        \
    }                                                                                  \
  } while (0)

static int write_file(const char* path, const void* a, size_t na, const void* b, size_t nb) {
  FILE* f = fopen(path, "wb");
  if (!f) return 0;
  int ok = fwrite(a, 1, na, f) == na && (nb == 0 || fwrite(b, 1, nb, f) == nb);
  return fclose(f) == 0 && ok;
}

int main(int argc, char** argv) {
  if (argc != 7) {
    fprintf(stderr, "usage: %s SPECTRUM NBINS ZMAX WMAX PLANE_OUT CANDIDATES_OUT\n", argv[0]);
    return 1;
  }
  const int64_t n = atoll(argv[2]);
  if (n < 1) return 1;
  float* h_spec = (float*)malloc((size_t)n * 8);
  FILE* f = fopen(argv[1], "rb");
  if (!h_spec || !f || fread(h_spec, 8, (size_t)n, f) != (size_t)n) {
    fprintf(stderr, "cannot read %lld complex64 values from %s\n", (long long)n, argv[1]);
    return 1;
  }
  fclose(f);

  jerk_plan_desc d = {0};
  d.nbins = n;
  d.zmax = atof(argv[3]);
  d.wmax = atof(argv[4]);
  d.dz = 2.0;
  d.dw = 20.0;
  d.numbetween = 2;
  d.margin_bins = 16;
  d.path = JERK_PATH_FFT_FP32;
  jerk_plan* plan = NULL;
  CHECK_JERK(jerk_plan_create(&d, &plan));
  jerk_plan_info_t info;
  CHECK_JERK(jerk_plan_info(plan, &info));
  const int32_t T = info.n_templates;
  const size_t plane_bytes = (size_t)T * (size_t)(2 * n) * sizeof(float);

  hipStream_t stream;
  CHECK_HIP(hipStreamCreate(&stream));
  void *bank = NULL, *spec = NULL, *ws = NULL;
  float* plane = NULL;
  CHECK_HIP(hipMalloc(&bank, info.bank_bytes));
  CHECK_HIP(hipMalloc(&spec, (size_t)n * 8));
  CHECK_HIP(hipMalloc((void**)&plane, plane_bytes));
  if (info.workspace_bytes) CHECK_HIP(hipMalloc(&ws, info.workspace_bytes));
  CHECK_HIP(hipMemcpyAsync(spec, h_spec, (size_t)n * 8, hipMemcpyHostToDevice, stream));
  CHECK_JERK(jerk_templates_build(plan, bank, info.bank_bytes, stream));
  CHECK_JERK(jerk_search(plan, bank, spec, n, plane, 2 * n, 0, T, ws, info.workspace_bytes, stream));

  const double k = 3.0, pre = 0.9 * (1.0 + k);
  const size_t cws_bytes = jerk_search_candidates_workspace_bytes(plan, n, 0, T, pre, 0);
  const int64_t capacity = (int64_t)T * n;  /* at most one peak in two points */
  void* cws = NULL;
  jerk_candidate* out = NULL;
  unsigned long long* count = NULL;
  double* stats = NULL;
  CHECK_HIP(hipMalloc(&cws, cws_bytes));
  CHECK_HIP(hipMalloc((void**)&out, (size_t)capacity * sizeof(jerk_candidate)));
  CHECK_HIP(hipMalloc((void**)&count, sizeof(unsigned long long)));
  CHECK_HIP(hipMalloc((void**)&stats, (size_t)T * 2 * sizeof(double)));
  CHECK_HIP(hipMemsetAsync(count, 0, sizeof(unsigned long long), stream));
  CHECK_JERK(jerk_search_candidates(plan, bank, spec, n, 0, T, k, pre, 0, stats, out, capacity, count, cws,
                                    cws_bytes, stream));
  CHECK_HIP(hipStreamSynchronize(stream));
  CHECK_JERK(jerk_stream_check(stream));

  float* h_plane = (float*)malloc(plane_bytes);
  unsigned long long h_count = 0;
  if (!h_plane) return 4;
  CHECK_HIP(hipMemcpy(h_plane, plane, plane_bytes, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(&h_count, count, sizeof h_count, hipMemcpyDeviceToHost));
  const size_t kept = h_count < (unsigned long long)capacity ? (size_t)h_count : (size_t)capacity;
  jerk_candidate* h_out = (jerk_candidate*)malloc(kept * sizeof(jerk_candidate) + 1);
  if (!h_out) return 4;
  CHECK_HIP(hipMemcpy(h_out, out, kept * sizeof(jerk_candidate), hipMemcpyDeviceToHost));
  const long long nk = (long long)kept;
  if (!write_file(argv[5], h_plane, plane_bytes, NULL, 0) ||
      !write_file(argv[6], &nk, sizeof nk, h_out, kept * sizeof(jerk_candidate))) {
    fprintf(stderr, "cannot write the outputs\n");
    return 5;
  }
  printf("templates %d, points %lld, candidates %llu\n", T, (long long)T * 2 * n, h_count);

  free(h_out);
  free(h_plane);
  free(h_spec);
  CHECK_HIP(hipFree(stats));
  CHECK_HIP(hipFree(count));
  CHECK_HIP(hipFree(out));
  CHECK_HIP(hipFree(cws));
  if (ws) CHECK_HIP(hipFree(ws));
  CHECK_HIP(hipFree(plane));
  CHECK_HIP(hipFree(spec));
  CHECK_HIP(hipFree(bank));
  CHECK_HIP(hipStreamDestroy(stream));
  CHECK_JERK(jerk_plan_destroy(plan));
  return 0;
}
