// Measured ceilings of the two arithmetic units the search uses, for the roofline fractions:
// v_mfma_f32_32x32x16_bf16 (four independent accumulators per wave) and plain FP32 FMA
// (v_fma_f32, sixteen independent chains per lane; packed FP32 is not used), each in a loop with
// no memory traffic over every SIMD at 8 waves per SIMD. Also the shader clock during each loop,
// from the cycle counter against the constant-rate wall clock. And the write bandwidth of
// plane-like tiles (a workgroup stores U float2 at offset seg U of one of 256 rows, 8 stores of
// 64 lanes, as the FFT epilogue does), plain and non-temporal, for U a multiple of 16 (whole
// 128-byte lines) and U odd (tiles share lines).
//
// Prints one JSON object. Built by build.py into peakprobe next to this file; bench.py runs it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
      std::exit(1);                                                           \
    }                                                                         \
  } while (0)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// clk[2 w], clk[2 w + 1]: cycle-counter and wall-clock ticks of wave w over its loop
__global__ void __launch_bounds__(256) mfma_loop(int iters, float* out, long long* clk) {
  f32x16 a0 = {}, a1 = {}, a2 = {}, a3 = {};
  bf16x8 x, y;
  for (int i = 0; i < 8; ++i) {
    x[i] = (__bf16)(threadIdx.x * 1e-3f + i);
    y[i] = (__bf16)(1e-3f * i);
  }
  const long long c0 = clock64(), w0 = wall_clock64();
  for (int it = 0; it < iters; ++it) {
    a0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, a0, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, a1, 0, 0, 0);
    a2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, a2, 0, 0, 0);
    a3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, a3, 0, 0, 0);
  }
  const long long c1 = clock64(), w1 = wall_clock64();
  float s = 0.f;
  for (int i = 0; i < 16; ++i) s += a0[i] + a1[i] + a2[i] + a3[i];
  const int gw = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
  if ((threadIdx.x & 63) == 0) {
    clk[2 * gw] = c1 - c0;
    clk[2 * gw + 1] = w1 - w0;
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) fma_loop(int iters, float* out, long long* clk) {
  float v[16];
  for (int i = 0; i < 16; ++i) v[i] = threadIdx.x * 1e-3f + i;
  const float m = 0.999f, c = 1e-4f;
  const long long c0 = clock64(), w0 = wall_clock64();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = fmaf(v[i], m, c);
  }
  const long long c1 = clock64(), w1 = wall_clock64();
  float s = 0.f;
  for (int i = 0; i < 16; ++i) s += v[i];
  const int gw = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
  if ((threadIdx.x & 63) == 0) {
    clk[2 * gw] = c1 - c0;
    clk[2 * gw + 1] = w1 - w0;
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// One tile per workgroup: row blk % rows, tile blk / rows of that row.
template <bool NT>
__global__ void __launch_bounds__(64) tile_store_kernel(float2* plane, long ld2, int U, int rows, long tiles) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const long blk = blockIdx.x;
  if (blk >= tiles) return;
  f2v* out = reinterpret_cast<f2v*>(plane + (blk % rows) * ld2 + (blk / rows) * U);
  const float v = (float)blk;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int lag = threadIdx.x + 64 * k;
    if (lag < U) {
      if (NT) __builtin_nontemporal_store(f2v{v, v}, out + lag);
      else out[lag] = f2v{v, v};
    }
  }
}

int main() {
  int dev = 0, cus = 0, wall_khz = 0;
  CHECK(hipGetDevice(&dev));
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  CHECK(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
  const int waves_per_simd = 8;
  const int threads = 256;  // one wave per SIMD per workgroup
  const int blocks = cus * waves_per_simd;
  const int waves = blocks * threads / 64;
  float* out = nullptr;
  long long* clk = nullptr;
  CHECK(hipMalloc(&out, sizeof(float) * (size_t)blocks * threads));
  CHECK(hipMalloc(&clk, sizeof(long long) * 2 * (size_t)waves));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  std::vector<long long> h(2 * (size_t)waves);
  std::printf("{\"cus\": %d, \"waves_per_simd\": %d", cus, waves_per_simd);
  for (int kind = 0; kind < 2; ++kind) {
    const int iters = kind == 0 ? 20000 : 200000;
    float best_ms = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      CHECK(hipEventRecord(e0, 0));
      if (kind == 0) hipLaunchKernelGGL(mfma_loop, dim3(blocks), dim3(threads), 0, 0, iters, out, clk);
      else hipLaunchKernelGGL(fma_loop, dim3(blocks), dim3(threads), 0, 0, iters, out, clk);
      CHECK(hipGetLastError());
      CHECK(hipEventRecord(e1, 0));
      CHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) best_ms = ms;
    }
    CHECK(hipMemcpy(h.data(), clk, sizeof(long long) * h.size(), hipMemcpyDeviceToHost));
    double cyc = 0, wall = 0;
    for (int w = 0; w < waves; ++w) {
      cyc += (double)h[2 * w];
      wall += (double)h[2 * w + 1];
    }
    const double mhz = cyc / (wall / (wall_khz * 1e3)) / 1e6;
    const double flops = kind == 0 ? (double)waves * iters * 4 * 32768.0 : (double)waves * 64 * iters * 16 * 2.0;
    std::printf(", \"%s\": {\"TFLOPs\": %.1f, \"ms\": %.3f, \"clock_MHz\": %.0f}",
                kind == 0 ? "mfma_bf16" : "fp32_fma", flops / (best_ms * 1e-3) / 1e12, best_ms, mhz);
  }
  CHECK(hipFree(out));
  CHECK(hipFree(clk));
  // plane-like stores: 256 rows of 2^22 float2 (8 GiB)
  const long ld2 = 1L << 22;
  const int rows = 256;
  float2* plane = nullptr;
  CHECK(hipMalloc(&plane, sizeof(float2) * ld2 * rows));
  std::printf(", \"tile_stores_TBps\": {");
  const int us[2] = {512, 481};
  for (int ui = 0; ui < 2; ++ui) {
    const int U = us[ui];
    const long tiles = (ld2 / U) * rows;  // seg < ld2 / U: every tile inside its row
    for (int nt = 0; nt < 2; ++nt) {
      float best_ms = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        CHECK(hipEventRecord(e0, 0));
        if (nt) hipLaunchKernelGGL(tile_store_kernel<true>, dim3((unsigned)tiles), dim3(64), 0, 0, plane, ld2, U, rows, tiles);
        else hipLaunchKernelGGL(tile_store_kernel<false>, dim3((unsigned)tiles), dim3(64), 0, 0, plane, ld2, U, rows, tiles);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) best_ms = ms;
      }
      const double bytes = (double)tiles * U * sizeof(float2);
      std::printf("%s\"U%d_%s\": %.2f", (ui | nt) ? ", " : "", U, nt ? "nt" : "plain", bytes / (best_ms * 1e-3) / 1e12);
    }
  }
  std::printf("}}\n");
  CHECK(hipFree(plane));
  return 0;
}
