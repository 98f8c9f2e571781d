// Issue-rate probe for gfx950: throughput of the VALU operations the halo-sum kernels are made
// of (FP32 add/mul/FMA, the FP32 reciprocal square root and reciprocal, FP64 FMA), their
// dependent-issue latency, and the shader clock while they run.  Every lane runs independent
// dependent chains; each wave's first lane records the shader-clock and constant-rate (100 MHz)
// counters around its work, so the host gets wave-instructions per SIMD per shader cycle at the
// clock the part actually ran.  A benchmark utility: nothing of the lensing library uses it.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

enum Kind {
  K_FMA32 = 0,     // 8 FMA chains
  K_RSQ32 = 1,     // 8 reciprocal-square-root chains
  K_RCP32 = 2,     // 8 reciprocal chains
  K_MIX2 = 3,      // 8 FMA chains x 4 FMAs + 2 reciprocal-square-root chains per iteration
  K_FMA64 = 4,     // 8 FP64 FMA chains
  K_LAT32 = 5,     // one FMA chain (dependent-issue latency)
  K_LATRSQ = 6,    // one reciprocal-square-root chain
  K_MUL32 = 7,     // 8 multiply chains
  K_MIX4 = 8,      // 8 FMA chains x 4 FMAs + 4 reciprocal-square-root chains per iteration
  K_MIX8 = 9,      // 8 FMA chains x 4 FMAs + 8 reciprocal-square-root chains per iteration
  K_FMAV = 10,     // 8 FMA chains, every operand a VGPR
  K_ADDV = 11,     // 8 add chains, every operand a VGPR
  K_FMA16 = 12,    // 16 FMA chains, every operand a VGPR
  K_MULV = 13,     // 8 multiply chains, every operand a VGPR
  K_MIXV = 14,     // 8 FMA chains x 4 FMAs (VGPR operands) + 4 reciprocal-square-root chains
};

struct Clk {
  unsigned long long core, real, waves;
};

template <int KIND>
__global__ __launch_bounds__(256) void k_rates(int iters, float a, float b, double da, double db, float* sink,
                                               Clk* clk) {
  const unsigned long long c0 = __builtin_amdgcn_s_memtime();
  const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
  float x[16], z[8];
  double y[8];
  // per-lane copies of the operands (VGPRs, not SGPRs)
  const float av = a + 1e-30f * (float)(threadIdx.x & 1), bv = b + 1e-30f * (float)(threadIdx.x & 2);
#pragma unroll
  for (int k = 0; k < 8; ++k) { x[k] = 1.0f + 0.01f * (k + (threadIdx.x & 7)); y[k] = x[k]; z[k] = x[k]; }
#pragma unroll
  for (int k = 8; k < 16; ++k) x[k] = 1.0f + 0.01f * (k + (threadIdx.x & 7));
  for (int it = 0; it < iters; ++it) {
    if constexpr (KIND == K_FMA32) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
    } else if constexpr (KIND == K_MUL32) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = x[k] * a;
    } else if constexpr (KIND == K_RSQ32) {
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_rsqf(x[k]);
    } else if constexpr (KIND == K_RCP32) {
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_rcpf(x[k]);
    } else if constexpr (KIND == K_MIX2 || KIND == K_MIX4 || KIND == K_MIX8) {
      constexpr int NR = KIND == K_MIX2 ? 2 : KIND == K_MIX4 ? 4 : 8;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
#pragma unroll
      for (int k = 0; k < NR; ++k) z[k] = __builtin_amdgcn_rsqf(z[k]);
    } else if constexpr (KIND == K_FMA64) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) y[k] = fma(y[k], da, db);
    } else if constexpr (KIND == K_FMAV) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], av, bv);
    } else if constexpr (KIND == K_ADDV) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = x[k] + bv;
    } else if constexpr (KIND == K_MULV) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = x[k] * av;
    } else if constexpr (KIND == K_MIXV) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], av, bv);
#pragma unroll
      for (int k = 0; k < 4; ++k) z[k] = __builtin_amdgcn_rsqf(z[k]);
    } else if constexpr (KIND == K_FMA16) {
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = fmaf(x[k], av, bv);
    } else if constexpr (KIND == K_LAT32) {
#pragma unroll
      for (int r = 0; r < 32; ++r) x[0] = fmaf(x[0], a, b);
    } else {
#pragma unroll
      for (int r = 0; r < 8; ++r) x[0] = __builtin_amdgcn_rsqf(x[0]);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k] + (float)y[k] + z[k] + x[k + 8];
  if (s == 1234.5f) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;   // keeps the chains alive
  const unsigned long long c1 = __builtin_amdgcn_s_memtime();
  const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&clk->core, c1 - c0);
    atomicAdd(&clk->real, r1 - r0);
    atomicAdd(&clk->waves, 1ull);
  }
}

}  // namespace

// Runs one probe kind: `blocks` workgroups of 256 threads, `iters` iterations each.  Returns the
// kernel time [ms] (HIP events), the mean shader clock over the waves [MHz] (shader-clock
// counter over the 100 MHz constant-rate counter) and 0, or a HIP error code.
extern "C" int lfr_run(int kind, int iters, int blocks, float* ms, double* mhz) {
  float* sink = nullptr;
  Clk* clk = nullptr;
  hipEvent_t e0, e1;
  if (hipMalloc(&sink, sizeof(float) * 256 * (size_t)blocks) != hipSuccess) return -1;
  if (hipMalloc(&clk, sizeof(Clk)) != hipSuccess) return -1;
  if (hipMemset(clk, 0, sizeof(Clk)) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    return -1;
  const float a = 0.999f, b = 0.001f;
  const double da = 0.999, db = 0.001;
  (void)hipEventRecord(e0, nullptr);
  switch (kind) {
#define LFR(K) case K: hipLaunchKernelGGL(k_rates<K>, dim3(blocks), dim3(256), 0, nullptr, iters, a, b, da, db, sink, clk); break;
    LFR(0) LFR(1) LFR(2) LFR(3) LFR(4) LFR(5) LFR(6) LFR(7) LFR(8) LFR(9) LFR(10) LFR(11) LFR(12) LFR(13) LFR(14)
#undef LFR
    default: break;
  }
  (void)hipEventRecord(e1, nullptr);
  hipError_t err = hipEventSynchronize(e1);
  (void)hipEventElapsedTime(ms, e0, e1);
  Clk h{};
  if (hipMemcpy(&h, clk, sizeof(Clk), hipMemcpyDeviceToHost) != hipSuccess) err = hipErrorUnknown;
  *mhz = h.real ? 100.0 * (double)h.core / (double)h.real : 0.0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  (void)hipFree(clk);
  return err == hipSuccess ? 0 : (int)err;
}
