// FP64 issue-rate probe: the rate of plain FP64 vector streams on one MI355X,
// measured the same way the step kernels are (HIP events around launches of
// 8 wavefronts per SIMD), as context for their roofline fractions.
//
//   fma   eight independent v_fma_f64 chains per lane
//   rcp   eight independent v_rcp_f64 chains per lane (the reciprocal seeds
//         of the Kepler solve and the interaction kick)
//   mix   per chain one v_rcp_f64 followed by eight v_fma_f64
//
// Prints one JSON line: the FMA stream's rate in TFLOP/s (2 flops per FMA
// lane), the time per wave64 instruction per SIMD of each stream, and the
// issue cost of a reciprocal seed inside an FMA stream in FMA units.
// Standalone program (no library, no inputs); exits non-zero on any HIP error.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                      \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));             \
      std::exit(2);                                                                   \
    }                                                                                 \
  } while (0)

namespace {

constexpr int CHAINS = 8;

template <int MODE>
__global__ __launch_bounds__(256) void k_probe(double* out, int n, int iters, double s) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double a[CHAINS];
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) a[j] = 1.0 + 1e-3 * (t & 63) + 0.01 * j;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < CHAINS; ++j) {
      if (MODE == 0) a[j] = fma(a[j], s, 0.25);
      if (MODE == 1) a[j] = __builtin_amdgcn_rcp(a[j]);
      if (MODE == 2) {
        a[j] = __builtin_amdgcn_rcp(a[j]);
#pragma unroll
        for (int u = 0; u < 8; ++u) a[j] = fma(a[j], s, 0.25);
      }
    }
  }
  double r = 0.0;
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) r += a[j];
  out[t] = r;
}

// Milliseconds per launch (mean of 5 after one warm-up launch).
template <int MODE>
float time_launch(double* d, int n, int blocks, int iters, hipEvent_t e0, hipEvent_t e1) {
  hipLaunchKernelGGL(k_probe<MODE>, dim3(blocks), dim3(256), 0, 0, d, n, iters, 0.75);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0, 0));
  for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(k_probe<MODE>, dim3(blocks), dim3(256), 0, 0, d, n, iters, 0.75);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms = 0.0f;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  return ms / 5.0f;
}

}  // namespace

int main() {
  int dev = 0, ncu = 0;
  CHECK(hipGetDevice(&dev));
  CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int simds = 4 * ncu;
  const int blocks = 8 * ncu;               // 256-thread blocks: 8 wavefronts per SIMD
  const int n = blocks * 256;
  const int iters = 4096;
  double* d = nullptr;
  CHECK(hipMalloc(&d, sizeof(double) * n));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const double wave_instr = (double)n / 64.0 / simds * iters * CHAINS;   // per SIMD, per instruction of a chain step
  const float t_fma = time_launch<0>(d, n, blocks, iters, e0, e1);
  const float t_rcp = time_launch<1>(d, n, blocks, iters, e0, e1);
  const float t_mix = time_launch<2>(d, n, blocks, iters, e0, e1);
  const double ns_fma = t_fma * 1e6 / wave_instr;
  const double ns_rcp = t_rcp * 1e6 / wave_instr;
  const double ns_mix = t_mix * 1e6 / wave_instr;                        // one rcp + 8 fma
  const double tflops = 2.0 * 64.0 * simds / (ns_fma * 1e-9) / 1e12;
  std::printf("{\"fma_tflops\": %.4f, \"ns_per_wave_fma\": %.5f, \"ns_per_wave_rcp\": %.5f, "
              "\"ns_per_wave_rcp_plus_8_fma\": %.5f, \"rcp_in_fma_stream_fma_units\": %.3f, "
              "\"simds\": %d, \"waves_per_simd\": 8}\n",
              tflops, ns_fma, ns_rcp, ns_mix, (ns_mix - 8.0 * ns_fma) / ns_fma, simds);
  CHECK(hipFree(d));
  return 0;
}
