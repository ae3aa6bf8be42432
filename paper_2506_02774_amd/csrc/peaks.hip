// Throughput probes that measure the chip's practical vector peaks, for the
// rooflines: FP32 fused multiply-add (8 independent chains per lane, built
// like every kernel here, so without packed FP32 instructions) and the
// hardware exponential v_exp_f32 (the transcendental unit). Each lane writes
// one value so that no chain is removed.
#include "vy_common.hpp"

namespace {

constexpr int kPeakBlocks = 256 * 8, kPeakThreads = 256, kChains = 8;

__global__ __launch_bounds__(kPeakThreads) void peak_fma(float* out, int iters, float a, float b) {
  float x[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) x[k] = (float)(threadIdx.x + k) * 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = fmaf(x[k], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += x[k];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kPeakThreads) void peak_exp(float* out, int iters) {
  float x[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) x[k] = (float)(threadIdx.x + k) * 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = __builtin_amdgcn_exp2f(-x[k]);   // stays in (0.5, 1]
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += x[k];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

}  // namespace

extern "C" size_t vy_measure_peaks_bytes(void) { return sizeof(float) * (size_t)kPeakBlocks * kPeakThreads; }

extern "C" int vy_measure_peaks(float* scratch, size_t scratch_bytes, double* fma_tflops, double* exp_gops,
                                void* stream) {
  if (!scratch || scratch_bytes < vy_measure_peaks_bytes() || !fma_tflops || !exp_gops)
    return vy::fail(VY_ERR_ARG, "vy_measure_peaks: bad argument");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e[4];
  for (int k = 0; k < 4; ++k) VY_HIP(hipEventCreate(&e[k]));
  const int iters = 4096;
  int rc = VY_OK;
  do {
    // one untimed launch of each, then the timed ones
    peak_fma<<<kPeakBlocks, kPeakThreads, 0, st>>>(scratch, 64, 0.999f, 1e-4f);
    peak_exp<<<kPeakBlocks, kPeakThreads, 0, st>>>(scratch, 64);
    if (hipEventRecord(e[0], st) != hipSuccess) { rc = VY_ERR_HIP; break; }
    peak_fma<<<kPeakBlocks, kPeakThreads, 0, st>>>(scratch, iters, 0.999f, 1e-4f);
    if (hipEventRecord(e[1], st) != hipSuccess) { rc = VY_ERR_HIP; break; }
    if (hipEventRecord(e[2], st) != hipSuccess) { rc = VY_ERR_HIP; break; }
    peak_exp<<<kPeakBlocks, kPeakThreads, 0, st>>>(scratch, iters);
    if (hipEventRecord(e[3], st) != hipSuccess) { rc = VY_ERR_HIP; break; }
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e[3]) != hipSuccess) { rc = VY_ERR_HIP; break; }
    float ms_fma = 0.f, ms_exp = 0.f;
    if (hipEventElapsedTime(&ms_fma, e[0], e[1]) != hipSuccess || hipEventElapsedTime(&ms_exp, e[2], e[3]) != hipSuccess) {
      rc = VY_ERR_HIP;
      break;
    }
    const double lanes = (double)kPeakBlocks * kPeakThreads * kChains * iters;
    *fma_tflops = 2.0 * lanes / (ms_fma * 1e-3) / 1e12;
    *exp_gops = lanes / (ms_exp * 1e-3) / 1e9;
  } while (0);
  for (int k = 0; k < 4; ++k) (void)hipEventDestroy(e[k]);
  return rc == VY_OK ? VY_OK : vy::fail(rc, "vy_measure_peaks: HIP failure");
}
