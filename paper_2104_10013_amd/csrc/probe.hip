// FP32 MFMA throughput probe: the matrix rate this device sustains on a pure
// v_mfma_f32_16x16x4f32 loop (four independent accumulators per wave, eight
// waves per SIMD, no memory traffic in the loop).  It is the attainable peak
// the train kernel is compared with beside the published one; the clock the
// part holds under a full MFMA load is below the rated 2.4 GHz.
#include <hip/hip_runtime.h>
#include "kernels.h"

namespace ddp {

typedef float probe_f4 __attribute__((ext_vector_type(4)));
constexpr int kProbeUnroll = 8;
constexpr int kProbeThreads = 256;
constexpr int kProbeBlocksPerCu = 8;

__global__ __launch_bounds__(kProbeThreads) void k_mfma_probe(float* out, int iters) {
  probe_f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
  const float a = 1e-3f * (float)(threadIdx.x & 63), b = 1.f - a;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, a, acc2, 0, 0, 0);
      acc3 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, b, acc3, 0, 0, 0);
    }
  }
  // one store per thread keeps the loop alive; the buffer holds grid x block floats
  out[blockIdx.x * kProbeThreads + threadIdx.x] = (acc0[0] + acc1[1]) + (acc2[2] + acc3[3]);
}

hipError_t mfma_probe(int iters, double* tflops) {
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int grid = n_cu * kProbeBlocksPerCu;
  float* out = nullptr;
  if ((e = hipMalloc(&out, (size_t)grid * kProbeThreads * sizeof(float))) != hipSuccess) return e;
  hipEvent_t ev[2] = {nullptr, nullptr};
  float ms = 0.f;
  e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_mfma_probe, dim3(grid), dim3(kProbeThreads), 0, 0, out, iters / 10 + 1);   // warm-up
    hipEventRecord(ev[0], 0);
    hipLaunchKernelGGL(k_mfma_probe, dim3(grid), dim3(kProbeThreads), 0, 0, out, iters);
    hipEventRecord(ev[1], 0);
    e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  }
  if (ev[0]) hipEventDestroy(ev[0]);
  if (ev[1]) hipEventDestroy(ev[1]);
  hipFree(out);
  if (e != hipSuccess) return e;
  // 2 * 16 * 16 * 4 flop per wave-level MFMA, 4 per unrolled step
  const double waves = (double)grid * (kProbeThreads / 64);
  const double flop = waves * iters * kProbeUnroll * 4 * (2.0 * 16 * 16 * 4);
  *tflops = ms > 0.f ? flop / (ms * 1e-3) / 1e12 : 0.0;
  return hipSuccess;
}

}  // namespace ddp
