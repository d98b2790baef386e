// Measured peaks of the GPU the library runs on, for reporting kernels
// against what this build can reach beside the datasheet: the FP32 FMA rate
// of independent chains (packed FP32 is disabled in every kernel here, so
// this is the non-packed rate) and the device-to-device copy bandwidth.
#include "nxs_internal.h"

namespace nxs {

namespace {

constexpr int kPeakThreads = 256;
constexpr int kPeakChains = 16;

// kPeakChains independent FMA chains per lane, `iters` steps each; the sum is
// stored so that nothing is dropped.
__global__ __launch_bounds__(kPeakThreads) void peak_fma_kernel(float* __restrict__ out,
                                                               int iters, float x, float y) {
  float a[kPeakChains];
#pragma unroll
  for (int k = 0; k < kPeakChains; ++k) a[k] = (float)threadIdx.x * 1e-3f + (float)k;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) a[k] = fmaf(a[k], x, y);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kPeakChains; ++k) s += a[k];
  out[(size_t)blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// One float4 per thread over a grid that covers the array (measured the
// fastest shape here, ahead of grid-stride loops and unrolled chunks).
__global__ __launch_bounds__(kPeakThreads) void peak_copy_kernel(const float4* __restrict__ src,
                                                                float4* __restrict__ dst,
                                                                int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * kPeakThreads + threadIdx.x;
  if (i < n4) dst[i] = src[i];
}

}  // namespace

int64_t peak_fma_flops(int groups, int iters) {
  return (int64_t)2 * kPeakChains * iters * groups * kPeakThreads;
}

size_t peak_fma_out_floats(int groups) { return (size_t)groups * kPeakThreads; }

void launch_peak_fma(float* out, int groups, int iters, hipStream_t s) {
  hipLaunchKernelGGL(peak_fma_kernel, dim3((unsigned)groups), dim3(kPeakThreads), 0, s, out,
                     iters, 0.999f, 0.001f);
}

void launch_peak_copy(const float4* src, float4* dst, int64_t n4, hipStream_t s) {
  hipLaunchKernelGGL(peak_copy_kernel, dim3((unsigned)((n4 + kPeakThreads - 1) / kPeakThreads)),
                     dim3(kPeakThreads), 0, s, src, dst, n4);
}

}  // namespace nxs
