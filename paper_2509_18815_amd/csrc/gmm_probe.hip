// Peak probes (diagnostics beside the coder): the issue rate of independent
// binary32 fused multiply-adds in the library's instruction forms (packed
// FP32 is disabled at compile time, so one fma per lane per instruction)
// and a plain device copy. The benchmark times them with HIP events to set
// the coder kernels' rates beside what the GPU sustains.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/flashgmm.h"

namespace {

constexpr int kChains = 8;

__global__ void __launch_bounds__(256) k_fma_probe(float* __restrict__ out, int32_t iters) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (float)(threadIdx.x + k) * 0x1p-10f;
  const float m = 0x1.000002p+0f, c = 0x1p-24f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = __builtin_fmaf(a[k], m, c);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[t] = s;
}

__global__ void __launch_bounds__(256) k_copy_probe(const float4* __restrict__ src,
                                                    float4* __restrict__ dst, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    dst[i] = src[i];
}

}  // namespace

extern "C" {

int gmm_fma_probe(float* out, int64_t threads, int32_t iters, void* stream) {
  if (!out || threads < 256 || threads % 256 != 0 || iters < 1) return GMM_EINVAL;
  hipLaunchKernelGGL(k_fma_probe, dim3((unsigned)(threads / 256)), dim3(256), 0,
                     (hipStream_t)stream, out, iters);
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

int gmm_copy_probe(const void* src, void* dst, int64_t bytes, void* stream) {
  if (!src || !dst || bytes < 16 || bytes % 16 != 0) return GMM_EINVAL;
  const int64_t n4 = bytes / 16;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      cus = prop.multiProcessorCount;
  }
  const int64_t grid = (int64_t)cus * 16;  // 16 workgroups of 256 per compute unit
  hipLaunchKernelGGL(k_copy_probe, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                     (const float4*)src, (float4*)dst, n4);
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

}  // extern "C"
