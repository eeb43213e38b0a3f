// Shared device pieces of the search-bracket MLP (training kernels and the
// decode-fused inference).
//
// Network: D = 3K+1 inputs -> 64 -> ReLU -> 64 -> ReLU -> 1. Inputs per
// element and slot: the K clamped weights, the K means, the K log-scales
// (natural log of the clamped scale) and slot / 2^P, each normalised as
// (x - mean) * inv_std with constants stored with the weights. The output,
// times out_std plus out_mean, predicts the decoded symbol. Flat parameter
// layout: W1 [64][D], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 [1].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fgmm {

constexpr int kMlpH = 64;
constexpr int kMlpMaxD = 16;

__host__ __device__ inline int mlp_num_params(int D) {
  return kMlpH * D + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;
}

// binary32 -> nearest bfloat16 (ties to even), returned as the float value.
__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

// Raw (unnormalised) feature d of one element: its parameters in registers.
template <int K>
__device__ __forceinline__ float mlp_raw_feature(int d, const float (&w)[K], const float (&mu)[K],
                                                 const float (&sg)[K], uint32_t slot,
                                                 float inv_m) {
  if (d < K) return (w[d] < 0x1p-60f) ? 0.0f : w[d];
  if (d < 2 * K) return mu[d - K];
  if (d < 3 * K) {
    const float s = __builtin_fminf(__builtin_fmaxf(sg[d - 2 * K], 0x1p-10f), 0x1p10f);
    return __logf(s);
  }
  if (d == 3 * K) return (float)slot * inv_m;
  return 0.0f;
}

}  // namespace fgmm
