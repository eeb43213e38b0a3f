// Device arithmetic of the quantized Gaussian-mixture CDF (gfx950).
//
// The quantity: the mass of integer symbol y under a K-component mixture is
// the mixture CDF difference across the half-integer boundaries y-1/2 and
// y+1/2 (FlashGMM paper, Eq. (1) with the mixture of Eq. (2)); FlashGMM
// evaluates that CDF only at the boundaries rANS needs (Sec. III-A), with a
// closed-form Gaussian CDF approximation (Sec. III-B).
//
// Binary32 contract (bit-exact between encoder and decoder, and with any
// conforming implementation): explicit fused multiply-adds only (the library
// is compiled with -ffp-contract=off), IEEE division, round-to-nearest-even,
// a fixed operation order. The constants are the binary32 values nearest the
// stated reals.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fgmm {

// Abramowitz & Stegun 26.2.17 (Handbook of Mathematical Functions).
constexpr float kAsP = 0x1.da6712p-3f;    // 0.2316419
constexpr float kAsB1 = 0x1.470bf4p-2f;   // 0.319381530
constexpr float kAsB2 = -0x1.6d1f0ep-2f;  // -0.356563782
constexpr float kAsB3 = 0x1.c80ef0p+0f;   // 1.781477937
constexpr float kAsB4 = -0x1.d23dd4p+0f;  // -1.821255978
constexpr float kAsB5 = 0x1.548cdep+0f;   // 1.330274429
constexpr float kInvSqrt2Pi = 0x1.988454p-2f;  // 1/sqrt(2 pi)
constexpr float kLogisticK = 0x1.b3b646p+0f;   // 1.702, logistic slope
// exp: Cody & Waite reduction with ln 2 split into a 16-significant-bit
// head (so n * head is exact for |n| < 2^8) and a rounded remainder.
constexpr float kLog2e = 0x1.715476p+0f;
constexpr float kLn2Hi = 0x1.62e4p-1f;
constexpr float kLn2Lo = 0x1.7f7d1cp-20f;
// Taylor coefficients 1/k!, k = 7..3.
constexpr float kF7 = 0x1.a01a02p-13f;
constexpr float kF6 = 0x1.6c16c2p-10f;
constexpr float kF5 = 0x1.111112p-7f;
constexpr float kF4 = 0x1.555556p-5f;
constexpr float kF3 = 0x1.555556p-3f;

constexpr int kMaxK = 8;

__device__ __forceinline__ float fma32(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// exp(g) for g in [-40.5, 0]: n = rint(g log2 e), r = g - n ln 2 in two
// fused steps, degree-7 Taylor polynomial of e^r by Horner, times 2^n
// (the result is always a normal float).
__device__ __forceinline__ float exp_tilde(float g) {
  const float n = __builtin_rintf(g * kLog2e);
  float r = fma32(-n, kLn2Hi, g);
  r = fma32(-n, kLn2Lo, r);
  float p = kF7;
  p = fma32(p, r, kF6);
  p = fma32(p, r, kF5);
  p = fma32(p, r, kF4);
  p = fma32(p, r, kF3);
  p = fma32(p, r, 0.5f);
  p = fma32(p, r, 1.0f);
  p = fma32(p, r, 1.0f);
  return __builtin_ldexpf(p, (int)n);
}

// Correctly rounded 1/u for u in [2^-10, 2^10]: hardware reciprocal estimate
// plus one fused Newton correction. The library checks bit-equality with
// IEEE division on every float of that range once per device and uses this
// form only if it holds, so it stands in for the division the contract
// specifies (t = 1/u with u in [1, 3.09], r = 1/sigma with sigma clamped to
// [2^-10, 2^10]).
__device__ __forceinline__ float recip_fast(float u) {
  const float y = __builtin_amdgcn_rcpf(u);
  const float e = fma32(-u, y, 1.0f);
  return fma32(e, y, y);
}

// Upper Gaussian tail 1 - Phi(a), a in [0, 9], by A&S 26.2.17:
// Z(a) (b1 t + ... + b5 t^5), t = 1 / (1 + p a).
template <bool kFastRecip>
__device__ __forceinline__ float tail_as(float a) {
  const float u = fma32(kAsP, a, 1.0f);
  const float t = kFastRecip ? recip_fast(u) : 1.0f / u;
  float q = fma32(kAsB5, t, kAsB4);
  q = fma32(q, t, kAsB3);
  q = fma32(q, t, kAsB2);
  q = fma32(q, t, kAsB1);
  q = q * t;
  const float m = a * a;
  const float g = m * -0.5f;
  const float e = exp_tilde(g);
  const float zf = kInvSqrt2Pi * e;
  return zf * q;
}

// Upper tail of the logistic approximation 1/(1+exp(-1.702 a)).
__device__ __forceinline__ float tail_logistic(float a) {
  const float g = a * -kLogisticK;
  const float e = exp_tilde(g);
  return e / (1.0f + e);
}

// Phi~(z): z clamped to [-9, 9]; Phi(-a) = tail(a), Phi(a) = 1 - tail(a);
// the tail is capped at 1/2 (the float A&S tail exceeds 1/2 by one ulp for
// tiny a), which keeps Phi~ non-decreasing across z = 0.
template <int kKind, bool kFastRecip>
__device__ __forceinline__ float phi_tilde(float z) {
  z = __builtin_fminf(__builtin_fmaxf(z, -9.0f), 9.0f);
  const float a = __builtin_fabsf(z);
  float tail = (kKind == 1) ? tail_logistic(a) : tail_as<kFastRecip>(a);
  tail = __builtin_fminf(tail, 0.5f);
  return (z < 0.0f) ? tail : 1.0f - tail;
}

// One element's parameters after the per-element clamps: scale clamped to
// [2^-10, 2^10] then reciprocated (IEEE division); weights below 2^-60
// (including negative ones) become 0. Parameter planes are [K][n].
template <int K>
struct Elem {
  float w[K], mu[K], r[K];
};

template <int K>
__device__ __forceinline__ void load_raw(const float* __restrict__ w, const float* __restrict__ mu,
                                         const float* __restrict__ sg, int64_t n, int64_t i,
                                         float (&rw)[K], float (&rm)[K], float (&rs)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    rw[k] = w[k * n + i];
    rm[k] = mu[k * n + i];
    rs[k] = sg[k * n + i];
  }
}

template <int K, bool kFastRecip>
__device__ __forceinline__ Elem<K> make_elem(const float (&rw)[K], const float (&rm)[K],
                                             const float (&rs)[K]) {
  Elem<K> e;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float s = __builtin_fminf(__builtin_fmaxf(rs[k], 0x1p-10f), 0x1p10f);
    e.r[k] = kFastRecip ? recip_fast(s) : 1.0f / s;
    e.w[k] = (rw[k] < 0x1p-60f) ? 0.0f : rw[k];
    e.mu[k] = rm[k];
  }
  return e;
}

// Quantization constants of one configuration.
struct QCfg {
  int32_t lo;      // smallest symbol
  int32_t N;       // alphabet size
  uint32_t M;      // 2^P
  float span;      // (float)(M - N)
};

// Quantized CDF c_j at boundary b_j = lo + j - 1/2 for j in [1, N-1]:
// F = sum_k w_k Phi~((b - mu_k) r_k) accumulated in component order with
// fused multiply-adds, clamped to 1; c_j = j + floor(F (M - N)).
template <int K, int kKind, bool kFastRecip>
__device__ __forceinline__ uint32_t cdf_inner(const Elem<K>& e, const QCfg& q, int32_t j) {
  const float b = (float)(q.lo + j) - 0.5f;
  float F = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float z = (b - e.mu[k]) * e.r[k];
    F = fma32(e.w[k], phi_tilde<kKind, kFastRecip>(z), F);
  }
  F = __builtin_fminf(F, 1.0f);
  return (uint32_t)j + (uint32_t)__builtin_floorf(F * q.span);
}

// c_j for any j in [0, N] (c_0 = 0, c_N = M). The mixture is evaluated for
// every j and the ends are selected afterwards, so a wavefront never
// branches on j.
template <int K, int kKind, bool kFastRecip>
__device__ __forceinline__ uint32_t cdf_at(const Elem<K>& e, const QCfg& q, int32_t j) {
  const uint32_t c = cdf_inner<K, kKind, kFastRecip>(e, q, j);
  const uint32_t lo_end = (j <= 0) ? 0u : c;
  return (j >= q.N) ? q.M : lo_end;
}

// Device status bits, folded into a status code by the last kernel.
enum : uint32_t { kStRange = 1u, kStCorrupt = 2u, kStNoSpace = 4u, kStInval = 8u };

}  // namespace fgmm
