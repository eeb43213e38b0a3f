// Device arithmetic of the quantized Gaussian-mixture CDF (gfx950).
//
// The quantity: the mass of integer symbol y under a K-component mixture is
// the mixture CDF difference across the half-integer boundaries y-1/2 and
// y+1/2 (FlashGMM paper, Eq. (1) with the mixture of Eq. (2)); FlashGMM
// evaluates that CDF only at the boundaries rANS needs (Sec. III-A), with a
// closed-form Gaussian CDF approximation (Sec. III-B: A&S 26.2.17, the
// logistic function, Polya's formula), or, as Table II's unapproximated
// baseline, a binary64 evaluation from series and continued fraction.
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
constexpr float kAsB1 = 0x1.470bf4p-2f;   // 0.319381530
constexpr float kAsB2 = -0x1.6d1f0ep-2f;  // -0.356563782
constexpr float kAsB3 = 0x1.c80ef0p+0f;   // 1.781477937
constexpr float kAsB4 = -0x1.d23dd4p+0f;  // -1.821255978
constexpr float kAsB5 = 0x1.548cdep+0f;   // 1.330274429
// A&S component form of the mixture (kind 0): the clamp |z| <= 9 becomes
// a = min(|b - mu| (r/9), 1), so 9 p and 81 log2(e)/2 scale a; the Gaussian
// density C 2^(-x), x = a^2 81 log2(e)/2, splits x into n = rint(x) and
// g = x - n in [-1/2, 1/2] (n by the round-to-integer of adding 1.5 2^23).
// C 2^(-g) is the degree-7 Taylor polynomial of C e^(-g ln 2) economized
// to degree 5 on [-1/2, 1/2] with the Chebyshev polynomials T7 and T6
// (Lanczos): with L = ln 2, c_k = C (-L)^k / k!,
//   G0 = c0 + c6/2048, G1 = c1 + (14/8192) c7, G2 = c2 - (72/2048) c6,
//   G3 = c3 - (448/8192) c7, G4 = c4 + (768/2048) c6, G5 = c5 + (3584/8192) c7.
constexpr float kAsP9 = 0x1.0ad9fap+1f;   // 9 p, p = 0.2316419
constexpr float kInv9 = 0x1.c71c72p-4f;   // 1/9
constexpr float kAsL2 = 0x1.d36ee6p+5f;   // 81 log2(e) / 2 = 58.429150
constexpr float kRound = 0x1.8p+23f;      // 1.5 2^23
constexpr float kG0 = 0x1.988456p-2f;
constexpr float kG1 = -0x1.1b2990p-2f;
constexpr float kG2 = 0x1.88899ap-4f;
constexpr float kG3 = -0x1.6ac8cep-6f;
constexpr float kG4 = 0x1.f9f438p-9f;
constexpr float kG5 = -0x1.184804p-11f;
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
constexpr float kF8 = 0x1.a01a02p-16f;  // 1/8!
// Polya: Phi(x) ~ (1 + sign(x) sqrt(1 - exp(-(2/pi) x^2))) / 2
constexpr float kPolyaC = 0x1.45f306p-1f;  // 2/pi
// lower bound of scales mapped from raw log-scale outputs
constexpr float kScaleMin = 0x1.c28f5cp-4f;  // 0.11

// binary64 reference CDF: exp with ln 2 split so that n * kLn2HiD is exact
// for |n| < 2^11; Taylor coefficients 1/k!, k = 0..13.
constexpr double kLog2eD = 0x1.71547652b82fep+0;
constexpr double kLn2HiD = 0x1.62e42fefa38p-1;
constexpr double kLn2LoD = 0x1.ef35793c7673p-45;
constexpr double kInvSqrt2D = 0x1.6a09e667f3bcdp-1;
constexpr double kInvSqrtPiD = 0x1.20dd750429b6dp-1;
constexpr double kHalfInvSqrtPiD = 0x1.20dd750429b6dp-2;
constexpr int kErfTerms = 32;     // Maclaurin terms of erf, x < 2
constexpr int kErfcCfDepth = 50;  // continued-fraction levels of erfc, x >= 2

constexpr int kMaxK = 8;

__device__ __forceinline__ float fma32(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// exp(g) for g in [-51.6, 7]: n = rint(g log2 e), r = g - n ln 2 in two
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

// Upper tail of the logistic approximation 1/(1+exp(-1.702 a)).
__device__ __forceinline__ float tail_logistic(float a) {
  const float g = a * -kLogisticK;
  const float e = exp_tilde(g);
  return e / (1.0f + e);
}

// Upper tail of Polya's approximation, (1 - sqrt(E)) / 2 with
// E = 1 - exp(-u), u = (2/pi) a^2, in the form (e/2) / (1 + sqrt(E)) that
// does not cancel for large a; E comes from the Taylor series of -expm1
// for u < 1/4 (where 1 - e would cancel) and from 1 - e above. Both
// candidates are computed and one is selected, so lanes do not diverge.
__device__ __forceinline__ float tail_polya(float a) {
  const float m = a * a;
  const float u = m * kPolyaC;
  const float g = -u;
  const float e = exp_tilde(g);
  float p = kF8;
  p = fma32(p, g, kF7);
  p = fma32(p, g, kF6);
  p = fma32(p, g, kF5);
  p = fma32(p, g, kF4);
  p = fma32(p, g, kF3);
  p = fma32(p, g, 0.5f);
  p = fma32(p, g, 1.0f);
  const float E = (u < 0.25f) ? u * p : 1.0f - e;
  const float s = __builtin_sqrtf(E);
  const float h = e * 0.5f;
  return h / (1.0f + s);
}

// Phi~(z) for the logistic (1) and Polya (2) kinds: z clamped to [-9, 9];
// Phi(-a) = tail(a), Phi(a) = 1 - tail(a); the tail is capped at 1/2, which
// keeps Phi~ non-decreasing across z = 0. (Kind 0 enters the mixture as
// as_half below.)
template <int kKind>
__device__ __forceinline__ float phi_tilde(float z) {
  z = __builtin_fminf(__builtin_fmaxf(z, -9.0f), 9.0f);
  const float a = __builtin_fabsf(z);
  float tail = (kKind == 1) ? tail_logistic(a) : tail_polya(a);
  tail = __builtin_fminf(tail, 0.5f);
  return (z < 0.0f) ? tail : 1.0f - tail;
}

// Signed half of one A&S component, Phi~(z) - 1/2, for kind 0, from
// d = b - mu and rn = r/9 (r = 1/sigma'):
//   a = min(|d| rn, 1),  t = 1 / (1 + 9p a),  q = t (b1 + t (b2 + ... b5)),
//   x2 = a a,  s = (1.5 2^23) - x2 L  (fused, = 1.5 2^23 - rint(x2 L)),
//   n = s - 1.5 2^23 (exact),  g = x2 L + n  (fused),
//   e = polynomial of C 2^(-g),  D = max(fma(-(e 2^n), q, 1/2), 0),
// and the result carries the sign of d. 2^n (n in [-59, 0]) is applied by
// adding the low bits of s, which hold n, to e's exponent field: e 2^n stays
// a normal float. D <= 1/2, so max(., 0) is the [0, 1] clamp and folds into
// the fused multiply-add; the clamp of a folds into its product the same
// way.
template <bool kFastRecip>
__device__ __forceinline__ float as_half(float d, float rn) {
  const float a = __builtin_fminf(__builtin_fmaxf(__builtin_fabsf(d) * rn, 0.0f), 1.0f);
  const float u = fma32(a, kAsP9, 1.0f);
  const float t = kFastRecip ? recip_fast(u) : 1.0f / u;
  float h = fma32(kAsB5, t, kAsB4);
  h = fma32(h, t, kAsB3);
  h = fma32(h, t, kAsB2);
  h = fma32(h, t, kAsB1);
  const float q = h * t;
  const float x2 = a * a;
  const float s = fma32(-x2, kAsL2, kRound);
  const float n = s - kRound;
  const float g = fma32(x2, kAsL2, n);
  float e = fma32(kG5, g, kG4);
  e = fma32(e, g, kG3);
  e = fma32(e, g, kG2);
  e = fma32(e, g, kG1);
  e = fma32(e, g, kG0);
  // bits(s) = bits(1.5 2^23) + n, and bits(1.5 2^23) << 23 wraps to 0
  const float E = __builtin_bit_cast(
      float, __builtin_bit_cast(uint32_t, e) + (__builtin_bit_cast(uint32_t, s) << 23));
  const float D = __builtin_fminf(__builtin_fmaxf(fma32(-E, q, 0.5f), 0.0f), 1.0f);
  return __builtin_copysignf(D, d);
}

// exp(g) in binary64 for g in [-686, 0]: Cody & Waite reduction, Taylor
// polynomial of degree 13 (|r| <= 0.35), times 2^n (normal result).
__device__ __forceinline__ double exp_d(double g) {
  constexpr double kInvFact[14] = {1.0,
                                   1.0,
                                   0x1p-1,
                                   0x1.5555555555555p-3,
                                   0x1.5555555555555p-5,
                                   0x1.1111111111111p-7,
                                   0x1.6c16c16c16c17p-10,
                                   0x1.a01a01a01a01ap-13,
                                   0x1.a01a01a01a01ap-16,
                                   0x1.71de3a556c734p-19,
                                   0x1.27e4fb7789f5cp-22,
                                   0x1.ae64567f544e4p-26,
                                   0x1.1eed8eff8d898p-29,
                                   0x1.6124613a86d09p-33};
  const double n = __builtin_rint(g * kLog2eD);
  double r = __builtin_fma(-n, kLn2HiD, g);
  r = __builtin_fma(-n, kLn2LoD, r);
  double p = kInvFact[13];
#pragma unroll
  for (int k = 12; k >= 0; --k) p = __builtin_fma(p, r, kInvFact[k]);
  return __builtin_ldexp(p, (int)n);
}

// Gaussian upper tail Q(a) = erfc(a / sqrt 2) / 2 in binary64, a in [0, 37].
// With x = a / sqrt 2, y = x^2: for x < 2 the Maclaurin series of erf,
// nested as s_{n-1} = 1/(2n-1) - (y/n) s_n from s_N = 1/(2N+1), gives
// Q = 1/2 - x s / sqrt(pi); for x >= 2 Laplace's continued fraction
// erfc(x) = exp(-y) / sqrt(pi) / (x + (1/2)/(x + 1/(x + (3/2)/(x + ...)))),
// evaluated bottom-up from a fixed depth, gives Q = exp(-y)/(2 sqrt pi)/u.
__device__ __forceinline__ double tail_ref(double a) {
  const double x = a * kInvSqrt2D;
  const double y = x * x;
  if (x < 2.0) {
    double s = 1.0 / (2 * kErfTerms + 1);
#pragma unroll
    for (int n = kErfTerms; n >= 1; --n) {
      const double v = y * (1.0 / n);
      s = __builtin_fma(-v, s, 1.0 / (2 * n - 1));
    }
    const double t1 = x * s;
    return __builtin_fma(-kInvSqrtPiD, t1, 0.5);
  }
  double u = x;
  for (int m = kErfcCfDepth; m >= 1; --m) u = x + (0.5 * m) / u;
  const double e = exp_d(-y);
  const double t2 = e * kHalfInvSqrtPiD;
  return t2 / u;
}

// Reference Phi(z) in binary64: z clamped to [-37, 37] (exp stays normal).
__device__ __forceinline__ double phi_ref(double z) {
  z = __builtin_fmin(__builtin_fmax(z, -37.0), 37.0);
  const double q = tail_ref(__builtin_fabs(z));
  return (z < 0.0) ? q : 1.0 - q;
}

// Quantization constants of one configuration.
struct QCfg {
  int32_t lo;      // smallest symbol
  int32_t N;       // alphabet size
  uint32_t M;      // 2^P
  float span;      // (float)(M - N)
  float lo_mh;     // (float)lo - 0.5, exact (|lo| <= 2^22)
  int32_t raw;     // 1: parameter planes hold raw outputs (weight logits, log-scales)
  int32_t prio;    // issue priority of the launch's wavefronts, 0..3
};

// Raises the calling wavefront's issue priority (s_setprio) to p in 1..3;
// 0 leaves the default. Among wavefronts sharing a SIMD the arbiter issues
// the higher-priority ones first; results do not depend on it.
__device__ __forceinline__ void set_wave_priority(int32_t p) {
  if (p >= 3)
    __builtin_amdgcn_s_setprio(3);
  else if (p == 2)
    __builtin_amdgcn_s_setprio(2);
  else if (p == 1)
    __builtin_amdgcn_s_setprio(1);
}

// Raw outputs of one element to weights and scales, in place: softmax of
// the logits (differences to the largest, in component order, floored at
// -40.5; the sum in component order; IEEE division) and
// sigma = max(exp~(clamp(t, -7, 7)), 0.11) of the log-scales t.
template <int K>
__device__ __forceinline__ void raw_to_params(float (&w)[K], float (&s)[K]) {
  float m = w[0];
#pragma unroll
  for (int k = 1; k < K; ++k) m = __builtin_fmaxf(m, w[k]);
  float e[K];
#pragma unroll
  for (int k = 0; k < K; ++k) e[k] = exp_tilde(__builtin_fmaxf(w[k] - m, -40.5f));
  float sum = e[0];
#pragma unroll
  for (int k = 1; k < K; ++k) sum = sum + e[k];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    w[k] = e[k] / sum;
    s[k] = __builtin_fmaxf(exp_tilde(__builtin_fminf(__builtin_fmaxf(s[k], -7.0f), 7.0f)),
                           kScaleMin);
  }
}

// One element's parameters after the per-element clamps: scale clamped to
// [2^-10, 2^10] then reciprocated (IEEE division; the binary64 reference
// kind keeps the clamped scale itself and divides in binary64); weights
// below 2^-60 (including negative ones) become 0. With q.raw the planes
// hold raw outputs, mapped first. Parameter planes are [K][n].
// Kind 0 also keeps rn = r (1/9) per component and hw = (sum_k w'_k) / 2,
// the sum in component order: the mixture starts from hw and adds
// w'_k (Phi~_k - 1/2).
template <int K>
struct Elem {
  float w[K], mu[K], r[K], rn[K];
  float hw;
  float sc[K];  // the clamped scale sigma' (the decoder's search bracket)
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

template <int K, bool kFastRecip, int kKind = 0>
__device__ __forceinline__ Elem<K> make_elem(const QCfg& q, const float (&rw)[K],
                                             const float (&rm)[K], const float (&rs)[K]) {
  float w[K], sc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    w[k] = rw[k];
    sc[k] = rs[k];
  }
  if (__builtin_expect(q.raw != 0, 0)) raw_to_params<K>(w, sc);
  Elem<K> e;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float s = __builtin_fminf(__builtin_fmaxf(sc[k], 0x1p-10f), 0x1p10f);
    e.r[k] = (kKind == 3) ? s : (kFastRecip ? recip_fast(s) : 1.0f / s);
    e.w[k] = (w[k] < 0x1p-60f) ? 0.0f : w[k];
    e.mu[k] = rm[k];
    e.rn[k] = e.r[k] * kInv9;
    e.sc[k] = s;
  }
  float ws = e.w[0];
#pragma unroll
  for (int k = 1; k < K; ++k) ws = ws + e.w[k];
  e.hw = ws * 0.5f;
  return e;
}

// The scaled mixture y = RN(F (M - N)) at a boundary b (kinds 0..2):
// F = sum_k w_k Phi~((b - mu_k) r_k) accumulated in component order with
// fused multiply-adds, clamped to [0, 1]. c_j = j + floor(y) at b = b_j.
template <int K, int kKind, bool kFastRecip>
__device__ __forceinline__ float cdf_scaled(const Elem<K>& e, const QCfg& q, float b) {
  float F = (kKind == 0) ? e.hw : 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if constexpr (kKind == 0) {
      F = fma32(e.w[k], as_half<kFastRecip>(b - e.mu[k], e.rn[k]), F);
    } else {
      const float z = (b - e.mu[k]) * e.r[k];
      F = fma32(e.w[k], phi_tilde<kKind>(z), F);
    }
  }
  // F clamped to [0, 1] (min(F, 1) of the contract; kind 0's sum of
  // signed halves can round a few ulps below 0), folded into the last
  // fused multiply-add as its output modifier
  F = __builtin_fminf(__builtin_fmaxf(F, 0.0f), 1.0f);
  return F * q.span;
}

// Quantized CDF c_j at boundary b_j = lo + j - 1/2 for j in [1, N-1]:
// c_j = j + floor(F (M - N)).
template <int K, int kKind, bool kFastRecip>
__device__ __forceinline__ uint32_t cdf_inner(const Elem<K>& e, const QCfg& q, int32_t j) {
  if constexpr (kKind == 3) {
    // binary64 reference: z = (b - mu) / sigma, F and its quantization in binary64
    const double b = (double)(q.lo + j) - 0.5;
    double F = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double z = (b - (double)e.mu[k]) / (double)e.r[k];
      F = __builtin_fma((double)e.w[k], phi_ref(z), F);
    }
    F = __builtin_fmin(F, 1.0);
    return (uint32_t)j + (uint32_t)__builtin_floor(F * (double)(q.M - (uint32_t)q.N));
  } else {
    // (float)j + ((float)lo - 1/2) is the exact value lo + j - 1/2 (both
    // terms and the sum are representable), i.e. the boundary b_j; the
    // scaled value is >= 0, so the truncating conversion is the floor
    const float b = (float)j + q.lo_mh;
    return (uint32_t)j + (uint32_t)cdf_scaled<K, kKind, kFastRecip>(e, q, b);
  }
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

// c_j for j >= 1, with c_j = M for every j >= N (the padded upper part of a
// power-of-two search range).
template <int K, int kKind, bool kFastRecip>
__device__ __forceinline__ uint32_t cdf_upper(const Elem<K>& e, const QCfg& q, int32_t j) {
  const uint32_t c = cdf_inner<K, kKind, kFastRecip>(e, q, j);
  return (j >= q.N) ? q.M : c;
}

// c_j for j in [0, N - 1].
template <int K, int kKind, bool kFastRecip>
__device__ __forceinline__ uint32_t cdf_lower(const Elem<K>& e, const QCfg& q, int32_t j) {
  const uint32_t c = cdf_inner<K, kKind, kFastRecip>(e, q, j);
  return (j <= 0) ? 0u : c;
}

// Device status bits, folded into a status code by the last kernel.
enum : uint32_t { kStRange = 1u, kStCorrupt = 2u, kStNoSpace = 4u, kStInval = 8u };

}  // namespace fgmm
