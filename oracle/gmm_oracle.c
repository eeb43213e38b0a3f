/*
 * CPU oracle for the GMM rANS entropy coder — TEST INFRASTRUCTURE ONLY.
 * (Loaded by the tests, the smoke check and the benchmark's CPU baseline;
 * never by the GPU library or its Python binding.)
 *
 * What it computes, and where the paper defines it (FlashGMM, Murai, Lin,
 * Katto, arXiv 2509.18815):
 *   - Sec. II-A, Eq. (1) and Eq. (2): a latent element's probability model
 *     is a K-component Gaussian mixture, and the mass of the integer symbol
 *     y is the mixture CDF difference across the half-integer boundaries
 *     y-1/2 and y+1/2.
 *   - Sec. II-C, Eqs. (4)-(6): the classic coder builds, per element, the
 *     table T_i of cumulative masses over the whole alphabet; by telescoping,
 *     its j-th entry is the mixture CDF at one boundary. This oracle builds
 *     that column for every element (O(K |y| |Y|)) and uses it for encode
 *     (lookup) and decode (linear search of the column).
 *   - Sec. II-B, Eq. (3): the rANS state map C(s,x) = m floor(x/l_s) + b_s +
 *     mod(x, l_s) with m = 2^P, l_s = the symbol's frequency, b_s = its
 *     cumulative frequency.
 *   - Sec. III-B: the Gaussian CDF is replaced by a closed-form approximation:
 *     the Abramowitz & Stegun 26.2.17 polynomial (default), the logistic
 *     function 1/(1+exp(-1.702 x)) or Polya's formula; Table II compares
 *     them with an unapproximated erfc, for which cdf_kind 3 evaluates the
 *     Gaussian CDF in binary64 from the Maclaurin series of erf and the
 *     Laplace continued fraction of erfc.
 *   - Sec. I and II-A: the mixture parameters come from a network; with
 *     param_kind 1 the inputs are its raw outputs (weight logits, means,
 *     log-scales), mapped here by a softmax and an exponential with the
 *     scale lower bound 0.11 that Sec. II-B quotes for scale tables.
 * The paper fixes no float format, rANS word size, stream layout or CDF
 * quantization; the readings taken here (binary32 with a fixed operation
 * order, 32-bit state with 16-bit renormalisation, round-robin interleaved
 * streams, c_j = j + floor(F (M-N))) are the written contract that the GPU
 * library also implements, independently.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp (no FMA
 * contraction: every fused multiply-add below is an explicit fmaf).
 */
#include "gmm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- constants: each is the binary32 value nearest the stated real ---- */
/* A&S 26.2.17 (Handbook of Mathematical Functions, Sec. 26.2.17). */
static const float AS_B1 = 0x1.470bf4p-2f; /* 0.319381530 */
static const float AS_B2 = -0x1.6d1f0ep-2f; /* -0.356563782 */
static const float AS_B3 = 0x1.c80ef0p+0f; /* 1.781477937 */
static const float AS_B4 = -0x1.d23dd4p+0f; /* -1.821255978 */
static const float AS_B5 = 0x1.548cdep+0f; /* 1.330274429 */
/* A&S in the variable a = |z| / 9 (so the clamp |z| <= 9 is a <= 1), with
 * the Gaussian density written C 2^(-x), x = (81 log2(e) / 2) a^2, C the
 * density at 0. */
static const float AS_P9 = 0x1.0ad9fap+1f;    /* 9 p, p = 0.2316419 */
static const float INV_NINE = 0x1.c71c72p-4f; /* 1/9 */
static const float AS_X = 0x1.d36ee6p+5f;     /* 81 log2(e) / 2 = 58.42915 */
static const float TWO23_HALF = 0x1.8p+23f;   /* 1.5 * 2^23 */
/* C 2^(-g) on [-1/2, 1/2]: the degree-7 Taylor polynomial sum_k c_k g^k,
 * c_k = C (-ln 2)^k / k!, economized (Lanczos) to degree 5 by replacing
 * g^7 and g^6 with their Chebyshev expansions on [-1/2, 1/2] less the T7
 * and T6 terms (g^7 = T7(2g)/8192 + (7/16) g^5 - (7/128) g^3 + (7/4096) g;
 * g^6 = T6(2g)/2048 + (3/8) g^4 - (9/256) g^2 + 1/2048):
 * coefficient k below is the binary32 nearest the resulting real. */
static const float DENS_T[6] = {0x1.988456p-2f,  -0x1.1b2990p-2f, 0x1.88899ap-4f,
                                -0x1.6ac8cep-6f, 0x1.f9f438p-9f,  -0x1.184804p-11f};
/* logistic approximation slope (paper Sec. III-B, third candidate) */
static const float LOGISTIC_K = 0x1.b3b646p+0f; /* 1.702 */
/* exp~: Cody & Waite argument reduction, ln 2 split in two parts. */
static const float LOG2E = 0x1.715476p+0f;   /* 1/ln 2 */
static const float LN2_HI = 0x1.62e4p-1f;    /* ln 2 truncated to 16 significant bits */
static const float LN2_LO = 0x1.7f7d1cp-20f; /* ln 2 - LN2_HI */
static const float INV_FACT3 = 0x1.555556p-3f;  /* 1/3! */
static const float INV_FACT4 = 0x1.555556p-5f;  /* 1/4! */
static const float INV_FACT5 = 0x1.111112p-7f;  /* 1/5! */
static const float INV_FACT6 = 0x1.6c16c2p-10f; /* 1/6! */
static const float INV_FACT7 = 0x1.a01a02p-13f; /* 1/7! */
static const float INV_FACT8 = 0x1.a01a02p-16f; /* 1/8! */
/* Polya: Phi(x) ~ (1 + sign(x) sqrt(1 - exp(-2 x^2 / pi))) / 2 */
static const float POLYA_C = 0x1.45f306p-1f; /* 2/pi */
/* raw-output mapping: scale lower bound and clamps */
static const float SCALE_MIN = 0x1.c28f5cp-4f; /* 0.11 */

/* binary64 reference CDF (cdf_kind 3): each the binary64 value nearest the
 * stated real; LN2_HI_D keeps 42 significant bits of ln 2, so n * LN2_HI_D
 * is exact for |n| < 2^11. */
static const double LOG2E_D = 0x1.71547652b82fep+0;
static const double LN2_HI_D = 0x1.62e42fefa38p-1;
static const double LN2_LO_D = 0x1.ef35793c7673p-45;
static const double INV_SQRT2_D = 0x1.6a09e667f3bcdp-1;     /* 1/sqrt(2) */
static const double INV_SQRT_PI_D = 0x1.20dd750429b6dp-1;   /* 1/sqrt(pi) */
static const double HALF_INV_SQRT_PI_D = 0x1.20dd750429b6dp-2; /* 1/(2 sqrt(pi)) */
/* 1/k! for k = 0..13 */
static const double INV_FACT_D[14] = {
    1.0, 1.0, 0x1p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5, 0x1.1111111111111p-7,
    0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16,
    0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26,
    0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};
#define ERF_TERMS 32  /* Maclaurin terms of erf(x), used for x < 2 */
#define ERFC_CF_DEPTH 50 /* Laplace continued-fraction levels, x >= 2 */

/* exp(g) for g in [-51.6, 7] (the range the contract uses; the result is a
 * normal float): n = rint(g / ln 2), r = g - n ln 2 (two fused steps, exact
 * high part), then the Taylor polynomial sum_{k<=7} r^k / k! by Horner,
 * scaled by 2^n. */
float gmm_oracle_exp(float g) {
  float n = rintf(g * LOG2E);
  float r = fmaf(-n, LN2_HI, g);
  r = fmaf(-n, LN2_LO, r);
  float p = INV_FACT7;
  p = fmaf(p, r, INV_FACT6);
  p = fmaf(p, r, INV_FACT5);
  p = fmaf(p, r, INV_FACT4);
  p = fmaf(p, r, INV_FACT3);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  return ldexpf(p, (int)n);
}

/* Kind 0's upper tail in the scaled variable a = |z|/9, a in [0, 1]
 * (A&S 26.2.17 with t = 1/(1 + 9p a)), as the two binary32 factors whose
 * product it is: the polynomial factor q and the density factor C 2^(-x),
 * x = AS_X a^2. The density is taken apart as x = n + g with n the integer
 * nearest x (read off the binary32 sum 1.5 2^23 - x, whose unit is 1) and
 * g = x - n in [-1/2, 1/2]; C 2^(-g) is the degree-5 polynomial above, and
 * 2^(-n) an exact power-of-two scaling. */
static void as_factors(float a, float* dens, float* q) {
  float u = fmaf(a, AS_P9, 1.0f);
  float t = 1.0f / u;
  float h = fmaf(AS_B5, t, AS_B4);
  h = fmaf(h, t, AS_B3);
  h = fmaf(h, t, AS_B2);
  h = fmaf(h, t, AS_B1);
  *q = h * t;
  float x2 = a * a;
  float s = fmaf(-x2, AS_X, TWO23_HALF); /* 1.5 2^23 - rint(x) */
  float negn = s - TWO23_HALF;           /* -rint(x), exact */
  float g = fmaf(x2, AS_X, negn);        /* x - rint(x) */
  float e = DENS_T[5];
  for (int k = 4; k >= 0; --k) e = fmaf(e, g, DENS_T[k]);
  *dens = ldexpf(e, (int)negn);
}

/* The tail as the exact product of its two factors (a binary64 holds the
 * product of two binary32 values exactly); the mixture uses it only inside
 * the fused 1/2 - dens q. */
double gmm_oracle_as_tail(float a) {
  float dens, q;
  as_factors(a, &dens, &q);
  return (double)dens * (double)q;
}

/* The kind-0 constants, for the tests that pin them to their definitions:
 * out[0..8] = 9p, 1/9, 81 log2(e)/2, then the density coefficients 0..5. */
void gmm_oracle_as_constants(float* out) {
  out[0] = AS_P9;
  out[1] = INV_NINE;
  out[2] = AS_X;
  for (int k = 0; k < 6; ++k) out[3 + k] = DENS_T[k];
}

/* One component's contribution Phi~(z) - 1/2 to the kind-0 mixture, from
 * d = b - mu and rn = r/9: a = min(|d| rn, 1); D = 1/2 - T rounded once
 * (a fused multiply-add of the two factors) and floored at 0 (the tail
 * exceeds 1/2 at tiny a), signed like d: Phi(z) - 1/2 = sign(z) (1/2 -
 * T(|z|)). */
float gmm_oracle_as_half(float d, float rn) {
  float a = fminf(fabsf(d) * rn, 1.0f);
  float dens, q;
  as_factors(a, &dens, &q);
  float D = fmaxf(fmaf(-dens, q, 0.5f), 0.0f);
  return copysignf(D, d);
}

/* Upper tail of the logistic approximation: 1 - 1/(1+exp(-k a)) =
 * e/(1+e) with e = exp(-k a). */
static float tail_logistic(float a) {
  float g = a * -LOGISTIC_K;
  float e = gmm_oracle_exp(g);
  return e / (1.0f + e);
}

/* Upper tail of Polya's approximation for a >= 0,
 *   T(a) = (1 - sqrt(1 - exp(-u))) / 2 = (exp(-u)/2) / (1 + sqrt(E)),
 *   u = (2/pi) a^2, E = 1 - exp(-u) = -expm1(-u),
 * in the rationalised form, so neither end cancels: E comes from its Taylor
 * series u (1 - u/2! + u^2/3! - ... - u^7/8!) for u < 1/4 and from
 * 1 - exp~(-u) above. T moves with e = exp~(-u) and against E, each step
 * being a correctly rounded monotone operation. */
float gmm_oracle_polya_E(float u) {
  float g = -u;
  if (u < 0.25f) {
    float p = INV_FACT8;
    p = fmaf(p, g, INV_FACT7);
    p = fmaf(p, g, INV_FACT6);
    p = fmaf(p, g, INV_FACT5);
    p = fmaf(p, g, INV_FACT4);
    p = fmaf(p, g, INV_FACT3);
    p = fmaf(p, g, 0.5f);
    p = fmaf(p, g, 1.0f);
    return u * p;
  }
  return 1.0f - gmm_oracle_exp(g);
}

static float tail_polya(float a) {
  float m = a * a;
  float u = m * POLYA_C;
  float e = gmm_oracle_exp(-u);
  float E = gmm_oracle_polya_E(u);
  float s = sqrtf(E);
  float h = e * 0.5f;
  return h / (1.0f + s);
}

/* exp(g) in binary64 for g in [-686, 0] (result normal): n = rint(g/ln 2),
 * r = g - n ln 2 in two fused steps, Taylor polynomial of degree 13 by
 * Horner (|r| <= 0.35, truncation below 2^-57), times 2^n. */
double gmm_oracle_exp_d(double g) {
  double n = rint(g * LOG2E_D);
  double r = fma(-n, LN2_HI_D, g);
  r = fma(-n, LN2_LO_D, r);
  double p = INV_FACT_D[13];
  for (int k = 12; k >= 0; --k) p = fma(p, r, INV_FACT_D[k]);
  return ldexp(p, (int)n);
}

/* Upper Gaussian tail Q(a) = erfc(a / sqrt 2) / 2 for a in [0, 37], binary64.
 * With x = a / sqrt 2 and y = x^2:
 *   x < 2:  erf(x) = (2/sqrt pi) x sum_{n>=0} (-y)^n / (n! (2n+1))  (Maclaurin
 *           series), the sum nested as s_{n-1} = 1/(2n-1) - (y/n) s_n from
 *           s_N = 1/(2N+1); Q = 1/2 - x s / sqrt pi;
 *   x >= 2: erfc(x) = exp(-y) / sqrt(pi) / (x + (1/2)/(x + 1/(x + (3/2)/(x +
 *           ...)))) (Laplace's continued fraction), evaluated bottom-up
 *           from a fixed depth; Q = exp(-y) / (2 sqrt pi) / u.
 * Relative error below 1e-12 on [0, 37] (series cancellation near x = 2 is
 * the largest term), far under the 7.5e-8 of A&S 26.2.17. */
double gmm_oracle_tail_ref(double a) {
  double x = a * INV_SQRT2_D;
  double y = x * x;
  if (x < 2.0) {
    double s = 1.0 / (2 * ERF_TERMS + 1);
    for (int n = ERF_TERMS; n >= 1; --n) {
      double v = y * (1.0 / n);
      s = fma(-v, s, 1.0 / (2 * n - 1));
    }
    double t1 = x * s;
    return fma(-INV_SQRT_PI_D, t1, 0.5);
  }
  double u = x;
  for (int m = ERFC_CF_DEPTH; m >= 1; --m) u = x + (0.5 * m) / u;
  double e = gmm_oracle_exp_d(-y);
  double t2 = e * HALF_INV_SQRT_PI_D;
  return t2 / u;
}

/* Reference Gaussian CDF, binary64: z clamped to [-37, 37] (so exp stays
 * normal); Phi(-a) = Q(a), Phi(a) = 1 - Q(a). */
double gmm_oracle_phi_ref(double z) {
  z = fmin(fmax(z, -37.0), 37.0);
  double a = fabs(z);
  double q = gmm_oracle_tail_ref(a);
  return (z < 0.0) ? q : 1.0 - q;
}

/* Phi~(z): clamp z to [-9, 9]; Phi(-a) = tail(a) and Phi(a) = 1 - tail(a).
 * The float A&S tail slightly exceeds 1/2 for tiny a (its coefficients sum
 * to just over sqrt(pi/2) after rounding), which would make Phi~ step down
 * across z = 0; capping the tail at 1/2 keeps Phi~ non-decreasing there.
 * Kind 0 enters the mixture as its signed half (above); as a function of z
 * on its own it is 1/2 + that half with rn = 1/9. */
float gmm_oracle_phi(float z, int32_t kind) {
  if (kind == 3) return (float)gmm_oracle_phi_ref((double)z);
  if (kind == 0) return 0.5f + gmm_oracle_as_half(z, INV_NINE);
  z = fminf(fmaxf(z, -9.0f), 9.0f);
  float a = fabsf(z);
  float tail = (kind == 1) ? tail_logistic(a) : tail_polya(a);
  tail = fminf(tail, 0.5f);
  return (z < 0.0f) ? tail : 1.0f - tail;
}

void gmm_oracle_phi_batch(const float* z, float* out, int64_t n, int32_t kind) {
  for (int64_t i = 0; i < n; ++i) out[i] = gmm_oracle_phi(z[i], kind);
}

void gmm_oracle_ref_batch(const double* x, double* out, int64_t n, int32_t which) {
  for (int64_t i = 0; i < n; ++i)
    out[i] = (which == 0) ? gmm_oracle_exp_d(x[i])
             : (which == 1) ? gmm_oracle_tail_ref(x[i])
                            : gmm_oracle_phi_ref(x[i]);
}

void gmm_oracle_exp_batch(const float* g, float* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = gmm_oracle_exp(g[i]);
}

int32_t gmm_oracle_num_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

void gmm_oracle_set_num_threads(int32_t n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------- configuration checks ---------------- */
static int check_cfg(const gmm_oracle_cfg* c, int64_t n) {
  if (!c || n < 0) return ORC_EINVAL;
  if (c->K < 1 || c->K > 8) return ORC_EINVAL;
  if (c->precision < 2 || c->precision > 16) return ORC_EINVAL;
  if (c->num_streams < 1) return ORC_EINVAL;
  if (c->cdf_kind < 0 || c->cdf_kind > 3) return ORC_EINVAL;
  if (c->param_kind != 0 && c->param_kind != 1) return ORC_EINVAL;
  if (c->lo < -(1 << 22) || c->hi > (1 << 22) || c->hi <= c->lo) return ORC_EINVAL;
  int64_t N = (int64_t)c->hi - c->lo + 1;
  int64_t M = (int64_t)1 << c->precision;
  if (N < 2 || N > M / 2) return ORC_EINVAL;
  return ORC_OK;
}

/* Raw network outputs of one element to mixture weights and scales:
 *   weights: softmax of the logits l_k, as m = max_k l_k (in component
 *            order), e_k = exp~(max(l_k - m, -40.5)), s = e_0 + e_1 + ...
 *            (in order), w_k = e_k / s;
 *   scales:  sigma_k = max(exp~(min(max(t_k, -7), 7)), 0.11) from the
 *            log-scale t_k. */
static void raw_to_params(int K, const float* l, const float* t, float* w, float* sg) {
  float m = l[0];
  for (int k = 1; k < K; ++k) m = fmaxf(m, l[k]);
  float e[8] = {0};
  for (int k = 0; k < K; ++k) e[k] = gmm_oracle_exp(fmaxf(l[k] - m, -40.5f));
  float s = e[0];
  for (int k = 1; k < K; ++k) s = s + e[k];
  for (int k = 0; k < K; ++k) w[k] = e[k] / s;
  for (int k = 0; k < K; ++k)
    sg[k] = fmaxf(gmm_oracle_exp(fminf(fmaxf(t[k], -7.0f), 7.0f)), SCALE_MIN);
}

int gmm_oracle_params_from_raw(int32_t K, int64_t n, const float* logits,
                               const float* log_scales, float* w_out, float* sigma_out) {
  if (K < 1 || K > 8 || n < 0) return ORC_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    float l[8], t[8], w[8], sg[8];
    for (int k = 0; k < K; ++k) {
      l[k] = logits[(int64_t)k * n + i];
      t[k] = log_scales[(int64_t)k * n + i];
    }
    raw_to_params(K, l, t, w, sg);
    for (int k = 0; k < K; ++k) {
      w_out[(int64_t)k * n + i] = w[k];
      sigma_out[(int64_t)k * n + i] = sg[k];
    }
  }
  return ORC_OK;
}

/* One element's parameters after the per-element clamps: scale to
 * [2^-10, 2^10] (kept in s) and its reciprocal r, weights below 2^-60 to
 * zero. With param_kind 1 the planes hold raw outputs, mapped first. */
typedef struct {
  float w[8], mu[8], r[8], s[8];
  float rn[8]; /* r/9 (kind 0) */
  float hw;    /* (w'_0 + ... + w'_{K-1}) / 2, summed in order (kind 0) */
} elem_params;

static void load_elem(const gmm_oracle_cfg* c, int64_t n, int64_t i, const float* w,
                      const float* mu, const float* sig, elem_params* e) {
  float wv[8], sv[8];
  for (int k = 0; k < c->K; ++k) {
    wv[k] = w[(int64_t)k * n + i];
    sv[k] = sig[(int64_t)k * n + i];
  }
  if (c->param_kind == 1) {
    float l[8], t[8];
    for (int k = 0; k < c->K; ++k) {
      l[k] = wv[k];
      t[k] = sv[k];
    }
    raw_to_params(c->K, l, t, wv, sv);
  }
  for (int k = 0; k < c->K; ++k) {
    float s = fminf(fmaxf(sv[k], 0x1p-10f), 0x1p10f);
    e->s[k] = s;
    e->r[k] = 1.0f / s;
    e->w[k] = (wv[k] < 0x1p-60f) ? 0.0f : wv[k];
    e->mu[k] = mu[(int64_t)k * n + i];
    e->rn[k] = e->r[k] * INV_NINE;
  }
  float ws = e->w[0];
  for (int k = 1; k < c->K; ++k) ws = ws + e->w[k];
  e->hw = 0.5f * ws;
}

/* Mixture CDF sum_k w_k Phi~((b - mu_k)/sigma_k) at boundary j, components
 * accumulated in order with fused multiply-adds, clamped to [0, 1]. Kind 0
 * writes each Phi~ as 1/2 + (Phi~ - 1/2): the halves sum to hw, the start
 * of the accumulation, and each component adds w_k times its signed half. */
static float mixture_F(const gmm_oracle_cfg* c, const elem_params* e, int64_t j) {
  float b = (float)(c->lo + j) - 0.5f;
  if (c->cdf_kind == 0) {
    float F = e->hw;
    for (int k = 0; k < c->K; ++k)
      F = fmaf(e->w[k], gmm_oracle_as_half(b - e->mu[k], e->rn[k]), F);
    return fminf(fmaxf(F, 0.0f), 1.0f);
  }
  float F = 0.0f;
  for (int k = 0; k < c->K; ++k) {
    float z = (b - e->mu[k]) * e->r[k];
    F = fmaf(e->w[k], gmm_oracle_phi(z, c->cdf_kind), F);
  }
  return fminf(F, 1.0f);
}

/* The same mixture in binary64 with the reference CDF (cdf_kind 3):
 * z_k = (b - mu_k) / sigma_k with a binary64 division. */
static double mixture_F_ref(const gmm_oracle_cfg* c, const elem_params* e, int64_t j) {
  double b = (double)(c->lo + j) - 0.5;
  double F = 0.0;
  for (int k = 0; k < c->K; ++k) {
    double z = (b - (double)e->mu[k]) / (double)e->s[k];
    F = fma((double)e->w[k], gmm_oracle_phi_ref(z), F);
  }
  return fmin(F, 1.0);
}

/* Quantized CDF column: c_0 = 0, c_N = M, and for 0 < j < N
 * c_j = j + floor(F_j (M - N)) (in binary64 for cdf_kind 3), which is
 * strictly increasing (every symbol keeps frequency >= 1) because F_j does
 * not decrease with j. */
static void build_column(const gmm_oracle_cfg* c, const elem_params* e, uint32_t* col) {
  int64_t N = (int64_t)c->hi - c->lo + 1;
  uint32_t M = 1u << c->precision;
  float span = (float)(M - (uint32_t)N);
  col[0] = 0;
  for (int64_t j = 1; j < N; ++j) {
    if (c->cdf_kind == 3) {
      double F = mixture_F_ref(c, e, j);
      col[j] = (uint32_t)j + (uint32_t)floor(F * (double)(M - (uint32_t)N));
    } else {
      float F = mixture_F(c, e, j);
      col[j] = (uint32_t)j + (uint32_t)floorf(F * span);
    }
  }
  col[N] = M;
}

int gmm_oracle_F_table(const gmm_oracle_cfg* c, int64_t n, const float* w, const float* mu,
                       const float* sig, float* out) {
  int st = check_cfg(c, n);
  if (st) return st;
  int64_t N = (int64_t)c->hi - c->lo + 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    elem_params e;
    load_elem(c, n, i, w, mu, sig, &e);
    for (int64_t j = 0; j <= N; ++j)
      out[i * (N + 1) + j] =
          (c->cdf_kind == 3) ? (float)mixture_F_ref(c, &e, j) : mixture_F(c, &e, j);
  }
  return ORC_OK;
}

int gmm_oracle_cdf_table(const gmm_oracle_cfg* c, int64_t n, const float* w, const float* mu,
                         const float* sig, uint32_t* out) {
  int st = check_cfg(c, n);
  if (st) return st;
  int64_t N = (int64_t)c->hi - c->lo + 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    elem_params e;
    load_elem(c, n, i, w, mu, sig, &e);
    build_column(c, &e, out + i * (N + 1));
  }
  return ORC_OK;
}

/* Element i belongs to stream i mod S at position i div S. */
static int64_t stream_len(int64_t n, int64_t S, int64_t s) {
  return (s < n) ? (n - 1 - s) / S + 1 : 0;
}

int gmm_oracle_inverse(const gmm_oracle_cfg* c, int64_t n, const float* w, const float* mu,
                       const float* sig, const uint32_t* slot, int32_t* j_out) {
  int st = check_cfg(c, n);
  if (st) return st;
  int64_t N = (int64_t)c->hi - c->lo + 1;
  uint32_t M = 1u << c->precision;
  for (int64_t i = 0; i < n; ++i)
    if (slot[i] >= M) return ORC_EINVAL;
#pragma omp parallel
  {
    uint32_t* col = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(N + 1));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      elem_params e;
      load_elem(c, n, i, w, mu, sig, &e);
      build_column(c, &e, col);
      int64_t j = 0;
      while (col[j + 1] <= slot[i]) ++j;
      j_out[i] = (int32_t)j;
    }
    free(col);
  }
  return ORC_OK;
}

int gmm_oracle_encode(const gmm_oracle_cfg* c, int64_t n, const int32_t* sym, const float* w,
                      const float* mu, const float* sig, uint16_t* bitstream,
                      int64_t capacity_words, int64_t* offsets) {
  int st = check_cfg(c, n);
  if (st) return st;
  for (int64_t i = 0; i < n; ++i)
    if (sym[i] < c->lo || sym[i] > c->hi) return ORC_ERANGE;
  const int64_t S = c->num_streams;
  const int64_t N = (int64_t)c->hi - c->lo + 1;
  const int P = c->precision;

  /* Words of stream s are kept in emission order in tmp[base[s] ...]. */
  int64_t* base = (int64_t*)malloc(sizeof(int64_t) * (size_t)(S + 1));
  int64_t* count = (int64_t*)malloc(sizeof(int64_t) * (size_t)S);
  uint32_t* xfin = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)S);
  base[0] = 0;
  for (int64_t s = 0; s < S; ++s) base[s + 1] = base[s] + stream_len(n, S, s);
  uint16_t* tmp = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)(n > 0 ? n : 1));

#pragma omp parallel
  {
    uint32_t* col = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(N + 1));
#pragma omp for schedule(dynamic, 16)
    for (int64_t s = 0; s < S; ++s) {
      uint32_t x = 1u << 16;
      int64_t cnt = 0;
      /* rANS codes in reverse so that the decoder reads forward. */
      for (int64_t p = stream_len(n, S, s) - 1; p >= 0; --p) {
        int64_t i = s + p * S;
        elem_params e;
        load_elem(c, n, i, w, mu, sig, &e);
        build_column(c, &e, col);
        int64_t j = sym[i] - c->lo;
        uint32_t cj = col[j];
        uint32_t f = col[j + 1] - col[j];
        /* keep x below f 2^(32-P) so the update stays in [2^16, 2^32) */
        if (x >= (f << (32 - P))) {
          tmp[base[s] + cnt++] = (uint16_t)(x & 0xFFFFu);
          x >>= 16;
        }
        x = ((x / f) << P) + (x % f) + cj; /* Eq. (3) */
      }
      xfin[s] = x;
      count[s] = cnt;
    }
    free(col);
  }

  offsets[0] = 0;
  for (int64_t s = 0; s < S; ++s) offsets[s + 1] = offsets[s] + 2 + count[s];
  if (offsets[S] > capacity_words) {
    st = ORC_ENOSPC;
  } else {
    for (int64_t s = 0; s < S; ++s) {
      uint16_t* seg = bitstream + offsets[s];
      seg[0] = (uint16_t)(xfin[s] & 0xFFFFu);
      seg[1] = (uint16_t)(xfin[s] >> 16);
      for (int64_t t = 0; t < count[s]; ++t) seg[2 + t] = tmp[base[s] + count[s] - 1 - t];
    }
  }
  free(base);
  free(count);
  free(xfin);
  free(tmp);
  return st;
}

int gmm_oracle_decode(const gmm_oracle_cfg* c, int64_t n, const uint16_t* bitstream,
                      int64_t total_words, const int64_t* offsets, const float* w,
                      const float* mu, const float* sig, int32_t* sym) {
  int st = check_cfg(c, n);
  if (st) return st;
  if (total_words < 0) return ORC_EINVAL;
  const int64_t S = c->num_streams;
  const int64_t N = (int64_t)c->hi - c->lo + 1;
  const int P = c->precision;
  const uint32_t M = 1u << P;
  int corrupt = 0;

#pragma omp parallel reduction(| : corrupt)
  {
    uint32_t* col = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(N + 1));
#pragma omp for schedule(dynamic, 16)
    for (int64_t s = 0; s < S; ++s) {
      int64_t ns = stream_len(n, S, s);
      int64_t a = offsets[s], b = offsets[s + 1];
      if (a < 0 || b < a + 2 || b > total_words) {
        for (int64_t p = 0; p < ns; ++p) sym[s + p * S] = c->lo;
        corrupt = 1;
        continue;
      }
      uint32_t x = (uint32_t)bitstream[a] | ((uint32_t)bitstream[a + 1] << 16);
      int64_t ptr = a + 2;
      int bad = (x < (1u << 16));
      for (int64_t p = 0; p < ns; ++p) {
        int64_t i = s + p * S;
        elem_params e;
        load_elem(c, n, i, w, mu, sig, &e);
        build_column(c, &e, col);
        uint32_t slot = x & (M - 1);
        int64_t j = 0;
        while (col[j + 1] <= slot) ++j; /* linear search of the column */
        sym[i] = (int32_t)(c->lo + j);
        uint32_t f = col[j + 1] - col[j];
        x = f * (x >> P) + slot - col[j];
        if (x < (1u << 16)) {
          uint32_t word = 0;
          if (ptr < b) word = bitstream[ptr++];
          else bad = 1;
          x = (x << 16) | word;
        }
      }
      if (x != (1u << 16) || ptr != b) bad = 1;
      if (bad) corrupt = 1;
    }
    free(col);
  }
  return corrupt ? ORC_ECORRUPT : ORC_OK;
}
