/*
 * Exhaustive checks behind the monotonicity lemma of the quantized CDF.
 *
 * Kind 0 (A&S): for every binary32 a in (0, 1] (a = |z|/9) it compares the
 * oracle's float tail with the same approximant in binary64 and records the
 * largest relative difference and the extreme tails. Logistic kind: the
 * same for the float tail Phi~(-a) over every binary32 a in [0, 9]. With the
 * hazard bound -d ln T/da >= h of the approximant (checked separately in
 * binary64) this proves that the float tail strictly decreases across every
 * step of at least d in a (2^-14 for kind 0, 2^-11 for the logistic kind);
 * the cap at 1/2 makes the step across z = 0 monotone.
 *
 * Built and run by the CPU tests against liboracle.so.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

float gmm_oracle_phi(float z, int32_t kind);

/* The logistic tail (kind 1) in binary64 with the binary32 slope. */
static double tail64(double a) {
  double e = exp(-(double)0x1.b3b646p+0f * a);
  return e / (1.0 + e);
}

/* Logistic kind: scans the float bit patterns [lo_bits, hi_bits] (non-negative floats).
 * out[0] = max relative error, out[1] = max float tail (a > 0),
 * out[2] = a at the max relative error, out[3] = min float tail (the tail at
 * the clamp a = 9 must be the smallest, since a neighbouring boundary can
 * be clamped onto it from an arbitrarily small distance). */
void lemma_scan(uint32_t lo_bits, uint32_t hi_bits, int kind, double* out) {
  double max_rel = 0.0, max_tail = 0.0, arg = 0.0, min_tail = 1.0;
#pragma omp parallel
  {
    double lrel = 0.0, ltail = 0.0, larg = 0.0, lmin = 1.0;
#pragma omp for schedule(static, 1 << 16)
    for (int64_t b = (int64_t)lo_bits; b <= (int64_t)hi_bits; ++b) {
      uint32_t bits = (uint32_t)b;
      float a;
      memcpy(&a, &bits, 4);
      if (a == 0.0f) continue;
      float tf = gmm_oracle_phi(-a, kind);
      double td = tail64((double)a);
      double rel = fabs((double)tf - td) / td;
      if (rel > lrel) { lrel = rel; larg = a; }
      if (tf > ltail) ltail = tf;
      if (tf < lmin) lmin = tf;
    }
#pragma omp critical
    {
      if (lrel > max_rel) { max_rel = lrel; arg = larg; }
      if (ltail > max_tail) max_tail = ltail;
      if (lmin < min_tail) min_tail = lmin;
    }
  }
  out[0] = max_rel;
  out[1] = max_tail;
  out[2] = arg;
  out[3] = min_tail;
}

float gmm_oracle_exp(float g);
double gmm_oracle_as_tail(float a);

/* Kind 0's tail approximant in binary64, in the scaled variable a = |z|/9
 * with the binary32 constants of the contract: C 2^(-x a^2) q(t),
 * t = 1/(1 + 9p a), q the A&S polynomial, C = 1/sqrt(2 pi). */
static double as_tail64(double a) {
  double t = 1.0 / (1.0 + (double)0x1.0ad9fap+1f * a);
  double q = (double)0x1.548cdep+0f;
  q = q * t + (double)-0x1.d23dd4p+0f;
  q = q * t + (double)0x1.c80ef0p+0f;
  q = q * t + (double)-0x1.6d1f0ep-2f;
  q = q * t + (double)0x1.470bf4p-2f;
  q = q * t;
  return exp2(-(double)0x1.d36ee6p+5f * a * a) / sqrt(2.0 * 3.14159265358979323846) * q;
}

/* Every float a in (0, a(hi_bits)] of kind 0's tail T(a) (the exact product
 * of its two float factors, before the cap): out[0] = largest relative error
 * against as_tail64, out[1] = largest T, out[2] = a there, out[3] = smallest
 * T. */
void as_lemma_scan(uint32_t hi_bits, double* out) {
  double max_rel = 0.0, max_tail = 0.0, arg = 0.0, min_tail = 1.0;
#pragma omp parallel
  {
    double lrel = 0.0, ltail = 0.0, larg = 0.0, lmin = 1.0;
#pragma omp for schedule(static, 1 << 16)
    for (int64_t b = 1; b <= (int64_t)hi_bits; ++b) {
      uint32_t bits = (uint32_t)b;
      float a;
      memcpy(&a, &bits, 4);
      double tf = gmm_oracle_as_tail(a);
      double td = as_tail64((double)a);
      double rel = fabs(tf - td) / td;
      if (rel > lrel) lrel = rel;
      if (tf > ltail) { ltail = tf; larg = a; }
      if (tf < lmin) lmin = tf;
    }
#pragma omp critical
    {
      if (lrel > max_rel) max_rel = lrel;
      if (ltail > max_tail) { max_tail = ltail; arg = larg; }
      if (lmin < min_tail) min_tail = lmin;
    }
  }
  out[0] = max_rel;
  out[1] = max_tail;
  out[2] = arg;
  out[3] = min_tail;
}

static float f_of(uint32_t bits) {
  float a;
  memcpy(&a, &bits, 4);
  return a;
}

/* Scan behind the Polya lemma, over every float u in [0, u(hi_bits)] with
 * g = -u: out[0] = max relative error of exp~(g) against binary64 exp(g);
 * out[1] = min of exp~(g) over u <= ua; out[2] = max of exp~(g) over
 * u >= ub. */
void polya_exp_scan(uint32_t hi_bits, double ua, double ub, double* out) {
  double eps = 0.0, mn = 2.0, mx = 0.0;
#pragma omp parallel for schedule(static, 1 << 16) reduction(max : eps, mx) reduction(min : mn)
  for (int64_t b = 0; b <= (int64_t)hi_bits; ++b) {
    const float u = f_of((uint32_t)b);
    const float e = gmm_oracle_exp(-u);
    const double ref = exp(-(double)u);
    const double rel = fabs((double)e - ref) / ref;
    if (rel > eps) eps = rel;
    if ((double)u <= ua && e < mn) mn = e;
    if ((double)u >= ub && e > mx) mx = e;
  }
  out[0] = eps;
  out[1] = mn;
  out[2] = mx;
}

float gmm_oracle_polya_E(float u);

/* Polya's E = 1 - exp(-u) over every float u in [0, u(hi_bits)]: the
 * largest relative error against binary64 -expm1(-u). */
double polya_E_scan(uint32_t hi_bits) {
  double eta = 0.0;
#pragma omp parallel for schedule(static, 1 << 16) reduction(max : eta)
  for (int64_t b = 1; b <= (int64_t)hi_bits; ++b) {
    const float u = f_of((uint32_t)b);
    const double ref = -expm1(-(double)u);
    const double rel = fabs((double)gmm_oracle_polya_E(u) - ref) / ref;
    if (rel > eta) eta = rel;
  }
  return eta;
}

/* The float tail Phi~(-a) of a CDF kind over every float a in
 * [0, a(hi_bits)]: out[0] = largest, out[1] = smallest value. */
void tail_range_scan(uint32_t hi_bits, int kind, double* out) {
  double mx = 0.0, mn = 1.0;
#pragma omp parallel for schedule(static, 1 << 16) reduction(max : mx) reduction(min : mn)
  for (int64_t b = 0; b <= (int64_t)hi_bits; ++b) {
    const float t = gmm_oracle_phi(-f_of((uint32_t)b), kind);
    if (t > mx) mx = t;
    if (t < mn) mn = t;
  }
  out[0] = mx;
  out[1] = mn;
}
