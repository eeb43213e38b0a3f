/*
 * Exhaustive check behind the monotonicity lemma of the quantized CDF.
 *
 * For every binary32 a in [0, 9] it compares the oracle's float upper tail
 * (Phi~(-a), the branch used for z < 0) with the same approximant evaluated
 * in binary64, and records the largest relative difference and the largest
 * float tail. With the hazard bound -d ln Q/da >= h of the approximant
 * (checked separately in binary64) this proves that the float tail strictly
 * decreases across every step of at least 2^-11 in a, and the bound
 * tail <= 1/2 makes the step across z = 0 monotone.
 *
 * Built and run by the CPU tests against liboracle.so.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

float gmm_oracle_phi(float z, int32_t kind);

static double tail64(double a, int kind) {
  if (kind == 1) {
    double e = exp(-(double)0x1.b3b646p+0f * a);
    return e / (1.0 + e);
  }
  double t = 1.0 / (1.0 + (double)0x1.da6712p-3f * a);
  double q = (double)0x1.548cdep+0f;
  q = q * t + (double)-0x1.d23dd4p+0f;
  q = q * t + (double)0x1.c80ef0p+0f;
  q = q * t + (double)-0x1.6d1f0ep-2f;
  q = q * t + (double)0x1.470bf4p-2f;
  q = q * t;
  return exp(-0.5 * a * a) / sqrt(2.0 * 3.14159265358979323846) * q;
}

/* Scans the float bit patterns [lo_bits, hi_bits] (non-negative floats).
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
      double td = tail64((double)a, kind);
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
