/*
 * CPU oracle for the GMM rANS entropy coder — TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. It is a plain, slow, obviously correct restatement
 * of the classic table method (FlashGMM paper, Sec. II-C, Eqs. (4)-(6)): the
 * whole quantized CDF column of every latent element is built, encode looks
 * the symbol's two entries up, and decode scans the column linearly.
 * It shares no code, header or constant table with the GPU library; both are
 * written independently from the same written contract (operation order,
 * constants, stream format).
 *
 * All pointers are host pointers. Status codes (same numbers as the GPU
 * library's, fixed by the contract): 0 ok, 1 invalid argument, 2 symbol
 * outside the support, 3 corrupt bitstream, 4 output capacity too small.
 */
#ifndef GMM_ORACLE_H
#define GMM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ERANGE = 2, ORC_ECORRUPT = 3, ORC_ENOSPC = 4 };

typedef struct {
  int32_t K;           /* mixture components, 1..8 */
  int32_t lo, hi;      /* alphabet = the integers lo..hi, N = hi-lo+1 */
  int32_t precision;   /* P: frequencies sum to M = 2^P, 2 <= P <= 16 */
  int32_t num_streams; /* S interleaved rANS streams, S >= 1 */
  int32_t cdf_kind;    /* 0: A&S 26.2.17; 1: logistic; 2: Polya;
                          3: binary64 reference (series / continued fraction) */
  int32_t param_kind;  /* 0: weights, means, scales; 1: raw outputs (weight
                          logits, means, log-scales) mapped per element */
} gmm_oracle_cfg;

/* Gaussian CDF approximation Phi~(z), binary32 contract arithmetic. */
float gmm_oracle_phi(float z, int32_t kind);
/* Kind 0 (A&S 26.2.17): the upper tail in a = |z|/9, a in [0, 1] (the exact
 * product of its two binary32 factors), and one component's signed half
 * Phi~ - 1/2 from d = b - mu and rn = r/9. */
double gmm_oracle_as_tail(float a);
/* out[0..8]: 9p, 1/9, 81 log2(e)/2 and the six density coefficients. */
void gmm_oracle_as_constants(float* out);
float gmm_oracle_as_half(float d, float rn);
/* exp~(g) for g in [-51.6, 7]: Cody-Waite reduction + degree-7 Taylor. */
float gmm_oracle_exp(float g);
/* binary64 exp for g in [-686, 0]; reference Gaussian tail Q(a) = erfc(a/sqrt2)/2
 * for a in [0, 37]; reference Phi(z) (z clamped to [-37, 37]). */
/* Polya's 1 - exp(-u) for u in [0, 51.6] (Taylor series below 1/4). */
float gmm_oracle_polya_E(float u);
double gmm_oracle_exp_d(double g);
double gmm_oracle_tail_ref(double a);
double gmm_oracle_phi_ref(double z);
/* which: 0 exp, 1 tail, 2 phi (the three binary64 functions above). */
void gmm_oracle_ref_batch(const double* x, double* out, int64_t n, int32_t which);
/* Raw network outputs to weights and scales (planes [K][n]): softmax of the
 * logits, sigma = max(exp~(clamp(t, -7, 7)), 0.11) of the log-scales. */
int gmm_oracle_params_from_raw(int32_t K, int64_t n, const float* logits,
                               const float* log_scales, float* w_out, float* sigma_out);
void gmm_oracle_phi_batch(const float* z, float* out, int64_t n, int32_t kind);
void gmm_oracle_exp_batch(const float* g, float* out, int64_t n);

/* Mixture CDF F at every boundary b_j = lo+j-1/2, j = 0..N, after the
 * clamp to 1: out is [n][N+1] row-major. */
int gmm_oracle_F_table(const gmm_oracle_cfg* cfg, int64_t n, const float* w,
                       const float* mu, const float* sig, float* out);
/* Quantized CDF table c_0..c_N per element: out is [n][N+1] row-major. */
int gmm_oracle_cdf_table(const gmm_oracle_cfg* cfg, int64_t n, const float* w,
                         const float* mu, const float* sig, uint32_t* out);

/* rANS encode; offsets has S+1 entries (in 16-bit words). On ORC_ENOSPC the
 * offsets are written (offsets[S] is the size needed), the bitstream is not. */
int gmm_oracle_encode(const gmm_oracle_cfg* cfg, int64_t n, const int32_t* sym,
                      const float* w, const float* mu, const float* sig,
                      uint16_t* bitstream, int64_t capacity_words, int64_t* offsets);
/* rANS decode by linear scan of each element's table column. On a corrupt
 * stream the remaining words read as zero and ORC_ECORRUPT is returned;
 * symbols of a stream whose segment bounds are invalid are set to lo. */
int gmm_oracle_decode(const gmm_oracle_cfg* cfg, int64_t n, const uint16_t* bitstream,
                      int64_t total_words, const int64_t* offsets, const float* w,
                      const float* mu, const float* sig, int32_t* sym);

/* Exact inverse of the quantized CDF at one slot per element (the symbol
 * index j with c_j <= slot < c_{j+1}), by linear scan. */
int gmm_oracle_inverse(const gmm_oracle_cfg* cfg, int64_t n, const float* w,
                       const float* mu, const float* sig, const uint32_t* slot,
                       int32_t* j_out);

int32_t gmm_oracle_num_threads(void);
/* Threads of the oracle's later parallel loops (OpenMP); n >= 1. */
void gmm_oracle_set_num_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
