/*
 * flashgmm.h — C ABI of libflashgmm.so, a GPU (MI355X, gfx950) entropy coder
 * for learned-image-compression latents under a Gaussian-mixture model.
 *
 * It implements the FlashGMM method (Murai, Lin, Katto, arXiv 2509.18815,
 * Sec. III-A): the quantized mixture CDF of every latent element is
 * evaluated on the fly, only where rANS needs it — the coded symbol's two
 * boundaries when encoding, a binary search over the monotone CDF when
 * decoding — instead of building the per-element CDF tables of the classic
 * coder (Sec. II-C, Eqs. (4)-(6)). The symbol model is the bin mass of the
 * K-component mixture of Eq. (2) across the half-integer boundaries of
 * Eq. (1); the coder is rANS with the state map of Eq. (3) (Sec. II-B);
 * the Gaussian CDF is the Abramowitz & Stegun 26.2.17 approximation or the
 * logistic approximation (Sec. III-B).
 *
 * Numerical contract: every CDF value is a fixed binary32 formula with a
 * fixed operation order, so encoder, decoder and any other conforming
 * implementation produce bit-identical bitstreams and symbols.
 *
 * Conventions for every entry point:
 *  - Pointers marked [device] are HIP device pointers; [host] are host
 *    pointers. The caller owns all buffers; the library never frees them.
 *  - Parameter planes are structure-of-arrays: weights, means and scales are
 *    float32 arrays of K*n values, component k of element i at k*n + i.
 *    Element i belongs to rANS stream i mod S at position i div S.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - `ws`/`ws_bytes`: a device workspace of at least gmm_workspace_bytes()
 *    bytes; if ws is NULL the library allocates it on the stream
 *    (hipMallocAsync) and frees it after the call.
 *  - `dev_status` [device, nullable]: if NULL the call synchronises the
 *    stream and returns the status found by the kernels; otherwise the call
 *    is asynchronous, returns GMM_OK after enqueueing, and the kernels store
 *    the call's final status code (an int32) at *dev_status.
 *  - Host-side argument errors are returned immediately, before any launch.
 *  - Preconditions (undefined output, but no out-of-bounds access, if
 *    violated): parameters finite; weights >= 0; scales > 0.
 */
#ifndef FLASHGMM_H
#define FLASHGMM_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define GMM_OK 0
#define GMM_EINVAL 1   /* invalid configuration or argument */
#define GMM_ERANGE 2   /* a symbol lies outside [lo, hi] (no escape coding) */
#define GMM_ECORRUPT 3 /* decode integrity check failed */
#define GMM_ENOSPC 4   /* bitstream capacity smaller than the encoded size */
#define GMM_EDEVICE 5  /* a HIP runtime call failed */
#define GMM_ENOMEM 6   /* workspace allocation failed */

/* Coder configuration (format parameters: encoder and decoder must agree).
 *  K           mixture components, 1..8
 *  lo, hi      alphabet = integers lo..hi, N = hi-lo+1, 2 <= N <= 2^(P-1),
 *              |lo|, |hi| <= 2^22
 *  precision   P, 2..16: quantized frequencies sum to M = 2^P
 *  num_streams S >= 1 interleaved rANS streams
 *  cdf_kind    0 = A&S 26.2.17 Gaussian CDF, 1 = logistic CDF (Sec. III-B) */
typedef struct gmm_cfg {
  int32_t K;
  int32_t lo, hi;
  int32_t precision;
  int32_t num_streams;
  int32_t cdf_kind;
} gmm_cfg;

/* Human-readable name of a status code (static string). */
const char* gmm_status_str(int status);

/* Library version as major*10000 + minor*100 + patch. */
int32_t gmm_version(void);

/* Upper bound of the encoded size of n symbols in S streams, in uint16 words
 * (at most one word per symbol plus the two state words per stream). */
int64_t gmm_encode_max_words(int64_t n, int32_t num_streams);

/* Device workspace needed by gmm_encode (op = 0) or gmm_decode (op = 1) for
 * n elements; -1 on an invalid configuration. */
int64_t gmm_workspace_bytes(const gmm_cfg* cfg, int64_t n, int32_t op);

/* Quantized CDF table c_0..c_N of every element (Sec. II-C, Eqs. (4)-(6),
 * evaluated boundary by boundary with the on-the-fly formula): table
 * [device] is uint32 [n][N+1] row-major. A reference/diagnostic entry point
 * (the coder itself never builds it). */
int gmm_cdf_table(const gmm_cfg* cfg, int64_t n, const float* weights, const float* means,
                  const float* scales, uint32_t* table, void* stream);

/* Inverse quantized CDF (Sec. III-A binary search): for each element i,
 * j_out[i] = the unique j with c_j <= slot[i] < c_{j+1}; slot [device]
 * uint32 [n], each < 2^P (else GMM_EINVAL on the device status); j_out
 * [device] int32 [n]. Synchronous. */
int gmm_inverse_cdf(const gmm_cfg* cfg, int64_t n, const float* weights, const float* means,
                    const float* scales, const uint32_t* slot, int32_t* j_out, void* stream);

/* Encode n symbols [device, int32] with parameter planes [device] into
 * bitstream [device, uint16, capacity_words] and offsets [device, int64,
 * S+1]: segment s occupies words offsets[s] .. offsets[s+1]-1 and
 * offsets[S] is the encoded size. GMM_ERANGE if a symbol is outside
 * [lo, hi]; GMM_ENOSPC if offsets[S] > capacity_words (offsets are still
 * written, the bitstream is not). Bitstream layout per segment: the final
 * 32-bit state as two little-endian uint16 words, then the renormalisation
 * words in the order the decoder reads them. */
int gmm_encode(const gmm_cfg* cfg, int64_t n, const int32_t* symbols, const float* weights,
               const float* means, const float* scales, uint16_t* bitstream,
               int64_t capacity_words, int64_t* offsets, void* ws, int64_t ws_bytes,
               int32_t* dev_status, void* stream);

/* Bracket-search model handle (learned search seed for decode); see
 * gmm_bracket_create. NULL selects the plain binary search. */
typedef struct gmm_bracket gmm_bracket;

/* Decode counters [device]: accumulated (added to) by gmm_decode when a
 * bracket is used. hits/misses count symbols whose bracket contained / did
 * not contain the symbol; wave_all_hit counts wavefront steps on which every
 * active lane hit; wave_steps counts all wavefront steps. */
typedef struct gmm_decode_stats {
  uint64_t hits, misses, wave_all_hit, wave_steps;
} gmm_decode_stats;

/* Decode n symbols [device, int32 out] from bitstream [device, uint16,
 * total_words] and offsets [device, int64, S+1] with the same parameter
 * planes and configuration used to encode. GMM_ECORRUPT if a segment lies
 * outside the bitstream, is shorter than two words, is read past its end
 * (missing words read as 0), does not end in the initial state 2^16, or has
 * unread words. The result equals the plain binary search whether or not a
 * bracket is given. stats [device, nullable]. */
int gmm_decode(const gmm_cfg* cfg, int64_t n, const uint16_t* bitstream, int64_t total_words,
               const int64_t* offsets, const float* weights, const float* means,
               const float* scales, int32_t* symbols, const gmm_bracket* bracket,
               gmm_decode_stats* stats, void* ws, int64_t ws_bytes, int32_t* dev_status,
               void* stream);

#ifdef __cplusplus
}
#endif
#endif
