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

/* ---- Batched coding of many latents (plans) ----
 * A plan fixes the common configuration (cfg with num_streams ignored) and
 * the shapes of B latents: n_b[b] elements coded in S_b[b] streams. Its
 * encode (op = 0) or decode (op = 1) of the whole batch runs as one hipGraph
 * of persistent kernels that share the latents' streams across the chip
 * (longest streams first from an atomic work queue). Each latent's
 * bitstream, offsets and symbols are exactly those of gmm_encode /
 * gmm_decode with cfg.num_streams = S_b[b]. Not part of the paper: a
 * throughput form for serving many images at once. */
typedef struct gmm_plan gmm_plan;

/* Flag for gmm_plan_create: time every candidate launch shape (lanes per
 * stream, schedule, waves per compute unit) on the real shapes at the first
 * gmm_plan_exec and keep the fastest; with the environment variable
 * FLASHGMM_TUNE_CACHE naming a file, results are cached there by shape
 * signature. Without it a fixed default shape is used. */
#define GMM_PLAN_AUTOTUNE 1

/* Buffers of one latent for gmm_plan_exec (all [device]):
 *  symbols   encode input, int32 [n]
 *  weights, means, scales   parameter planes, float32 [K][n]
 *  bitstream encode output / decode input, uint16
 *  words     encode: capacity of bitstream in words; decode: its length
 *  offsets   int64 [S+1]: encode output / decode input
 *  decoded   decode output, int32 [n] */
typedef struct gmm_latent_io {
  const int32_t* symbols;
  const float* weights;
  const float* means;
  const float* scales;
  uint16_t* bitstream;
  int64_t words;
  int64_t* offsets;
  int32_t* decoded;
} gmm_latent_io;

/* Chosen launch shape of a plan (after its first execution). schedule:
 * 0 one work item per workgroup, 1 persistent with an atomic queue,
 * 2 persistent with a static round-robin assignment. */
typedef struct gmm_plan_info_t {
  int32_t tuned, lanes_per_stream, schedule, waves_per_cu, candidates, graph_captured;
  double best_ms;
} gmm_plan_info_t;

/* Creates a plan (allocates its device workspace and tables). *out [host]
 * receives the handle; release it with gmm_plan_destroy. */
int gmm_plan_create(const gmm_cfg* common, int32_t B, const int64_t* n_b, const int32_t* S_b,
                    int32_t op, int32_t flags, gmm_plan** out);

/* Runs the plan on io [host array of B]. dev_status [device, int32 [B],
 * nullable]: if NULL the call synchronises and returns the first failing
 * latent's status (or GMM_OK); otherwise it is asynchronous and the
 * per-latent status codes are stored there. The first call tunes (with
 * GMM_PLAN_AUTOTUNE) and captures the graph; a call with buffers different
 * from the previous call's synchronises the stream before refreshing the
 * plan's descriptor table. */
int gmm_plan_exec(gmm_plan* plan, const gmm_latent_io* io, int32_t* dev_status, void* stream);

/* Reports the plan's chosen launch shape. */
int gmm_plan_info(const gmm_plan* plan, gmm_plan_info_t* info);

/* Forces a launch shape (skipping the tuner) and drops the captured graph;
 * the next gmm_plan_exec captures again. lanes 1, 2, 4, 8 or 16 (decode
 * only; encode requires 1), schedule 0..2, waves_per_cu 1..64. For tests
 * and sweeps: the output never depends on it. */
int gmm_plan_set_config(gmm_plan* plan, int32_t lanes, int32_t schedule, int32_t waves_per_cu);

/* The tuner's candidate launch shapes: writes up to max_count triples
 * (lanes, schedule, waves_per_cu) to out [host, int32 3*max_count] and
 * returns the number of candidates (-1 on a NULL plan). */
int gmm_plan_candidates(const gmm_plan* plan, int32_t* out, int32_t max_count);

/* Releases a plan (waits for its work to finish). */
int gmm_plan_destroy(gmm_plan* plan);

/* Launch shape of later gmm_decode calls in this process (all threads):
 * lanes = 1 runs one wavefront lane per stream with a binary search
 * (ceil(log2 N) CDF evaluations per symbol); lanes = 2, 4, 8, 16 or 32 lets
 * that many lanes share a stream and search (lanes+1)-ary, cutting the
 * sequential rounds to ceil(log_{lanes+1} N) at the cost of more total
 * evaluations (for latents with few streams); 0 (default) chooses from the
 * stream count. Output is identical for every choice. GMM_EINVAL otherwise. */
int gmm_set_decode_lanes(int32_t lanes);

/* Diagnostic: number of floats u in [2^-10, 2^10] on which the coder's fused
 * reciprocal differs from IEEE division (*count [host]); the library uses
 * the fused form on a device only when this is 0. Synchronous. */
int gmm_fast_recip_mismatches(uint64_t* count, void* stream);

#ifdef __cplusplus
}
#endif
#endif
