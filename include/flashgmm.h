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
#define GMM_E2BIG 7    /* gmm_encode_noalloc: the call needs more workspace than
                          GMM_NOALLOC_SCRATCH_BYTES */

/* Coder configuration (format parameters: encoder and decoder must agree).
 *  K           mixture components, 1..8
 *  lo, hi      alphabet = integers lo..hi, N = hi-lo+1, 2 <= N <= 2^(P-1),
 *              |lo|, |hi| <= 2^22
 *  precision   P, 2..16: quantized frequencies sum to M = 2^P
 *  num_streams S >= 1 interleaved rANS streams
 *  cdf_kind    Gaussian CDF used inside the mixture (Sec. III-B, Table II):
 *              0 = A&S 26.2.17, 1 = logistic 1/(1+exp(-1.702 z)),
 *              2 = Polya (1 + sign(z) sqrt(1 - exp(-2 z^2/pi)))/2,
 *              3 = binary64 reference (erf series / erfc continued
 *              fraction, error below 1e-12). Kinds 2 and 3 are built for
 *              gmm_encode, gmm_decode without bracket, gmm_cdf_table and
 *              gmm_inverse_cdf (decode with 1 or 16 lanes per stream);
 *              plans and subset passes take kinds 0 and 1.
 *  param_kind  0 = the planes hold weights, means, scales; 1 = they hold a
 *              network's raw outputs (weight logits, means, log-scales),
 *              mapped per element inside the coder kernels exactly as
 *              gmm_params_from_raw maps them (no bracket with 1). */
typedef struct gmm_cfg {
  int32_t K;
  int32_t lo, hi;
  int32_t precision;
  int32_t num_streams;
  int32_t cdf_kind;
  int32_t param_kind;
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

/* Encode (Sec. III-A: each element's quantized mixture CDF evaluated at the
 * coded symbol's two boundaries, then the rANS state map of Eq. (3) per
 * stream, last element first). Encode n symbols [device, int32] with
 * parameter planes [device] into
 * bitstream [device, uint16, capacity_words] and offsets [device, int64,
 * S+1]: segment s occupies words offsets[s] .. offsets[s+1]-1 and
 * offsets[S] is the encoded size. GMM_ERANGE if a symbol is outside
 * [lo, hi]; GMM_ENOSPC if offsets[S] > capacity_words (offsets are still
 * written; no word at or beyond capacity_words is written, the words below
 * it are unspecified). Bitstream layout per segment: the final
 * 32-bit state as two little-endian uint16 words, then the renormalisation
 * words in the order the decoder reads them. */
int gmm_encode(const gmm_cfg* cfg, int64_t n, const int32_t* symbols, const float* weights,
               const float* means, const float* scales, uint16_t* bitstream,
               int64_t capacity_words, int64_t* offsets, void* ws, int64_t ws_bytes,
               int32_t* dev_status, void* stream);

/* Allocation-free encode, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): gmm_encode without the ws and ws_bytes arguments, with the
 * same kernels, output and status codes; the workspace is a static device
 * array of
 * GMM_NOALLOC_SCRATCH_BYTES that each device holds from the library's first
 * use on it until the process ends. The call allocates nothing (no
 * hipMalloc, hipMallocAsync or hipFree). GMM_E2BIG, before any launch, if
 * gmm_workspace_bytes(cfg, n, 0) exceeds GMM_NOALLOC_SCRATCH_BYTES (the
 * 320x135x240 latent with 65,536 streams needs 63.1 MB and fits).
 * Every call on a device shares that device's array: calls that overlap on
 * one device (concurrent streams or host threads) race and must be ordered
 * by the caller. The first call on a device (unless another entry point ran
 * there before) also runs the library's one-time check of its fused
 * reciprocal, which synchronizes the stream; under stream capture make one
 * call before capturing and pass dev_status (the synchronous form waits on
 * the stream). */
#define GMM_NOALLOC_SCRATCH_BYTES (64LL << 20)
int gmm_encode_noalloc(const gmm_cfg* cfg, int64_t n, const int32_t* symbols,
                       const float* weights, const float* means, const float* scales,
                       uint16_t* bitstream, int64_t capacity_words, int64_t* offsets,
                       int32_t* dev_status, void* stream);

/* Subset passes (the paper's two-pass Checkerboard context model, Sec. IV-A:
 * anchors are coded first, then the other elements with parameters that
 * the context model computes from the decoded anchors). A pass codes the m
 * elements idx[0..m) [device, int32, each in [0, n_total)] of a latent of
 * n_total < 2^31 elements in that order: pass position k reads element
 * idx[k] of symbols [device, int32 [n_total]] and of the parameter planes
 * [device, float32 [K][n_total]], belongs to stream k mod S, and decode
 * writes only symbols[idx[k]]. The bitstream equals gmm_encode of the
 * gathered m-element latent. An index out of range gives GMM_EINVAL (and no
 * out-of-bounds access). Workspace as gmm_encode / gmm_decode with n = m. */
int gmm_encode_subset(const gmm_cfg* cfg, int64_t n_total, const int32_t* idx, int64_t m,
                      const int32_t* symbols, const float* weights, const float* means,
                      const float* scales, uint16_t* bitstream, int64_t capacity_words,
                      int64_t* offsets, void* ws, int64_t ws_bytes, int32_t* dev_status,
                      void* stream);
int gmm_decode_subset(const gmm_cfg* cfg, int64_t n_total, const int32_t* idx, int64_t m,
                      const uint16_t* bitstream, int64_t total_words, const int64_t* offsets,
                      const float* weights, const float* means, const float* scales,
                      int32_t* symbols, void* ws, int64_t ws_bytes, int32_t* dev_status,
                      void* stream);

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

/* Description of a bracket model for gmm_bracket_create (all [host]).
 * The network maps D = 3K+1 features of an element and its rANS slot —
 * the K clamped weights, the K means, the K natural-log clamped scales and
 * slot / 2^P, each normalised as (x - in_mean) / in_std — through
 * D -> 64 -> ReLU -> 64 -> ReLU -> 1 to t, and predicts the symbol
 * t * out_std + out_mean. params: float32, W1 [64][D], b1 [64], W2 [64][64],
 * b2 [64], w3 [64], b3 [1] (rounded to bfloat16 on load). radius R: the
 * decoder checks the bracket [p - R, p + R] around the prediction p. */
typedef struct gmm_bracket_desc {
  int32_t K;
  int32_t radius;
  const float* params;
  const float* in_mean;
  const float* in_std;
  float out_mean, out_std;
} gmm_bracket_desc;

/* Uploads a bracket model (K 1..5). *out [host] receives the handle. */
int gmm_bracket_create(const gmm_bracket_desc* desc, gmm_bracket** out);
/* Releases a bracket model (waits for the device to be idle). */
int gmm_bracket_destroy(gmm_bracket* bracket);
/* Diagnostic: the model's symbol prediction for each element i at slot[i]
 * [device, uint32 [n]] as the decoder computes it (matrix cores, bfloat16
 * weights and inputs, float32 accumulation), into pred [device, float32
 * [n]]. Synchronous. */
int gmm_bracket_predict(const gmm_bracket* bracket, int32_t precision, int64_t n,
                        const float* weights, const float* means, const float* scales,
                        const uint32_t* slot, float* pred, void* stream);

/* ---- Training of the bracket model on the GPU ----
 * Parameter count of the D-input network (64 D + 4289). */
int gmm_mlp_num_params(int32_t D);
/* Device workspace bytes of gmm_mlp_loss_grad for n samples. */
int64_t gmm_mlp_workspace_bytes(int32_t D, int64_t n);
/* Features X [device, float32 [n][3K+1]] of element i at slot[i] [device,
 * uint32 [n]], normalised with mean / inv_std [device, float32 [3K+1]] when
 * given (both or neither), rounded to bfloat16 when round_bf16. K 1..5. */
int gmm_mlp_features(int32_t K, int64_t n, const float* weights, const float* means,
                     const float* scales, const uint32_t* slot, int32_t precision,
                     const float* mean, const float* inv_std, int32_t round_bf16, float* X,
                     void* stream);
/* Sum over the n samples of the Huber loss (threshold delta) of the network
 * output against y [device, float32 [n]] and its gradient: grad_loss
 * [device, float32 [P + 1]] receives the P parameter gradients then the
 * loss. params [device, float32 [P]] in the bracket layout. With round_act
 * the first hidden layer's activations are rounded to bfloat16 (as the
 * decoder's matrix cores see them; the gradient passes straight through).
 * The reduction order is fixed: results are bit-reproducible. */
int gmm_mlp_loss_grad(int32_t D, int64_t n, const float* X, const float* y, const float* params,
                      float delta, int32_t round_act, float* grad_loss, void* ws,
                      int64_t ws_bytes, void* stream);
/* Network output per sample into out [device, float32 [n]]. */
int gmm_mlp_forward(int32_t D, int64_t n, const float* X, const float* params, int32_t round_act,
                    float* out, void* stream);
/* One Adam step (bias-corrected, step >= 1) on float32 params with
 * gradient grad * grad_scale; m, v are the moment buffers; shadow
 * [device, nullable] receives the bfloat16-rounded parameters. */
int gmm_mlp_adam(int32_t P, float* params, const float* grad, float* m, float* v, float lr,
                 float beta1, float beta2, float eps, int32_t step, float grad_scale,
                 float* shadow, void* stream);

/* Decode (Sec. III-A: per symbol a binary search for the slot over the
 * monotone quantized CDF evaluated on the fly, then the inverse of the
 * state map of Eq. (3)). Decode n symbols [device, int32 out] from
 * bitstream [device, uint16,
 * total_words] and offsets [device, int64, S+1] with the same parameter
 * planes and configuration used to encode. GMM_ECORRUPT if a segment lies
 * outside the bitstream, is shorter than two words, is read past its end
 * (missing words read as 0), does not end in the initial state 2^16, or has
 * unread words. The result equals the plain binary search whether or not a
 * bracket is given. With one lane per stream, the A&S kind and 65 to 1,024
 * symbols and no learned bracket, the search proposes the symbol from the
 * components' quantiles and an approximate-Phi search and confirms it with
 * the exact c_j and c_{j+1} (exact binary search where the candidate
 * fails); c_j being strictly increasing, the symbols are the same.
 * stats [device, nullable]. */
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

/* Flag for gmm_plan_create: time every candidate launch shape
 * (gmm_plan_config) on the real shapes at the first
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

/* Launch shape of a plan (the autotuner's search space; the output never
 * depends on it):
 *  lanes_per_stream  decode: 1, 2, 4, 8 or 16 lanes share a stream and
 *                    search (lanes+1)-ary; encode and bracket decode: 1
 *  streams_per_lane  1, or 2 streams coded by one lane in lock-step (two
 *                    independent rANS chains per lane, half the wavefronts):
 *                    encode with lds_staging, and plain decode with one
 *                    lane per stream; otherwise 1
 *  schedule          0 one work item per workgroup, 1 persistent workgroups
 *                    with an atomic queue, 2 persistent with a static
 *                    round-robin assignment
 *  waves_per_cu      wavefronts per compute unit of the persistent grids,
 *                    1..64
 *  lds_staging       encode: 1 = each work item keeps its streams'
 *                    renormalisation words in LDS and writes offsets and
 *                    segments itself (per-latent decoupled look-back; streams
 *                    of at most 300 symbols; schedules 0 and 1), 0 = words
 *                    through scratch rows, then scan and pack kernels */
typedef struct gmm_plan_config {
  int32_t lanes_per_stream, streams_per_lane, schedule, waves_per_cu, lds_staging;
} gmm_plan_config;

/* State of a plan after its first execution: the chosen launch shape. */
typedef struct gmm_plan_info_t {
  int32_t tuned, candidates, graph_captured;
  gmm_plan_config config;
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

/* Decode plans only: decode with the learned bracket (NULL = plain search)
 * and add the bracket counters to stats [device, nullable]. Drops the
 * captured graph and the tuned shape (the next execution tunes again). The
 * output is identical with or without the bracket. */
int gmm_plan_set_bracket(gmm_plan* plan, const gmm_bracket* bracket, gmm_decode_stats* stats);

/* Forces a launch shape (skipping the tuner) and drops the captured graph;
 * the next gmm_plan_exec captures again. GMM_EINVAL for a shape outside
 * gmm_plan_config's ranges or not built for the plan (lds_staging with
 * decode, schedule 2 or streams over 300 symbols; streams_per_lane 2 for
 * an encode without lds_staging, a bracket decode or lanes_per_stream > 1).
 * For tests and sweeps: the output never depends on it. */
int gmm_plan_set_config(gmm_plan* plan, const gmm_plan_config* config);

/* The tuner's candidate launch shapes: writes up to max_count of them to out
 * [host, nullable] and returns the number of candidates (-1 on a NULL
 * plan). */
int gmm_plan_candidates(const gmm_plan* plan, gmm_plan_config* out, int32_t max_count);

/* Releases a plan (waits for its work to finish). */
int gmm_plan_destroy(gmm_plan* plan);

/* Launch shape of later gmm_decode calls in this process (all threads):
 * lanes = 1 runs one wavefront lane per stream with a binary search
 * (ceil(log2 N) CDF evaluations per symbol, or the bracketed search of
 * gmm_decode); lanes = 2, 4, 8, 16 or 32 lets
 * that many lanes share a stream and search (lanes+1)-ary, cutting the
 * sequential rounds to ceil(log_{lanes+1} N) at the cost of more total
 * evaluations (for latents with few streams); 0 (default) chooses from the
 * stream count: the smallest power of two up to 32 that gives at least
 * 65,536 lanes, which is then halved, down to 2, while the (lanes+1)-ary
 * search needs no more rounds. With a bracket, 16 or more lanes select the
 * group form with 16 lanes per stream (the network's prediction seeds one
 * round that evaluates 16 consecutive boundaries, with a 17-ary search as
 * fallback), 8 lanes the group form with 8 (8 boundaries, 9-ary fallback),
 * fewer the one-lane form (a verified bracket of radius R, then a binary
 * search).
 * Output is identical for every choice. GMM_EINVAL otherwise. */
int gmm_set_decode_lanes(int32_t lanes);

/* Lanes per stream that a gmm_decode of cfg [host] without a bracket uses
 * now (the gmm_set_decode_lanes choice, or the automatic one for cfg's
 * stream count and alphabet); -GMM_EINVAL for an invalid cfg. */
int gmm_decode_lanes(const gmm_cfg* cfg);

/* Issue priority, 0 (default) to 3, of the wavefronts of later
 * gmm_encode / gmm_decode calls (subset passes and bracket decodes included;
 * not the batched plans) made from the calling host thread. It matters only
 * when kernels of several calls share the SIMDs (calls on different HIP
 * streams): each SIMD issues the higher-priority wavefronts first, so
 * latency-bound work of a low-priority call fills the issue slots that an
 * issue-bound high-priority call leaves idle instead of taking its slots.
 * Output is identical for every value. GMM_EINVAL outside 0..3. */
int gmm_set_wave_priority(int32_t priority);

/* Diagnostic: number of floats u in [2^-10, 2^10] on which the coder's fused
 * reciprocal differs from IEEE division (*count [host]); the library uses
 * the fused form on a device only when this is 0. Synchronous. */
int gmm_fast_recip_mismatches(uint64_t* count, void* stream);

/* Raw network outputs to mixture parameters, one element per thread (the
 * entropy parameters come from a network, Sec. I and II-A; the scale lower
 * bound 0.11 is the one Sec. II-B quotes for scale tables). Planes [K][n]
 * [device]: weights = softmax over k of logits (differences to the largest
 * logit floored at -40.5, exp~ of the binary32 contract, sum in component
 * order, IEEE division); scales = max(exp~(clamp(log_scales, -7, 7)), 0.11).
 * Asynchronous on stream; outputs may not alias inputs. EINVAL for K outside
 * 1..8, n < 0 or NULL planes with n > 0. */
int gmm_params_from_raw(int32_t K, int64_t n, const float* logits, const float* log_scales,
                        float* weights, float* scales, void* stream);

/* ---- Peak probes (diagnostics; not part of the coder) ----
 * gmm_fma_probe: `threads` lanes (a multiple of 256) each run 8 independent
 * chains of `iters` binary32 fused multiply-adds (one fma per lane per
 * instruction, as the library is compiled) and store a sum to out [device,
 * float32 [threads]]; lane-fmas = threads * iters * 8. gmm_copy_probe:
 * copies `bytes` (a multiple of 16) from src to dst [device]. Both are
 * asynchronous on stream; the caller times them. GMM_EINVAL on bad sizes. */
int gmm_fma_probe(float* out, int64_t threads, int32_t iters, void* stream);
int gmm_copy_probe(const void* src, void* dst, int64_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif
