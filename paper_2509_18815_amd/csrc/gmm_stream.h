// Per-element and per-stream device routines of the GMM rANS coder, shared
// by the single-latent kernels (gmm_coder.hip) and the batched persistent
// kernels (gmm_batch.hip).
//
// Stream format (the coder's contract): element i of a latent with S streams
// belongs to stream i mod S at position i div S; a stream is coded last
// element first with a 32-bit state x starting at 2^16 and 16-bit
// renormalisation (emit x & 0xFFFF and shift when x >= f << (32-P)), the
// state map of FlashGMM Eq. (3) x <- (x div f) 2^P + (x mod f) + c; its
// segment is [x & 0xFFFF, x >> 16, words in the order the decoder reads].
#pragma once
#include "../../include/flashgmm.h"
#include "gmm_device.h"

namespace fgmm {

__device__ __forceinline__ int64_t stream_len(int64_t n, int64_t S, int64_t s) {
  return (s < n) ? (n - 1 - s) / S + 1 : 0;
}

// Third word of a raw buffer resource (stride 0, 32-bit elements, range
// checked against the byte count) on gfx9-family parts.
constexpr int kRsrcWord3 = 0x00020000;

// Whether every byte offset of decode_stream's buffer path fits the
// resources' 32-bit range: the K planes of n elements, positions up to
// three steps past a stream's last element (clamped, but counted before
// the clamp), the bitstream's words and the symbols.
__host__ __device__ inline bool buffer_offsets_fit(int K, int64_t n, int64_t S,
                                                   int64_t total_words) {
  const int64_t lim = 0xFFFFFFFFll;
  return n >= 0 && S >= 1 && 4 * ((int64_t)K * n + 4 * S) <= lim && 2 * (total_words + 1) <= lim;
}

// The same for the encode's buffer path: the K planes, and the (c, f) words
// of positions down to a block (8 steps) before a stream's first element,
// whose offsets wrap below 0 to values past the words (read as 0: those
// steps are not live).
__host__ __device__ inline bool encode_offsets_fit(int K, int64_t n, int64_t S) {
  const int64_t lim = 0xFFFFFFFFll;
  return n >= 0 && S >= 1 && 4 * ((int64_t)K * n) <= lim && 4 * (n + 8 * S) <= lim;
}

// Element of a subset pass, clamped into the latent so that an invalid
// index (reported as EINVAL by the pass's index check) never reads or
// writes outside the buffers.
__device__ __forceinline__ int64_t gather_index(const int32_t* __restrict__ idx, int64_t i,
                                                int64_t n_total) {
  const int64_t v = (int64_t)idx[i];
  return v < 0 ? 0 : (v >= n_total ? n_total - 1 : v);
}

// Branch-uniform binary search for the j with c_j <= slot < c_{j+1}, over
// the power-of-two range [0, 2^rounds) with 2^rounds >= N and c_j = M for
// every j >= N: round r tests lo + 2^(rounds-1-r), so every lane runs
// exactly `rounds` CDF evaluations and the same instruction stream. Before
// the round testing lo + h, c_lo = c(lo) <= slot < c_hi = c(lo + 2h), so
// on return c_lo = c_j and c_hi = c_{j+1}; since slot < M, lo never reaches
// N.
//
// A midpoint lo + h is at most 2^rounds - h, so only the rounds with
// h <= 2^rounds - N can test an index >= N (for N = 2^rounds - 1 only the
// last one); the others skip that select (a wavefront-uniform branch).
//
// Leading rounds whose midpoints stay below N: those with 2^r > 2^rounds - N.
__device__ __forceinline__ int free_rounds(int rounds, int32_t N) {
  const int32_t pad = (1 << rounds) - N;
  int nfree = 0;
  while (nfree < rounds && (1 << (rounds - 1 - nfree)) > pad) ++nfree;
  return nfree;
}

// Exact binary search over [0, 2^rounds): the first nfree rounds probe
// boundaries below N, the rest clamp c_j to M for j >= N.
template <int K, int kKind, bool kFast>
__device__ __forceinline__ int32_t search_loop(const Elem<K>& e, const QCfg& q, int rounds,
                                               int nfree, uint32_t slot, uint32_t& c_lo,
                                               uint32_t& c_hi) {
  int32_t lo = 0;
  c_lo = 0;
  c_hi = q.M;
  int r = rounds - 1;
  for (int i = 0; i < nfree; ++i, --r) {
    const int32_t mid = lo + (1 << r);
    const uint32_t c = cdf_inner<K, kKind, kFast>(e, q, mid);
    const bool right = slot >= c;
    lo = right ? mid : lo;
    c_lo = right ? c : c_lo;
    c_hi = right ? c_hi : c;
  }
  for (; r >= 0; --r) {
    const int32_t mid = lo + (1 << r);
    const uint32_t c = cdf_upper<K, kKind, kFast>(e, q, mid);
    const bool right = slot >= c;
    lo = right ? mid : lo;
    c_lo = right ? c : c_lo;
    c_hi = right ? c_hi : c;
  }
  return lo;
}

// ---------------------------------------------------------------------
// Bracketed search (one lane per stream, A&S kind). The decoder has to
// find the j with c_j <= slot < c_{j+1}; since c_j is strictly increasing
// that j is unique, and any procedure that proposes a candidate and then
// confirms it with the exact c_j and c_{j+1} returns what the binary search
// returns. The candidate comes from two steps that are not part of the
// coding contract and may err (an error only costs time):
//  1. a bracket from component quantiles: if every component has CDF value
//     u at its own quantile mu_k + sigma_k z(u), the mixture's u-quantile
//     lies between the smallest and the largest of them, so a rough z(u)
//     (A&S 26.2.23, |error| < 4.5e-4) and the slot's position u give an
//     index range [jl, jh] that usually holds j;
//  2. a binary search over that range with an approximate Phi (A&S 26.2.16,
//     |error| < 1e-5, on the hardware reciprocal and exp2, no clamps): its
//     comparisons differ from the exact ones only where the slot lies
//     within about 1e-5 (M - N) counts of a boundary.
// Two exact evaluations then confirm the candidate; a lane whose candidate
// fails runs the exact binary search (the looped form: it is rare, and one
// copy keeps the unrolled decode loop small). The wavefront runs as many
// approximate rounds as its widest bracket needs (at most the exact
// search's), so it pays off when brackets are narrow: the components'
// quantiles close together relative to their scales.
constexpr float kQ23C0 = 2.515517f, kQ23C1 = 0.802853f, kQ23C2 = 0.010328f;
constexpr float kQ23D1 = 1.432788f, kQ23D2 = 0.189269f, kQ23D3 = 0.001308f;
// A&S 26.2.16: Q(x) = Z(x) (a1 t + a2 t^2 + a3 t^3), t = 1 / (1 + p x)
constexpr float kA16P = 0.33267f, kA16A1 = 0.4361836f, kA16A2 = -0.1201676f,
                kA16A3 = 0.9372980f;
constexpr float kInvSqrt2Pi = 0.3989422804014327f;
// z is carried pre-scaled by kappa = sqrt(log2(e) / 2), so that the
// density factor exp(-z^2 / 2) is exp2(-(kappa z)^2)
constexpr float kKappa = 0.8493218002880191f;
constexpr float kNeg2Ln2 = -1.3862943611198906f;       // -2 ln 2
// below 7 exact rounds (N <= 64) the plain search is as cheap; above 10
// (N > 1024) the looped search serves
constexpr int kBracketMinRounds = 7, kBracketMaxRounds = 10;

// Approximate Phi(z) - 1/2 (|error| ~1e-5): the A&S 26.2.16 tail with the
// hardware reciprocal and exp2. (The five-term 26.2.17, error ~1e-7, costs
// two more instructions per component, which its rarer fallbacks do not
// repay: 4K decode 254 against 250 us, 256-latent plan 12.9 against
// 12.2 ms.)
__device__ __forceinline__ float approx_half(float zk) {  // zk = kappa z
  const float x = __builtin_fabsf(zk);
  const float t = __builtin_amdgcn_rcpf(fma32(x, kA16P / kKappa, 1.0f));
  float h = fma32(kA16A3 * kInvSqrt2Pi, t, kA16A2 * kInvSqrt2Pi);
  h = fma32(h, t, kA16A1 * kInvSqrt2Pi);
  const float g = __builtin_amdgcn_exp2f(-(zk * zk));
  return __builtin_copysignf(fma32(-g, h * t, 0.5f), zk);
}

// Maximum / minimum over the 16 lanes of a DPP row (every lane receives
// it): rotations of the row by 1, 2, 4 and 8 lanes.
__device__ __forceinline__ int32_t row16_max(int32_t v) {
  v = max(v, __builtin_amdgcn_mov_dpp(v, 0x121, 0xF, 0xF, true));  // row_ror:1
  v = max(v, __builtin_amdgcn_mov_dpp(v, 0x122, 0xF, 0xF, true));  // row_ror:2
  v = max(v, __builtin_amdgcn_mov_dpp(v, 0x124, 0xF, 0xF, true));  // row_ror:4
  v = max(v, __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true));  // row_ror:8
  return v;
}
__device__ __forceinline__ int32_t row16_min(int32_t v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x121, 0xF, 0xF, true));
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x122, 0xF, 0xF, true));
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x124, 0xF, 0xF, true));
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true));
  return v;
}

// The largest value over the wavefront's lanes of a small non-negative v
// (lanes outside exec may contribute stale values: callers clamp).
__device__ __forceinline__ int32_t wave_max_small(int32_t v) {
  v = row16_max(v);
  const int32_t a = max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16));
  const int32_t b = max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48));
  return max(a, b);
}

template <int K, bool kFast>
__device__ __forceinline__ int32_t search_bracketed(const Elem<K>& e, const QCfg& q, int rounds,
                                                    int nfree, uint32_t slot, uint32_t& c_lo,
                                                    uint32_t& c_hi) {
  const int32_t N = (int32_t)q.N;
  // 1. bracket. The slot sits near j + F(b_j)(M - N) for the symbol j, so
  // u = (slot + 1/2 - jbar) / (M - N), with jbar the index of the
  // mixture's mean, approximates F at the symbol.
  float wm = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) wm = fma32(e.w[k], e.mu[k], wm);
  const float jbar = wm * (0.5f * __builtin_amdgcn_rcpf(e.hw)) - q.lo_mh;
  const float u = ((float)slot + 0.5f - jbar) * __builtin_amdgcn_rcpf(q.span);
  const float pu = __builtin_fmaxf(__builtin_fminf(u, 1.0f - u), 0x1p-30f);
  const float t = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(pu) * kNeg2Ln2);
  const float num = fma32(fma32(kQ23C2, t, kQ23C1), t, kQ23C0);
  const float den = fma32(fma32(fma32(kQ23D3, t, kQ23D2), t, kQ23D1), t, 1.0f);
  const float xq = t - num * __builtin_amdgcn_rcpf(den);
  const float z = (u < 0.5f) ? -xq : xq;
  float qmin = fma32(e.sc[0], z, e.mu[0]), qmax = qmin;
#pragma unroll
  for (int k = 1; k < K; ++k) {
    const float v = fma32(e.sc[k], z, e.mu[k]);
    qmin = __builtin_fminf(qmin, v);
    qmax = __builtin_fmaxf(qmax, v);
  }
  // symbol index of a value v: floor(v - (lo - 1/2)); one index of margin.
  // The indices stay floats (integers below 2^23, exact); the rounds the
  // lane needs are the bit length of jh - jl, the exponent of its frexp
  // (0 for 0).
  const float fN1 = (float)(N - 1);
  const float jl = __builtin_fminf(
      __builtin_fmaxf(__builtin_floorf(qmin - q.lo_mh) - 1.0f, 0.0f), fN1);
  const float jh = __builtin_fminf(
      __builtin_fmaxf(__builtin_floorf(qmax - q.lo_mh) + 1.0f, jl), fN1);
  const int32_t rl = __builtin_amdgcn_frexp_expf(jh - jl);
  const int32_t rw = min(wave_max_small(rl), rounds);
  // 2. approximate binary search over [jl, jh]
  // the boundaries as floats b = j + lo - 1/2 (exact: integers and
  // half-integers below 2^23), so a round costs no conversions
  float ws[K], zr[K], zo[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ws[k] = e.w[k] * q.span;
    zr[k] = e.r[k] * kKappa;
    zo[k] = -e.mu[k] * zr[k];
  }
  const float h0 = e.hw * q.span;
  const float s1 = (float)(slot + 1u) + q.lo_mh;
  const float bh = jh + q.lo_mh;
  float bj = jl + q.lo_mh;
  for (int i = rw - 1; i >= 0; --i) {
    // 2^i as float bits built on the scalar unit; a midpoint past jh is
    // evaluated anyway (the approximation needs no range) and not taken
    const float b = bj + __builtin_bit_cast(float, (uint32_t)(127 + i) << 23);
    float y = h0;
#pragma unroll
    for (int k = 0; k < K; ++k) y = fma32(ws[k], approx_half(fma32(b, zr[k], zo[k])), y);
    bj = (b <= bh && y < s1 - b) ? b : bj;
  }
  const int32_t j = (int32_t)(bj - q.lo_mh);
  // 3. confirm with the exact c_j and c_{j+1} (cdf_inner's values: bj is
  // exactly j + lo - 1/2 and bj + 1 the next boundary; j < N, so only c_0
  // and c_N need their ends)
  const float y0 = cdf_scaled<K, 0, kFast>(e, q, bj);
  const float y1 = cdf_scaled<K, 0, kFast>(e, q, bj + 1.0f);
  const uint32_t cl = (j <= 0) ? 0u : (uint32_t)j + (uint32_t)y0;
  const uint32_t ch = (j + 1 >= N) ? q.M : (uint32_t)(j + 1) + (uint32_t)y1;
  if (__builtin_expect(cl <= slot && slot < ch, 1)) {
    c_lo = cl;
    c_hi = ch;
    return j;
  }
  return search_loop<K, 0, kFast>(e, q, rounds, nfree, slot, c_lo, c_hi);
}

// nfree = free_rounds(rounds, N), computed once by the caller. With
// kBracket (A&S kind, one lane per stream) alphabets of 65 to 1024 symbols
// take the bracketed search (a wavefront-uniform branch on the kernel's
// arguments); other kinds and sizes the exact loop.
template <int K, int kKind, bool kFast, bool kBracket = false>
__device__ __forceinline__ int32_t search_bs(const Elem<K>& e, const QCfg& q, int rounds,
                                             int nfree, uint32_t slot, uint32_t& c_lo,
                                             uint32_t& c_hi) {
  if constexpr (kKind == 0 && kBracket) {
    if (__builtin_expect(rounds >= kBracketMinRounds && rounds <= kBracketMaxRounds, 1))
      return search_bracketed<K, kFast>(e, q, rounds, nfree, slot, c_lo, c_hi);
  }
  return search_loop<K, kKind, kFast>(e, q, rounds, nfree, slot, c_lo, c_hi);
}

// (L+1)-ary search by a group of L lanes (lane g of the group, group mask
// gmask, first lane gbase): each round the lanes evaluate the CDF at L split
// points of [lo, hi); the interval shrinks to the part between the last
// point at or below the slot and the first one above it. The split points
// are non-decreasing in g and below hi, so the points at or below the slot
// are a prefix of the group. With 16 lanes (a group is a DPP row) the new
// bounds are row maxima and minima (lo' = max over lanes of (at or below ?
// m : lo), hi' = min of (at or below ? hi : m), and the same for the CDF
// values), which needs no LDS round trip; otherwise a ballot counts the
// points at or below the slot and shuffles fetch the bounds.
template <int K, int kKind, bool kFast, int L>
__device__ __forceinline__ int32_t search_group(const Elem<K>& e, const QCfg& q, int rounds,
                                                uint32_t slot, int g, int gbase, uint64_t gmask,
                                                int32_t lo, int32_t hi, uint32_t& c_lo,
                                                uint32_t& c_hi) {
  if constexpr (L == 16) {
    for (int r = 0; r < rounds; ++r) {
      const uint32_t sz = (uint32_t)(hi - lo);
      const int32_t m = lo + (int32_t)((sz * (uint32_t)(g + 1)) / (uint32_t)(L + 1));
      const uint32_t c = cdf_lower<K, kKind, kFast>(e, q, m);  // m < hi <= N
      const bool le = slot >= c;
      const int32_t nlo = row16_max(le ? m : lo);
      const int32_t nclo = row16_max((int32_t)(le ? c : c_lo));
      const int32_t nhi = row16_min(le ? hi : m);
      const int32_t nchi = row16_min((int32_t)(le ? c_hi : c));
      lo = nlo;
      hi = nhi;
      c_lo = (uint32_t)nclo;
      c_hi = (uint32_t)nchi;
    }
    return lo;
  }
  for (int r = 0; r < rounds; ++r) {
    const uint32_t sz = (uint32_t)(hi - lo);
    const int32_t m = lo + (int32_t)((sz * (uint32_t)(g + 1)) / (uint32_t)(L + 1));
    const uint32_t c = cdf_lower<K, kKind, kFast>(e, q, m);  // m < hi <= N
    const uint64_t bal = __ballot(slot >= c) & gmask;
    const int cnt = __popcll(bal);
    const int src_lo = gbase + (cnt > 0 ? cnt - 1 : 0);
    const int src_hi = gbase + (cnt < L ? cnt : L - 1);
    const int32_t m_lo = __shfl(m, src_lo, 64);
    const uint32_t c_l = __shfl(c, src_lo, 64);
    const int32_t m_hi = __shfl(m, src_hi, 64);
    const uint32_t c_h = __shfl(c, src_hi, 64);
    if (cnt > 0) {
      lo = m_lo;
      c_lo = c_l;
    }
    if (cnt < L) {
      hi = m_hi;
      c_hi = c_h;
    }
  }
  return lo;
}

// Encode phase 1 for element i: (c_j << 16) | f_j of its symbol (both fit
// 16 bits: c_j < M <= 2^16 for j < N, f_j <= M - N + 1 < 2^16). A symbol
// outside [lo, hi] sets kStRange in *status, or with kSentinel gives the
// word 0 (f = 0, which no valid symbol has), which the rANS pass reports.
// With kBuf the symbol and the parameters are read through buffer resources
// (one 32-bit offset, plane rows at scalar offsets k n 4; the caller checks
// encode_offsets_fit).
template <int K, int kKind, bool kFast, bool kSentinel = false, bool kBuf = false>
__device__ __forceinline__ uint32_t enc_cdf_elem(const QCfg& q, int64_t n, int64_t i,
                                                 const int32_t* __restrict__ sym,
                                                 const float* __restrict__ w,
                                                 const float* __restrict__ mu,
                                                 const float* __restrict__ sg, uint32_t* status) {
  float rw[K], rm[K], rs[K];
  int32_t j;
  if constexpr (kBuf) {
    const int nb = (int)(uint32_t)(K * n * 4);
    const __amdgpu_buffer_rsrc_t bw_ = __builtin_amdgcn_make_buffer_rsrc((void*)w, (short)0, nb, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t bm_ = __builtin_amdgcn_make_buffer_rsrc((void*)mu, (short)0, nb, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t bsg_ = __builtin_amdgcn_make_buffer_rsrc((void*)sg, (short)0, nb, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t bsy_ = __builtin_amdgcn_make_buffer_rsrc(
        (void*)sym, (short)0, (int)(uint32_t)(n * 4), kRsrcWord3);
    const uint32_t o = (uint32_t)i * 4u, plane = (uint32_t)(n * 4);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      rw[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(bw_, o, k * plane, 0));
      rm[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(bm_, o, k * plane, 0));
      rs[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(bsg_, o, k * plane, 0));
    }
    j = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(bsy_, o, 0, 0) - q.lo;
  } else {
    load_raw<K>(w, mu, sg, n, i, rw, rm, rs);
    j = sym[i] - q.lo;
  }
  const bool out = j < 0 || j >= q.N;
  if (out) {
    if (!kSentinel) atomicOr(status, kStRange);
    j = 0;
  }
  const Elem<K> e = make_elem<K, kFast, kKind>(q, rw, rm, rs);
  const uint32_t c0 = cdf_at<K, kKind, kFast>(e, q, j);
  const uint32_t c1 = cdf_at<K, kKind, kFast>(e, q, j + 1);
  return (kSentinel && out) ? 0u : ((c0 << 16) | (c1 - c0));
}

// s_waitcnt immediate: vector memory count 0, the other counters unlimited.
constexpr int kWaitVm0 = 0x0F70;

// One encode step of the rANS recurrence for the packed word cfw = (c << 16)
// | f: renormalise (emit = whether the low 16 bits of x, returned in word,
// leave the state), then x <- (x div f) 2^P + (x mod f) + c (Eq. (3)).
__device__ __forceinline__ void rans_put(uint32_t& x, uint32_t cfw, int P, int shift, bool& emit,
                                         uint32_t& word) {
  const uint32_t c = cfw >> 16;
  const uint32_t f = cfw & 0xFFFFu;
  // 1/f in binary64 off the chain: hardware estimate, one Newton step
  const double fd = (double)f;
  const double y0 = __builtin_amdgcn_rcp(fd);
  const double rf = __builtin_fma(__builtin_fma(-fd, y0, 1.0), y0, y0);
  emit = x >= (f << shift);
  word = x & 0xFFFFu;
  x = emit ? (x >> 16) : x;
  // x <- (x div f) 2^P + (x mod f) + c, exactly: with rf within 2^-50 of
  // 1/f, x rf is within 2^-17 of x / f < 2^32, while a non-integer
  // x / f lies at least 1/f >= 2^-16 below the next integer, so
  // q0 = trunc(x rf) is the quotient q or q - 1; then r0 = x - q0 f
  // (exact) is the remainder or the remainder + f, and one comparison
  // fixes both. Every binary64 value here is an integer below 2^53.
  const double xd = (double)x;
  const double q0 = __builtin_trunc(xd * rf);
  const double r0 = __builtin_fma(-q0, fd, xd);
  const double fix = (r0 >= fd) ? (double)((1u << P) - f) : 0.0;
  x = (uint32_t)(__builtin_fma(q0, (double)(1u << P), r0 + (double)c) + fix);
}

// Encode phase 2 for stream s: the integer rANS recurrence over the packed
// (c, f) words cf[s + p S], p = n_s-1 .. 0. The k-th emitted word goes to
// region_end[-k], so the words end up in the order the decoder reads them.
// Returns the final state; *count receives the number of words, *zero_f
// whether a word had f = 0 (an out-of-range symbol, see enc_cdf_elem).
//
// Memory operations are arranged so that every wait is for work issued a
// whole block of kDepth steps earlier: the (c, f) words are loaded a block
// ahead with a fixed number of loads, and the words a block emits are held
// in registers and stored at the start of the next block.
__device__ __forceinline__ uint32_t rans_stream(int64_t n, int64_t S, int P, int64_t s,
                                                const uint32_t* __restrict__ cf,
                                                uint16_t* __restrict__ region_end,
                                                uint32_t* count, bool* zero_f) {
  const int64_t ns = stream_len(n, S, s);
  uint32_t x = 1u << 16;
  uint32_t cnt = 0;
  const int shift = 32 - P;
  // the word of position p sits at s + p S, walked down by running indices
  constexpr int kDepth = 8;
  int64_t dS[kDepth];
#pragma unroll
  for (int d = 0; d < kDepth; ++d) dS[d] = (int64_t)d * S;
  uint32_t buf[kDepth];
  int64_t base = s + (ns - 1) * S;  // position ns - 1
#pragma unroll
  for (int d = 0; d < kDepth; ++d) buf[d] = (ns - 1 - d >= 0) ? cf[base - dS[d]] : 0u;
  const int64_t step = (int64_t)kDepth * S;
  uint32_t pend[kDepth];   // words emitted by the previous block (bit d of pmask: step d emitted)
  uint32_t pmask = 0, pbase = 0;
  bool zf = false;
  for (int64_t p = ns - 1; p >= 0; p -= kDepth) {
    base -= step;  // position p - kDepth
    // everything issued so far is a block old: the loads of this block's
    // words and the previous block's stores (a wait issued after the new
    // stores and loads would also wait for them, the counter being shared)
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    uint32_t cur[kDepth];
#pragma unroll
    for (int d = 0; d < kDepth; ++d) cur[d] = buf[d];
#pragma unroll
    for (int d = 0; d < kDepth; ++d)
      if ((pmask >> d) & 1u)
        region_end[-(int64_t)(pbase + __builtin_popcount(pmask & ((1u << d) - 1u)))] =
            (uint16_t)pend[d];
    pbase = cnt;
    pmask = 0;
    asm volatile("" ::: "memory");
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      // unconditional (positions below 0 reload position 0)
      const int64_t at = base - dS[d];
      buf[d] = cf[at >= s ? at : s];
    }
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      if (p - d < 0) break;
      bool emit;
      zf = zf || (cur[d] & 0xFFFFu) == 0u;
      rans_put(x, cur[d], P, shift, emit, pend[d]);
      pmask |= (emit ? 1u : 0u) << d;
      cnt += emit ? 1u : 0u;
    }
  }
#pragma unroll
  for (int d = 0; d < kDepth; ++d)
    if ((pmask >> d) & 1u)
      region_end[-(int64_t)(pbase + __builtin_popcount(pmask & ((1u << d) - 1u)))] =
          (uint16_t)pend[d];
  *count = cnt;
  *zero_f = zf;
  return x;
}

// Encode phase 2 for stream s with the emitted words kept in LDS: the k-th
// emitted word goes to col[k stride] (a column of the workgroup's word
// array, so that the lanes of a step write neighbouring LDS words). The
// (c, f) words are loaded a block of kDepth steps ahead as in rans_stream;
// the LDS stores do not count on the vector-memory counter, so the one wait
// per block is for those loads only. Returns the final state; *count
// receives the number of words (at most n_s), *zero_f whether a word had
// f = 0.
template <bool kBuf = false>
__device__ __forceinline__ uint32_t rans_stream_lds(int64_t n, int64_t S, int P, int64_t s,
                                                    const uint32_t* __restrict__ cf,
                                                    uint16_t* col, int stride, int trash_row,
                                                    uint32_t* count, bool* zero_f) {
  const int64_t ns = stream_len(n, S, s);
  uint32_t x = 1u << 16;
  uint32_t cnt = 0;
  const int shift = 32 - P;
  constexpr int kDepth = 8;
  int64_t dS[kDepth];
#pragma unroll
  for (int d = 0; d < kDepth; ++d) dS[d] = (int64_t)d * S;
  uint32_t buf[kDepth];
  int64_t base = s + (ns - 1) * S;  // position ns - 1
  // kBuf: the words through a buffer resource, offsets in bytes; a position
  // below 0 wraps to an offset past the words (encode_offsets_fit), which
  // reads 0 (such steps are not live)
  [[maybe_unused]] __amdgpu_buffer_rsrc_t bcf_;
  [[maybe_unused]] uint32_t ob = 0;
  const uint32_t dS4 = (uint32_t)S * 4u;
  if constexpr (kBuf) {
    bcf_ = __builtin_amdgcn_make_buffer_rsrc((void*)cf, (short)0, (int)(uint32_t)(n * 4),
                                             kRsrcWord3);
    ob = (uint32_t)base * 4u;
#pragma unroll
    for (int d = 0; d < kDepth; ++d)
      buf[d] = __builtin_amdgcn_raw_buffer_load_b32(bcf_, ob - (uint32_t)d * dS4, 0, 0);
  } else {
#pragma unroll
    for (int d = 0; d < kDepth; ++d) buf[d] = (ns - 1 - d >= 0) ? cf[base - dS[d]] : 0u;
  }
  const int64_t step = (int64_t)kDepth * S;
  bool zf = false;
  for (int64_t p = ns - 1; p >= 0; p -= kDepth) {
    base -= step;  // position p - kDepth
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    uint32_t cur[kDepth];
#pragma unroll
    for (int d = 0; d < kDepth; ++d) cur[d] = buf[d];
    if constexpr (kBuf) {
      ob -= (uint32_t)kDepth * dS4;
#pragma unroll
      for (int d = 0; d < kDepth; ++d)
        buf[d] = __builtin_amdgcn_raw_buffer_load_b32(bcf_, ob - (uint32_t)d * dS4, 0, 0);
    } else {
#pragma unroll
      for (int d = 0; d < kDepth; ++d) {
        // unconditional (positions below 0 reload position 0)
        const int64_t at = base - dS[d];
        buf[d] = cf[at >= s ? at : s];
      }
    }
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      // every step of the block runs (no branch per step): a step past the
      // stream's start leaves the state as it is, and a step that emits no
      // word stores its word to the trash row
      const bool live = p - d >= 0;
      bool emit;
      uint32_t word, xn = x;
      rans_put(xn, cur[d], P, shift, emit, word);
      emit = emit && live;
      zf = zf || (live && (cur[d] & 0xFFFFu) == 0u);
      col[(emit ? (int)cnt : trash_row) * stride] = (uint16_t)word;
      x = live ? xn : x;
      cnt += emit ? 1u : 0u;
    }
  }
  *count = cnt;
  *zero_f = zf;
  return x;
}

// rans_stream_lds for two streams a and b of one latent in one lane, stepped
// in turn at the same positions (their lengths differ by at most one), so
// that the lane carries two independent dependency chains; the (c, f) words
// of both are loaded a block ahead.
__device__ __forceinline__ void rans_stream_lds2(int64_t n, int64_t S, int P, int64_t sa,
                                                 int64_t sb, const uint32_t* __restrict__ cf,
                                                 uint16_t* cola, uint16_t* colb, int stride,
                                                 int trash_row, uint32_t& xa, uint32_t& xb,
                                                 uint32_t& ca,
                                                 uint32_t& cb, bool& zero_f) {
  const int64_t na = stream_len(n, S, sa), nb = stream_len(n, S, sb);
  const int64_t nmax = na > nb ? na : nb;
  xa = xb = 1u << 16;
  ca = cb = 0;
  const int shift = 32 - P;
  constexpr int kDepth = 8;
  int64_t dS[kDepth];
#pragma unroll
  for (int d = 0; d < kDepth; ++d) dS[d] = (int64_t)d * S;
  // positions past a stream's end (or below 0) reload its first element
  auto at = [&](int64_t s, int64_t ns, int64_t pos) -> int64_t {
    return (pos >= 0 && pos < ns) ? s + pos * S : s;
  };
  uint32_t bufa[kDepth], bufb[kDepth];
#pragma unroll
  for (int d = 0; d < kDepth; ++d) {
    bufa[d] = cf[at(sa, na, nmax - 1 - d)];
    bufb[d] = cf[at(sb, nb, nmax - 1 - d)];
  }
  bool zf = false;
  for (int64_t p = nmax - 1; p >= 0; p -= kDepth) {
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    uint32_t cura[kDepth], curb[kDepth];
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      cura[d] = bufa[d];
      curb[d] = bufb[d];
    }
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      bufa[d] = cf[at(sa, na, p - kDepth - d)];
      bufb[d] = cf[at(sb, nb, p - kDepth - d)];
    }
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      const int64_t q = p - d;
      const bool la = q >= 0 && q < na, lb = q >= 0 && q < nb;
      bool ea, eb;
      uint32_t wa, wb, xna = xa, xnb = xb;
      rans_put(xna, cura[d], P, shift, ea, wa);
      rans_put(xnb, curb[d], P, shift, eb, wb);
      ea = ea && la;
      eb = eb && lb;
      zf = zf || (la && (cura[d] & 0xFFFFu) == 0u) || (lb && (curb[d] & 0xFFFFu) == 0u);
      cola[(ea ? (int)ca : trash_row) * stride] = (uint16_t)wa;
      colb[(eb ? (int)cb : trash_row) * stride] = (uint16_t)wb;
      xa = la ? xna : xa;
      xb = lb ? xnb : xb;
      ca += ea ? 1u : 0u;
      cb += eb ? 1u : 0u;
    }
  }
  zero_f = zf;
}

// Sum of v over the 64 lanes of a wavefront (every lane receives it).
__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Decoupled look-back: the sum of the totals of every workgroup with a
// smaller ticket (workgroups take tickets in the order they start, from an
// atomic counter). slots[t] is 0 until workgroup t publishes (1 << 62) |
// its total, and later (2 << 62) | its inclusive prefix; the slots are
// zeroed before the launch. The ticket order guarantees that every
// workgroup waited on has started, and a workgroup publishes its total
// before it waits on anyone, so the waits end. Called by all 64 lanes of
// one wavefront; every lane receives the result. The slots are read and
// written with device-scope atomics (coherent across XCDs).
constexpr uint64_t kLbAggregate = 1ull << 62, kLbInclusive = 2ull << 62;
constexpr uint64_t kLbValue = (1ull << 62) - 1;
__device__ __forceinline__ int64_t lookback_prefix(uint64_t* slots, int64_t ticket,
                                                   int64_t total) {
  const int lane = threadIdx.x & 63;
  if (lane == 0)
    __hip_atomic_store(&slots[ticket], kLbAggregate | (uint64_t)total, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  int64_t excl = 0;
  int64_t j = ticket - 1;  // the newest slot not yet summed
  while (j >= 0) {
    // lane i looks at slot j - i; slots before 0 act as an inclusive 0
    const int64_t k = j - lane;
    const uint64_t v = (k >= 0) ? __hip_atomic_load(&slots[k], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT)
                                : kLbInclusive;
    const uint64_t flag = v >> 62;
    const uint64_t notready = __ballot(flag == 0);
    const uint64_t incl = __ballot(flag == 2);
    const int first_nr = notready ? __ffsll((long long)notready) - 1 : 64;
    const int first_in = incl ? __ffsll((long long)incl) - 1 : 64;
    if (first_in < first_nr) {  // lanes 0..first_in reach an inclusive prefix
      excl += wave_sum64(lane <= first_in ? (int64_t)(v & kLbValue) : 0);
      break;
    }
    // lanes 0..first_nr-1 hold totals: add them and look further back
    excl += wave_sum64(lane < first_nr ? (int64_t)(v & kLbValue) : 0);
    j -= first_nr;
    if (first_nr == 0) __builtin_amdgcn_s_sleep(1);
  }
  if (lane == 0)
    __hip_atomic_store(&slots[ticket], kLbInclusive | (uint64_t)(excl + total),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// Inclusive prefix sum across the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Block-wide exclusive scan of len over kBlock threads (wavefront scans, then
// the wavefront totals through LDS). Returns the exclusive prefix; *total
// receives the block sum. Every thread of the block must call it.
template <int kBlock>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t len, uint32_t* total) {
  __shared__ uint32_t wave_sum[kBlock / 64];
  const uint32_t incl = wave_incl_scan(len);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) wave_sum[wv] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    base += (k < wv) ? wave_sum[k] : 0u;
    tot += wave_sum[k];
  }
  *total = tot;
  return base + incl - len;
}

// Exclusive scan of nblk int64 block totals by one workgroup of kBlock
// threads, tile by tile with a running carry; returns the sum (every
// thread). Every thread of the workgroup must call it. With kAtomic the
// totals are read with device-scope atomics (written by other workgroups of
// the same launch with atomics).
constexpr int kScanBlock = 1024;
template <int kBlock = kScanBlock, bool kAtomic = false>
__device__ __forceinline__ int64_t scan_totals(int64_t nblk, const int64_t* __restrict__ tot,
                                               int64_t* __restrict__ pre) {
  __shared__ int64_t wsum[kBlock / 64];
  __shared__ int64_t carry_sh;
  if (threadIdx.x == 0) carry_sh = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t base = 0; base < nblk; base += kBlock) {
    const int64_t i = base + threadIdx.x;
    int64_t v = 0;
    if (i < nblk)
      v = kAtomic ? (int64_t)atomicAdd((unsigned long long*)(tot + i), 0ull) : tot[i];
    int64_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t t = __shfl_up(incl, d, 64);
      if (lane >= d) incl += t;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int64_t off = carry_sh;
    for (int k = 0; k < wv; ++k) off += wsum[k];
    if (i < nblk) pre[i] = off + incl - v;
    __syncthreads();
    if (threadIdx.x == kBlock - 1) carry_sh = off + incl;
    __syncthreads();
  }
  return carry_sh;
}

// Status code of a call from its status bits (first match wins).
__device__ __forceinline__ int32_t status_code(uint32_t b) {
  if (b & kStInval) return GMM_EINVAL;
  if (b & kStRange) return GMM_ERANGE;
  if (b & kStNoSpace) return GMM_ENOSPC;
  if (b & kStCorrupt) return GMM_ECORRUPT;
  return GMM_OK;
}

// True in every thread of the workgroup that finishes last among the
// grid's workgroups (all threads call it once, at the end). The counter is
// zeroed before the launch. Data that the last workgroup reads from the
// others must be written and read with device-scope atomics (performed at
// the point of coherence of all XCDs): each thread waits for its own memory
// operations to complete before the workgroup counts itself, so every such
// atomic precedes the increment that lets the last workgroup through. (A
// release fence would write back the XCD's whole L2 in every workgroup.)
__device__ __forceinline__ bool grid_last_block(uint32_t* counter) {
  __shared__ uint32_t last_sh;
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t total = gridDim.x * gridDim.y * gridDim.z;
    last_sh = (atomicAdd(counter, 1u) == total - 1u) ? 1u : 0u;
  }
  __syncthreads();
  return last_sh != 0u;
}

// The last workgroup of a launch writes the call's status code from the
// status bits (bits[0]; bits[1] is the workgroup counter) to dev_status,
// when given. All threads call it once, at the end of the kernel.
__device__ __forceinline__ void grid_finish_status(uint32_t* bits, int32_t* dev_status) {
  if (dev_status == nullptr) return;
  if (grid_last_block(bits + 1) && threadIdx.x == 0)
    *dev_status = status_code(atomicOr(bits, 0u));
}

// Copies stream segment [x lo, x hi, cnt words] to dst with `lanes` lanes
// (lane l handles words l, l+lanes, ...).
__device__ __forceinline__ void pack_segment(uint16_t* __restrict__ dst, uint32_t x,
                                             const uint16_t* __restrict__ src, uint32_t cnt,
                                             int l, int lanes) {
  for (int64_t t = l; t < (int64_t)cnt + 2; t += lanes) {
    uint16_t wv;
    if (t == 0) wv = (uint16_t)(x & 0xFFFFu);
    else if (t == 1) wv = (uint16_t)(x >> 16);
    else wv = src[t - 2];
    dst[t] = wv;
  }
}

// Register copy the compiler cannot coalesce away (an early-clobber output
// never shares a register with the input).
__device__ __forceinline__ float opaque_copy(float v) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=&v"(r) : "v"(v));
  return r;
}

// Decode of stream s of one latent by one lane (binary search) or by a
// group of L lanes ((L+1)-ary search); lane g == 0 of the group writes the
// symbols. The next element's parameters and the next renormalisation word
// are loaded ahead of the dependent chain. Returns true if the stream fails
// the integrity checks.
//
// With kGather the coded sequence is the subset idx[0..n) of a latent of
// n_total elements: pass position i reads its parameters at element idx[i]
// of the [K][n_total] planes and writes its symbol to sym[idx[i]].
// kBracket selects the bracketed search for one lane per stream (search_bs);
// kRing1 the depth of the parameter ring with one lane per stream.
// With kBuf the parameters, the refill words and the symbols go through
// buffer resources with 32-bit byte offsets: one offset per step for all
// 3K parameter loads (the plane rows at constant scalar offsets k n 4), no
// 64-bit address arithmetic, and no clamp for the refill word (a word past
// the bitstream reads 0 by the resource's range check). The caller selects
// it only when every offset fits: buffer_offsets_fit below.
template <int K, int kKind, bool kFast, int L, bool kGather = false, bool kBracket = false,
          bool kBuf = false, int kRing1 = 3>
__device__ __forceinline__ bool decode_stream(const QCfg& q, int P, int rounds, int64_t n,
                                              int64_t S, int64_t s, int g,
                                              const uint16_t* __restrict__ bs, int64_t total_words,
                                              const int64_t* __restrict__ offsets,
                                              const float* __restrict__ w,
                                              const float* __restrict__ mu,
                                              const float* __restrict__ sg,
                                              int32_t* __restrict__ sym,
                                              const int32_t* __restrict__ idx = nullptr,
                                              int64_t n_total = 0) {
  const int64_t np = kGather ? n_total : n;  // plane stride
  const int lane = threadIdx.x & 63;
  const int gbase = lane - g;
  const uint64_t gmask = (L >= 64) ? ~0ull : (((1ull << L) - 1ull) << gbase);
  const int64_t ns = stream_len(n, S, s);
  const int64_t a = offsets[s], b = offsets[s + 1];
  if (a < 0 || b < a + 2 || b > total_words) {
    if (g == 0)
      for (int64_t p = 0; p < ns; ++p) sym[kGather ? gather_index(idx, s + p * S, n_total) : s + p * S] = q.lo;
    return true;
  }
  uint32_t x = (uint32_t)bs[a] | ((uint32_t)bs[a + 1] << 16);
  int64_t ptr = a + 2;
  uint32_t nword = (ptr < b) ? bs[ptr] : 0u;
  bool bad = x < (1u << 16);
  const uint32_t mask = q.M - 1;
  if (ns == 0) return bad || x != (1u << 16) || ptr != b;
  const int nfree = (L == 1) ? free_rounds(rounds, q.N) : 0;
  // Software pipeline over the stream's steps. Each step issues, after its
  // own refill, first the bitstream word the next step's refill may need and
  // then the parameters of the element kRing steps ahead into a ring of
  // register sets. Vector loads retire in issue order, so with this order a
  // wait for the word never waits for parameters issued after it, and the
  // parameters get kRing - 1 whole steps to arrive. Every load is
  // unconditional (positions past the end reload the last element or word)
  // so the number of loads per step is fixed and the wait counts stay exact.
  // kRing1 is the depth with one lane per stream: 4 for the whole-latent
  // decode on buffer resources (4K decode 244.9 -> 236.3 us alternated on
  // one box; 2, 5 and 6 steps 248.6, 236.6 and 235.4 us), 3 elsewhere
  // (the batched kernels, which share SIMDs among several wavefronts, lost
  // on the 256-latent plan with 4: 11.71 -> 11.99 ms).
  constexpr int kRing = (L == 1) ? kRing1 : 2;
  const int64_t last = ns - 1;
  static_assert(!(kBuf && kGather), "the buffer path reads the planes in stream order");
  [[maybe_unused]] __amdgpu_buffer_rsrc_t bw_, bm_, bsg_, bbs_, bsym_;
  [[maybe_unused]] uint32_t off_next = 0, off_last = 0, plane = 0;
  [[maybe_unused]] uint32_t ro[kRing] = {};
  if constexpr (kBuf) {
    const int nb = (int)(uint32_t)(K * n * 4);
    bw_ = __builtin_amdgcn_make_buffer_rsrc((void*)w, (short)0, nb, kRsrcWord3);
    bm_ = __builtin_amdgcn_make_buffer_rsrc((void*)mu, (short)0, nb, kRsrcWord3);
    bsg_ = __builtin_amdgcn_make_buffer_rsrc((void*)sg, (short)0, nb, kRsrcWord3);
    bbs_ = __builtin_amdgcn_make_buffer_rsrc((void*)bs, (short)0,
                                             (int)(uint32_t)(total_words * 2), kRsrcWord3);
    bsym_ = __builtin_amdgcn_make_buffer_rsrc((void*)sym, (short)0, (int)(uint32_t)(n * 4),
                                              kRsrcWord3);
    plane = (uint32_t)(n * 4);
    off_next = (uint32_t)s * 4u;  // the element of position 0
    off_last = (uint32_t)(s + last * S) * 4u;
  }
  auto elem_at = [&](int64_t p) -> int64_t {
    const int64_t pp = p < last ? p : last;
    return kGather ? gather_index(idx, s + pp * S, n_total) : s + pp * S;
  };
  // The first pass (p0 = -kRing) only issues the ring's first loads, so
  // every load comes from the loop body in one fixed order.
  float rw[kRing][K] = {}, rm[kRing][K] = {}, rs[kRing][K] = {};
  int64_t rg[kRing] = {};
  for (int64_t p0 = -kRing; p0 < ns; p0 += kRing) {
#pragma unroll
    for (int d = 0; d < kRing; ++d) {
      const int64_t p = p0 + d;
      const bool live = p >= 0 && p < ns;
      const uint32_t slot = x & mask;
      uint32_t cl = 0, ch = q.M;
      if (live) {
        // With 64-bit addresses: copies that the register allocator cannot
        // merge with the ring slot, so that the slot keeps one register set
        // and the wait for its loads lands here instead of at the loop's
        // back edge. With buffer loads plain copies measured faster (4K
        // decode 268-270 -> 262-265 us, 8-lane decode of the 4,096-stream
        // latent 124.3-125.3 -> 121.8-122.0 us).
        float cw[K], cm[K], cs[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if constexpr (kBuf) {
            cw[k] = rw[d][k];
            cm[k] = rm[d][k];
            cs[k] = rs[d][k];
          } else {
            cw[k] = opaque_copy(rw[d][k]);
            cm[k] = opaque_copy(rm[d][k]);
            cs[k] = opaque_copy(rs[d][k]);
          }
        }
        const Elem<K> e = make_elem<K, kFast, kKind>(q, cw, cm, cs);
        int32_t j;
        if (L == 1)
          j = search_bs<K, kKind, kFast, kBracket>(e, q, rounds, nfree, slot, cl, ch);
        else
          j = search_group<K, kKind, kFast, L>(e, q, rounds, slot, g, gbase, gmask, 0, q.N, cl,
                                               ch);
        if constexpr (kBuf) {
          if (g == 0)
            __builtin_amdgcn_raw_buffer_store_b32((uint32_t)(q.lo + j), bsym_, ro[d], 0, 0);
        } else {
          if (g == 0) sym[rg[d]] = q.lo + j;
        }
      }
      // State update and refill outside the branch, as selects: the word is
      // then used on every path, which keeps its load where it is issued.
      const uint32_t xs = (ch - cl) * (x >> P) + slot - cl;
      const bool refill = live && xs < (1u << 16);
      const bool have = ptr < b;
      const uint32_t xr = refill ? ((xs << 16) | (have ? nword : 0u)) : xs;
      x = live ? xr : x;
      bad = bad || (refill && !have);
      ptr += (refill && have) ? 1 : 0;
      if constexpr (kBuf) {
        // ptr <= b <= total_words: a word past the bitstream reads 0
        nword = __builtin_amdgcn_raw_buffer_load_b16(bbs_, (uint32_t)ptr * 2u, 0, 0);
        asm volatile("" ::: "memory");  // keep the word's load ahead of the ring's
        // the element of position p + kRing, clamped to the stream's last
        const uint32_t o = off_next < off_last ? off_next : off_last;
        ro[d] = o;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          rw[d][k] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(bw_, o, k * plane, 0));
          rm[d][k] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(bm_, o, k * plane, 0));
          rs[d][k] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(bsg_, o, k * plane, 0));
        }
        off_next += (uint32_t)S * 4u;
      } else {
        nword = bs[ptr < b ? ptr : b - 1];
        asm volatile("" ::: "memory");  // keep the word's load ahead of the ring's
        rg[d] = elem_at(p + kRing);
        load_raw<K>(w, mu, sg, np, rg[d], rw[d], rm[d], rs[d]);
      }
    }
  }
  return bad || x != (1u << 16) || ptr != b;
}

// The looped binary search of search_bs for two elements at once: both run
// the same rounds, so each round holds two independent CDF evaluations.
template <int K, int kKind, bool kFast>
__device__ __forceinline__ void search_bs2(const Elem<K>& ea, const Elem<K>& eb, const QCfg& q,
                                           int rounds, int nfree, uint32_t sla, uint32_t slb,
                                           int32_t& ja, uint32_t& cla, uint32_t& cha,
                                           int32_t& jb, uint32_t& clb, uint32_t& chb) {
  int32_t la = 0, lb = 0;
  cla = 0;
  clb = 0;
  cha = q.M;
  chb = q.M;
  int r = rounds - 1;
  for (int i = 0; i < nfree; ++i, --r) {
    const int32_t ma = la + (1 << r), mb = lb + (1 << r);
    const uint32_t ca = cdf_inner<K, kKind, kFast>(ea, q, ma);
    const uint32_t cb = cdf_inner<K, kKind, kFast>(eb, q, mb);
    const bool ra = sla >= ca, rb = slb >= cb;
    la = ra ? ma : la;
    cla = ra ? ca : cla;
    cha = ra ? cha : ca;
    lb = rb ? mb : lb;
    clb = rb ? cb : clb;
    chb = rb ? chb : cb;
  }
  for (; r >= 0; --r) {
    const int32_t ma = la + (1 << r), mb = lb + (1 << r);
    const uint32_t ca = cdf_upper<K, kKind, kFast>(ea, q, ma);
    const uint32_t cb = cdf_upper<K, kKind, kFast>(eb, q, mb);
    const bool ra = sla >= ca, rb = slb >= cb;
    la = ra ? ma : la;
    cla = ra ? ca : cla;
    cha = ra ? cha : ca;
    lb = rb ? mb : lb;
    clb = rb ? cb : clb;
    chb = rb ? chb : cb;
  }
  ja = la;
  jb = lb;
}

// Decode of two streams sa < sb of one latent by one lane (two streams per
// lane): the streams' steps run in lock-step in one loop and a step's two
// searches share their rounds, so every step holds two independent
// dependency chains, with half the wavefronts of one stream per lane. The
// software pipeline is decode_stream's with a ring of two steps per stream.
// sb >= S leaves the lane one stream: the second chain then repeats sa's
// loads and never writes. sb's stream is never longer than sa's. A lane
// whose offsets fail the checks decodes its streams one at a time with
// decode_stream, which writes and reports them. Returns true if either
// stream fails the integrity checks.
template <int K, int kKind, bool kFast>
__device__ __forceinline__ bool decode_stream2(const QCfg& q, int P, int rounds, int64_t n,
                                               int64_t S, int64_t sa, int64_t sb,
                                               const uint16_t* __restrict__ bs,
                                               int64_t total_words,
                                               const int64_t* __restrict__ offsets,
                                               const float* __restrict__ w,
                                               const float* __restrict__ mu,
                                               const float* __restrict__ sg,
                                               int32_t* __restrict__ sym) {
  const bool two = sb < S;
  const int64_t a0 = offsets[sa], a1 = offsets[sa + 1];
  const int64_t b0 = two ? offsets[sb] : a0, b1 = two ? offsets[sb + 1] : a1;
  if (a0 < 0 || a1 < a0 + 2 || a1 > total_words || b0 < 0 || b1 < b0 + 2 || b1 > total_words) {
    bool bad = false;
    for (int j = 0; j < (two ? 2 : 1); ++j)
      bad = decode_stream<K, kKind, kFast, 1>(q, P, rounds, n, S, j ? sb : sa, 0, bs,
                                              total_words, offsets, w, mu, sg, sym) ||
            bad;
    return bad;
  }
  const int64_t na = stream_len(n, S, sa), nb = two ? stream_len(n, S, sb) : 0;
  uint32_t xa = (uint32_t)bs[a0] | ((uint32_t)bs[a0 + 1] << 16);
  uint32_t xb = (uint32_t)bs[b0] | ((uint32_t)bs[b0 + 1] << 16);
  int64_t pa = a0 + 2, pb = b0 + 2;
  uint32_t wa = (pa < a1) ? bs[pa] : 0u, wb = (pb < b1) ? bs[pb] : 0u;
  bool bad = xa < (1u << 16) || (two && xb < (1u << 16));
  const uint32_t mask = q.M - 1;
  if (na > 0) {
    const int nfree = free_rounds(rounds, q.N);
    constexpr int kRing = 2;
    // element of position p of each stream, clamped to its last element (an
    // empty second stream follows the first, so every load stays in the latent)
    auto elem_a = [&](int64_t p) -> int64_t { return sa + (p < na - 1 ? p : na - 1) * S; };
    auto elem_b = [&](int64_t p) -> int64_t {
      return nb > 0 ? sb + (p < nb - 1 ? p : nb - 1) * S : elem_a(p);
    };
    float aw[kRing][K] = {}, am[kRing][K] = {}, as[kRing][K] = {};
    float bw[kRing][K] = {}, bm[kRing][K] = {}, bsg[kRing][K] = {};
    int64_t ga[kRing] = {}, gb[kRing] = {};
    for (int64_t p0 = -kRing; p0 < na; p0 += kRing) {
#pragma unroll
      for (int d = 0; d < kRing; ++d) {
        const int64_t p = p0 + d;
        const bool liva = p >= 0 && p < na, livb = p >= 0 && p < nb;
        const uint32_t sla = xa & mask, slb = xb & mask;
        uint32_t cla = 0, cha = q.M, clb = 0, chb = q.M;
        if (liva) {
          float cw[K], cm[K], cs[K], dw[K], dm[K], ds[K];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            cw[k] = opaque_copy(aw[d][k]);
            cm[k] = opaque_copy(am[d][k]);
            cs[k] = opaque_copy(as[d][k]);
            dw[k] = opaque_copy(bw[d][k]);
            dm[k] = opaque_copy(bm[d][k]);
            ds[k] = opaque_copy(bsg[d][k]);
          }
          const Elem<K> ea = make_elem<K, kFast, kKind>(q, cw, cm, cs);
          const Elem<K> eb = make_elem<K, kFast, kKind>(q, dw, dm, ds);
          int32_t ja, jb;
          search_bs2<K, kKind, kFast>(ea, eb, q, rounds, nfree, sla, slb, ja, cla, cha, jb, clb,
                                      chb);
          sym[ga[d]] = q.lo + ja;
          if (livb) sym[gb[d]] = q.lo + jb;
        }
        const uint32_t xsa = (cha - cla) * (xa >> P) + sla - cla;
        const uint32_t xsb = (chb - clb) * (xb >> P) + slb - clb;
        const bool ra = liva && xsa < (1u << 16), rb = livb && xsb < (1u << 16);
        const bool ha = pa < a1, hb = pb < b1;
        const uint32_t xra = ra ? ((xsa << 16) | (ha ? wa : 0u)) : xsa;
        const uint32_t xrb = rb ? ((xsb << 16) | (hb ? wb : 0u)) : xsb;
        xa = liva ? xra : xa;
        xb = livb ? xrb : xb;
        bad = bad || (ra && !ha) || (rb && !hb);
        pa += (ra && ha) ? 1 : 0;
        pb += (rb && hb) ? 1 : 0;
        wa = bs[pa < a1 ? pa : a1 - 1];
        wb = bs[pb < b1 ? pb : b1 - 1];
        asm volatile("" ::: "memory");  // keep the words' loads ahead of the rings'
        ga[d] = elem_a(p + kRing);
        gb[d] = elem_b(p + kRing);
        load_raw<K>(w, mu, sg, n, ga[d], aw[d], am[d], as[d]);
        load_raw<K>(w, mu, sg, n, gb[d], bw[d], bm[d], bsg[d]);
      }
    }
  }
  bad = bad || xa != (1u << 16) || pa != a1;
  if (two) bad = bad || xb != (1u << 16) || pb != b1;
  return bad;
}

}  // namespace fgmm
