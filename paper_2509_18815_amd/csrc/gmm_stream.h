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
#include "gmm_device.h"

namespace fgmm {

__device__ __forceinline__ int64_t stream_len(int64_t n, int64_t S, int64_t s) {
  return (s < n) ? (n - 1 - s) / S + 1 : 0;
}

// Branch-uniform binary search for the j with c_j <= slot < c_{j+1}:
// exactly `rounds` = ceil(log2 N) CDF evaluations; on return c_lo = c_j and
// c_hi = c_{j+1}. Once the interval holds one symbol, mid = lo re-evaluates
// c_lo and changes nothing, so every lane runs the same instruction stream.
template <int K, int kKind, bool kFast>
__device__ __forceinline__ int32_t search_bs(const Elem<K>& e, const QCfg& q, int rounds,
                                             uint32_t slot, uint32_t& c_lo, uint32_t& c_hi) {
  int32_t lo = 0, hi = q.N;
  c_lo = 0;
  c_hi = q.M;
  for (int r = 0; r < rounds; ++r) {
    const int32_t mid = (lo + hi) >> 1;
    const uint32_t c = cdf_at<K, kKind, kFast>(e, q, mid);
    const bool right = slot >= c;
    lo = right ? mid : lo;
    c_lo = right ? c : c_lo;
    hi = right ? hi : mid;
    c_hi = right ? c_hi : c;
  }
  return lo;
}

// (L+1)-ary search by a group of L lanes (lane g of the group, group mask
// gmask, first lane gbase): each round the lanes evaluate the CDF at L split
// points of [lo, hi); a ballot counts the points at or below the slot and the
// interval shrinks to one of the L+1 parts. The split points are
// non-decreasing in g and below hi, so the count selects the right part.
template <int K, int kKind, bool kFast, int L>
__device__ __forceinline__ int32_t search_group(const Elem<K>& e, const QCfg& q, int rounds,
                                                uint32_t slot, int g, int gbase, uint64_t gmask,
                                                int32_t lo, int32_t hi, uint32_t& c_lo,
                                                uint32_t& c_hi) {
  for (int r = 0; r < rounds; ++r) {
    const uint32_t sz = (uint32_t)(hi - lo);
    const int32_t m = lo + (int32_t)((sz * (uint32_t)(g + 1)) / (uint32_t)(L + 1));
    const uint32_t c = cdf_at<K, kKind, kFast>(e, q, m);
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
// 16 bits: c_j < M <= 2^16 for j < N, f_j <= M - N + 1 < 2^16).
template <int K, int kKind, bool kFast>
__device__ __forceinline__ uint32_t enc_cdf_elem(const QCfg& q, int64_t n, int64_t i,
                                                 const int32_t* __restrict__ sym,
                                                 const float* __restrict__ w,
                                                 const float* __restrict__ mu,
                                                 const float* __restrict__ sg, uint32_t* status) {
  float rw[K], rm[K], rs[K];
  load_raw<K>(w, mu, sg, n, i, rw, rm, rs);
  int32_t j = sym[i] - q.lo;
  if (j < 0 || j >= q.N) {
    atomicOr(status, kStRange);
    j = 0;
  }
  const Elem<K> e = make_elem<K, kFast>(rw, rm, rs);
  const uint32_t c0 = cdf_at<K, kKind, kFast>(e, q, j);
  const uint32_t c1 = cdf_at<K, kKind, kFast>(e, q, j + 1);
  return (c0 << 16) | (c1 - c0);
}

// Encode phase 2 for stream s: the integer rANS recurrence over the packed
// (c, f) words cf[s + p S], p = n_s-1 .. 0. The k-th emitted word goes to
// region_end[-k], so the words end up in the order the decoder reads them.
// Returns the final state; *count receives the number of words.
__device__ __forceinline__ uint32_t rans_stream(int64_t n, int64_t S, int P, int64_t s,
                                                const uint32_t* __restrict__ cf,
                                                uint16_t* __restrict__ region_end,
                                                uint32_t* count) {
  const int64_t ns = stream_len(n, S, s);
  uint32_t x = 1u << 16;
  uint32_t cnt = 0;
  const int shift = 32 - P;
  // (c, f) words are fetched kDepth steps ahead of the dependent chain
  constexpr int kDepth = 8;
  uint32_t buf[kDepth];
#pragma unroll
  for (int d = 0; d < kDepth; ++d) {
    const int64_t pp = ns - 1 - d;
    buf[d] = (pp >= 0) ? cf[s + pp * S] : 0u;
  }
  for (int64_t p = ns - 1; p >= 0; p -= kDepth) {
    uint32_t cur[kDepth];
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      cur[d] = buf[d];
      const int64_t pp = p - kDepth - d;
      buf[d] = (pp >= 0) ? cf[s + pp * S] : 0u;
    }
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      if (p - d < 0) break;
      const uint32_t c = cur[d] >> 16;
      const uint32_t f = cur[d] & 0xFFFFu;
      if (x >= (f << shift)) {
        region_end[-(int64_t)cnt] = (uint16_t)(x & 0xFFFFu);
        ++cnt;
        x >>= 16;
      }
      const uint32_t qd = x / f;
      x = (qd << P) + (x - qd * f) + c;
    }
  }
  *count = cnt;
  return x;
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

// Exclusive scan of nblk int64 block totals in one workgroup of 1024
// threads, tile by tile with a running carry.
constexpr int kScanBlock = 1024;
__device__ __forceinline__ void scan_totals(int64_t nblk, const int64_t* __restrict__ tot,
                                            int64_t* __restrict__ pre) {
  __shared__ int64_t wsum[kScanBlock / 64];
  __shared__ int64_t carry_sh;
  if (threadIdx.x == 0) carry_sh = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t base = 0; base < nblk; base += kScanBlock) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = (i < nblk) ? tot[i] : 0;
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
    if (threadIdx.x == kScanBlock - 1) carry_sh = off + incl;
    __syncthreads();
  }
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

// Decode of stream s of one latent by one lane (binary search) or by a
// group of L lanes ((L+1)-ary search); lane g == 0 of the group writes the
// symbols. The next element's parameters and the next renormalisation word
// are loaded ahead of the dependent chain. Returns true if the stream fails
// the integrity checks.
template <int K, int kKind, bool kFast, int L>
__device__ __forceinline__ bool decode_stream(const QCfg& q, int P, int rounds, int64_t n,
                                              int64_t S, int64_t s, int g,
                                              const uint16_t* __restrict__ bs, int64_t total_words,
                                              const int64_t* __restrict__ offsets,
                                              const float* __restrict__ w,
                                              const float* __restrict__ mu,
                                              const float* __restrict__ sg,
                                              int32_t* __restrict__ sym) {
  const int lane = threadIdx.x & 63;
  const int gbase = lane - g;
  const uint64_t gmask = (L >= 64) ? ~0ull : (((1ull << L) - 1ull) << gbase);
  const int64_t ns = stream_len(n, S, s);
  const int64_t a = offsets[s], b = offsets[s + 1];
  if (a < 0 || b < a + 2 || b > total_words) {
    if (g == 0)
      for (int64_t p = 0; p < ns; ++p) sym[s + p * S] = q.lo;
    return true;
  }
  uint32_t x = (uint32_t)bs[a] | ((uint32_t)bs[a + 1] << 16);
  int64_t ptr = a + 2;
  uint32_t nword = (ptr < b) ? bs[ptr] : 0u;
  bool bad = x < (1u << 16);
  const uint32_t mask = q.M - 1;
  float nw[K], nm[K], nsg[K];
  if (ns > 0) load_raw<K>(w, mu, sg, n, s, nw, nm, nsg);
  for (int64_t p = 0; p < ns; ++p) {
    const int64_t i = s + p * S;
    float cw[K], cm[K], cs[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      cw[k] = nw[k];
      cm[k] = nm[k];
      cs[k] = nsg[k];
    }
    if (p + 1 < ns) load_raw<K>(w, mu, sg, n, i + S, nw, nm, nsg);
    const Elem<K> e = make_elem<K, kFast>(cw, cm, cs);
    const uint32_t slot = x & mask;
    uint32_t cl = 0, ch = q.M;
    int32_t j;
    if (L == 1)
      j = search_bs<K, kKind, kFast>(e, q, rounds, slot, cl, ch);
    else
      j = search_group<K, kKind, kFast, L>(e, q, rounds, slot, g, gbase, gmask, 0, q.N, cl, ch);
    if (g == 0) sym[i] = q.lo + j;
    x = (ch - cl) * (x >> P) + slot - cl;
    if (x < (1u << 16)) {
      if (ptr < b) {
        x = (x << 16) | nword;
        ++ptr;
        nword = (ptr < b) ? bs[ptr] : 0u;
      } else {
        bad = true;
        x <<= 16;
      }
    }
  }
  return bad || x != (1u << 16) || ptr != b;
}

}  // namespace fgmm
