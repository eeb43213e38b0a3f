// Device side of the learned search bracket (shared by the single-latent
// and the batched decode kernels).
//
// Per decoded symbol an MLP predicts the symbol from the element's mixture
// parameters and the rANS slot. The decoder evaluates the exact quantized
// CDF at both ends of the bracket [p - R, p + R] around the prediction
// (clamped to [slot - (M - N), slot], the only indices the quantization
// allows for this slot) and, if the slot falls inside, finishes with a
// binary search of the bracket; otherwise on the side the slot fell. The
// decoded symbol is the unique j with c_j <= slot < c_{j+1} either way, so
// the output is bit-identical to the plain binary search.
//
// The MLP (D -> 64 -> 64 -> 1, bfloat16 weights, float32 accumulation) runs
// on the matrix cores for the 64 lanes of a wavefront at once: hidden units
// are rows and samples columns, layer 1 is four and layer 2 sixteen
// v_mfma_f32_32x32x16_bf16. Hidden units are permuted when the model is
// loaded so that layer 1's accumulator registers are exactly layer 2's B
// operand in every lane (no LDS transpose).
//
// Wavefront-cooperative fallback: after the bracket's binary rounds the
// lanes whose slot fell outside their bracket (m of them) get 64/m lanes
// each, which finish the search (L+1)-ary — one or two rounds instead of
// five when few lanes miss.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gmm_device.h"
#include "gmm_mlp.h"
#include "gmm_stream.h"

namespace fgmm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Device image of a bracket model. Operand fragment (lane l, block m) holds
// the bfloat16 pair words of A[l % 32][8 (l / 32) + e], e = 0..7 (the
// v_mfma_f32_32x32x16_bf16 A-operand layout).
struct BracketDev {
  uint32_t wa1[64][2][4];     // W1 rows 32 mb + (l % 32), inputs 8 (l / 32) + e
  uint32_t wa2[64][2][4][4];  // W2 rows 32 mb2 + (l % 32), k block kb (permuted inputs)
  float b1v[2][32];           // [lane half][16 mb + r]: bias of accumulator row
  float b2v[2][32];
  float w3v[2][32];
  float b3, out_mean, out_std, pad0;
  float in_mean[16], in_inv_std[16];
  int32_t K, D, radius, pad1;
};

// Per-wavefront LDS: the model's per-lane-half bias and output weights
// (read with lane-half-uniform addresses, i.e. broadcast) and the table of
// the cooperative fallback.
struct BracketLds {
  float b1[2][32], b2[2][32], w3[2][32];
  int32_t owner[64];
};

struct LaneModel {
  bf16x8 a1[2];
  bf16x8 a2[2][4];
};

__device__ __forceinline__ bf16x8 bracket_frag(const uint32_t* p) {
  u32x4 v;
  v[0] = p[0];
  v[1] = p[1];
  v[2] = p[2];
  v[3] = p[3];
  return __builtin_bit_cast(bf16x8, v);
}

// Loads the lane's operand fragments into registers and the vectors into
// LDS (the workgroup is one wavefront).
__device__ __forceinline__ void load_lane_model(const BracketDev* __restrict__ br, LaneModel& m,
                                                BracketLds& lds) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) m.a1[mb] = bracket_frag(br->wa1[l][mb]);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) m.a2[mb][kb] = bracket_frag(br->wa2[l][mb][kb]);
  (&lds.b1[0][0])[l] = (&br->b1v[0][0])[l];
  (&lds.b2[0][0])[l] = (&br->b2v[0][0])[l];
  (&lds.w3[0][0])[l] = (&br->w3v[0][0])[l];
  __syncthreads();
}

// Prediction for this lane's sample from its normalised features x (all 64
// lanes of the wavefront call it together).
__device__ __forceinline__ float mlp_wave(const BracketDev* __restrict__ br, const LaneModel& m,
                                          const BracketLds& lds, const float (&x)[16]) {
  const int l = threadIdx.x & 63;
  const int hh = l >> 5;
  bf16x8 lo8, hi8;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    lo8[e] = (__bf16)x[e];
    hi8[e] = (__bf16)x[8 + e];
  }
  // The B operand of column block nb holds features 8 hh .. 8 hh + 7 of
  // sample 32 nb + l % 32: lanes trade the half they do not keep with l ^ 32.
  const u32x4 send = __builtin_bit_cast(u32x4, hh ? lo8 : hi8);
  u32x4 recv;
#pragma unroll
  for (int j = 0; j < 4; ++j) recv[j] = __shfl_xor(send[j], 32, 64);
  const bf16x8 other = __builtin_bit_cast(bf16x8, recv);
  float res = 0.0f;
  // one column block at a time keeps the accumulators of only one live
#pragma unroll 1
  for (int nb = 0; nb < 2; ++nb) {
    const bf16x8 bx = (nb == 0) ? (hh ? other : lo8) : (hh ? hi8 : other);
    f32x16 acc1[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) acc1[mb][r] = lds.b1[hh][16 * mb + r];
      acc1[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m.a1[mb], bx, acc1[mb], 0, 0, 0);
    }
    bf16x8 b2op[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        b2op[kb][e] = (__bf16)__builtin_fmaxf(acc1[kb >> 1][8 * (kb & 1) + e], 0.0f);
    float part = 0.0f;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      f32x16 acc2;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc2[r] = lds.b2[hh][16 * mb + r];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m.a2[mb][kb], b2op[kb], acc2, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) part = fmaf(lds.w3[hh][16 * mb + r], __builtin_fmaxf(acc2[r], 0.0f), part);
    }
    part += __shfl_xor(part, 32, 64);
    if (nb == hh) res = part;
  }
  return fmaf(res + br->b3, br->out_std, br->out_mean);
}

template <int K>
__device__ __forceinline__ void lane_features(const BracketDev* __restrict__ br,
                                              const float (&w)[K], const float (&mu)[K],
                                              const float (&sg)[K], uint32_t slot, float inv_m,
                                              float (&x)[16]) {
#pragma unroll
  for (int d = 0; d < 16; ++d)
    x[d] = (d <= 3 * K) ? (mlp_raw_feature<K>(d, w, mu, sg, slot, inv_m) - br->in_mean[d]) *
                              br->in_inv_std[d]
                        : 0.0f;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Rounds of an (L+1)-ary search to shrink an interval of size sz to one.
__device__ __forceinline__ int rounds_for(int32_t sz, int L) {
  int r = 0;
  int32_t reach = 1;
  while (reach < sz) {
    reach *= (L + 1);
    ++r;
  }
  return r;
}

// Decodes streams s0 .. s0+63 (those below S) of one latent with the bracket.
// Every lane runs every step of the wavefront's longest stream (finished
// lanes compute on placeholder data and store nothing): the matrix-core
// inference and the cooperative fallback need all 64 lanes.
// Counters (per lane): hit / miss symbols; lane 0 also counts wavefront
// steps and the steps on which every active lane hit.
template <int K, int kKind, bool kFast>
__device__ __forceinline__ void bracket_decode_wave(
    const QCfg& q, int P, int64_t n, int64_t S, int64_t s0, const uint16_t* __restrict__ bs,
    int64_t total_words, const int64_t* __restrict__ offsets, const float* __restrict__ w,
    const float* __restrict__ mu, const float* __restrict__ sg, int32_t* __restrict__ sym,
    uint32_t* status, const BracketDev* __restrict__ br, const LaneModel& model,
    BracketLds& lds, unsigned long long (&cnt)[4]) {
  const int l = threadIdx.x & 63;
  const int64_t s = s0 + l;
  const int R = br->radius;
  const int64_t ns_max = stream_len(n, S, s0);  // lower-index streams are never shorter
  const int64_t ns = (s < S) ? stream_len(n, S, s) : 0;
  bool seg_ok = false;
  int64_t a = 0, b = 0;
  if (s < S) {
    a = offsets[s];
    b = offsets[s + 1];
    seg_ok = !(a < 0 || b < a + 2 || b > total_words);
  }
  bool bad = (s < S) && !seg_ok;
  if (bad)
    for (int64_t p = 0; p < ns; ++p) sym[s + p * S] = q.lo;
  uint32_t x = seg_ok ? ((uint32_t)bs[a] | ((uint32_t)bs[a + 1] << 16)) : (1u << 16);
  int64_t ptr = a + 2;
  uint32_t nword = (seg_ok && ptr < b) ? bs[ptr] : 0u;
  if (seg_ok && x < (1u << 16)) bad = true;
  const uint32_t mask = q.M - 1;
  const float inv_m = 1.0f / (float)q.M;
  float nw[K], nm[K], nsg[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    nw[k] = 0.0f;
    nm[k] = 0.0f;
    nsg[k] = 1.0f;
  }
  if (seg_ok && ns > 0) load_raw<K>(w, mu, sg, n, s, nw, nm, nsg);
  for (int64_t p = 0; p < ns_max; ++p) {
    const bool act = seg_ok && p < ns;
    const int64_t i = s + p * S;
    float cw[K], cm[K], cs[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      cw[k] = nw[k];
      cm[k] = nm[k];
      cs[k] = nsg[k];
    }
    if (seg_ok) load_raw<K>(w, mu, sg, n, (p + 1 < ns) ? i + S : s + (ns > 0 ? ns - 1 : 0) * S,
                            nw, nm, nsg);
    const Elem<K> e = make_elem<K, kFast, kKind>(q, cw, cm, cs);
    const uint32_t slot = x & mask;
    float feat[16];
    lane_features<K>(br, cw, cm, cs, slot, inv_m, feat);
    const float pred = mlp_wave(br, model, lds, feat);
    // bracket around the prediction, inside [slot - (M - N), slot]
    const int32_t jmin = max(0, (int32_t)slot - (int32_t)(q.M - (uint32_t)q.N));
    const int32_t jmax = min(q.N - 1, (int32_t)slot);
    const float pc = __builtin_fminf(__builtin_fmaxf(pred - (float)q.lo, -1.0f), (float)q.N);
    const int32_t jh = min(max((int32_t)__builtin_rintf(pc), jmin), jmax);
    const int32_t ba = max(jh - R, 0), bb = min(jh + R, q.N - 1);
    const uint32_t c_a = cdf_at<K, kKind, kFast>(e, q, ba);
    const uint32_t c_b = cdf_at<K, kKind, kFast>(e, q, bb + 1);
    const bool hit = (c_a <= slot) && (slot < c_b);
    int32_t lo, hi;
    uint32_t c_lo, c_hi;
    if (hit) {
      lo = ba; hi = bb + 1; c_lo = c_a; c_hi = c_b;
    } else if (slot < c_a) {
      lo = 0; hi = ba; c_lo = 0; c_hi = c_a;
    } else {
      lo = bb + 1; hi = q.N; c_lo = c_b; c_hi = q.M;
    }
    if (!act) {
      lo = 0; hi = 1; c_lo = 0; c_hi = q.M;
    }
    // binary rounds that finish every bracket (a miss interval shrinks too)
    const int r1 = rounds_for(2 * R + 1, 1);
    for (int r = 0; r < r1; ++r) {
      const int32_t mid = (lo + hi) >> 1;
      const uint32_t c = cdf_at<K, kKind, kFast>(e, q, mid);
      const bool right = slot >= c;
      lo = right ? mid : lo;
      c_lo = right ? c : c_lo;
      hi = right ? hi : mid;
      c_hi = right ? c_hi : c;
    }
    // cooperative fallback for the lanes still holding more than one symbol
    const uint64_t open = __ballot(hi - lo > 1);
    if (open) {
      const int m = __popcll(open);
      int L = 64 / m;
      L = (L >= 32) ? 32 : (L >= 16) ? 16 : (L >= 8) ? 8 : (L >= 4) ? 4 : (L >= 2) ? 2 : 1;
      const int rank = __popcll(open & ((1ull << l) - 1ull));
      if (hi - lo > 1) lds.owner[rank] = l;
      __syncthreads();
      const int grp = l / L, gl = l % L;
      const int owner = (grp < m) ? lds.owner[grp] : l;
      // the owner's element, slot and interval
      Elem<K> eo;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        eo.w[k] = __shfl(e.w[k], owner, 64);
        eo.mu[k] = __shfl(e.mu[k], owner, 64);
        eo.r[k] = __shfl(e.r[k], owner, 64);
      }
      const uint32_t so = __shfl(slot, owner, 64);
      int32_t glo = __shfl(lo, owner, 64), ghi = __shfl(hi, owner, 64);
      uint32_t gclo = __shfl(c_lo, owner, 64), gchi = __shfl(c_hi, owner, 64);
      const int rounds = wave_max(rounds_for(ghi - glo, L));
      const int gbase = grp * L;
      const uint64_t gmask = (L == 64) ? ~0ull : (((1ull << L) - 1ull) << (gbase & 63));
      for (int r = 0; r < rounds; ++r) {
        const uint32_t sz = (uint32_t)(ghi - glo);
        const int32_t mpt = glo + (int32_t)((sz * (uint32_t)(gl + 1)) / (uint32_t)(L + 1));
        const uint32_t c = cdf_at<K, kKind, kFast>(eo, q, mpt);
        const int cntb = __popcll(__ballot(so >= c) & gmask);
        const int src_lo = gbase + (cntb > 0 ? cntb - 1 : 0);
        const int src_hi = gbase + (cntb < L ? cntb : L - 1);
        const int32_t m_lo = __shfl(mpt, src_lo, 64);
        const uint32_t c_l = __shfl(c, src_lo, 64);
        const int32_t m_hi = __shfl(mpt, src_hi, 64);
        const uint32_t c_h = __shfl(c, src_hi, 64);
        if (cntb > 0) {
          glo = m_lo;
          gclo = c_l;
        }
        if (cntb < L) {
          ghi = m_hi;
          gchi = c_h;
        }
      }
      // each open lane takes its result from the first lane of its group
      const int src = (hi - lo > 1) ? rank * L : l;
      const int32_t rlo = __shfl(glo, src, 64);
      const uint32_t rclo = __shfl(gclo, src, 64), rchi = __shfl(gchi, src, 64);
      if (hi - lo > 1) {
        lo = rlo;
        c_lo = rclo;
        c_hi = rchi;
      }
      __syncthreads();  // lds.owner is rewritten next step
    }
    const uint64_t act_mask = __ballot(act);
    const uint64_t hit_mask = __ballot(act && hit);
    cnt[0] += (act && hit) ? 1 : 0;
    cnt[1] += (act && !hit) ? 1 : 0;
    if (l == 0 && act_mask) {
      ++cnt[3];
      if (hit_mask == act_mask) ++cnt[2];
    }
    if (act) {
      sym[i] = q.lo + lo;
      x = (c_hi - c_lo) * (x >> P) + slot - c_lo;
      if (x < (1u << 16)) {
        const bool have = ptr < b;
        x = (x << 16) | (have ? nword : 0u);
        bad = bad || !have;
        ptr += have ? 1 : 0;
      }
      nword = bs[ptr < b ? ptr : b - 1];
    }
  }
  if (seg_ok && (x != (1u << 16) || ptr != b)) bad = true;
  if (bad) atomicOr(status, kStCorrupt);
}

// Adds the wavefront's counters to stats[0..3] (one atomic each).
__device__ __forceinline__ void bracket_flush_stats(unsigned long long (&cnt)[4],
                                                    unsigned long long* stats) {
  if (!stats) return;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    cnt[0] += __shfl_xor(cnt[0], o, 64);
    cnt[1] += __shfl_xor(cnt[1], o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&stats[0], cnt[0]);
    atomicAdd(&stats[1], cnt[1]);
    atomicAdd(&stats[2], cnt[2]);
    atomicAdd(&stats[3], cnt[3]);
  }
}

}  // namespace fgmm

// Host handle of a loaded bracket model (declared opaque in flashgmm.h).
struct gmm_bracket {
  fgmm::BracketDev* dev = nullptr;
  int32_t K = 0, D = 0, radius = 4;
};
