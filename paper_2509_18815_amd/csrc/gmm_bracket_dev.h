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
  // Group form (v_mfma_f32_16x16x32_bf16, hidden units as rows in four
  // 16-row tiles t, samples as columns). The input normalisation is folded
  // into layer 1, which takes the element's raw inputs: the K flushed
  // weights, the K means, the K values log2(1 / scale') (the reciprocals the
  // CDF uses), slot / 2^P, and in input 16 a constant 1 that carries the
  // folded bias. Lane l holds
  //   ga1[l][t]: W1'[16 t + l % 16][8 (l / 16) + 2 w, +1], w = 0..3;
  //   ga2[l][t][kb]: W2[16 t + l % 16][phys(kb, 8 (l / 16) + 2 w, +1)], the
  //              physical hidden unit of logical input q of k block kb being
  //              the layer-1 accumulator row that lane holds there;
  //   ga3[l][kb]: w3[phys(kb, 8 (l / 16) + 2 w, +1)] (every row of the
  //              layer-3 tile is w3, so every accumulator register of a
  //              lane holds the output of its column);
  //   gb2[l][4 t + r]: b2 of accumulator row 16 t + 4 (l / 16) + r.
  uint32_t ga1[64][4][4];
  uint32_t ga2[64][4][2][4];
  uint32_t ga3[64][2][4];
  float gb2[64][16];
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
        eo.rn[k] = __shfl(e.rn[k], owner, 64);
      }
      eo.hw = __shfl(e.hw, owner, 64);
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

// ---------------------------------------------------------------- group form
// Streams with 16 lanes each (four per wavefront), for latents with few
// streams, where the decode is bound by the latency of each stream's chain
// of steps rather than by issue: the network runs on the matrix cores for
// the wavefront's four samples (columns 0..3 of 16x16 tiles), then the 16
// lanes of a stream evaluate the CDF at 16 consecutive boundaries around the
// prediction in one round. If the slot lies between the first and the last
// of them the symbol is known; otherwise the group finishes with the
// 17-ary search over the side the slot fell on.

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef short s16x2 __attribute__((ext_vector_type(2)));

struct GroupModel {
  bf16x8 a1[4];
  bf16x8 a2[4][2];
  bf16x8 a3[2];
  f32x4 b2[4];
};

__device__ __forceinline__ void load_group_model(const BracketDev* __restrict__ br,
                                                 GroupModel& m) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    m.a1[t] = bracket_frag(br->ga1[l][t]);
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) m.a2[t][kb] = bracket_frag(br->ga2[l][t][kb]);
#pragma unroll
    for (int r = 0; r < 4; ++r) m.b2[t][r] = br->gb2[l][4 * t + r];
  }
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) m.a3[kb] = bracket_frag(br->ga3[l][kb]);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two floats to a packed bfloat16 pair (round to nearest even), one
// conversion instruction.
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  const f32x2 f = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
}

// ReLU of a packed bfloat16 pair: as 16-bit integers, negative values
// (sign bit set, -0 included) are below 0 and positive ones above, so an
// integer max with 0 is the ReLU.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v) {
  const s16x2 x = __builtin_bit_cast(s16x2, v);
  const s16x2 z = {0, 0};
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(x, z));
}

// Next layer's B operand from two accumulator tiles: inputs 0..3 of the
// lane's group of eight from tile lo, 4..7 from tile hi, ReLU then bfloat16.
__device__ __forceinline__ bf16x8 relu_operand(const f32x4& lo, const f32x4& hi) {
  u32x4 v;
  v[0] = relu_bf16x2(pack_bf16x2(lo[0], lo[1]));
  v[1] = relu_bf16x2(pack_bf16x2(lo[2], lo[3]));
  v[2] = relu_bf16x2(pack_bf16x2(hi[0], hi[1]));
  v[3] = relu_bf16x2(pack_bf16x2(hi[2], hi[3]));
  return __builtin_bit_cast(bf16x8, v);
}

// B operand of layer 1 (inputs as rows, samples as columns) for groups of
// LG lanes (64 / LG streams per wavefront): lane l feeds column c = l % 16
// with inputs 8 (l / 16) .. 8 (l / 16) + 7. Column c < 64 / LG is the sample
// of lane group c, whose lanes all hold its inputs x; the upper half of a
// group serves inputs 8..15, the lower half inputs 0..7. Input 16 is the
// constant 1 of the folded bias; the other columns carry copies and are not
// read.
template <int LG>
__device__ __forceinline__ bf16x8 group_operand(const float (&x)[16]) {
  constexpr int G = 64 / LG;  // streams per wavefront
  const int l = threadIdx.x & 63;
  const bool upper = (l % LG) >= LG / 2;
  uint32_t wv[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    // both halves packed with constant indices, then one select per word
    const uint32_t lo = pack_bf16x2(x[2 * w], x[2 * w + 1]);
    const uint32_t hi = pack_bf16x2(x[8 + 2 * w], x[9 + 2 * w]);
    wv[w] = upper ? hi : lo;
  }
  const int kh = l >> 4;
  const int src = LG * ((l & 15) % G) + (LG / 2) * (kh & 1);
  u32x4 rv;
#pragma unroll
  for (int w = 0; w < 4; ++w) rv[w] = __shfl(wv[w], src, 64);
  if (kh >= 2) {
    rv[0] = (kh == 2) ? pack_bf16x2(1.0f, 0.0f) : 0u;
    rv[1] = 0u;
    rv[2] = 0u;
    rv[3] = 0u;
  }
  return __builtin_bit_cast(bf16x8, rv);
}

// Network output for column l % 16 (every lane holds its column's value):
// three layers on the matrix cores, ReLU between them on packed bfloat16.
__device__ __forceinline__ float mlp_group(const BracketDev* __restrict__ br, const GroupModel& m,
                                           const bf16x8& bx) {
  const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  f32x4 acc1[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
    acc1[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.a1[t], bx, zero, 0, 0, 0);
  // k block kb of layer 2 takes rows 32 kb + 4 (l / 16) + 0..3 (tile 2 kb)
  // and 32 kb + 16 + 4 (l / 16) + 0..3 (tile 2 kb + 1) of this lane
  const bf16x8 op2[2] = {relu_operand(acc1[0], acc1[1]), relu_operand(acc1[2], acc1[3])};
  f32x4 acc2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    acc2[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.a2[t][0], op2[0], m.b2[t], 0, 0, 0);
    acc2[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.a2[t][1], op2[1], acc2[t], 0, 0, 0);
  }
  const bf16x8 op3[2] = {relu_operand(acc2[0], acc2[1]), relu_operand(acc2[2], acc2[3])};
  f32x4 acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.a3[0], op3[0], zero, 0, 0, 0);
  acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(m.a3[1], op3[1], acc3, 0, 0, 0);
  return fmaf(acc3[0] + br->b3, br->out_std, br->out_mean);
}

// Decodes streams s0 .. s0 + 64/LG - 1 of one latent, LG = 16 or 8 lanes
// each (lane group l / LG takes stream s0 + l / LG); the window holds LG
// boundaries around the prediction. Every lane runs every step of the
// wavefront's longest stream (finished groups compute on placeholder data
// and store nothing): the matrix-core inference needs all 64 lanes.
// Counters (lane 0 of each group): hit / miss symbols; lane 0 of the
// wavefront also counts wavefront steps and steps on which every active
// stream hit. kBuf: parameters, refill words and symbols through buffer
// resources with 32-bit offsets, as decode_stream's buffer path (the caller
// checks buffer_offsets_fit; loads are then unconditional, the resources'
// range checks covering groups past S).
template <int K, int kKind, bool kFast, int LG, bool kBuf = false>
__device__ __forceinline__ void bracket_group_decode(
    const QCfg& q, int P, int64_t n, int64_t S, int64_t s0, const uint16_t* __restrict__ bs,
    int64_t total_words, const int64_t* __restrict__ offsets, const float* __restrict__ w,
    const float* __restrict__ mu, const float* __restrict__ sg, int32_t* __restrict__ sym,
    uint32_t* status, const BracketDev* __restrict__ br, const GroupModel& gm,
    unsigned long long (&cnt)[4]) {
  constexpr int L = LG;
  constexpr int kHalf = LG / 2 - 1;  // window [p - kHalf, p + kHalf + 1]: LG boundaries
  const int l = threadIdx.x & 63;
  const int gi = l / L, g = l % L, gbase = gi * L;
  const uint64_t gmask = ((1ull << L) - 1ull) << gbase;
  const int64_t s = s0 + gi;
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
  if (bad && g == 0)
    for (int64_t p = 0; p < ns; ++p) sym[s + p * S] = q.lo;
  uint32_t x = seg_ok ? ((uint32_t)bs[a] | ((uint32_t)bs[a + 1] << 16)) : (1u << 16);
  int64_t ptr = a + 2;
  const int64_t bl = seg_ok ? b - 1 : 0;  // last word of the segment (clamped reads)
  uint32_t nword = (seg_ok && ptr < b) ? bs[ptr] : 0u;
  if (seg_ok && x < (1u << 16)) bad = true;
  const uint32_t mask = q.M - 1;
  const float inv_m = 1.0f / (float)q.M;
  const int64_t last = ns > 0 ? ns - 1 : 0;
  // parameters one and two steps ahead (ring of two register sets); every
  // load is unconditional, positions past the end reload the last element
  constexpr int kRing = 2;
  float rw[kRing][K], rm[kRing][K], rs[kRing][K];
  [[maybe_unused]] __amdgpu_buffer_rsrc_t bw_, bm_, bsg_, bbs_, bsym_;
  [[maybe_unused]] uint32_t off_next = 0, off_last = 0, off_cur = 0, plane = 0;
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
    off_cur = (uint32_t)s * 4u;
    off_last = (uint32_t)(s + last * S) * 4u;
    off_next = off_cur;
  }
#pragma unroll
  for (int d = 0; d < kRing; ++d) {
    if constexpr (kBuf) {
      const uint32_t o = off_next < off_last ? off_next : off_last;
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
      const int64_t pp = (d < last) ? d : last;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        rw[d][k] = 0.0f;
        rm[d][k] = 0.0f;
        rs[d][k] = 1.0f;
      }
      if (seg_ok && ns > 0) load_raw<K>(w, mu, sg, n, s + pp * S, rw[d], rm[d], rs[d]);
    }
  }
  for (int64_t p0 = 0; p0 < ns_max; p0 += kRing) {
#pragma unroll
    for (int d = 0; d < kRing; ++d) {
      const int64_t p = p0 + d;
      if (p >= ns_max) break;
      const bool act = seg_ok && p < ns;
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
      const uint32_t slot = x & mask;
      // raw inputs (the normalisation is folded into layer 1)
      float feat[16];
#pragma unroll
      for (int d = 0; d < 16; ++d) feat[d] = 0.0f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        feat[k] = e.w[k];
        feat[K + k] = e.mu[k];
        feat[2 * K + k] = __builtin_amdgcn_logf(e.r[k]);  // log2(1 / scale')
      }
      feat[3 * K] = (float)slot * inv_m;
      const float pred_col = mlp_group(br, gm, group_operand<LG>(feat));
      const float pred = __shfl(pred_col, gi, 64);  // column gi = this group's sample
      // window of 16 boundaries around the prediction, inside the indices
      // [slot - (M - N), slot] that the quantization allows for this slot
      const int32_t jmin = max(0, (int32_t)slot - (int32_t)(q.M - (uint32_t)q.N));
      const int32_t jmax = min(q.N - 1, (int32_t)slot);
      const float pc = __builtin_fminf(__builtin_fmaxf(pred - (float)q.lo, -1.0f), (float)q.N);
      const int32_t jh = min(max((int32_t)__builtin_rintf(pc), jmin), jmax);
      const int32_t ws = max(0, min(jh - kHalf, q.N - (L - 1)));
      const uint32_t c = cdf_at<K, kKind, kFast>(e, q, ws + g);
      const int cb = __popcll(__ballot(slot >= c) & gmask);  // c rises with g
      const uint32_t c_l = __shfl(c, gbase + (cb > 0 ? cb - 1 : 0), 64);
      const uint32_t c_h = __shfl(c, gbase + (cb < L ? cb : L - 1), 64);
      const bool hit = cb > 0 && cb < L;
      int32_t lo, hi;
      uint32_t c_lo, c_hi;
      if (hit) {
        lo = ws + cb - 1; hi = lo + 1; c_lo = c_l; c_hi = c_h;
      } else if (cb == 0) {
        lo = 0; hi = ws; c_lo = 0; c_hi = c_h;
      } else {
        lo = ws + L - 1; hi = q.N; c_lo = c_l; c_hi = q.M;
      }
      if (!act) {
        lo = 0; hi = 1; c_lo = 0; c_hi = q.M;
      }
      if (hi - lo > 1)  // uniform within the group
        lo = search_group<K, kKind, kFast, L>(e, q, rounds_for(hi - lo, L), slot, g, gbase, gmask,
                                              lo, hi, c_lo, c_hi);
      const uint64_t lead = __ballot(g == 0 && act);
      const uint64_t lead_hit = __ballot(g == 0 && act && hit);
      if (g == 0) {
        cnt[0] += (act && hit) ? 1 : 0;
        cnt[1] += (act && !hit) ? 1 : 0;
      }
      if (l == 0 && lead) {
        ++cnt[3];
        if (lead_hit == lead) ++cnt[2];
      }
      if constexpr (kBuf) {
        if (act && g == 0)
          __builtin_amdgcn_raw_buffer_store_b32((uint32_t)(q.lo + lo), bsym_, off_cur, 0, 0);
        off_cur += (uint32_t)S * 4u;
      } else {
        if (act && g == 0) sym[s + p * S] = q.lo + lo;
      }
      // state update and refill as selects (all lanes of a group agree)
      const uint32_t xs = (c_hi - c_lo) * (x >> P) + slot - c_lo;
      const bool refill = act && xs < (1u << 16);
      const bool have = ptr < b;
      const uint32_t xr = refill ? ((xs << 16) | (have ? nword : 0u)) : xs;
      x = act ? xr : x;
      bad = bad || (refill && !have);
      ptr += (refill && have) ? 1 : 0;
      if constexpr (kBuf) {
        // ptr <= b <= total_words (a word past the bitstream reads 0)
        nword = __builtin_amdgcn_raw_buffer_load_b16(bbs_, (uint32_t)ptr * 2u, 0, 0);
        asm volatile("" ::: "memory");  // keep the word's load ahead of the ring's
        const uint32_t o = off_next < off_last ? off_next : off_last;
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
        nword = seg_ok ? bs[ptr < b ? ptr : bl] : 0u;
        asm volatile("" ::: "memory");  // keep the word's load ahead of the ring's
        const int64_t pn = p + kRing;
        if (seg_ok)
          load_raw<K>(w, mu, sg, n, s + (pn < last ? pn : last) * S, rw[d], rm[d], rs[d]);
      }
    }
  }
  if (seg_ok && (x != (1u << 16) || ptr != b)) bad = true;
  if (bad && g == 0) atomicOr(status, kStCorrupt);
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
