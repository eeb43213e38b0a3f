// Batched coding of many latents of uneven sizes (plans).
//
// A plan fixes the common configuration and the shapes (n_b, S_b) of B
// latents. Its kernels address the latents through a device descriptor
// table and flattened index spaces in which every latent's elements and
// streams start on a block boundary, so a block always belongs to one
// latent (found through a block -> latent table):
//   encode: kb_enc_cdf (one thread per element of every latent)
//           kb_enc_rans_lds (256 streams per work item, words in LDS, one
//                        pass with a per-latent look-back; persistent
//                        workgroups pull items from an atomic queue, longest
//                        streams first, or one item per workgroup)  kb_finalize
//           or kb_enc_rans (words through scratch rows; queue, static or one
//                        item per block)  kb_scan (one workgroup per latent)
//           kb_pack  kb_finalize
//   decode: kb_decode (one wavefront per work item of 64/L streams, L lanes
//                      per stream; persistent/dynamic, persistent/static or
//                      one item per block)          kb_finalize
// The launch shape (lanes per stream, streams per lane, schedule, waves per
// compute unit, LDS staging of the encoder's words) is chosen by timing
// every candidate on the real shapes at the first
// execution (the output is identical for every candidate), optionally
// cached in a file keyed by the shape signature, and the chosen sequence is
// captured once into a hipGraph that later executions launch.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/flashgmm.h"
#include "gmm_device.h"
#include "gmm_host.h"
#include "gmm_stream.h"
#include "gmm_bracket_dev.h"

using namespace fgmm;

namespace {

constexpr int kCdfBlock = 256;   // elements per encode-phase-1 block
constexpr int kRBlock = 256;     // streams per rANS block
constexpr int kPLanes = 16;      // lanes per stream when packing
constexpr int kPBlock = 256;     // threads per pack block (16 streams)

enum Sched : int32_t { kFlat = 0, kDynamic = 1, kStatic = 2 };

struct LatentDesc {
  int64_t n, S, cap;
  int64_t elem_base;     // first flattened element (multiple of kCdfBlock)
  int64_t cdf_blk0;      // first phase-1 block
  int64_t rans_blk0;     // first rANS block; stream_base = rans_blk0 * kRBlock
  int64_t nblk;          // rANS blocks of the latent
  int64_t pack_blk0;     // first pack block
  int64_t scratch_base;  // first scratch word
  const int32_t* sym;
  const float* w;
  const float* mu;
  const float* sg;
  uint16_t* bs;
  int64_t words;  // encode: capacity; decode: total words
  int64_t* offsets;
  int32_t* dec;
};

__global__ void kb_reset(uint32_t* p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

// kBuf: every latent's offsets fit enc_cdf_elem's buffer path
// (encode_offsets_fit).
template <int K, int kKind, bool kFast, bool kBuf = false>
__global__ void __launch_bounds__(kCdfBlock)
    kb_enc_cdf(const LatentDesc* __restrict__ desc, QCfg q, const int32_t* __restrict__ blk_latent,
               uint32_t* __restrict__ cf, uint32_t* status) {
  const int b = blk_latent[blockIdx.x];
  const LatentDesc& d = desc[b];
  const int64_t i = ((int64_t)blockIdx.x - d.cdf_blk0) * kCdfBlock + threadIdx.x;
  if (i >= d.n) return;
  cf[d.elem_base + i] = enc_cdf_elem<K, kKind, kFast, false, kBuf>(q, d.n, i, d.sym, d.w, d.mu,
                                                                   d.sg, &status[b]);
}

// Work item = one rANS block (256 streams of one latent).
__global__ void __launch_bounds__(kRBlock)
    kb_enc_rans(const LatentDesc* __restrict__ desc, int P, const int32_t* __restrict__ items,
                int64_t n_items, int sched, uint32_t* queue,
                const int32_t* __restrict__ blk_latent, const uint32_t* __restrict__ cf,
                uint16_t* __restrict__ scratch, uint32_t* __restrict__ xfin,
                uint32_t* __restrict__ count, uint32_t* __restrict__ local_off,
                int64_t* __restrict__ blk_total) {
  __shared__ int64_t item_sh;
  int64_t it = blockIdx.x;
  for (;;) {
    int64_t item;
    if (sched == kDynamic) {
      if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(queue, 1u);
      __syncthreads();
      item = item_sh;
    } else {
      item = it;
    }
    if (item >= n_items) break;
    const int64_t blk = items[item];
    const LatentDesc& d = desc[blk_latent[blk]];
    const int64_t s = (blk - d.rans_blk0) * kRBlock + threadIdx.x;
    const int64_t gs = blk * kRBlock + threadIdx.x;
    uint32_t cnt = 0;
    if (s < d.S) {
      bool zf;  // phase 1 of plans reports ranges itself and never writes f = 0
      xfin[gs] = rans_stream(d.n, d.S, P, s, cf + d.elem_base,
                             scratch + d.scratch_base + s * d.cap + (d.cap - 1), &cnt, &zf);
      count[gs] = cnt;
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<kRBlock>((s < d.S) ? cnt + 2u : 0u, &tot);
    if (s < d.S) local_off[gs] = ex;
    if (threadIdx.x == 0) blk_total[blk] = tot;
    if (sched == kFlat) break;
    if (sched == kStatic) it += gridDim.x;
    __syncthreads();  // the scan's LDS and item_sh are reused next item
  }
}

__global__ void __launch_bounds__(kScanBlock)
    kb_scan(const LatentDesc* __restrict__ desc, const int64_t* __restrict__ blk_total,
            int64_t* __restrict__ blk_pre) {
  const LatentDesc& d = desc[blockIdx.x];
  scan_totals(d.nblk, blk_total + d.rans_blk0, blk_pre + d.rans_blk0);
}

__global__ void __launch_bounds__(kPBlock)
    kb_pack(const LatentDesc* __restrict__ desc, const int32_t* __restrict__ blk_latent,
            const uint16_t* __restrict__ scratch, const uint32_t* __restrict__ xfin,
            const uint32_t* __restrict__ count, const uint32_t* __restrict__ local_off,
            const int64_t* __restrict__ blk_pre, const int64_t* __restrict__ blk_total,
            uint32_t* status) {
  const int b = blk_latent[blockIdx.x];
  const LatentDesc& d = desc[b];
  const int64_t s = ((int64_t)blockIdx.x - d.pack_blk0) * (kPBlock / kPLanes) +
                    threadIdx.x / kPLanes;
  const int l = threadIdx.x % kPLanes;
  const int64_t last = d.rans_blk0 + d.nblk - 1;
  const int64_t total = blk_pre[last] + blk_total[last];
  const bool fits = total <= d.words;
  if (!fits && (int64_t)blockIdx.x == d.pack_blk0 && threadIdx.x == 0)
    atomicOr(&status[b], kStNoSpace);
  if (s >= d.S) return;
  const int64_t gs = d.rans_blk0 * kRBlock + s;
  const int64_t off = blk_pre[d.rans_blk0 + s / kRBlock] + (int64_t)local_off[gs];
  if (l == 0) {
    d.offsets[s] = off;
    if (s == d.S - 1) d.offsets[d.S] = total;
  }
  if (!fits) return;
  const uint32_t cnt = count[gs];
  pack_segment(d.bs + off, xfin[gs], scratch + d.scratch_base + s * d.cap + (d.cap - cnt), cnt,
               l, kPLanes);
}

// rANS pass with the renormalisation words staged in LDS, one pass per work
// item (a rANS block: 256 streams of one latent), in place of kb_enc_rans,
// kb_scan and kb_pack. SPL streams per lane: 1 (256 threads) or 2 (128
// threads, each stepping streams t and t + 128 in turn: two independent
// chains per lane). Items are taken from the queue in its order, which
// keeps each latent's items in stream order, so the item's offset in its
// latent comes from a decoupled look-back over the latent's earlier items
// (slots of the latent, zeroed before the launch); every item waited on has
// been taken by a running workgroup. The item writes its streams' offsets
// and, when its range fits the latent's capacity, their segments straight
// into the latent's bitstream; the item with the latent's last streams
// writes offsets[S] and flags ENOSPC. Dynamic LDS: words[cap][256] for the
// largest cap of the plan. Schedules: flat (one item per workgroup, taken
// by ticket) and dynamic.
template <int SPL, bool kBuf = false>
__global__ void __launch_bounds__(kRBlock / SPL)
    kb_enc_rans_lds(const LatentDesc* __restrict__ desc, int P, int trash_row,
                    const int32_t* __restrict__ items,
                    int64_t n_items, int sched, uint32_t* queue,
                    const int32_t* __restrict__ blk_latent, const uint32_t* __restrict__ cf,
                    uint64_t* slots, uint32_t* status) {
  extern __shared__ uint16_t words[];  // [cap + 1][kRBlock], row cap: trash
  __shared__ int64_t item_sh, excl_sh;
  __shared__ uint32_t tot_a_sh;
  constexpr int T = kRBlock / SPL;
  for (;;) {
    if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(queue, 1u);
    __syncthreads();
    // wavefront-uniform in a scalar register: the latent's descriptor and
    // the buffer resource built from it stay scalar
    const int64_t item = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)item_sh);
    if (item >= n_items) break;
    const int64_t blk = items[item];
    const int b = blk_latent[blk];
    const LatentDesc& d = desc[b];
    const int64_t k = blk - d.rans_blk0;  // item index within its latent
    const uint32_t* lcf = cf + d.elem_base;
    const int64_t sa = k * kRBlock + threadIdx.x, sb = sa + T;
    uint32_t xa = 1u << 16, xb = 1u << 16, ca = 0, cb = 0;
    bool zf = false;
    if (SPL == 1) {
      if (sa < d.S)
        xa = rans_stream_lds<kBuf>(d.n, d.S, P, sa, lcf, words + threadIdx.x, kRBlock, trash_row,
                                   &ca, &zf);
    } else if (sa < d.S) {
      // a lane whose second stream lies past S steps its first one twice;
      // the copy's words go to an unused column and are dropped
      rans_stream_lds2(d.n, d.S, P, sa, sb < d.S ? sb : sa, lcf, words + threadIdx.x,
                       words + threadIdx.x + T, kRBlock, trash_row, xa, xb, ca, cb, zf);
      if (sb >= d.S) cb = 0;
    }
    (void)zf;  // plans report ranges in phase 1 (no f = 0 words)
    uint32_t tot, la, lb = 0;
    la = block_excl_scan<T>((sa < d.S) ? ca + 2u : 0u, &tot);
    if (SPL == 2) {
      if (threadIdx.x == 0) tot_a_sh = tot;
      __syncthreads();
      uint32_t tot_b;
      lb = tot_a_sh + block_excl_scan<T>((sb < d.S) ? cb + 2u : 0u, &tot_b);
      tot += tot_b;
    }
    if (threadIdx.x < 64) {
      const int64_t e = lookback_prefix(slots + d.rans_blk0, k, (int64_t)tot);
      if (threadIdx.x == 0) excl_sh = e;
    }
    __syncthreads();
    const int64_t excl = excl_sh;
    if (sa < d.S) d.offsets[sa] = excl + (int64_t)la;
    if (SPL == 2 && sb < d.S) d.offsets[sb] = excl + (int64_t)lb;
    if (k == d.nblk - 1 && threadIdx.x == 0) {
      const int64_t total = excl + (int64_t)tot;
      d.offsets[d.S] = total;
      if (total > d.words) atomicOr(&status[b], kStNoSpace);
    }
    if (excl + (int64_t)tot <= d.words) {
      // each lane writes its own streams' segments: the state words, then the
      // renormalisation words in decoder order (newest first)
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        const int64_t s = j ? sb : sa;
        if (s < d.S) {
          const uint32_t x = j ? xb : xa, cnt = j ? cb : ca;
          const int64_t o = excl + (int64_t)(j ? lb : la);
          d.bs[o] = (uint16_t)(x & 0xFFFFu);
          d.bs[o + 1] = (uint16_t)(x >> 16);
          const uint16_t* col = words + threadIdx.x + j * T;
          for (uint32_t t = 0; t < cnt; ++t) d.bs[o + 2 + t] = col[(cnt - 1u - t) * kRBlock];
        }
      }
    }
    if (sched == kFlat) break;
    __syncthreads();  // LDS words, the scans' LDS and item_sh are reused next item
  }
}

// Work item = (latent, first stream) of 64/L streams; one wavefront each.
// With kBuf (every latent's offsets fit 32 bits) decode_stream's buffer
// path; the item index is wavefront-uniform (read from the first lane into
// a scalar register), so the latent's descriptor and the buffer resources
// built from it stay scalar.
template <int K, int kKind, bool kFast, int L, bool kBuf = false>
__global__ void __launch_bounds__(64)
    kb_decode(const LatentDesc* __restrict__ desc, QCfg q, int P, int rounds,
              const int2* __restrict__ items, int64_t n_items, int sched, uint32_t* queue,
              uint32_t* status) {
  const int lane = threadIdx.x;
  int64_t it = blockIdx.x;
  for (;;) {
    int64_t item;
    if (sched == kDynamic) {
      uint32_t v = 0;
      if (lane == 0) v = atomicAdd(queue, 1u);
      item = (int64_t)__builtin_amdgcn_readfirstlane(v);
    } else {
      item = it;
    }
    if (item >= n_items) break;
    const int2 t = items[item];
    const LatentDesc& d = desc[t.x];
    const int64_t s = (int64_t)t.y + lane / L;
    const int g = lane % L;
    if (s < d.S) {
      const bool bad = decode_stream<K, kKind, kFast, L, false, L == 1, kBuf>(
          q, P, rounds, d.n, d.S, s, g, d.bs, d.words, d.offsets, d.w, d.mu, d.sg, d.dec);
      if (bad && g == 0) atomicOr(&status[t.x], kStCorrupt);
    }
    if (sched == kFlat) break;
    if (sched == kStatic) it += gridDim.x;
  }
}

// Two streams per lane: work item = (latent, first stream) of 128 streams;
// lane l decodes streams first + l and first + 64 + l together.
template <int K, int kKind, bool kFast>
__global__ void __launch_bounds__(64)
    kb_decode2(const LatentDesc* __restrict__ desc, QCfg q, int P, int rounds,
               const int2* __restrict__ items, int64_t n_items, int sched, uint32_t* queue,
               uint32_t* status) {
  const int lane = threadIdx.x;
  int64_t it = blockIdx.x;
  for (;;) {
    int64_t item;
    if (sched == kDynamic) {
      uint32_t v = 0;
      if (lane == 0) v = atomicAdd(queue, 1u);
      item = (int64_t)__shfl(v, 0, 64);
    } else {
      item = it;
    }
    if (item >= n_items) break;
    const int2 t = items[item];
    const LatentDesc& d = desc[t.x];
    const int64_t sa = (int64_t)t.y + lane;
    if (sa < d.S) {
      const bool bad = decode_stream2<K, kKind, kFast>(q, P, rounds, d.n, d.S, sa, sa + 64, d.bs,
                                                       d.words, d.offsets, d.w, d.mu, d.sg,
                                                       d.dec);
      if (bad) atomicOr(&status[t.x], kStCorrupt);
    }
    if (sched == kFlat) break;
    if (sched == kStatic) it += gridDim.x;
  }
}

// Decode with the learned bracket: work item = (latent, first stream) of 64
// streams, one wavefront each (the matrix-core inference needs all lanes).
template <int K, int kKind, bool kFast>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
    kb_decode_bracket(const LatentDesc* __restrict__ desc, QCfg q, int P,
                      const int2* __restrict__ items, int64_t n_items, int sched, uint32_t* queue,
                      uint32_t* status, const BracketDev* __restrict__ br,
                      unsigned long long* stats) {
  __shared__ BracketLds lds;
  LaneModel model;
  load_lane_model(br, model, lds);
  unsigned long long cnt[4] = {0, 0, 0, 0};
  const int lane = threadIdx.x;
  int64_t it = blockIdx.x;
  for (;;) {
    int64_t item;
    if (sched == kDynamic) {
      uint32_t v = 0;
      if (lane == 0) v = atomicAdd(queue, 1u);
      item = (int64_t)__shfl(v, 0, 64);
    } else {
      item = it;
    }
    if (item >= n_items) break;
    const int2 t = items[item];
    const LatentDesc& d = desc[t.x];
    bracket_decode_wave<K, kKind, kFast>(q, P, d.n, d.S, (int64_t)t.y, d.bs, d.words, d.offsets,
                                         d.w, d.mu, d.sg, d.dec, &status[t.x], br, model, lds,
                                         cnt);
    if (sched == kFlat) break;
    if (sched == kStatic) it += gridDim.x;
  }
  bracket_flush_stats(cnt, stats);
}

__global__ void kb_finalize(const uint32_t* __restrict__ bits, int32_t B,
                            int32_t* __restrict__ codes) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const uint32_t v = bits[b];
  int32_t c = GMM_OK;
  if (v & kStInval) c = GMM_EINVAL;
  else if (v & kStRange) c = GMM_ERANGE;
  else if (v & kStNoSpace) c = GMM_ENOSPC;
  else if (v & kStCorrupt) c = GMM_ECORRUPT;
  codes[b] = c;
}

struct Config {
  int32_t lanes = 1, spl = 1, sched = kDynamic, waves_per_cu = 8, lds = 0;
};

// Largest dynamic LDS of kb_enc_rans_lds (words of a work item's 256
// streams): streams of up to 300 symbols.
constexpr int64_t kRansLdsMax = (300 + 1) * kRBlock * 2;

bool same_io(const gmm_latent_io& a, const gmm_latent_io& b) {
  return memcmp(&a, &b, sizeof(gmm_latent_io)) == 0;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::mutex g_cache_mu;

}  // namespace

struct gmm_plan {
  gmm_cfg cfg;
  int32_t op = 0, B = 0, flags = 0;
  bool fast = false;
  int num_cus = 256;
  QCfg q;
  std::vector<int64_t> n, S;
  std::vector<LatentDesc> h_desc;
  LatentDesc* d_desc = nullptr;
  LatentDesc* pinned_desc = nullptr;
  // encode tables and workspace
  int64_t n_cdf_blk = 0, n_rans_blk = 0, n_pack_blk = 0;
  int32_t *d_cdf_blk = nullptr, *d_rans_blk = nullptr, *d_pack_blk = nullptr;
  int32_t* d_rans_items = nullptr;
  uint32_t *d_cf = nullptr, *d_xfin = nullptr, *d_count = nullptr, *d_local = nullptr;
  uint16_t* d_scratch = nullptr;
  int64_t *d_blk_total = nullptr, *d_blk_pre = nullptr;
  // decode: whether every latent's offsets fit decode_stream's buffer path
  // (set from the buffers of the latest execution; a change recaptures)
  bool buf = false;
  // decode items (for the chosen lanes and streams per lane)
  int2* d_items = nullptr;
  int64_t n_items = 0;
  int32_t items_per = 0;  // streams per item of the current list (0: none built)
  // learned bracket for decode (nullable) and its counters
  const gmm_bracket* bracket = nullptr;
  unsigned long long* stats = nullptr;
  // status
  uint32_t* d_bits = nullptr;  // [B] status bits, the queue counter, look-back slots
  uint64_t* d_slots = nullptr; // [n_rans_blk] look-back slots (inside d_bits)
  int64_t reset_words = 0;     // words of d_bits cleared before each execution
  int64_t cap_max = 1;         // longest stream of the plan (LDS words per stream)
  int32_t* d_codes = nullptr;  // [B]
  // chosen configuration and graph
  Config conf;
  bool tuned = false;
  double best_ms = -1.0;
  int32_t candidates = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<gmm_latent_io> last_io;
  std::string signature;
  std::vector<void*> allocs;
};

namespace {

template <typename T>
int dev_alloc(gmm_plan* p, T** out, int64_t count) {
  void* ptr = nullptr;
  const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
  if (hipMalloc(&ptr, bytes) != hipSuccess) return GMM_ENOMEM;
  p->allocs.push_back(ptr);
  *out = (T*)ptr;
  return GMM_OK;
}

// Streams per decode work item: one wavefront's 64 lanes, L lanes per
// stream, spl streams per lane.
int item_streams(const Config& c) { return 64 / c.lanes * c.spl; }

int build_decode_items(gmm_plan* p, int per, hipStream_t st) {
  if (p->items_per == per) return GMM_OK;
  struct It {
    int2 v;
    int64_t cost;
  };
  std::vector<It> v;
  for (int b = 0; b < p->B; ++b)
    for (int64_t s0 = 0; s0 < p->S[b]; s0 += per) {
      const int64_t ns = (s0 < p->n[b]) ? (p->n[b] - 1 - s0) / p->S[b] + 1 : 0;
      v.push_back({make_int2(b, (int)s0), ns});
    }
  std::stable_sort(v.begin(), v.end(), [](const It& a, const It& b) { return a.cost > b.cost; });
  std::vector<int2> h(v.size());
  for (size_t i = 0; i < v.size(); ++i) h[i] = v[i].v;
  if (!p->d_items) {
    // room for the most items any lanes-per-stream choice produces
    int64_t cap = 0;
    for (int b = 0; b < p->B; ++b) cap += p->S[b];
    int r = dev_alloc(p, &p->d_items, cap);
    if (r) return r;
  }
  if (hipMemcpyAsync(p->d_items, h.data(), h.size() * sizeof(int2), hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return GMM_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return GMM_EDEVICE;
  p->n_items = (int64_t)h.size();
  p->items_per = per;
  return GMM_OK;
}

// Enqueues one execution of the plan with configuration c on stream st.
int enqueue(gmm_plan* p, const Config& c, hipStream_t st) {
  const int B = p->B;
  hipLaunchKernelGGL(kb_reset, dim3((unsigned)((p->reset_words + 255) / 256)), dim3(256), 0, st,
                     p->d_bits, p->reset_words);
  uint32_t* queue = p->d_bits + B;
  const int64_t persist_grid = (int64_t)p->num_cus * c.waves_per_cu;
  if (p->op == 0) {
    // buffer resources when every latent's offsets fit 32 bits
    bool ebuf = true;
    for (int b = 0; b < B; ++b) ebuf = ebuf && encode_offsets_fit(p->cfg.K, p->n[b], p->S[b]);
    if (p->n_cdf_blk > 0) {
      dispatch(p->cfg.K, p->cfg.cdf_kind, p->fast, [&](auto Kc, auto kc, auto fc) {
        constexpr int K_ = decltype(Kc)::value, KI = decltype(kc)::value;
        constexpr bool F = decltype(fc)::value;
        if (ebuf)
          hipLaunchKernelGGL((kb_enc_cdf<K_, KI, F, true>), dim3((unsigned)p->n_cdf_blk),
                             dim3(kCdfBlock), 0, st, p->d_desc, p->q, p->d_cdf_blk, p->d_cf,
                             p->d_bits);
        else
          hipLaunchKernelGGL((kb_enc_cdf<K_, KI, F>), dim3((unsigned)p->n_cdf_blk),
                             dim3(kCdfBlock), 0, st, p->d_desc, p->q, p->d_cdf_blk, p->d_cf,
                             p->d_bits);
      });
    }
    if (c.lds) {
      // one pass per item, words in LDS; workgroups of 256 / spl threads
      const int wpb = (kRBlock / c.spl) / 64;
      const int64_t grid =
          (c.sched == kFlat) ? p->n_rans_blk
                             : std::min<int64_t>(p->n_rans_blk,
                                                 std::max<int64_t>(1, persist_grid / wpb));
      const size_t lds = (size_t)((p->cap_max + 1) * kRBlock * 2);  // and a trash row
      if (c.spl == 2)
        hipLaunchKernelGGL(kb_enc_rans_lds<2>, dim3((unsigned)grid), dim3(kRBlock / 2), lds, st,
                           p->d_desc, p->cfg.precision, (int)p->cap_max, p->d_rans_items,
                           p->n_rans_blk, c.sched,
                           queue, p->d_rans_blk, p->d_cf, p->d_slots, p->d_bits);
      else if (ebuf)
        hipLaunchKernelGGL((kb_enc_rans_lds<1, true>), dim3((unsigned)grid), dim3(kRBlock), lds,
                           st, p->d_desc, p->cfg.precision, (int)p->cap_max, p->d_rans_items,
                           p->n_rans_blk, c.sched, queue, p->d_rans_blk, p->d_cf, p->d_slots,
                           p->d_bits);
      else
        hipLaunchKernelGGL(kb_enc_rans_lds<1>, dim3((unsigned)grid), dim3(kRBlock), lds, st,
                           p->d_desc, p->cfg.precision, (int)p->cap_max, p->d_rans_items,
                           p->n_rans_blk, c.sched,
                           queue, p->d_rans_blk, p->d_cf, p->d_slots, p->d_bits);
      hipLaunchKernelGGL(kb_finalize, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, st,
                         p->d_bits, B, p->d_codes);
      return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
    }
    // persistent grids of 4-wave workgroups: waves_per_cu / 4 per compute unit
    int64_t grid = (c.sched == kFlat) ? p->n_rans_blk
                                      : std::min<int64_t>(p->n_rans_blk,
                                                          std::max<int64_t>(1, persist_grid / 4));
    hipLaunchKernelGGL(kb_enc_rans, dim3((unsigned)grid), dim3(kRBlock), 0, st, p->d_desc,
                       p->cfg.precision, p->d_rans_items, p->n_rans_blk, c.sched, queue,
                       p->d_rans_blk, p->d_cf, p->d_scratch, p->d_xfin, p->d_count, p->d_local,
                       p->d_blk_total);
    hipLaunchKernelGGL(kb_scan, dim3((unsigned)B), dim3(kScanBlock), 0, st, p->d_desc,
                       p->d_blk_total, p->d_blk_pre);
    hipLaunchKernelGGL(kb_pack, dim3((unsigned)p->n_pack_blk), dim3(kPBlock), 0, st, p->d_desc,
                       p->d_pack_blk, p->d_scratch, p->d_xfin, p->d_count, p->d_local,
                       p->d_blk_pre, p->d_blk_total, p->d_bits);
  } else if (p->bracket) {
    const int64_t grid = (c.sched == kFlat) ? p->n_items : std::min(p->n_items, persist_grid);
    if (grid > 0) {
      dispatch(p->cfg.K, p->cfg.cdf_kind, p->fast, [&](auto Kc, auto kc, auto fc) {
        constexpr int K_ = decltype(Kc)::value;
        if constexpr (K_ <= 5) {
          hipLaunchKernelGGL((kb_decode_bracket<K_, decltype(kc)::value, decltype(fc)::value>),
                             dim3((unsigned)grid), dim3(64), 0, st, p->d_desc, p->q,
                             p->cfg.precision, p->d_items, p->n_items, c.sched, queue, p->d_bits,
                             p->bracket->dev, p->stats);
        }
      });
    }
  } else if (c.spl == 2) {
    const int rounds = search_rounds(p->q.N);
    const int64_t grid = (c.sched == kFlat) ? p->n_items : std::min(p->n_items, persist_grid);
    if (grid > 0) {
      dispatch(p->cfg.K, p->cfg.cdf_kind, p->fast, [&](auto Kc, auto kc, auto fc) {
        hipLaunchKernelGGL((kb_decode2<decltype(Kc)::value, decltype(kc)::value,
                                       decltype(fc)::value>),
                           dim3((unsigned)grid), dim3(64), 0, st, p->d_desc, p->q,
                           p->cfg.precision, rounds, p->d_items, p->n_items, c.sched, queue,
                           p->d_bits);
      });
    }
  } else {
    const int L = c.lanes;
    const int rounds = (L == 1) ? search_rounds(p->q.N) : search_rounds_lps(p->q.N, L);
    const int64_t grid = (c.sched == kFlat) ? p->n_items : std::min(p->n_items, persist_grid);
    if (grid > 0) {
      dispatch(p->cfg.K, p->cfg.cdf_kind, p->fast, [&](auto Kc, auto kc, auto fc) {
        constexpr int K_ = decltype(Kc)::value, KI = decltype(kc)::value;
        constexpr bool F = decltype(fc)::value;
#define FG_BDEC(LL)                                                                        \
  if (p->buf)                                                                              \
    hipLaunchKernelGGL((kb_decode<K_, KI, F, LL, true>), dim3((unsigned)grid), dim3(64), 0, \
                       st, p->d_desc, p->q, p->cfg.precision, rounds, p->d_items,          \
                       p->n_items, c.sched, queue, p->d_bits);                             \
  else                                                                                     \
    hipLaunchKernelGGL((kb_decode<K_, KI, F, LL>), dim3((unsigned)grid), dim3(64), 0, st,  \
                       p->d_desc, p->q, p->cfg.precision, rounds, p->d_items, p->n_items,  \
                       c.sched, queue, p->d_bits)
        switch (L) {
          case 1: FG_BDEC(1); break;
          case 2: FG_BDEC(2); break;
          case 4: FG_BDEC(4); break;
          case 8: FG_BDEC(8); break;
          default: FG_BDEC(16); break;
        }
#undef FG_BDEC
      });
    }
  }
  hipLaunchKernelGGL(kb_finalize, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, st, p->d_bits, B,
                     p->d_codes);
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

// Lets kb_enc_rans_lds use more than the default dynamic LDS (once).
bool lds_ready() {
  static const bool ok =
      hipFuncSetAttribute((const void*)kb_enc_rans_lds<1>,
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kRansLdsMax) == hipSuccess &&
      hipFuncSetAttribute((const void*)kb_enc_rans_lds<2>,
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kRansLdsMax) == hipSuccess &&
      hipFuncSetAttribute((const void*)kb_enc_rans_lds<1, true>,
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kRansLdsMax) == hipSuccess;
  return ok;
}

std::vector<Config> candidates(const gmm_plan* p) {
  std::vector<Config> v;
  const int wpcs[] = {4, 8, 16};
  if (p->op == 0) {
    v.push_back({1, 1, kFlat, 8, 0});
    for (int w : wpcs) {
      v.push_back({1, 1, kDynamic, w, 0});
      v.push_back({1, 1, kStatic, w, 0});
    }
    // words staged in LDS, one pass per item (flat by ticket or dynamic;
    // a static assignment could wait on an item not yet started), one or
    // two streams per lane
    if ((p->cap_max + 1) * kRBlock * 2 <= kRansLdsMax && lds_ready()) {
      for (int spl : {1, 2}) {
        v.push_back({1, spl, kFlat, 8, 1});
        for (int w : wpcs) v.push_back({1, spl, kDynamic, w, 1});
      }
    }
  } else {
    int64_t streams = 0;
    for (int b = 0; b < p->B; ++b) streams += p->S[b];
    for (int L : {1, 2, 4, 8, 16}) {
      if (p->bracket && L != 1) continue;  // the bracket kernel runs one lane per stream
      if (L > 1 && streams * L > (int64_t)p->num_cus * 64 * 64) continue;  // > 16 waves / SIMD
      v.push_back({L, 1, kFlat, 8, 0});
      for (int w : wpcs) {
        v.push_back({L, 1, kDynamic, w, 0});
        v.push_back({L, 1, kStatic, w, 0});
      }
    }
    // two streams per lane (one lane per stream, plain decode)
    if (!p->bracket) {
      v.push_back({1, 2, kFlat, 8, 0});
      for (int w : wpcs) {
        v.push_back({1, 2, kDynamic, w, 0});
        v.push_back({1, 2, kStatic, w, 0});
      }
    }
  }
  return v;
}

std::string shape_signature(const gmm_plan* p) {
  uint64_t h = 1469598103934665603ull;
  const int32_t hdr[8] = {p->op, p->cfg.K, p->cfg.lo, p->cfg.hi, p->cfg.precision,
                          p->cfg.cdf_kind, p->B, p->bracket ? 1 : 0};
  h = fnv1a(h, hdr, sizeof(hdr));
  h = fnv1a(h, p->n.data(), p->n.size() * sizeof(int64_t));
  h = fnv1a(h, p->S.data(), p->S.size() * sizeof(int64_t));
  h = fnv1a(h, &p->num_cus, sizeof(p->num_cus));
  char buf[40];
  snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  return buf;
}

// Tuning cache: one line per signature,
// "<sig> <lanes> <streams_per_lane> <sched> <waves_per_cu> <lds> <ms>".
bool cache_lookup(const std::string& sig, Config* c, double* ms) {
  const char* path = getenv("FLASHGMM_TUNE_CACHE");
  if (!path || !*path) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char s[64];
  int L, spl, sc, w, lds;
  double t;
  bool found = false;
  while (fscanf(f, "%63s %d %d %d %d %d %lf", s, &L, &spl, &sc, &w, &lds, &t) == 7) {
    if (sig == s) {
      c->lanes = L;
      c->spl = spl;
      c->sched = sc;
      c->waves_per_cu = w;
      c->lds = lds;
      *ms = t;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void cache_store(const std::string& sig, const Config& c, double ms) {
  const char* path = getenv("FLASHGMM_TUNE_CACHE");
  if (!path || !*path) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d %d %d %d %.6f\n", sig.c_str(), c.lanes, c.spl, c.sched, c.waves_per_cu,
          c.lds, ms);
  fclose(f);
}

Config default_config(const gmm_plan* p) {
  Config c;
  // encode: words staged in LDS where the streams fit (measured 2-4% faster
  // than the scratch rows on the 64- and 256-latent batches)
  if (p->op == 0 && (p->cap_max + 1) * kRBlock * 2 <= kRansLdsMax && lds_ready()) c.lds = 1;
  if (p->op == 1 && !p->bracket) {
    int64_t streams = 0;
    for (int b = 0; b < p->B; ++b) streams += p->S[b];
    c.lanes = default_lanes_per_stream(streams);
    if (c.lanes > 16) c.lanes = 16;
  }
  return c;
}

int time_config(gmm_plan* p, const Config& c, hipStream_t st, double* ms) {
  int r = GMM_OK;
  if (p->op == 1) r = build_decode_items(p, item_streams(c), st);
  if (r) return r;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return GMM_EDEVICE;
  r = enqueue(p, c, st);  // warm-up
  float best = 1e30f;
  for (int rep = 0; rep < 2 && r == GMM_OK; ++rep) {
    (void)hipEventRecord(a, st);
    r = enqueue(p, c, st);
    (void)hipEventRecord(b, st);
    if (hipEventSynchronize(b) != hipSuccess) r = GMM_EDEVICE;
    float t = 0;
    (void)hipEventElapsedTime(&t, a, b);
    best = std::min(best, t);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = best;
  return r;
}

int tune(gmm_plan* p, hipStream_t st) {
  Config c = default_config(p);
  double ms = -1.0;
  if (p->flags & GMM_PLAN_AUTOTUNE) {
    if (!cache_lookup(p->signature, &c, &ms)) {
      double best = 1e30;
      Config bestc = c;
      const std::vector<Config> cand = candidates(p);
      for (const Config& k : cand) {
        double t;
        int r = time_config(p, k, st, &t);
        if (r) return r;
        if (t < best) {
          best = t;
          bestc = k;
        }
      }
      c = bestc;
      ms = best;
      p->candidates = (int32_t)cand.size();
      cache_store(p->signature, c, ms);
    }
  }
  p->conf = c;
  p->best_ms = ms;
  if (p->op == 1) {
    int r = build_decode_items(p, item_streams(c), st);
    if (r) return r;
  }
  p->tuned = true;
  return GMM_OK;
}

int capture(gmm_plan* p) {
  if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return GMM_EDEVICE;
  int r = enqueue(p, p->conf, p->cap_stream);
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(p->cap_stream, &g) != hipSuccess || r != GMM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r ? r : GMM_EDEVICE;
  }
  if (hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return GMM_EDEVICE;
  }
  p->graph = g;
  return GMM_OK;
}

}  // namespace

extern "C" {

int gmm_plan_create(const gmm_cfg* common, int32_t B, const int64_t* n_b, const int32_t* S_b,
                    int32_t op, int32_t flags, gmm_plan** out) {
  if (!out || !common || B < 1 || !n_b || !S_b || (op != 0 && op != 1)) return GMM_EINVAL;
  *out = nullptr;
  gmm_cfg c = *common;
  c.num_streams = 1;
  int st = check_cfg(&c, 0);
  if (st) return st;
  if (c.cdf_kind >= 2) return GMM_EINVAL;  // plans build the A&S and logistic kinds
  for (int b = 0; b < B; ++b)
    if (n_b[b] < 0 || S_b[b] < 1) return GMM_EINVAL;
  gmm_plan* p = new gmm_plan();
  p->cfg = c;
  p->op = op;
  p->B = B;
  p->flags = flags;
  p->q = make_qcfg(&c);
  p->q.prio = 0;  // the batched kernels run at the default priority
  p->n.assign(n_b, n_b + B);
  p->S.assign(S_b, S_b + B);
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    p->num_cus = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete p;
    return GMM_EDEVICE;
  }
  p->fast = use_fast_recip(p->cap_stream);
  // flattened layout
  p->h_desc.resize(B);
  std::vector<int32_t> cdf_blk, rans_blk, pack_blk;
  int64_t scratch = 0;
  for (int b = 0; b < B; ++b) {
    LatentDesc& d = p->h_desc[b];
    memset(&d, 0, sizeof(d));
    d.n = p->n[b];
    d.S = p->S[b];
    d.cap = (d.n > 0) ? (d.n + d.S - 1) / d.S : 1;
    d.cdf_blk0 = (int64_t)cdf_blk.size();
    d.elem_base = d.cdf_blk0 * kCdfBlock;
    for (int64_t k = 0; k < (d.n + kCdfBlock - 1) / kCdfBlock; ++k) cdf_blk.push_back(b);
    d.rans_blk0 = (int64_t)rans_blk.size();
    d.nblk = (d.S + kRBlock - 1) / kRBlock;
    for (int64_t k = 0; k < d.nblk; ++k) rans_blk.push_back(b);
    d.pack_blk0 = (int64_t)pack_blk.size();
    const int64_t per = kPBlock / kPLanes;
    for (int64_t k = 0; k < (d.S + per - 1) / per; ++k) pack_blk.push_back(b);
    d.scratch_base = scratch;
    scratch += d.S * d.cap;
    p->cap_max = std::max<int64_t>(p->cap_max, d.cap);
  }
  p->n_cdf_blk = (int64_t)cdf_blk.size();
  p->n_rans_blk = (int64_t)rans_blk.size();
  p->n_pack_blk = (int64_t)pack_blk.size();
  int r = GMM_OK;
  r = r ? r : dev_alloc(p, &p->d_desc, B);
  // status bits [B], the queue counter, then (encode) the look-back slots
  // of the LDS-staged rANS pass at an 8-byte aligned offset
  const int64_t slot_off = (B + 2) & ~(int64_t)1;
  p->reset_words = (op == 0) ? slot_off + 2 * p->n_rans_blk : B + 1;
  r = r ? r : dev_alloc(p, &p->d_bits, p->reset_words);
  if (!r && op == 0) p->d_slots = (uint64_t*)(p->d_bits + slot_off);
  r = r ? r : dev_alloc(p, &p->d_codes, B);
  if (!r && hipHostMalloc((void**)&p->pinned_desc, sizeof(LatentDesc) * B, 0) != hipSuccess)
    r = GMM_ENOMEM;
  if (!r && op == 0) {
    r = r ? r : dev_alloc(p, &p->d_cdf_blk, p->n_cdf_blk);
    r = r ? r : dev_alloc(p, &p->d_rans_blk, p->n_rans_blk);
    r = r ? r : dev_alloc(p, &p->d_pack_blk, p->n_pack_blk);
    r = r ? r : dev_alloc(p, &p->d_rans_items, p->n_rans_blk);
    r = r ? r : dev_alloc(p, &p->d_cf, p->n_cdf_blk * kCdfBlock);
    r = r ? r : dev_alloc(p, &p->d_scratch, scratch);
    r = r ? r : dev_alloc(p, &p->d_xfin, p->n_rans_blk * kRBlock);
    r = r ? r : dev_alloc(p, &p->d_count, p->n_rans_blk * kRBlock);
    r = r ? r : dev_alloc(p, &p->d_local, p->n_rans_blk * kRBlock);
    r = r ? r : dev_alloc(p, &p->d_blk_total, p->n_rans_blk);
    r = r ? r : dev_alloc(p, &p->d_blk_pre, p->n_rans_blk);
    if (!r) {
      // rANS work items, longest streams first
      std::vector<int32_t> items(p->n_rans_blk);
      for (int64_t k = 0; k < p->n_rans_blk; ++k) items[k] = (int32_t)k;
      std::stable_sort(items.begin(), items.end(), [&](int32_t x, int32_t y) {
        const LatentDesc& a = p->h_desc[rans_blk[x]];
        const LatentDesc& bb = p->h_desc[rans_blk[y]];
        return a.cap > bb.cap;
      });
      hipStream_t s = p->cap_stream;
      if (hipMemcpyAsync(p->d_cdf_blk, cdf_blk.data(), cdf_blk.size() * 4, hipMemcpyHostToDevice,
                         s) != hipSuccess ||
          hipMemcpyAsync(p->d_rans_blk, rans_blk.data(), rans_blk.size() * 4,
                         hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(p->d_pack_blk, pack_blk.data(), pack_blk.size() * 4,
                         hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(p->d_rans_items, items.data(), items.size() * 4, hipMemcpyHostToDevice,
                         s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        r = GMM_EDEVICE;
    }
  }
  if (r) {
    gmm_plan_destroy(p);
    return r;
  }
  p->signature = shape_signature(p);
  *out = p;
  return GMM_OK;
}

int gmm_plan_exec(gmm_plan* p, const gmm_latent_io* io, int32_t* dev_status, void* stream) {
  if (!p || !io) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  // validate and refresh the descriptor table when the buffers change
  bool changed = p->last_io.size() != (size_t)p->B;
  for (int b = 0; b < p->B && !changed; ++b) changed = !same_io(io[b], p->last_io[b]);
  if (changed) {
    for (int b = 0; b < p->B; ++b) {
      const gmm_latent_io& x = io[b];
      const bool need_params = p->n[b] > 0;
      if (need_params && (!x.weights || !x.means || !x.scales)) return GMM_EINVAL;
      if (!x.offsets || x.words < 0) return GMM_EINVAL;
      if (p->op == 0 && need_params && !x.symbols) return GMM_EINVAL;
      if (p->op == 1 && need_params && !x.decoded) return GMM_EINVAL;
      if (x.words > 0 && !x.bitstream) return GMM_EINVAL;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return GMM_EDEVICE;
    for (int b = 0; b < p->B; ++b) {
      LatentDesc& d = p->h_desc[b];
      const gmm_latent_io& x = io[b];
      d.sym = x.symbols;
      d.w = x.weights;
      d.mu = x.means;
      d.sg = x.scales;
      d.bs = x.bitstream;
      d.words = x.words;
      d.offsets = x.offsets;
      d.dec = x.decoded;
      p->pinned_desc[b] = d;
    }
    if (hipMemcpyAsync(p->d_desc, p->pinned_desc, sizeof(LatentDesc) * p->B,
                       hipMemcpyHostToDevice, st) != hipSuccess)
      return GMM_EDEVICE;
    p->last_io.assign(io, io + p->B);
    if (p->op == 1) {
      bool fit = true;
      for (int b = 0; b < p->B; ++b)
        fit = fit && buffer_offsets_fit(p->cfg.K, p->n[b], p->S[b], io[b].words);
      if (fit != p->buf) {  // the captured graph launches the other decode kernel
        p->buf = fit;
        if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->gexec = nullptr;
        p->graph = nullptr;
      }
    }
  }
  int r;
  if (!p->tuned) {
    r = tune(p, st);
    if (r) return r;
  }
  if (!p->gexec) {
    if (hipStreamSynchronize(st) != hipSuccess) return GMM_EDEVICE;
    r = capture(p);
    if (r) return r;
  }
  if (hipGraphLaunch(p->gexec, st) != hipSuccess) return GMM_EDEVICE;
  if (dev_status) {
    if (hipMemcpyAsync(dev_status, p->d_codes, sizeof(int32_t) * p->B, hipMemcpyDeviceToDevice,
                       st) != hipSuccess)
      return GMM_EDEVICE;
    return GMM_OK;
  }
  std::vector<int32_t> codes(p->B);
  if (hipMemcpyAsync(codes.data(), p->d_codes, sizeof(int32_t) * p->B, hipMemcpyDeviceToHost,
                     st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return GMM_EDEVICE;
  int worst = GMM_OK;
  for (int32_t c : codes)
    if (c != GMM_OK && (worst == GMM_OK || c < worst)) worst = c;
  return worst;
}

int gmm_plan_info(const gmm_plan* p, gmm_plan_info_t* info) {
  if (!p || !info) return GMM_EINVAL;
  info->tuned = p->tuned ? 1 : 0;
  info->candidates = p->candidates;
  info->graph_captured = p->gexec ? 1 : 0;
  info->config.lanes_per_stream = p->conf.lanes;
  info->config.streams_per_lane = p->conf.spl;
  info->config.schedule = p->conf.sched;
  info->config.waves_per_cu = p->conf.waves_per_cu;
  info->config.lds_staging = p->conf.lds;
  info->best_ms = p->best_ms;
  return GMM_OK;
}

int gmm_plan_set_config(gmm_plan* p, const gmm_plan_config* config) {
  if (!p || !config) return GMM_EINVAL;
  const int32_t lanes = config->lanes_per_stream, spl = config->streams_per_lane;
  const int32_t schedule = config->schedule, waves_per_cu = config->waves_per_cu;
  const int32_t lds = config->lds_staging;
  if (lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16) return GMM_EINVAL;
  if ((p->op == 0 || p->bracket) && lanes != 1) return GMM_EINVAL;
  if (schedule < kFlat || schedule > kStatic || waves_per_cu < 1 || waves_per_cu > 64)
    return GMM_EINVAL;
  if (lds != 0 && lds != 1) return GMM_EINVAL;
  if (lds && (p->op != 0 || schedule == kStatic || (p->cap_max + 1) * kRBlock * 2 > kRansLdsMax ||
              !lds_ready()))
    return GMM_EINVAL;
  // two streams per lane: the LDS-staged encode pass, or the plain decode
  // with one lane per stream
  if (spl != 1 && !(spl == 2 && (p->op == 0 ? lds == 1 : (!p->bracket && lanes == 1))))
    return GMM_EINVAL;
  if (p->cap_stream) (void)hipStreamSynchronize(p->cap_stream);
  (void)hipDeviceSynchronize();
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
  p->conf.lanes = lanes;
  p->conf.spl = spl;
  p->conf.sched = schedule;
  p->conf.waves_per_cu = waves_per_cu;
  p->conf.lds = lds;
  p->best_ms = -1.0;
  if (p->op == 1) {
    int r = build_decode_items(p, item_streams(p->conf), p->cap_stream);
    if (r) return r;
  }
  p->tuned = true;
  return GMM_OK;
}

int gmm_plan_set_bracket(gmm_plan* p, const gmm_bracket* bracket, gmm_decode_stats* stats) {
  if (!p || p->op != 1) return GMM_EINVAL;
  if (bracket && (bracket->K != p->cfg.K || p->cfg.K > 5 || p->cfg.param_kind != 0))
    return GMM_EINVAL;
  if (p->cap_stream) (void)hipStreamSynchronize(p->cap_stream);
  (void)hipDeviceSynchronize();
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
  p->bracket = bracket;
  p->stats = (unsigned long long*)stats;
  p->tuned = false;
  p->items_per = 0;
  p->signature = shape_signature(p);
  return GMM_OK;
}

int gmm_plan_candidates(const gmm_plan* p, gmm_plan_config* out, int32_t max_count) {
  if (!p) return -1;
  const std::vector<Config> v = candidates(p);
  for (int32_t i = 0; i < (int32_t)v.size() && out && i < max_count; ++i)
    out[i] = {v[i].lanes, v[i].spl, v[i].sched, v[i].waves_per_cu, v[i].lds};
  return (int32_t)v.size();
}

int gmm_plan_destroy(gmm_plan* p) {
  if (!p) return GMM_OK;
  if (p->cap_stream) (void)hipStreamSynchronize(p->cap_stream);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  (void)hipDeviceSynchronize();
  for (void* a : p->allocs) (void)hipFree(a);
  if (p->pinned_desc) (void)hipHostFree(p->pinned_desc);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
  return GMM_OK;
}

}  // extern "C"
