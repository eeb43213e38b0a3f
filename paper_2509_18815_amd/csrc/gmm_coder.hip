// GMM rANS coder kernels for gfx950 and the C ABI of libflashgmm.so
// (declarations and argument contracts: include/flashgmm.h).
//
// Encode (FlashGMM Sec. III-A: the CDF is evaluated only at the coded
// symbol's two boundaries) runs as
//   k_enc_cdf   one thread per element: c_j and f_j of its symbol, packed
//               into one uint32 (fully parallel over all n elements);
//   k_enc_rans  one lane per stream: the integer rANS recurrence of Eq. (3)
//               in reverse element order, renormalisation words written to
//               the stream's scratch region in decoder order, then a
//               wavefront/block prefix sum of the segment lengths; the
//               workgroup that finishes last scans the block totals and
//               writes the call's status;
//   k_pack      stream offsets and the compacted bitstream.
// Decode (Sec. III-A: binary search over the monotone CDF) runs one lane per
// stream with a branch-uniform search (every lane executes exactly
// ceil(log2 N) CDF evaluations per symbol, with no early exit), or L lanes
// per stream with an (L+1)-ary search when streams are few; its last
// workgroup writes the call's status.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <mutex>

#include "../../include/flashgmm.h"
#include "gmm_device.h"
#include "gmm_host.h"
#include "gmm_kernels.h"
#include "gmm_stream.h"

using namespace fgmm;

// ------------------------------------------------------------------ kernels

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}


// Exhaustive check of recip_fast against IEEE division on every float in
// [lo_bits, lo_bits + count).
__global__ void k_recip_check(uint32_t lo_bits, uint32_t count, unsigned long long* mismatches) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const float u = __uint_as_float(lo_bits + t);
  const float a = recip_fast(u);
  const float b = 1.0f / u;
  if (__float_as_uint(a) != __float_as_uint(b)) atomicAdd(mismatches, 1ull);
}

constexpr int kRansBlock = 256;

// Encode phase 2: one lane per stream; stream s owns scratch words
// [s cap, (s+1) cap). Then the block's exclusive scan of the segment
// lengths 2 + count (the wavefront prefix sums that place the streams).
// The workgroup that finishes last scans the block totals into blk_pre,
// flags a total above the capacity, and writes the call's status code
// (bits[0]: status bits, bits[1]: workgroup counter, zeroed before).
__global__ void __launch_bounds__(kRansBlock)
    k_enc_rans(int64_t n, int64_t S, int P, const uint32_t* __restrict__ cf,
               uint16_t* __restrict__ scratch, int64_t cap, uint32_t* __restrict__ xfin,
               uint32_t* __restrict__ count, uint32_t* __restrict__ local_off,
               int64_t* __restrict__ blk_total, int64_t* __restrict__ blk_pre, int64_t capacity,
               uint32_t* bits, int32_t* dev_status) {
  const int64_t s = (int64_t)blockIdx.x * kRansBlock + threadIdx.x;
  uint32_t cnt = 0;
  if (s < S) {
    bool zf;
    xfin[s] = rans_stream(n, S, P, s, cf, scratch + s * cap + (cap - 1), &cnt, &zf);
    count[s] = cnt;
    if (zf) atomicOr(bits, kStRange);  // an out-of-range symbol (phase 1 wrote f = 0)
  }
  uint32_t tot;
  const uint32_t excl = block_excl_scan<kRansBlock>((s < S) ? cnt + 2u : 0u, &tot);
  if (s < S) local_off[s] = excl;
  if (threadIdx.x == 0) atomicExch((unsigned long long*)(blk_total + blockIdx.x), (unsigned long long)tot);
  if (!grid_last_block(bits + 1)) return;
  const int64_t total = scan_totals<kRansBlock, true>(gridDim.x, blk_total, blk_pre);
  if (threadIdx.x == 0) {
    uint32_t b = atomicOr(bits, (total > capacity) ? kStNoSpace : 0u);
    if (total > capacity) b |= kStNoSpace;
    if (dev_status) *dev_status = status_code(b);
  }
}

// Encode phase 2 with the renormalisation words staged in LDS, in one pass:
// a workgroup of 256 streams (taken in start order from a ticket counter,
// bits[1]) runs the recurrence with each lane's emitted words in a column
// of the dynamic LDS array words[cap][256], scans its segment lengths
// (2 + count), gets the exclusive prefix of the words of all earlier
// workgroups by decoupled look-back over slots[] (zeroed before the launch),
// and writes its streams' offsets and, when its range fits the capacity,
// their segments straight into the bitstream (each lane its own stream's;
// a copy by whole wavefronts, 64 consecutive words per store, took longer
// for its per-stream shuffles). The workgroup holding the last streams
// writes offsets[S], flags ENOSPC and writes the call's status code
// (bits[0]: status bits).
template <bool kBuf>
__global__ void __launch_bounds__(kRansBlock)
    k_enc_rans_lds(int64_t n, int64_t S, int P, int trash_row,
                   const uint32_t* __restrict__ cf,
                   int64_t* __restrict__ offsets, uint16_t* __restrict__ bitstream,
                   int64_t capacity, uint64_t* slots, uint32_t* bits, int32_t* dev_status) {
  extern __shared__ uint16_t words[];  // [cap + 1][kRansBlock], row cap: trash
  __shared__ int64_t ticket_sh, excl_sh;
  if (threadIdx.x == 0) ticket_sh = (int64_t)atomicAdd(bits + 1, 1u);
  __syncthreads();
  const int64_t ticket = ticket_sh;
  const int64_t s = ticket * kRansBlock + threadIdx.x;
  uint32_t cnt = 0, x = 1u << 16;
  bool zf = false;
  if (s < S)
    x = rans_stream_lds<kBuf>(n, S, P, s, cf, words + threadIdx.x, kRansBlock, trash_row, &cnt,
                              &zf);
  uint32_t tot;
  const uint32_t len = (s < S) ? cnt + 2u : 0u;
  const uint32_t local = block_excl_scan<kRansBlock>(len, &tot);
  // an out-of-range symbol (phase 1 wrote f = 0): the status bit is set,
  // and complete, before this workgroup publishes its total, so the
  // workgroup of the last streams sees it once its look-back has ended
  if (__syncthreads_or(zf ? 1 : 0) && threadIdx.x == 0) {
    atomicOr(bits, kStRange);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
  }
  if (threadIdx.x < 64) {
    const int64_t e = lookback_prefix(slots, ticket, (int64_t)tot);
    if (threadIdx.x == 0) excl_sh = e;
  }
  __syncthreads();
  const int64_t excl = excl_sh;
  if (s < S) offsets[s] = excl + (int64_t)local;
  const int64_t nblk = (S + kRansBlock - 1) / kRansBlock;
  if (ticket == nblk - 1 && threadIdx.x == 0) {
    const int64_t total = excl + (int64_t)tot;
    offsets[S] = total;
    const uint32_t nospace = (total > capacity) ? kStNoSpace : 0u;
    const uint32_t b = atomicOr(bits, nospace) | nospace;
    if (dev_status) *dev_status = status_code(b);
  }
  if (excl + (int64_t)tot > capacity) return;
  // copy out: each lane writes its own stream's segment, the state words
  // and then the renormalisation words in decoder order (newest first)
  if (s < S) {
    const int64_t o = excl + (int64_t)local;
    bitstream[o] = (uint16_t)(x & 0xFFFFu);
    bitstream[o + 1] = (uint16_t)(x >> 16);
    const uint16_t* col = words + threadIdx.x;
    for (uint32_t t = 0; t < cnt; ++t) bitstream[o + 2 + t] = col[(cnt - 1u - t) * kRansBlock];
  }
}

// Offsets and compaction: 16 lanes per stream.
constexpr int kPackBlock = 256, kPackLanes = 16;
__global__ void __launch_bounds__(kPackBlock)
    k_pack(int64_t S, int64_t nblk, int64_t cap, const uint16_t* __restrict__ scratch,
           const uint32_t* __restrict__ xfin, const uint32_t* __restrict__ count,
           const uint32_t* __restrict__ local_off, const int64_t* __restrict__ blk_pre,
           const int64_t* __restrict__ blk_total, int64_t* __restrict__ offsets,
           uint16_t* __restrict__ bitstream, int64_t capacity) {
  const int64_t s = (int64_t)blockIdx.x * (kPackBlock / kPackLanes) + threadIdx.x / kPackLanes;
  const int l = threadIdx.x % kPackLanes;
  const int64_t total = blk_pre[nblk - 1] + blk_total[nblk - 1];
  const bool fits = total <= capacity;  // (k_enc_rans flagged ENOSPC)
  if (s >= S) return;
  const int64_t off = blk_pre[s / kRansBlock] + (int64_t)local_off[s];
  const uint32_t cnt = count[s];
  if (l == 0) {
    offsets[s] = off;
    if (s == S - 1) offsets[S] = total;
  }
  if (!fits) return;
  pack_segment(bitstream + off, xfin[s], scratch + s * cap + (cap - (int64_t)cnt), cnt, l,
               kPackLanes);
}

// Raw network outputs to mixture parameters as a pass of its own (the
// coder kernels apply the same mapping per element when param_kind = 1):
// weights [K][n] from logits, scales [K][n] from log-scales.
template <int K>
__global__ void k_params_from_raw(int64_t n, const float* __restrict__ logits,
                                  const float* __restrict__ log_scales, float* __restrict__ w,
                                  float* __restrict__ sg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float a[K], b[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    a[k] = logits[k * n + i];
    b[k] = log_scales[k * n + i];
  }
  fgmm::raw_to_params<K>(a, b);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    w[k * n + i] = a[k];
    sg[k * n + i] = b[k];
  }
}

// Subset (gather) pass of a latent: validates idx (every entry in
// [0, n_total)) before the coder runs.
__global__ void k_check_idx(const int32_t* __restrict__ idx, int64_t m, int64_t n_total,
                            uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m && (idx[i] < 0 || (int64_t)idx[i] >= n_total)) atomicOr(status, kStInval);
}

// ------------------------------------------------------------- host side

namespace {

int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

struct EncLayout {
  int64_t status, look, cf, scratch, xfin, count, local_off, blk_total, blk_pre, bytes;
  int64_t cap, nblk;
};

EncLayout enc_layout(int64_t n, int64_t S) {
  EncLayout L;
  L.cap = (n > 0) ? (n + S - 1) / S : 1;
  L.nblk = (S + kRansBlock - 1) / kRansBlock;
  int64_t o = 0;
  L.status = o; o += 256;
  L.look = o; o += align256(8 * L.nblk);  // look-back slots, zeroed with the status words
  L.cf = o; o += align256(4 * n);
  L.scratch = o; o += align256(2 * S * L.cap);
  L.xfin = o; o += align256(4 * S);
  L.count = o; o += align256(4 * S);
  L.local_off = o; o += align256(4 * S);
  L.blk_total = o; o += align256(8 * L.nblk);
  L.blk_pre = o; o += align256(8 * L.nblk);
  L.bytes = o;
  return L;
}

}  // namespace

namespace fgmm {

int check_cfg(const gmm_cfg* c, int64_t n) {
  if (!c || n < 0) return GMM_EINVAL;
  if (c->K < 1 || c->K > kMaxK) return GMM_EINVAL;
  if (c->precision < 2 || c->precision > 16) return GMM_EINVAL;
  if (c->num_streams < 1) return GMM_EINVAL;
  if (c->cdf_kind < 0 || c->cdf_kind > 3) return GMM_EINVAL;
  if (c->param_kind != 0 && c->param_kind != 1) return GMM_EINVAL;
  if (c->lo < -(1 << 22) || c->hi > (1 << 22) || c->hi <= c->lo) return GMM_EINVAL;
  const int64_t N = (int64_t)c->hi - c->lo + 1;
  const int64_t M = (int64_t)1 << c->precision;
  if (N < 2 || N > M / 2) return GMM_EINVAL;
  return GMM_OK;
}

// Wavefront priority of this host thread's later encode and decode launches
// (gmm_set_wave_priority).
thread_local int32_t g_wave_priority = 0;

QCfg make_qcfg(const gmm_cfg* c) {
  QCfg q;
  q.prio = g_wave_priority;
  q.lo = c->lo;
  q.N = c->hi - c->lo + 1;
  q.M = 1u << c->precision;
  q.span = (float)(q.M - (uint32_t)q.N);
  q.lo_mh = (float)c->lo - 0.5f;
  q.raw = c->param_kind;
  return q;
}

int search_rounds(int32_t N) {
  int r = 0;
  while ((1 << r) < N) ++r;
  return r;
}

// Per-device flag: recip_fast matches IEEE division on [2^-10, 2^10]
// (checked once per device, exhaustively, before the first coder launch).
static std::mutex g_init_mu;
static int g_fast_ok[64];  // 0 unknown, 1 verified, -1 mismatch

// counter [device, nullable]: 8 bytes for the mismatch count; when NULL the
// check allocates it on the stream.
int fast_recip_mismatches(unsigned long long* count, hipStream_t st, void* counter) {
  unsigned long long* d = (unsigned long long*)counter;
  if (!d && hipMallocAsync((void**)&d, sizeof(unsigned long long), st) != hipSuccess)
    return GMM_ENOMEM;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t*)d, 0u, (int64_t)2);
  const uint32_t lo = 0x3a800000u;            // 2^-10
  const uint32_t cnt = 0x44800000u - lo + 1;  // every float in [2^-10, 2^10]
  hipLaunchKernelGGL(k_recip_check, dim3((cnt + 255) / 256), dim3(256), 0, st, lo, cnt, d);
  unsigned long long h = 0;
  hipError_t e1 = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, st);
  hipError_t e2 = hipStreamSynchronize(st);
  if (!counter) (void)hipFreeAsync(d, st);
  if (e1 != hipSuccess || e2 != hipSuccess) return GMM_EDEVICE;
  *count = h;
  return GMM_OK;
}

bool use_fast_recip(hipStream_t st, void* counter) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (g_fast_ok[dev] == 0) {
    unsigned long long mm = 1;
    if (fast_recip_mismatches(&mm, st, counter) != GMM_OK) return false;
    g_fast_ok[dev] = (mm == 0) ? 1 : -1;
  }
  return g_fast_ok[dev] == 1;
}

int finish(uint32_t* bits, int32_t* dev_status, hipStream_t st) {
  // with a device status the last workgroup of the call's last kernel has
  // written the code already
  if (dev_status) return GMM_OK;
  uint32_t h = 0;
  if (hipMemcpyAsync(&h, bits, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess)
    return GMM_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return GMM_EDEVICE;
  if (h & kStInval) return GMM_EINVAL;
  if (h & kStRange) return GMM_ERANGE;
  if (h & kStNoSpace) return GMM_ENOSPC;
  if (h & kStCorrupt) return GMM_ECORRUPT;
  return GMM_OK;
}

// Largest dynamic LDS of k_enc_rans_lds (words of a workgroup's streams):
// streams of up to 300 symbols; longer ones take the scratch-row path.
constexpr int64_t kRansLdsMax = (300 + 1) * kRansBlock * 2;

// Lets k_enc_rans_lds use more than the default dynamic LDS (once).
bool enc_lds_ready() {
  static const bool ok = hipFuncSetAttribute((const void*)k_enc_rans_lds<false>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)kRansLdsMax) == hipSuccess &&
                         hipFuncSetAttribute((const void*)k_enc_rans_lds<true>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)kRansLdsMax) == hipSuccess;
  return ok;
}

// Encode with an explicit workspace (used by the C entry point and plans).
int encode_launch(const gmm_cfg* cfg, int64_t n, const int32_t* symbols, const float* w,
                  const float* mu, const float* sg, uint16_t* bitstream, int64_t capacity,
                  int64_t* offsets, char* ws, bool fast, hipStream_t st, const int32_t* idx,
                  int64_t n_total, int32_t* dev_status) {
  const int64_t S = cfg->num_streams;
  const EncLayout L = enc_layout(n, S);
  const QCfg q = make_qcfg(cfg);
  uint32_t* status = (uint32_t*)(ws + L.status);
  uint32_t* cf = (uint32_t*)(ws + L.cf);
  uint16_t* scratch = (uint16_t*)(ws + L.scratch);
  uint32_t* xfin = (uint32_t*)(ws + L.xfin);
  uint32_t* count = (uint32_t*)(ws + L.count);
  uint32_t* local_off = (uint32_t*)(ws + L.local_off);
  int64_t* blk_total = (int64_t*)(ws + L.blk_total);
  int64_t* blk_pre = (int64_t*)(ws + L.blk_pre);
  // status bits, the workgroup counter (or ticket counter) of the rANS
  // pass and the look-back slots: zeroed by the first workgroup of phase 1
  // when phase 1 is the plain-kind, non-gather kernel (nothing before it
  // writes them), else by a fill kernel first
  const int64_t nclear = (L.look + 8 * L.nblk) / 4;
  const bool clear_in_cdf = n > 0 && !idx && cfg->cdf_kind < 2;
  // buffer resources for the whole-latent encode when its offsets fit 32 bits
  const bool buf = !idx && encode_offsets_fit(cfg->K, n, S);
  if (!clear_in_cdf)
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((nclear + 255) / 256)), dim3(256), 0, st,
                       status, 0u, nclear);
  if (n > 0) {
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (idx) hipLaunchKernelGGL(k_check_idx, grid, block, 0, st, idx, n, n_total, status);
    if (cfg->cdf_kind >= 2)
      ablation_enc_cdf(q, cfg->K, cfg->cdf_kind, n, symbols, w, mu, sg, cf, status, st);
    else
    dispatch(cfg->K, cfg->cdf_kind, fast, [&](auto Kc, auto kc, auto fc) {
      constexpr int K_ = decltype(Kc)::value, KI = decltype(kc)::value;
      constexpr bool F = decltype(fc)::value;
      if (idx)
        hipLaunchKernelGGL((k_enc_cdf<K_, KI, F, true>), grid, block, 0, st, q, n, symbols, w,
                           mu, sg, cf, status, idx, n_total);
      else if (buf)
        hipLaunchKernelGGL((k_enc_cdf<K_, KI, F, false, true>), grid, block, 0, st, q, n,
                           symbols, w, mu, sg, cf, status, nullptr, (int64_t)0, status, nclear);
      else
        hipLaunchKernelGGL((k_enc_cdf<K_, KI, F, false>), grid, block, 0, st, q, n, symbols, w,
                           mu, sg, cf, status, nullptr, (int64_t)0, status, nclear);
    });
  }
  const int64_t lds = (L.cap + 1) * kRansBlock * 2;  // the words and a trash row
  if (lds <= kRansLdsMax && enc_lds_ready()) {
    if (buf)
      hipLaunchKernelGGL(k_enc_rans_lds<true>, dim3((unsigned)L.nblk), dim3(kRansBlock),
                         (size_t)lds, st, n, S, cfg->precision, (int)L.cap, cf, offsets,
                         bitstream, capacity, (uint64_t*)(ws + L.look), status, dev_status);
    else
      hipLaunchKernelGGL(k_enc_rans_lds<false>, dim3((unsigned)L.nblk), dim3(kRansBlock),
                         (size_t)lds, st, n, S, cfg->precision, (int)L.cap, cf, offsets,
                         bitstream, capacity, (uint64_t*)(ws + L.look), status, dev_status);
    return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
  }
  // streams too long for LDS: words through the scratch rows, then k_pack
  hipLaunchKernelGGL(k_enc_rans, dim3((unsigned)L.nblk), dim3(kRansBlock), 0, st, n, S,
                     cfg->precision, cf, scratch, L.cap, xfin, count, local_off, blk_total,
                     blk_pre, capacity, status, dev_status);
  const int64_t per = kPackBlock / kPackLanes;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((S + per - 1) / per)), dim3(kPackBlock), 0, st, S,
                     L.nblk, L.cap, scratch, xfin, count, local_off, blk_pre, blk_total, offsets,
                     bitstream, capacity);
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

// Rounds of an (L+1)-ary search over N symbols: smallest R with (L+1)^R >= N.
int search_rounds_lps(int32_t N, int L) {
  int r = 0;
  int64_t reach = 1;
  while (reach < N) {
    reach *= (L + 1);
    ++r;
  }
  return r;
}

// Lanes per stream when the caller does not choose: enough lanes to give
// the chip about 64K lanes (one wave per SIMD), at most 32 per stream.
int default_lanes_per_stream(int64_t S) {
  int L = 1;
  while (L < 32 && S * L < 65536) L <<= 1;
  return L;
}

// Lanes per stream of a plain decode (lanes > 0: the caller's choice).
int plain_decode_lanes(const gmm_cfg* cfg, int lanes) {
  const int32_t N = cfg->hi - cfg->lo + 1;
  int L = (lanes > 0) ? lanes : default_lanes_per_stream(cfg->num_streams);
  // The automatic choice then halves the group while that needs no more
  // rounds: a smaller group makes fewer evaluations per symbol, exchanges its
  // bounds in fewer DPP steps (16 lanes: a DPP row, no LDS) and leaves SIMDs
  // free for concurrent work. 192x16x16 latent (256 streams, N = 256): 16
  // lanes 0.145 ms against 32 lanes 0.158 ms; 320x48x32 latent (4,096
  // streams, N = 511, three rounds at 8 and 16 lanes): 8 lanes 0.135 ms
  // against 0.150 ms on its own, and 0.388 against 0.39-0.44 ms per plain
  // step of the two paper-scale latents on two streams.
  if (lanes <= 0 && L > 2) {
    const int r = search_rounds_lps(N, L);
    while (L > 2 && search_rounds_lps(N, L / 2) == r) L >>= 1;
  }
  if (cfg->cdf_kind >= 2) L = (L == 1) ? 1 : 16;  // the comparison kinds build L = 1 and 16
  return L;
}

int decode_launch(const gmm_cfg* cfg, int64_t n, const uint16_t* bs, int64_t total_words,
                  const int64_t* offsets, const float* w, const float* mu, const float* sg,
                  int32_t* symbols, uint32_t* status, bool fast, hipStream_t st, int lanes,
                  const int32_t* idx, int64_t n_total, int32_t* dev_status) {
  const int64_t S = cfg->num_streams;
  const QCfg q = make_qcfg(cfg);
  const int L = plain_decode_lanes(cfg, lanes);
  const int rounds = (L == 1) ? search_rounds(q.N) : search_rounds_lps(q.N, L);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, status, 0u, (int64_t)2);
  if (idx && n > 0)
    hipLaunchKernelGGL(k_check_idx, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, idx, n,
                       n_total, status);
  const int64_t threads = S * L;
  // 256-thread workgroups: the four wavefronts of a workgroup land on the
  // four SIMDs of a CU, while single-wavefront workgroups were measured to
  // leave up to ~9% of the SIMDs with two wavefronts (and as many idle)
  // after other work, which stretched a one-wavefront-per-SIMD decode by
  // about 1.4x.
  const int blk = 256;
  const dim3 grid((unsigned)((threads + blk - 1) / blk)), block(blk);
  if (cfg->cdf_kind >= 2) {
    if (idx) return GMM_EINVAL;
    ablation_decode(q, cfg->K, cfg->cdf_kind, cfg->precision, rounds, L, n, S, bs, total_words,
                    offsets, w, mu, sg, symbols, status, dev_status, st);
    return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
  }
  // buffer resources for the whole-latent decode when its offsets fit 32 bits
  const bool buf = !idx && buffer_offsets_fit(cfg->K, n, S, total_words);
  dispatch(cfg->K, cfg->cdf_kind, fast, [&](auto Kc, auto kc, auto fc) {
    constexpr int K_ = decltype(Kc)::value, KI = decltype(kc)::value;
    constexpr bool F = decltype(fc)::value;
#define FG_DEC(LL)                                                                              \
  if (idx)                                                                                      \
    hipLaunchKernelGGL((k_decode<K_, KI, F, LL, true>), grid, block, 0, st, q, cfg->precision,  \
                       rounds, n, S, bs, total_words, offsets, w, mu, sg, symbols, status,      \
                       dev_status, idx, n_total);                                               \
  else if (buf)                                                                                 \
    hipLaunchKernelGGL((k_decode<K_, KI, F, LL, false, true>), grid, block, 0, st, q,           \
                       cfg->precision, rounds, n, S, bs, total_words, offsets, w, mu, sg,       \
                       symbols, status, dev_status, nullptr, (int64_t)0);                       \
  else                                                                                          \
    hipLaunchKernelGGL((k_decode<K_, KI, F, LL, false>), grid, block, 0, st, q, cfg->precision, \
                       rounds, n, S, bs, total_words, offsets, w, mu, sg, symbols, status,      \
                       dev_status, nullptr, (int64_t)0)
    switch (L) {
      case 1: FG_DEC(1); break;
      case 2: FG_DEC(2); break;
      case 4: FG_DEC(4); break;
      case 8: FG_DEC(8); break;
      case 16: FG_DEC(16); break;
      default: FG_DEC(32); break;
    }
#undef FG_DEC
  });
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

int64_t encode_ws_bytes(int64_t n, int64_t S) { return enc_layout(n, S).bytes; }

}  // namespace fgmm

// -------------------------------------------------------------- C ABI

// Lanes per stream chosen by gmm_set_decode_lanes (0 = automatic).
static int g_lanes_override = 0;

extern "C" {

int gmm_set_decode_lanes(int32_t lanes) {
  if (lanes != 0 && lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16 &&
      lanes != 32)
    return GMM_EINVAL;
  g_lanes_override = lanes;
  return GMM_OK;
}


int gmm_decode_lanes(const gmm_cfg* cfg) {
  if (fgmm::check_cfg(cfg, 0)) return -GMM_EINVAL;
  return fgmm::plain_decode_lanes(cfg, g_lanes_override);
}

int gmm_set_wave_priority(int32_t priority) {
  if (priority < 0 || priority > 3) return GMM_EINVAL;
  fgmm::g_wave_priority = priority;
  return GMM_OK;
}

const char* gmm_status_str(int s) {
  switch (s) {
    case GMM_OK: return "ok";
    case GMM_EINVAL: return "invalid argument";
    case GMM_ERANGE: return "symbol outside the support";
    case GMM_ECORRUPT: return "corrupt bitstream";
    case GMM_ENOSPC: return "bitstream capacity too small";
    case GMM_EDEVICE: return "HIP runtime error";
    case GMM_ENOMEM: return "out of device memory";
    case GMM_E2BIG: return "input too large for the static workspace of the allocation-free entry point";
    default: return "unknown status";
  }
}

int32_t gmm_version(void) { return 10000; }

int64_t gmm_encode_max_words(int64_t n, int32_t S) {
  if (n < 0 || S < 1) return -1;
  return n + 2 * (int64_t)S;
}

int64_t gmm_workspace_bytes(const gmm_cfg* cfg, int64_t n, int32_t op) {
  if (fgmm::check_cfg(cfg, n) != GMM_OK) return -1;
  if (op == 0) return fgmm::encode_ws_bytes(n, cfg->num_streams);
  if (op == 1) return 256;
  return -1;
}

int gmm_cdf_table(const gmm_cfg* cfg, int64_t n, const float* w, const float* mu,
                  const float* sg, uint32_t* table, void* stream) {
  int st0 = fgmm::check_cfg(cfg, n);
  if (st0) return st0;
  if (n > 0 && (!w || !mu || !sg || !table)) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const bool fast = fgmm::use_fast_recip(st);
  const fgmm::QCfg q = fgmm::make_qcfg(cfg);
  const int64_t total = n * ((int64_t)q.N + 1);
  if (total == 0) return GMM_OK;
  if (cfg->cdf_kind >= 2)
    fgmm::ablation_cdf_table(q, cfg->K, cfg->cdf_kind, n, w, mu, sg, table, st);
  else
  fgmm::dispatch(cfg->K, cfg->cdf_kind, fast, [&](auto Kc, auto kc, auto fc) {
    hipLaunchKernelGGL((k_cdf_table<decltype(Kc)::value, decltype(kc)::value,
                                    decltype(fc)::value>),
                       dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, q, n, w, mu, sg,
                       table);
  });
  if (hipGetLastError() != hipSuccess) return GMM_EDEVICE;
  return hipStreamSynchronize(st) == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

int gmm_inverse_cdf(const gmm_cfg* cfg, int64_t n, const float* w, const float* mu,
                    const float* sg, const uint32_t* slot, int32_t* jout, void* stream) {
  int st0 = fgmm::check_cfg(cfg, n);
  if (st0) return st0;
  if (n > 0 && (!w || !mu || !sg || !slot || !jout)) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const bool fast = fgmm::use_fast_recip(st);
  const fgmm::QCfg q = fgmm::make_qcfg(cfg);
  const int rounds = fgmm::search_rounds(q.N);
  uint32_t* status = nullptr;
  if (hipMallocAsync((void**)&status, 256, st) != hipSuccess) return GMM_ENOMEM;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, status, 0u, (int64_t)1);
  if (n > 0 && cfg->cdf_kind >= 2) {
    fgmm::ablation_inverse(q, cfg->K, cfg->cdf_kind, rounds, n, w, mu, sg, slot, jout, status, st);
  } else if (n > 0) {
    fgmm::dispatch(cfg->K, cfg->cdf_kind, fast, [&](auto Kc, auto kc, auto fc) {
      hipLaunchKernelGGL((k_inverse<decltype(Kc)::value, decltype(kc)::value,
                                    decltype(fc)::value>),
                         dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, q, rounds, n, w,
                         mu, sg, slot, jout, status);
    });
  }
  int r = fgmm::finish(status, nullptr, st);
  (void)hipFreeAsync(status, st);
  return r;
}

int gmm_encode(const gmm_cfg* cfg, int64_t n, const int32_t* symbols, const float* w,
               const float* mu, const float* sg, uint16_t* bitstream, int64_t capacity_words,
               int64_t* offsets, void* ws, int64_t ws_bytes, int32_t* dev_status,
               void* stream) {
  int st0 = fgmm::check_cfg(cfg, n);
  if (st0) return st0;
  if (!offsets || capacity_words < 0) return GMM_EINVAL;
  if (n > 0 && (!symbols || !w || !mu || !sg)) return GMM_EINVAL;
  if (capacity_words > 0 && !bitstream) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int64_t need = fgmm::encode_ws_bytes(n, cfg->num_streams);
  char* wsp = (char*)ws;
  bool own = false;
  if (!wsp) {
    if (hipMallocAsync((void**)&wsp, need, st) != hipSuccess) return GMM_ENOMEM;
    own = true;
  } else if (ws_bytes < need) {
    return GMM_EINVAL;
  }
  const bool fast = fgmm::use_fast_recip(st);
  int r = fgmm::encode_launch(cfg, n, symbols, w, mu, sg, bitstream, capacity_words, offsets,
                              wsp, fast, st, nullptr, 0, dev_status);
  if (r == GMM_OK) r = fgmm::finish((uint32_t*)wsp, dev_status, st);
  if (own) (void)hipFreeAsync(wsp, st);
  return r;
}

int gmm_decode(const gmm_cfg* cfg, int64_t n, const uint16_t* bitstream, int64_t total_words,
               const int64_t* offsets, const float* w, const float* mu, const float* sg,
               int32_t* symbols, const gmm_bracket* bracket, gmm_decode_stats* stats, void* ws,
               int64_t ws_bytes, int32_t* dev_status, void* stream) {
  int st0 = fgmm::check_cfg(cfg, n);
  if (st0) return st0;
  if (!offsets || total_words < 0) return GMM_EINVAL;
  if (n > 0 && (!symbols || !w || !mu || !sg)) return GMM_EINVAL;
  if (total_words > 0 && !bitstream) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  char* wsp = (char*)ws;
  bool own = false;
  if (!wsp) {
    if (hipMallocAsync((void**)&wsp, 256, st) != hipSuccess) return GMM_ENOMEM;
    own = true;
  } else if (ws_bytes < 256) {
    return GMM_EINVAL;
  }
  if (bracket && (cfg->cdf_kind >= 2 || cfg->param_kind != 0)) {
    if (own) (void)hipFreeAsync(wsp, st);
    return GMM_EINVAL;
  }
  const bool fast = fgmm::use_fast_recip(st);
  int r;
  if (bracket) {
    r = fgmm::decode_bracket_launch(cfg, n, bitstream, total_words, offsets, w, mu, sg, symbols,
                                    bracket, stats, (uint32_t*)wsp, fast, st, g_lanes_override,
                                    dev_status);
  } else {
    r = fgmm::decode_launch(cfg, n, bitstream, total_words, offsets, w, mu, sg, symbols,
                            (uint32_t*)wsp, fast, st, g_lanes_override, nullptr, 0, dev_status);
  }
  if (r == GMM_OK) r = fgmm::finish((uint32_t*)wsp, dev_status, st);
  if (own) (void)hipFreeAsync(wsp, st);
  return r;
}

int gmm_encode_subset(const gmm_cfg* cfg, int64_t n_total, const int32_t* idx, int64_t m,
                      const int32_t* symbols, const float* w, const float* mu, const float* sg,
                      uint16_t* bitstream, int64_t capacity_words, int64_t* offsets, void* ws,
                      int64_t ws_bytes, int32_t* dev_status, void* stream) {
  int st0 = fgmm::check_cfg(cfg, m);
  if (st0) return st0;
  if (cfg->cdf_kind >= 2) return GMM_EINVAL;  // subset passes build the plain kinds only
  if (n_total < 0 || m > n_total || (m > 0 && (!idx || n_total > INT32_MAX))) return GMM_EINVAL;
  if (!offsets || capacity_words < 0) return GMM_EINVAL;
  if (m > 0 && (!symbols || !w || !mu || !sg)) return GMM_EINVAL;
  if (capacity_words > 0 && !bitstream) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int64_t need = fgmm::encode_ws_bytes(m, cfg->num_streams);
  char* wsp = (char*)ws;
  bool own = false;
  if (!wsp) {
    if (hipMallocAsync((void**)&wsp, need, st) != hipSuccess) return GMM_ENOMEM;
    own = true;
  } else if (ws_bytes < need) {
    return GMM_EINVAL;
  }
  const bool fast = fgmm::use_fast_recip(st);
  int r = fgmm::encode_launch(cfg, m, symbols, w, mu, sg, bitstream, capacity_words, offsets,
                              wsp, fast, st, idx, n_total, dev_status);
  if (r == GMM_OK) r = fgmm::finish((uint32_t*)wsp, dev_status, st);
  if (own) (void)hipFreeAsync(wsp, st);
  return r;
}

int gmm_decode_subset(const gmm_cfg* cfg, int64_t n_total, const int32_t* idx, int64_t m,
                      const uint16_t* bitstream, int64_t total_words, const int64_t* offsets,
                      const float* w, const float* mu, const float* sg, int32_t* symbols,
                      void* ws, int64_t ws_bytes, int32_t* dev_status, void* stream) {
  int st0 = fgmm::check_cfg(cfg, m);
  if (st0) return st0;
  if (cfg->cdf_kind >= 2) return GMM_EINVAL;  // subset passes build the plain kinds only
  if (n_total < 0 || m > n_total || (m > 0 && (!idx || n_total > INT32_MAX))) return GMM_EINVAL;
  if (!offsets || total_words < 0) return GMM_EINVAL;
  if (m > 0 && (!symbols || !w || !mu || !sg)) return GMM_EINVAL;
  if (total_words > 0 && !bitstream) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  char* wsp = (char*)ws;
  bool own = false;
  if (!wsp) {
    if (hipMallocAsync((void**)&wsp, 256, st) != hipSuccess) return GMM_ENOMEM;
    own = true;
  } else if (ws_bytes < 256) {
    return GMM_EINVAL;
  }
  const bool fast = fgmm::use_fast_recip(st);
  int r = fgmm::decode_launch(cfg, m, bitstream, total_words, offsets, w, mu, sg, symbols,
                              (uint32_t*)wsp, fast, st, g_lanes_override, idx, n_total,
                              dev_status);
  if (r == GMM_OK) r = fgmm::finish((uint32_t*)wsp, dev_status, st);
  if (own) (void)hipFreeAsync(wsp, st);
  return r;
}

int gmm_params_from_raw(int32_t K, int64_t n, const float* logits, const float* log_scales,
                        float* weights, float* scales, void* stream) {
  if (K < 1 || K > fgmm::kMaxK || n < 0) return GMM_EINVAL;
  if (n > 0 && (!logits || !log_scales || !weights || !scales)) return GMM_EINVAL;
  if (n == 0) return GMM_OK;
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (K) {
#define FG_RAW(KK) \
  case KK: hipLaunchKernelGGL(k_params_from_raw<KK>, grid, block, 0, st, n, logits, log_scales, weights, scales); break;
    FG_RAW(1) FG_RAW(2) FG_RAW(3) FG_RAW(4) FG_RAW(5) FG_RAW(6) FG_RAW(7) FG_RAW(8)
#undef FG_RAW
  }
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

int gmm_fast_recip_mismatches(uint64_t* count, void* stream) {
  if (!count) return GMM_EINVAL;
  unsigned long long c = 0;
  int r = fgmm::fast_recip_mismatches(&c, (hipStream_t)stream, nullptr);
  *count = c;
  return r;
}

}  // extern "C"
