// Templated coder kernels shared by the translation units that instantiate
// them: the plain path for the A&S and logistic CDFs (gmm_coder.hip) and the
// Polya / binary64-reference kinds of the Table II comparison
// (gmm_ablation.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gmm_device.h"
#include "gmm_stream.h"

// (global namespace, so that profiles name the kernels briefly)

template <int K, int kKind, bool kFast>
__global__ void k_cdf_table(fgmm::QCfg q, int64_t n, const float* __restrict__ w,
                            const float* __restrict__ mu, const float* __restrict__ sg,
                            uint32_t* __restrict__ table) {
  using namespace fgmm;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cols = (int64_t)q.N + 1;
  if (t >= n * cols) return;
  const int64_t i = t / cols;
  const int32_t j = (int32_t)(t - i * cols);
  float rw[K], rm[K], rs[K];
  load_raw<K>(w, mu, sg, n, i, rw, rm, rs);
  const Elem<K> e = make_elem<K, kFast, kKind>(q, rw, rm, rs);
  table[t] = cdf_at<K, kKind, kFast>(e, q, j);
}

template <int K, int kKind, bool kFast>
__global__ void k_inverse(fgmm::QCfg q, int rounds, int64_t n, const float* __restrict__ w,
                          const float* __restrict__ mu, const float* __restrict__ sg,
                          const uint32_t* __restrict__ slot, int32_t* __restrict__ jout,
                          uint32_t* status) {
  using namespace fgmm;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float rw[K], rm[K], rs[K];
  load_raw<K>(w, mu, sg, n, i, rw, rm, rs);
  const Elem<K> e = make_elem<K, kFast, kKind>(q, rw, rm, rs);
  uint32_t s = slot[i];
  if (s >= q.M) {
    atomicOr(status, kStInval);
    s = q.M - 1;
  }
  uint32_t cl, ch;
  jout[i] = search_bs<K, kKind, kFast>(e, q, rounds, free_rounds(rounds, q.N), s, cl, ch);
}

// Encode phase 1: one thread per element (per pass position with kGather:
// element idx[i] of a latent of n_total elements). An out-of-range symbol
// gives the word 0, which the rANS pass reports as GMM_ERANGE. With clear,
// the first workgroup also zeroes clear[0 .. nclear) (the call's status
// words and the rANS pass's look-back slots, used only by the kernels
// after this one), which saves a launch.
template <int K, int kKind, bool kFast, bool kGather = false, bool kBuf = false>
__global__ void k_enc_cdf(fgmm::QCfg q, int64_t n, const int32_t* __restrict__ sym,
                          const float* __restrict__ w, const float* __restrict__ mu,
                          const float* __restrict__ sg, uint32_t* __restrict__ cf,
                          uint32_t* status, const int32_t* __restrict__ idx = nullptr,
                          int64_t n_total = 0, uint32_t* clear = nullptr, int64_t nclear = 0) {
  using namespace fgmm;
  set_wave_priority(q.prio);
  if (clear && blockIdx.x == 0)
    for (int64_t k = threadIdx.x; k < nclear; k += blockDim.x) clear[k] = 0u;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (kGather)
    cf[i] = enc_cdf_elem<K, kKind, kFast, true>(q, n_total, gather_index(idx, i, n_total), sym,
                                                 w, mu, sg, status);
  else
    cf[i] = enc_cdf_elem<K, kKind, kFast, true, kBuf>(q, n, i, sym, w, mu, sg, status);
}

// Decode with L lanes per stream (L = 1: one lane per stream and a binary
// search; L > 1: an (L+1)-ary search, ceil(log_{L+1} N) rounds). status[0]
// collects the status bits, status[1] counts finished workgroups (both
// zeroed before the launch); the last workgroup writes the call's status
// code to dev_status when given.
template <int K, int kKind, bool kFast, int L, bool kGather = false, bool kBuf = false>
__global__ void __launch_bounds__(256)
    k_decode(fgmm::QCfg q, int P, int rounds, int64_t n, int64_t S, const uint16_t* __restrict__ bs,
             int64_t total_words, const int64_t* __restrict__ offsets,
             const float* __restrict__ w, const float* __restrict__ mu,
             const float* __restrict__ sg, int32_t* __restrict__ sym, uint32_t* status,
             int32_t* dev_status, const int32_t* __restrict__ idx = nullptr,
             int64_t n_total = 0) {
  using namespace fgmm;
  set_wave_priority(q.prio);
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = gt / L;
  const int g = (int)(gt % L);
  // groups never straddle the S boundary (S * L lanes, L divides 64)
  if (s < S) {
    const bool bad = decode_stream<K, kKind, kFast, L, kGather, L == 1, kBuf, kBuf ? 4 : 3>(
        q, P, rounds, n, S, s, g, bs, total_words, offsets, w, mu, sg, sym, idx, n_total);
    if (bad && g == 0) atomicOr(status, kStCorrupt);
  }
  grid_finish_status(status, dev_status);
}

