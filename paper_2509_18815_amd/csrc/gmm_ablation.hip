// Kernels of the Gaussian-CDF kinds compared in the paper's Table II besides
// the plain path: Polya's approximation (binary32) and the binary64
// reference that stands in for an unapproximated erfc. They run the same
// coder kernels as A&S and logistic; only the CDF differs. Built in a
// translation unit of their own (decode with one lane per stream or with
// 16 lanes per stream, no subset passes, no plans).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

#include "gmm_host.h"
#include "gmm_kernels.h"

namespace fgmm {
namespace {

template <typename Fn>
void dispatch_ablation(int K, int kind, Fn&& fn) {
  auto by_kind = [&](auto Kc) {
    if (kind == 2)
      fn(Kc, std::integral_constant<int, 2>{});
    else
      fn(Kc, std::integral_constant<int, 3>{});
  };
  switch (K) {
    case 1: by_kind(std::integral_constant<int, 1>{}); break;
    case 2: by_kind(std::integral_constant<int, 2>{}); break;
    case 3: by_kind(std::integral_constant<int, 3>{}); break;
    case 4: by_kind(std::integral_constant<int, 4>{}); break;
    case 5: by_kind(std::integral_constant<int, 5>{}); break;
    case 6: by_kind(std::integral_constant<int, 6>{}); break;
    case 7: by_kind(std::integral_constant<int, 7>{}); break;
    default: by_kind(std::integral_constant<int, 8>{}); break;
  }
}

}  // namespace

void ablation_cdf_table(const QCfg& q, int K, int kind, int64_t n, const float* w,
                        const float* mu, const float* sg, uint32_t* table, hipStream_t st) {
  const int64_t total = n * ((int64_t)q.N + 1);
  dispatch_ablation(K, kind, [&](auto Kc, auto kc) {
    hipLaunchKernelGGL((k_cdf_table<decltype(Kc)::value, decltype(kc)::value, false>),
                       dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, q, n, w, mu, sg,
                       table);
  });
}

void ablation_inverse(const QCfg& q, int K, int kind, int rounds, int64_t n, const float* w,
                      const float* mu, const float* sg, const uint32_t* slot, int32_t* jout,
                      uint32_t* status, hipStream_t st) {
  dispatch_ablation(K, kind, [&](auto Kc, auto kc) {
    hipLaunchKernelGGL((k_inverse<decltype(Kc)::value, decltype(kc)::value, false>),
                       dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, q, rounds, n, w, mu,
                       sg, slot, jout, status);
  });
}

void ablation_enc_cdf(const QCfg& q, int K, int kind, int64_t n, const int32_t* sym,
                      const float* w, const float* mu, const float* sg, uint32_t* cf,
                      uint32_t* status, hipStream_t st) {
  dispatch_ablation(K, kind, [&](auto Kc, auto kc) {
    hipLaunchKernelGGL((k_enc_cdf<decltype(Kc)::value, decltype(kc)::value, false, false>),
                       dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, q, n, sym, w, mu, sg,
                       cf, status, nullptr, (int64_t)0);
  });
}

void ablation_decode(const QCfg& q, int K, int kind, int P, int rounds, int L, int64_t n,
                     int64_t S, const uint16_t* bs, int64_t total_words, const int64_t* offsets,
                     const float* w, const float* mu, const float* sg, int32_t* sym,
                     uint32_t* status, int32_t* dev_status, hipStream_t st) {
  // 256-thread workgroups: the four wavefronts of a workgroup land on the
  // four SIMDs of a CU, while single-wavefront workgroups were measured to
  // leave up to ~9% of the SIMDs with two wavefronts (and as many idle)
  // after other work, which stretched a one-wavefront-per-SIMD decode by
  // about 1.4x.
  const int blk = 256;
  const int64_t threads = S * L;
  const dim3 grid((unsigned)((threads + blk - 1) / blk)), block(blk);
  dispatch_ablation(K, kind, [&](auto Kc, auto kc) {
    constexpr int K_ = decltype(Kc)::value, KI = decltype(kc)::value;
    if (L == 1)
      hipLaunchKernelGGL((k_decode<K_, KI, false, 1, false>), grid, block, 0, st, q, P, rounds, n,
                         S, bs, total_words, offsets, w, mu, sg, sym, status, dev_status,
                         nullptr, (int64_t)0);
    else
      hipLaunchKernelGGL((k_decode<K_, KI, false, 16, false>), grid, block, 0, st, q, P, rounds,
                         n, S, bs, total_words, offsets, w, mu, sg, sym, status, dev_status,
                         nullptr, (int64_t)0);
  });
}

}  // namespace fgmm
