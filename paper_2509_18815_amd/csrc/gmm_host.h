// Host-side helpers shared by the translation units of libflashgmm.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/flashgmm.h"
#include "gmm_device.h"

namespace fgmm {

int check_cfg(const gmm_cfg* c, int64_t n);
QCfg make_qcfg(const gmm_cfg* c);
int search_rounds(int32_t N);
// Whether the fused reciprocal equals IEEE division on this device (checked
// once per device, exhaustively; counter: optional 8-byte device buffer for
// the check, else it allocates one on the stream).
bool use_fast_recip(hipStream_t st, void* counter = nullptr);
int fast_recip_mismatches(unsigned long long* count, hipStream_t st, void* counter);
int finish(uint32_t* bits, int32_t* dev_status, hipStream_t st);
int64_t encode_ws_bytes(int64_t n, int64_t S);
int encode_launch(const gmm_cfg* cfg, int64_t n, const int32_t* symbols, const float* w,
                  const float* mu, const float* sg, uint16_t* bitstream, int64_t capacity,
                  int64_t* offsets, char* ws, bool fast, hipStream_t st,
                  const int32_t* idx = nullptr, int64_t n_total = 0,
                  int32_t* dev_status = nullptr);
int decode_launch(const gmm_cfg* cfg, int64_t n, const uint16_t* bs, int64_t total_words,
                  const int64_t* offsets, const float* w, const float* mu, const float* sg,
                  int32_t* symbols, uint32_t* status, bool fast, hipStream_t st, int lanes,
                  const int32_t* idx = nullptr, int64_t n_total = 0,
                  int32_t* dev_status = nullptr);
int search_rounds_lps(int32_t N, int L);
int default_lanes_per_stream(int64_t S);
// Lanes per stream of a decode of cfg (lanes > 0: the caller's choice; else
// the automatic one: default_lanes_per_stream halved while the search needs
// no more rounds).
int plain_decode_lanes(const gmm_cfg* cfg, int lanes);
int decode_bracket_launch(const gmm_cfg* cfg, int64_t n, const uint16_t* bs, int64_t total_words,
                          const int64_t* offsets, const float* w, const float* mu,
                          const float* sg, int32_t* symbols, const gmm_bracket* bracket,
                          gmm_decode_stats* stats, uint32_t* status, bool fast, hipStream_t st,
                          int lanes, int32_t* dev_status);

// Launchers of the Polya (kind 2) and binary64-reference (kind 3) CDF
// kernels (gmm_ablation.hip); launch errors are left for hipGetLastError.
void ablation_cdf_table(const QCfg& q, int K, int kind, int64_t n, const float* w,
                        const float* mu, const float* sg, uint32_t* table, hipStream_t st);
void ablation_inverse(const QCfg& q, int K, int kind, int rounds, int64_t n, const float* w,
                      const float* mu, const float* sg, const uint32_t* slot, int32_t* jout,
                      uint32_t* status, hipStream_t st);
void ablation_enc_cdf(const QCfg& q, int K, int kind, int64_t n, const int32_t* sym,
                      const float* w, const float* mu, const float* sg, uint32_t* cf,
                      uint32_t* status, hipStream_t st);
void ablation_decode(const QCfg& q, int K, int kind, int P, int rounds, int L, int64_t n,
                     int64_t S, const uint16_t* bs, int64_t total_words, const int64_t* offsets,
                     const float* w, const float* mu, const float* sg, int32_t* sym,
                     uint32_t* status, int32_t* dev_status, hipStream_t st);

// Calls fn(integral_constant<K>, integral_constant<kind>, bool_constant<fast>)
// for the runtime (K, kind, fast) (the logistic kind has no division to
// replace, so its fast flag is always false).
template <int K, typename Fn>
void dispatch_kind(int kind, bool fast, Fn&& fn) {
  if (kind == 1)
    fn(std::integral_constant<int, K>{}, std::integral_constant<int, 1>{}, std::false_type{});
  else if (fast)
    fn(std::integral_constant<int, K>{}, std::integral_constant<int, 0>{}, std::true_type{});
  else
    fn(std::integral_constant<int, K>{}, std::integral_constant<int, 0>{}, std::false_type{});
}

template <typename Fn>
void dispatch(int K, int kind, bool fast, Fn&& fn) {
  switch (K) {
    case 1: dispatch_kind<1>(kind, fast, fn); break;
    case 2: dispatch_kind<2>(kind, fast, fn); break;
    case 3: dispatch_kind<3>(kind, fast, fn); break;
    case 4: dispatch_kind<4>(kind, fast, fn); break;
    case 5: dispatch_kind<5>(kind, fast, fn); break;
    case 6: dispatch_kind<6>(kind, fast, fn); break;
    case 7: dispatch_kind<7>(kind, fast, fn); break;
    default: dispatch_kind<8>(kind, fast, fn); break;
  }
}

}  // namespace fgmm
