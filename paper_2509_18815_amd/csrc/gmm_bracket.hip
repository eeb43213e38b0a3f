// Learned search bracket for decode: model loading, the single-latent
// decode kernel and a prediction diagnostic (device code in
// gmm_bracket_dev.h; not part of the paper's method).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "../../include/flashgmm.h"
#include "gmm_device.h"
#include "gmm_host.h"
#include "gmm_mlp.h"
#include "gmm_stream.h"
#include "gmm_bracket_dev.h"

using namespace fgmm;

namespace {

uint16_t host_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  u = u + 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Row of the 32x32 accumulator held in register r of a lane in half hh.
inline int acc_row(int r, int hh) { return 8 * (r / 4) + 4 * hh + (r % 4); }

// Physical hidden unit feeding logical input q (0..15) of a layer-2 k block:
// the accumulator row order of layer 1 re-read in B-operand order.
inline int phys_of_logical(int q) {
  const int hh = q / 8, t = q % 8;
  return 8 * (t / 4) + 4 * hh + (t % 4);
}

// Physical hidden unit feeding logical input q (0..31) of k block kb of
// layer 2 in the group form: the layer-1 accumulator rows of a lane in
// 16x16 tiles 2 kb (inputs 0..3 of its group of eight) and 2 kb + 1 (4..7).
inline int phys16(int kb, int q) {
  const int kh = q / 8, e = q % 8;
  return 32 * kb + (e < 4 ? 4 * kh + e : 16 + 4 * kh + (e - 4));
}

// Zeroes the status bits and the workgroup counter.
__global__ void k_fill_u32_bracket(uint32_t* p) {
  if (threadIdx.x < 2 && blockIdx.x == 0) p[threadIdx.x] = 0u;
}

template <int K, int kKind, bool kFast>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
    k_decode_bracket(QCfg q, int P, int64_t n, int64_t S, const uint16_t* __restrict__ bs,
                     int64_t total_words, const int64_t* __restrict__ offsets,
                     const float* __restrict__ w, const float* __restrict__ mu,
                     const float* __restrict__ sg, int32_t* __restrict__ sym, uint32_t* status,
                     const BracketDev* __restrict__ br, unsigned long long* stats,
                     int32_t* dev_status) {
  set_wave_priority(q.prio);
  __shared__ BracketLds lds;
  LaneModel model;
  load_lane_model(br, model, lds);
  unsigned long long cnt[4] = {0, 0, 0, 0};
  bracket_decode_wave<K, kKind, kFast>(q, P, n, S, (int64_t)blockIdx.x * 64, bs, total_words,
                                       offsets, w, mu, sg, sym, status, br, model, lds, cnt);
  bracket_flush_stats(cnt, stats);
  grid_finish_status(status, dev_status);
}

// Group form: LG = 16 or 8 lanes per stream, 64 / LG streams per wavefront.
template <int K, int kKind, bool kFast, int LG, bool kBuf = false>
__global__ void __launch_bounds__(256)
    k_decode_bracket_group(QCfg q, int P, int64_t n, int64_t S, const uint16_t* __restrict__ bs,
                           int64_t total_words, const int64_t* __restrict__ offsets,
                           const float* __restrict__ w, const float* __restrict__ mu,
                           const float* __restrict__ sg, int32_t* __restrict__ sym,
                           uint32_t* status, const BracketDev* __restrict__ br,
                           unsigned long long* stats, int32_t* dev_status) {
  set_wave_priority(q.prio);
  const int64_t s0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64 * (64 / LG);
  if (s0 < S) {  // whole wavefronts
    GroupModel gm;
    load_group_model(br, gm);
    unsigned long long cnt[4] = {0, 0, 0, 0};
    bracket_group_decode<K, kKind, kFast, LG, kBuf>(q, P, n, S, s0, bs, total_words, offsets, w,
                                                    mu, sg, sym, status, br, gm, cnt);
    bracket_flush_stats(cnt, stats);
  }
  grid_finish_status(status, dev_status);
}

template <int K>
__global__ void __launch_bounds__(64)
    k_bracket_predict(int64_t n, int P, const float* __restrict__ w, const float* __restrict__ mu,
                      const float* __restrict__ sg, const uint32_t* __restrict__ slot,
                      const BracketDev* __restrict__ br, float* __restrict__ pred) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  __shared__ BracketLds lds;
  LaneModel model;
  load_lane_model(br, model, lds);
  float rw[K], rm[K], rs[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    rw[k] = 0.0f;
    rm[k] = 0.0f;
    rs[k] = 1.0f;
  }
  uint32_t sl = 0;
  if (i < n) {
    load_raw<K>(w, mu, sg, n, i, rw, rm, rs);
    sl = slot[i];
  }
  float feat[16];
  lane_features<K>(br, rw, rm, rs, sl, 1.0f / (float)(1u << P), feat);
  const float pv = mlp_wave(br, model, lds, feat);
  if (i < n) pred[i] = pv;
}

}  // namespace

namespace fgmm {

int decode_bracket_launch(const gmm_cfg* cfg, int64_t n, const uint16_t* bs, int64_t total_words,
                          const int64_t* offsets, const float* w, const float* mu,
                          const float* sg, int32_t* symbols, const gmm_bracket* br,
                          gmm_decode_stats* stats, uint32_t* status, bool fast, hipStream_t st,
                          int lanes, int32_t* dev_status) {
  if (!br || br->K != cfg->K) return GMM_EINVAL;
  const int64_t S = cfg->num_streams;
  const QCfg q = make_qcfg(cfg);
  hipLaunchKernelGGL(k_fill_u32_bracket, dim3(1), dim3(64), 0, st, status);
  // the plain decode's choice (4,096 streams, N = 511: the 8-lane group
  // form, 124.8-126.3 us on the 320x48x32 latent against 132.9-133.1 us
  // for 16 lanes and 130.1-130.5 us for the plain 8-lane search)
  const int L = plain_decode_lanes(cfg, lanes);
  const bool buf = buffer_offsets_fit(cfg->K, n, S, total_words);
  dispatch(cfg->K, cfg->cdf_kind, fast, [&](auto Kc, auto kc, auto fc) {
    constexpr int K_ = decltype(Kc)::value;
    if constexpr (K_ <= 5) {
      constexpr int KI = decltype(kc)::value;
      constexpr bool F = decltype(fc)::value;
#define FG_GRP(LG, BUF)                                                                      \
  hipLaunchKernelGGL((k_decode_bracket_group<K_, KI, F, LG, BUF>),                          \
                     dim3((unsigned)((S + 256 / LG - 1) / (256 / LG))), dim3(256),           \
                     0, st, q, cfg->precision, n, S, bs, total_words, offsets, w, mu, sg,    \
                     symbols, status, br->dev, (unsigned long long*)stats, dev_status)
      if (L >= 16 && buf)
        FG_GRP(16, true);
      else if (L >= 16)
        FG_GRP(16, false);
      else if (L == 8 && buf)
        FG_GRP(8, true);
      else if (L == 8)
        FG_GRP(8, false);
#undef FG_GRP
      else
        hipLaunchKernelGGL((k_decode_bracket<K_, decltype(kc)::value, decltype(fc)::value>),
                           dim3((unsigned)((S + 63) / 64)), dim3(64), 0, st, q, cfg->precision,
                           n, S, bs, total_words, offsets, w, mu, sg, symbols, status, br->dev,
                           (unsigned long long*)stats, dev_status);
    }
  });
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

}  // namespace fgmm

extern "C" {

int gmm_bracket_create(const gmm_bracket_desc* d, gmm_bracket** out) {
  if (!d || !out || d->K < 1 || d->K > 5 || !d->params || !d->in_mean || !d->in_std ||
      d->radius < 0 || d->radius > 64 || !(d->out_std > 0.0f))
    return GMM_EINVAL;
  *out = nullptr;
  const int K = d->K, D = 3 * K + 1;
  const float* W1 = d->params;
  const float* b1 = W1 + kMlpH * D;
  const float* W2 = b1 + kMlpH;
  const float* b2 = W2 + kMlpH * kMlpH;
  const float* w3 = b2 + kMlpH;
  BracketDev h;
  memset(&h, 0, sizeof(h));
  auto pack = [](uint32_t* dst, const float* v8) {
    for (int j = 0; j < 4; ++j)
      dst[j] = (uint32_t)host_bf16(v8[2 * j]) | ((uint32_t)host_bf16(v8[2 * j + 1]) << 16);
  };
  for (int l = 0; l < 64; ++l) {
    const int i = l % 32, hh = l / 32;
    for (int mb = 0; mb < 2; ++mb) {
      float v[8];
      for (int e = 0; e < 8; ++e) {
        const int k = 8 * hh + e;
        v[e] = (k < D) ? W1[(32 * mb + i) * D + k] : 0.0f;
      }
      pack(h.wa1[l][mb], v);
      for (int kb = 0; kb < 4; ++kb) {
        for (int e = 0; e < 8; ++e) {
          const int src = 16 * kb + phys_of_logical(8 * hh + e);
          v[e] = W2[(32 * mb + i) * kMlpH + src];
        }
        pack(h.wa2[l][mb][kb], v);
      }
    }
  }
  // group form (16x16x32 tiles): layer 1 takes raw inputs, so the input
  // normalisation (x - mean) / std and the scalings of the log-scale inputs
  // (ln s = -ln 2 log2(1 / s)) are folded into W1 and the bias, in binary64
  std::vector<double> w1f((size_t)kMlpH * 17, 0.0);
  for (int r = 0; r < kMlpH; ++r) {
    double bias = b1[r];
    for (int k = 0; k < D; ++k) {
      const double inv = (d->in_std[k] > 0.0f) ? 1.0 / (double)d->in_std[k] : 0.0;
      const double a = (k >= 2 * K && k < 3 * K) ? -M_LN2 : 1.0;
      w1f[(size_t)r * 17 + k] = (double)W1[r * D + k] * inv * a;
      bias -= (double)W1[r * D + k] * inv * (double)d->in_mean[k];
    }
    w1f[(size_t)r * 17 + 16] = bias;
  }
  for (int l = 0; l < 64; ++l) {
    const int i = l % 16, kh = l / 16;
    for (int t = 0; t < 4; ++t) {
      const int row = 16 * t + i;
      float v[8];
      for (int e = 0; e < 8; ++e) {
        const int k = 8 * kh + e;
        v[e] = (k <= 16) ? (float)w1f[(size_t)row * 17 + k] : 0.0f;
      }
      pack(h.ga1[l][t], v);
      for (int kb = 0; kb < 2; ++kb) {
        for (int e = 0; e < 8; ++e) v[e] = W2[row * kMlpH + phys16(kb, 8 * kh + e)];
        pack(h.ga2[l][t][kb], v);
      }
      for (int r = 0; r < 4; ++r) h.gb2[l][4 * t + r] = b2[16 * t + 4 * kh + r];
    }
    for (int kb = 0; kb < 2; ++kb) {
      float v[8];
      for (int e = 0; e < 8; ++e) v[e] = w3[phys16(kb, 8 * kh + e)];
      pack(h.ga3[l][kb], v);
    }
  }
  for (int hh = 0; hh < 2; ++hh)
    for (int mb = 0; mb < 2; ++mb)
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * mb + acc_row(r, hh);
        h.b1v[hh][16 * mb + r] = b1[row];
        h.b2v[hh][16 * mb + r] = b2[row];
        h.w3v[hh][16 * mb + r] = w3[row];
      }
  h.b3 = w3[kMlpH];
  h.out_mean = d->out_mean;
  h.out_std = d->out_std;
  for (int k = 0; k < 16; ++k) {
    h.in_mean[k] = (k < D) ? d->in_mean[k] : 0.0f;
    h.in_inv_std[k] = (k < D && d->in_std[k] > 0.0f) ? 1.0f / d->in_std[k] : 0.0f;
  }
  h.K = K;
  h.D = D;
  h.radius = d->radius;
  gmm_bracket* br = new gmm_bracket();
  br->K = K;
  br->D = D;
  br->radius = d->radius;
  if (hipMalloc((void**)&br->dev, sizeof(BracketDev)) != hipSuccess) {
    delete br;
    return GMM_ENOMEM;
  }
  if (hipMemcpy(br->dev, &h, sizeof(BracketDev), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(br->dev);
    delete br;
    return GMM_EDEVICE;
  }
  *out = br;
  return GMM_OK;
}

int gmm_bracket_destroy(gmm_bracket* br) {
  if (!br) return GMM_OK;
  (void)hipDeviceSynchronize();
  if (br->dev) (void)hipFree(br->dev);
  delete br;
  return GMM_OK;
}

int gmm_bracket_predict(const gmm_bracket* br, int32_t precision, int64_t n, const float* w,
                        const float* mu, const float* sg, const uint32_t* slot, float* pred,
                        void* stream) {
  if (!br || n < 0 || precision < 2 || precision > 16) return GMM_EINVAL;
  if (n == 0) return GMM_OK;
  if (!w || !mu || !sg || !slot || !pred) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const dim3 g((unsigned)((n + 63) / 64)), b(64);
  switch (br->K) {
    case 1: hipLaunchKernelGGL(k_bracket_predict<1>, g, b, 0, st, n, precision, w, mu, sg, slot,
                               br->dev, pred); break;
    case 2: hipLaunchKernelGGL(k_bracket_predict<2>, g, b, 0, st, n, precision, w, mu, sg, slot,
                               br->dev, pred); break;
    case 3: hipLaunchKernelGGL(k_bracket_predict<3>, g, b, 0, st, n, precision, w, mu, sg, slot,
                               br->dev, pred); break;
    case 4: hipLaunchKernelGGL(k_bracket_predict<4>, g, b, 0, st, n, precision, w, mu, sg, slot,
                               br->dev, pred); break;
    default: hipLaunchKernelGGL(k_bracket_predict<5>, g, b, 0, st, n, precision, w, mu, sg, slot,
                                br->dev, pred); break;
  }
  if (hipGetLastError() != hipSuccess) return GMM_EDEVICE;
  return hipStreamSynchronize(st) == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

}  // extern "C"
