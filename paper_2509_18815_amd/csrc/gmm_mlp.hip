// Training kernels of the search-bracket MLP (not part of the paper's
// method: the network only seeds the decoder's search, whose result is
// verified against the exact integer CDF).
//
//   k_mlp_features  per element: normalised features, optionally rounded
//                   to bfloat16 (what the decode-fused inference sees)
//   k_mlp_fwdbwd    64 samples per workgroup: forward, Huber loss and the
//                   backward pass, per-workgroup partial gradient sums
//   k_mlp_reduce    fixed-order sum of the partials (deterministic)
//   k_mlp_forward   one thread per sample (evaluation)
//   k_mlp_adam      Adam on the float32 master weights, writing the
//                   bfloat16-rounded copy used by the forward pass
// Weights and activations are held in binary32; with round_act the hidden
// activations after the first layer are rounded to bfloat16 as the fused
// inference's matrix cores see them (the gradient passes straight through).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/flashgmm.h"
#include "gmm_host.h"
#include "gmm_mlp.h"

using namespace fgmm;

namespace {

constexpr int kTS = 64;   // samples per workgroup
constexpr int kMT = 256;  // threads per workgroup

template <int K>
__global__ void k_mlp_features(int64_t n, const float* __restrict__ w, const float* __restrict__ mu,
                               const float* __restrict__ sg, const uint32_t* __restrict__ slot,
                               float inv_m, const float* __restrict__ mean,
                               const float* __restrict__ inv_std, int round_bf16,
                               float* __restrict__ X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  constexpr int D = 3 * K + 1;
  float rw[K], rm[K], rs[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    rw[k] = w[k * n + i];
    rm[k] = mu[k * n + i];
    rs[k] = sg[k * n + i];
  }
  const uint32_t s = slot[i];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    float v = mlp_raw_feature<K>(d, rw, rm, rs, s, inv_m);
    if (mean) v = (v - mean[d]) * inv_std[d];
    X[i * D + d] = round_bf16 ? bf16_round(v) : v;
  }
}

// Partial row layout per workgroup: the P parameter gradients, then the loss.
__global__ void __launch_bounds__(kMT)
    k_mlp_fwdbwd(int D, int64_t n, const float* __restrict__ X, const float* __restrict__ y,
                 const float* __restrict__ prm, float delta, int round_act,
                 float* __restrict__ part) {
  __shared__ float sW1[kMlpH * kMlpMaxD], sb1[kMlpH], sW2[kMlpH * kMlpH], sb2[kMlpH], sw3[kMlpH];
  __shared__ float sX[kTS * kMlpMaxD];
  __shared__ float sA1[kTS * kMlpH];  // h1, then d1
  __shared__ float sA2[kTS * kMlpH];  // h2, then d2
  __shared__ float sG[kTS];           // dLoss/dout
  __shared__ float sL[kTS];           // per-sample loss
  const int P = mlp_num_params(D);
  const int tid = threadIdx.x;
  const float* pW1 = prm;
  const float* pb1 = pW1 + kMlpH * D;
  const float* pW2 = pb1 + kMlpH;
  const float* pb2 = pW2 + kMlpH * kMlpH;
  const float* pw3 = pb2 + kMlpH;
  const float b3 = pw3[kMlpH];
  for (int i = tid; i < kMlpH * D; i += kMT) sW1[i] = pW1[i];
  for (int i = tid; i < kMlpH * kMlpH; i += kMT) sW2[i] = pW2[i];
  if (tid < kMlpH) {
    sb1[tid] = pb1[tid];
    sb2[tid] = pb2[tid];
    sw3[tid] = pw3[tid];
  }
  const int64_t base = (int64_t)blockIdx.x * kTS;
  const int ts = (int)((n - base) < kTS ? (n - base) : kTS);
  for (int i = tid; i < kTS * D; i += kMT) {
    const int s = i / D, d = i % D;
    sX[s * kMlpMaxD + d] = (s < ts) ? X[(base + s) * D + d] : 0.0f;
  }
  __syncthreads();
  for (int o = tid; o < kTS * kMlpH; o += kMT) {
    const int s = o / kMlpH, h = o % kMlpH;
    float a = sb1[h];
    for (int d = 0; d < D; ++d) a = fmaf(sW1[h * D + d], sX[s * kMlpMaxD + d], a);
    a = fmaxf(a, 0.0f);
    sA1[o] = round_act ? bf16_round(a) : a;
  }
  __syncthreads();
  for (int o = tid; o < kTS * kMlpH; o += kMT) {
    const int s = o / kMlpH, h = o % kMlpH;
    float a = sb2[h];
    for (int k = 0; k < kMlpH; ++k) a = fmaf(sW2[h * kMlpH + k], sA1[s * kMlpH + k], a);
    sA2[o] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  if (tid < kTS) {
    const int s = tid;
    float out = b3;
    for (int h = 0; h < kMlpH; ++h) out = fmaf(sw3[h], sA2[s * kMlpH + h], out);
    float g = 0.0f, l = 0.0f;
    if (s < ts) {
      const float r = out - y[base + s];
      const float ar = fabsf(r);
      l = (ar <= delta) ? 0.5f * r * r : delta * (ar - 0.5f * delta);
      g = (ar <= delta) ? r : copysignf(delta, r);
    }
    sG[s] = g;
    sL[s] = l;
  }
  __syncthreads();
  float* row = part + (int64_t)blockIdx.x * (P + 1);
  float* gW1 = row;
  float* gb1 = gW1 + kMlpH * D;
  float* gW2 = gb1 + kMlpH;
  float* gb2 = gW2 + kMlpH * kMlpH;
  float* gw3 = gb2 + kMlpH;
  if (tid < kMlpH) {  // w3 gradient
    float a = 0.0f;
    for (int s = 0; s < kTS; ++s) a = fmaf(sG[s], sA2[s * kMlpH + tid], a);
    gw3[tid] = a;
  } else if (tid == kMlpH) {
    float a = 0.0f, l = 0.0f;
    for (int s = 0; s < kTS; ++s) {
      a += sG[s];
      l += sL[s];
    }
    gw3[kMlpH] = a;  // b3
    row[P] = l;
  }
  __syncthreads();
  for (int o = tid; o < kTS * kMlpH; o += kMT) {  // d2
    const int s = o / kMlpH, h = o % kMlpH;
    sA2[o] = (sA2[o] > 0.0f) ? sG[s] * sw3[h] : 0.0f;
  }
  __syncthreads();
  for (int o = tid; o < kMlpH * kMlpH; o += kMT) {  // W2 gradient
    const int h = o / kMlpH, k = o % kMlpH;
    float a = 0.0f;
    for (int s = 0; s < kTS; ++s) a = fmaf(sA2[s * kMlpH + h], sA1[s * kMlpH + k], a);
    gW2[o] = a;
  }
  if (tid < kMlpH) {
    float a = 0.0f;
    for (int s = 0; s < kTS; ++s) a += sA2[s * kMlpH + tid];
    gb2[tid] = a;
  }
  __syncthreads();
  // d1 = (W2^T d2) masked by h1 > 0, written over h1 after every thread
  // has read h1 for the W2 gradient
  float d1v[kTS * kMlpH / kMT];
  for (int o = tid, q = 0; o < kTS * kMlpH; o += kMT, ++q) {
    const int s = o / kMlpH, k = o % kMlpH;
    float a = 0.0f;
    for (int h = 0; h < kMlpH; ++h) a = fmaf(sA2[s * kMlpH + h], sW2[h * kMlpH + k], a);
    d1v[q] = (sA1[o] > 0.0f) ? a : 0.0f;
  }
  __syncthreads();
  for (int o = tid, q = 0; o < kTS * kMlpH; o += kMT, ++q) sA1[o] = d1v[q];
  __syncthreads();
  for (int o = tid; o < kMlpH * D; o += kMT) {  // W1 gradient
    const int h = o / D, d = o % D;
    float a = 0.0f;
    for (int s = 0; s < kTS; ++s) a = fmaf(sA1[s * kMlpH + h], sX[s * kMlpMaxD + d], a);
    gW1[o] = a;
  }
  if (tid < kMlpH) {
    float a = 0.0f;
    for (int s = 0; s < kTS; ++s) a += sA1[s * kMlpH + tid];
    gb1[tid] = a;
  }
}

__global__ void k_mlp_reduce(int64_t nblk, int P1, const float* __restrict__ part,
                             float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P1) return;
  double a = 0.0;
  for (int64_t b = 0; b < nblk; ++b) a += (double)part[b * P1 + i];
  out[i] = (float)a;
}

__global__ void __launch_bounds__(256)
    k_mlp_forward(int D, int64_t n, const float* __restrict__ X, const float* __restrict__ prm,
                  int round_act, float* __restrict__ out) {
  __shared__ float sW1[kMlpH * kMlpMaxD], sb1[kMlpH], sW2[kMlpH * kMlpH], sb2[kMlpH], sw3[kMlpH];
  const int tid = threadIdx.x;
  const float* pW1 = prm;
  const float* pb1 = pW1 + kMlpH * D;
  const float* pW2 = pb1 + kMlpH;
  const float* pb2 = pW2 + kMlpH * kMlpH;
  const float* pw3 = pb2 + kMlpH;
  for (int i = tid; i < kMlpH * D; i += blockDim.x) sW1[i] = pW1[i];
  for (int i = tid; i < kMlpH * kMlpH; i += blockDim.x) sW2[i] = pW2[i];
  if (tid < kMlpH) {
    sb1[tid] = pb1[tid];
    sb2[tid] = pb2[tid];
    sw3[tid] = pw3[tid];
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
  if (i >= n) return;
  float x[kMlpMaxD];
  for (int d = 0; d < kMlpMaxD; ++d) x[d] = (d < D) ? X[i * D + d] : 0.0f;
  float h1[kMlpH];
  for (int h = 0; h < kMlpH; ++h) {
    float a = sb1[h];
    for (int d = 0; d < D; ++d) a = fmaf(sW1[h * D + d], x[d], a);
    a = fmaxf(a, 0.0f);
    h1[h] = round_act ? bf16_round(a) : a;
  }
  float o = pw3[kMlpH];
  for (int h = 0; h < kMlpH; ++h) {
    float a = sb2[h];
    for (int k = 0; k < kMlpH; ++k) a = fmaf(sW2[h * kMlpH + k], h1[k], a);
    o = fmaf(sw3[h], fmaxf(a, 0.0f), o);
  }
  out[i] = o;
}

__global__ void k_mlp_adam(int P, float* __restrict__ prm, const float* __restrict__ grad,
                           float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                           float b2, float eps, float c1, float c2, float gscale,
                           float* __restrict__ shadow) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float g = grad[i] * gscale;
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float p = prm[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  prm[i] = p;
  if (shadow) shadow[i] = bf16_round(p);
}

}  // namespace

extern "C" {

int gmm_mlp_num_params(int32_t D) {
  if (D < 1 || D > kMlpMaxD) return -1;
  return mlp_num_params(D);
}

int64_t gmm_mlp_workspace_bytes(int32_t D, int64_t n) {
  if (D < 1 || D > kMlpMaxD || n < 0) return -1;
  const int64_t nblk = (n + kTS - 1) / kTS;
  return (nblk > 0 ? nblk : 1) * (int64_t)(mlp_num_params(D) + 1) * 4;
}

int gmm_mlp_features(int32_t K, int64_t n, const float* w, const float* mu, const float* sg,
                     const uint32_t* slot, int32_t precision, const float* mean,
                     const float* inv_std, int32_t round_bf16, float* X, void* stream) {
  if (K < 1 || K > 5 || n < 0 || precision < 2 || precision > 16) return GMM_EINVAL;
  if (n == 0) return GMM_OK;
  if (!w || !mu || !sg || !slot || !X || (!mean) != (!inv_std)) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const float inv_m = 1.0f / (float)(1u << precision);
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  switch (K) {
    case 1: hipLaunchKernelGGL(k_mlp_features<1>, g, b, 0, st, n, w, mu, sg, slot, inv_m, mean,
                               inv_std, round_bf16, X); break;
    case 2: hipLaunchKernelGGL(k_mlp_features<2>, g, b, 0, st, n, w, mu, sg, slot, inv_m, mean,
                               inv_std, round_bf16, X); break;
    case 3: hipLaunchKernelGGL(k_mlp_features<3>, g, b, 0, st, n, w, mu, sg, slot, inv_m, mean,
                               inv_std, round_bf16, X); break;
    case 4: hipLaunchKernelGGL(k_mlp_features<4>, g, b, 0, st, n, w, mu, sg, slot, inv_m, mean,
                               inv_std, round_bf16, X); break;
    default: hipLaunchKernelGGL(k_mlp_features<5>, g, b, 0, st, n, w, mu, sg, slot, inv_m, mean,
                                inv_std, round_bf16, X); break;
  }
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

int gmm_mlp_loss_grad(int32_t D, int64_t n, const float* X, const float* y, const float* params,
                      float delta, int32_t round_act, float* grad_loss, void* ws,
                      int64_t ws_bytes, void* stream) {
  if (D < 1 || D > kMlpMaxD || n < 1 || !X || !y || !params || !grad_loss || !ws)
    return GMM_EINVAL;
  if (ws_bytes < gmm_mlp_workspace_bytes(D, n)) return GMM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int64_t nblk = (n + kTS - 1) / kTS;
  const int P1 = mlp_num_params(D) + 1;
  hipLaunchKernelGGL(k_mlp_fwdbwd, dim3((unsigned)nblk), dim3(kMT), 0, st, D, n, X, y, params,
                     delta, round_act, (float*)ws);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)((P1 + 255) / 256)), dim3(256), 0, st, nblk,
                     P1, (const float*)ws, grad_loss);
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

int gmm_mlp_forward(int32_t D, int64_t n, const float* X, const float* params, int32_t round_act,
                    float* out, void* stream) {
  if (D < 1 || D > kMlpMaxD || n < 0 || (n > 0 && (!X || !params || !out))) return GMM_EINVAL;
  if (n == 0) return GMM_OK;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, D, n, X, params, round_act, out);
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

int gmm_mlp_adam(int32_t P, float* params, const float* grad, float* m, float* v, float lr,
                 float beta1, float beta2, float eps, int32_t step, float grad_scale,
                 float* shadow, void* stream) {
  if (P < 1 || !params || !grad || !m || !v || step < 1) return GMM_EINVAL;
  const float c1 = 1.0f - powf(beta1, (float)step);
  const float c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((P + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, P, params, grad, m, v, lr, beta1, beta2, eps, c1, c2,
                     grad_scale, shadow);
  return hipGetLastError() == hipSuccess ? GMM_OK : GMM_EDEVICE;
}

}  // extern "C"
