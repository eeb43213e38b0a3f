// Allocation-free encode (gmm_encode_noalloc): gmm_encode with its
// workspace in a static device array, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation). The kernels are gmm_encode's; only
// where the workspace lives differs.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>

#include "../../include/flashgmm.h"
#include "gmm_host.h"

namespace {

// The workspace of every gmm_encode_noalloc call on a device: each device
// holds its own copy of this array until the process ends, and successive
// calls reuse it (encode_launch clears the status words it reads before any
// other use; every other part is written before it is read). In host code
// the name is only a stand-in: the device address comes from
// hipGetSymbolAddress, resolved once per device below.
static __device__ __align__(256) unsigned char scratch[GMM_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64];  // device address of scratch on each device (null: not resolved)

// Device address of this device's scratch, resolved at the first call on
// the device (with the device current).
int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return GMM_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GMM_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GMM_OK;
}

}  // namespace

extern "C" int gmm_encode_noalloc(const gmm_cfg* cfg, int64_t n, const int32_t* symbols,
                                  const float* w, const float* mu, const float* sg,
                                  uint16_t* bitstream, int64_t capacity_words, int64_t* offsets,
                                  int32_t* dev_status, void* stream) {
  int st0 = fgmm::check_cfg(cfg, n);
  if (st0) return st0;
  if (!offsets || capacity_words < 0) return GMM_EINVAL;
  if (n > 0 && (!symbols || !w || !mu || !sg)) return GMM_EINVAL;
  if (capacity_words > 0 && !bitstream) return GMM_EINVAL;
  if (fgmm::encode_ws_bytes(n, cfg->num_streams) > (int64_t)GMM_NOALLOC_SCRATCH_BYTES)
    return GMM_E2BIG;
  void* ws = nullptr;
  int r = scratch_address(&ws);
  if (r) return r;
  hipStream_t st = (hipStream_t)stream;
  // the once-per-device check of the fused reciprocal counts its mismatches
  // in the array's first words (before this call's encode uses them)
  const bool fast = fgmm::use_fast_recip(st, ws);
  r = fgmm::encode_launch(cfg, n, symbols, w, mu, sg, bitstream, capacity_words, offsets,
                          (char*)ws, fast, st, nullptr, 0, dev_status);
  if (r == GMM_OK) r = fgmm::finish((uint32_t*)ws, dev_status, st);
  return r;
}
