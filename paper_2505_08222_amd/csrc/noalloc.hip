// Guarded learned inference without a caller workspace: the scratch the
// kernels need (MFMA-ready weight copies, the fallback counter and the
// fallback list) lives in one statically sized device array per GPU.
//
// The array's host-side name is only a stand-in: its device address is looked
// up once per device with hipGetSymbolAddress (that device current) and only
// that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "learned_internal.h"
#include "mi_lrauv.h"

extern "C" int mil_set_error(int code, const char *msg);  // abi.cpp

namespace {

constexpr int64_t kAlign = 256;
constexpr int64_t align_up(int64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// layout: BF16 weight copies (the FP32 size bounds them), counter, list
constexpr int64_t kPrepOff = 0;
constexpr int64_t kCountOff = align_up(kPrepOff + mil::kPrepBytes);
constexpr int64_t kListOff = align_up(kCountOff + 4);
constexpr int64_t kScratchBytes = align_up(kListOff + (int64_t)MIL_NOALLOC_MAX_WINDOWS * 4);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on first use).
int scratch_ptr(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return mil_set_error(MIL_EHIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return mil_set_error(MIL_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return mil_set_error(MIL_EHIP, "hipGetSymbolAddress of the scratch array failed");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return MIL_OK;
}

int num_cus_noalloc() {
  int dev = 0, n = 0;
  hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
    n = 256;
  return n;
}

}  // namespace

extern "C" {

int mlp_infer_noalloc(const float *d_win, int64_t N, int32_t W, const float *d_params,
                      const float *d_sigma, float k_sigma, int32_t gn_iters, float tau,
                      float *d_out, uint8_t *d_flag, void *stream) {
  if (N < 0 || W < 3 || 3 * W + 1 > mil::kIn)
    return mil_set_error(MIL_EINVAL, "need N >= 0, 3 <= W <= 21");
  if (N > MIL_NOALLOC_MAX_WINDOWS)
    return mil_set_error(MIL_EINVAL,
                         "N exceeds MIL_NOALLOC_MAX_WINDOWS, the no-allocation scratch "
                         "capacity; use mlp_infer with a workspace");
  if (gn_iters < 0 || gn_iters > 64) return mil_set_error(MIL_EINVAL, "gn_iters must be in 0..64");
  if (N == 0) return MIL_OK;
  if (!d_win || !d_params || !d_sigma || !d_out || !d_flag)
    return mil_set_error(MIL_EINVAL, "null argument");
  void *base = nullptr;
  int rc = scratch_ptr(&base);
  if (rc) return rc;
  char *ws = (char *)base;
  // the weight copies are rewritten and the counter cleared (by a kernel) on
  // every call; list entries are read only below the count this call wrote
  if (mil::launch_prepare(d_params, 0, ws + kPrepOff, stream) ||
      mil::launch_infer(d_win, N, W, d_params, ws + kPrepOff, d_sigma, k_sigma, gn_iters, tau,
                        d_out, d_flag, (int32_t *)(ws + kCountOff), (int32_t *)(ws + kListOff),
                        num_cus_noalloc(), stream))
    return mil_set_error(MIL_EHIP, "inference launch failed");
  return MIL_OK;
}

}  // extern "C"
