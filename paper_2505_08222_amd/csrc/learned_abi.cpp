// C ABI of the learned range-only estimator (declared in include/mi_lrauv.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "learned_internal.h"
#include "mi_lrauv.h"

namespace {

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

struct WorkLayout {
  int64_t prep, partial, loss_partial, fb_count, fb_list, total;
};

WorkLayout work_layout(int64_t N, int precision) {
  WorkLayout w{};
  int64_t o = 0;
  w.prep = o;
  o = align256(o + mil::kPrepBytes);
  const int64_t nb = mil::train_blocks(N > 0 ? N : 1, precision);
  w.partial = o;
  o = align256(o + nb * mil::train_partial_floats(precision) * 4);
  w.loss_partial = o;
  o = align256(o + nb * 4);
  w.fb_count = o;
  o = align256(o + 4);
  w.fb_list = o;
  o = align256(o + (N > 0 ? N : 1) * 4);
  w.total = o;
  return w;
}

int set_error(int code, const char *msg);

int num_cus() {
  static int n = 0;
  if (n == 0) {
    int dev = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
  }
  return n;
}

}  // namespace

extern "C" int mil_set_error(int code, const char *msg);  // abi.cpp

namespace {
int set_error(int code, const char *msg) { return mil_set_error(code, msg); }

int check_work(void *d_work, int64_t work_bytes, int64_t need) {
  if (!d_work) return set_error(MIL_EINVAL, "null workspace");
  if (((uintptr_t)d_work) & 255) return set_error(MIL_EALIGN, "workspace must be 256-byte aligned");
  if (work_bytes < need) return set_error(MIL_ESHAPE, "workspace too small (see mlp_workspace_bytes)");
  return MIL_OK;
}
}  // namespace

extern "C" {

int64_t mlp_num_params(void) { return mil::kNumParams; }

int mlp_init(float *d_params, uint64_t seed, void *stream) {
  if (!d_params) return set_error(MIL_EINVAL, "null argument");
  if (mil::launch_init(d_params, seed, stream)) return set_error(MIL_EHIP, "init launch failed");
  return MIL_OK;
}

int64_t mlp_workspace_bytes(int64_t N, int32_t precision) {
  return work_layout(N, precision == 0 ? 0 : 1).total;
}

int mlp_features(const float *d_win, int64_t N, int32_t W, float *d_x, float *d_frame,
                 void *stream) {
  if (N < 0 || W < 3 || 3 * W + 1 > mil::kIn) return set_error(MIL_EINVAL, "need N >= 0, 3 <= W <= 21");
  if (N == 0) return MIL_OK;
  if (!d_win || !d_x || !d_frame) return set_error(MIL_EINVAL, "null argument");
  if (((uintptr_t)d_x) & 15) return set_error(MIL_EALIGN, "features must be 16-byte aligned");
  if (mil::launch_features(d_win, N, W, d_x, d_frame, stream)) return set_error(MIL_EHIP, "launch failed");
  return MIL_OK;
}

int mlp_targets(const float *d_frame, const float *d_p, int64_t N, float *d_y, void *stream) {
  if (N < 0) return set_error(MIL_EINVAL, "N must be >= 0");
  if (N == 0) return MIL_OK;
  if (!d_frame || !d_p || !d_y) return set_error(MIL_EINVAL, "null argument");
  if (mil::launch_targets(d_frame, d_p, N, d_y, stream)) return set_error(MIL_EHIP, "launch failed");
  return MIL_OK;
}

int mlp_forward(int64_t N, const float *d_x, const float *d_params, float *d_y, int32_t precision,
                void *d_work, int64_t work_bytes, void *stream) {
  if (N < 0 || (precision != 0 && precision != 1)) return set_error(MIL_EINVAL, "bad N or precision");
  if (N == 0) return MIL_OK;
  if (!d_x || !d_params || !d_y) return set_error(MIL_EINVAL, "null argument");
  const WorkLayout w = work_layout(N, precision);
  int rc = check_work(d_work, work_bytes, w.prep + mil::kPrepBytes);
  if (rc) return rc;
  char *ws = (char *)d_work;
  if (mil::launch_prepare(d_params, precision, ws + w.prep, stream) ||
      mil::launch_forward(N, d_x, d_params, precision, ws + w.prep, d_y, stream))
    return set_error(MIL_EHIP, "forward launch failed");
  return MIL_OK;
}

int mlp_backward(int64_t N, const float *d_x, const int64_t *d_index, const float *d_target,
                 const float *d_params, float *d_grad, float *d_loss, int32_t precision,
                 void *d_work, int64_t work_bytes, void *stream) {
  if (N < 1 || (precision != 0 && precision != 1)) return set_error(MIL_EINVAL, "bad N or precision");
  if (!d_x || !d_target || !d_params || !d_grad) return set_error(MIL_EINVAL, "null argument");
  if (precision == 0 && ((((uintptr_t)d_x) | ((uintptr_t)d_params)) & 15))
    return set_error(MIL_EALIGN, "d_x and d_params must be 16-byte aligned");
  const WorkLayout w = work_layout(N, precision);
  int rc = check_work(d_work, work_bytes, w.fb_count);
  if (rc) return rc;
  char *ws = (char *)d_work;
  // BF16: the training kernel converts its weight fragments itself
  if ((precision != 0 && mil::launch_prepare(d_params, precision, ws + w.prep, stream)) ||
      mil::launch_train(N, d_x, d_index, d_target, d_params, precision, ws + w.prep,
                        (float *)(ws + w.partial), (float *)(ws + w.loss_partial), d_grad, d_loss,
                        stream))
    return set_error(MIL_EHIP, "backward launch failed");
  return MIL_OK;
}

int mlp_adam_step(int64_t P, float *d_params, const float *d_grad, float *d_m, float *d_v,
                  float lr, float beta1, float beta2, float eps, int32_t step, void *stream) {
  if (P < 1 || step < 1) return set_error(MIL_EINVAL, "need P >= 1 and step >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return set_error(MIL_EINVAL, "bad Adam constants");
  if (!d_params || !d_grad || !d_m || !d_v) return set_error(MIL_EINVAL, "null argument");
  if (mil::launch_adam(P, d_params, d_grad, d_m, d_v, lr, beta1, beta2, eps, step, stream))
    return set_error(MIL_EHIP, "adam launch failed");
  return MIL_OK;
}

int mlp_train_step(int64_t N, const float *d_x, const int64_t *d_index, const float *d_target,
                   float *d_params, float *d_m, float *d_v, float lr, float beta1, float beta2,
                   float eps, int32_t step, float *d_grad, float *d_loss, void *d_work,
                   int64_t work_bytes, void *stream) {
  if (N < 1 || step < 1) return set_error(MIL_EINVAL, "need N >= 1 and step >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return set_error(MIL_EINVAL, "bad Adam constants");
  if (!d_x || !d_target || !d_params || !d_m || !d_v) return set_error(MIL_EINVAL, "null argument");
  if ((((uintptr_t)d_x) | ((uintptr_t)d_params)) & 15)
    return set_error(MIL_EALIGN, "d_x and d_params must be 16-byte aligned");
  const WorkLayout w = work_layout(N, 0);
  int rc = check_work(d_work, work_bytes, w.fb_count);
  if (rc) return rc;
  char *ws = (char *)d_work;
  if (mil::launch_train_step(N, d_x, d_index, d_target, d_params, d_m, d_v, lr, beta1, beta2, eps,
                             step, (float *)(ws + w.partial), (float *)(ws + w.loss_partial),
                             d_grad, d_loss, stream))
    return set_error(MIL_EHIP, "training step launch failed");
  return MIL_OK;
}

int mlp_infer(const float *d_win, int64_t N, int32_t W, const float *d_params,
              const float *d_sigma, float k_sigma, int32_t gn_iters, float tau, float *d_out,
              uint8_t *d_flag, void *d_work, int64_t work_bytes, void *stream) {
  if (N < 0 || W < 3 || 3 * W + 1 > mil::kIn) return set_error(MIL_EINVAL, "need N >= 0, 3 <= W <= 21");
  if (gn_iters < 0 || gn_iters > 64) return set_error(MIL_EINVAL, "gn_iters must be in 0..64");
  if (N == 0) return MIL_OK;
  if (N > INT32_MAX) return set_error(MIL_EINVAL, "N must fit in int32");
  if (!d_win || !d_params || !d_sigma || !d_out || !d_flag) return set_error(MIL_EINVAL, "null argument");
  const WorkLayout w = work_layout(N, 0);
  int rc = check_work(d_work, work_bytes, w.total);
  if (rc) return rc;
  char *ws = (char *)d_work;
  if (mil::launch_prepare(d_params, 0, ws + w.prep, stream) ||
      mil::launch_infer(d_win, N, W, d_params, ws + w.prep, d_sigma, k_sigma, gn_iters, tau, d_out,
                        d_flag, (int32_t *)(ws + w.fb_count), (int32_t *)(ws + w.fb_list),
                        num_cus(), stream))
    return set_error(MIL_EHIP, "inference launch failed");
  return MIL_OK;
}

}  // extern "C"
