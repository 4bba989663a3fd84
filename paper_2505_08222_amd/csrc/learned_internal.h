// Constants and launchers of the learned estimator (learned_kernels.hip).
#pragma once
#include <stdint.h>

namespace mil {

// 64 -> 128 -> 128 -> 2. Parameter vector (FP32 master copy), row-major
// (out, in) weight matrices: W1, b1, W2, b2, W3, b3.
constexpr int kIn = 64;
constexpr int kHidden = 128;
constexpr int kOut = 2;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHidden * kIn;
constexpr int kOffW2 = kOffB1 + kHidden;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kOut * kHidden;
constexpr int kNumParams = kOffB3 + kOut;
// padded row strides of the MFMA-ready weight copies
constexpr int kLdIn = kIn + 8;
constexpr int kLdH = kHidden + 8;
// samples per training tile
constexpr int kTileBf16 = 32;
constexpr int kTileF32 = 16;
// most blocks (partial gradients) of the persistent BF16 training kernel:
// batches beyond kTrainBlocks tiles give each block several tiles
constexpr int kTrainBlocks = 128;
// bytes of the MFMA-ready weights (W1, W2, W2^T) for FP32 operands (the
// larger of the two precisions)
constexpr int64_t kPrepBytes = (int64_t)(kHidden * kLdIn + 2 * kHidden * kLdH) * 4;

int launch_init(float *th, uint64_t seed, void *stream);
int launch_prepare(const float *th, int precision, void *prep, void *stream);
int launch_features(const float *win, int64_t N, int32_t W, float *x, float *frame, void *stream);
int launch_targets(const float *frame, const float *p, int64_t N, float *y, void *stream);
int launch_forward(int64_t N, const float *x, const float *th, int precision, const void *prep,
                   float *y, void *stream);
int64_t train_blocks(int64_t N, int precision);
// floats of one block's partial gradient
int64_t train_partial_floats(int precision);
int launch_train(int64_t N, const float *x, const int64_t *index, const float *target,
                 const float *th, int precision, const void *prep, float *partial,
                 float *loss_partial, float *grad, float *loss, void *stream);
// BF16 training step: gradient (d_grad may be null) and, when m and v are
// given, the Adam update of th, in two kernels
int launch_train_step(int64_t N, const float *x, const int64_t *index, const float *target,
                      float *th, float *m, float *v, float lr, float b1, float b2, float eps,
                      int32_t step, float *partial, float *loss_partial, float *grad, float *loss,
                      void *stream);
int launch_adam(int64_t P, float *th, const float *g, float *m, float *v, float lr, float b1,
                float b2, float eps, int32_t step, void *stream);
int launch_infer(const float *win, int64_t N, int32_t W, const float *th, const void *prep,
                 const float *sigma, float k_sigma, int32_t gn_iters, float tau, float *out,
                 uint8_t *flag, int32_t *fb_count, int32_t *fb_list, int num_cus, void *stream);

// env_kernels.hip: tracker windows of a bound environment
struct DevState;
// slots = the largest pair count of an env (max agents x max targets)
int launch_env_windows(const DevState &s, int32_t W, int32_t slots, float *win, float *sigma,
                       float *truth, void *stream);

}  // namespace mil
