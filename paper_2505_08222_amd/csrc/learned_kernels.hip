// Learned range-only estimator on gfx950: a 64 -> 128 -> 128 -> 2 MLP with
// GELU (tanh form), BF16 operands on MFMA with FP32 accumulation (or FP32
// operands on the FP32 MFMA, for gradient checks), trained by hand-written
// forward/backward kernels and Adam; inference is fused with the window
// features, a residual test against the measured ranges and a compacted
// exact-LS fallback (arXiv 2505.08222, Sec. III-A, is the exact estimator it
// stands in for).
//
// MFMA operand layout (16x16 output tile, lane l = 0..63): lane l supplies
// row (l % 16) of A and column (l % 16) of B for the K-slice (l / 16), i.e.
// 8 consecutive K for v_mfma_f32_16x16x32_bf16 and 1 for
// v_mfma_f32_16x16x4_f32; it receives D rows 4 * (l / 16) + j, column l % 16.
// Both operands are therefore read K-contiguous: A as [m][k], B as [n][k].
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <math.h>

#include "learned_internal.h"
#include "mfma_tile.h"
#include "ls_device.h"
#include "rng.h"

namespace mil {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu_f(float x) {
  const float c = 0.7978845608028654f;
  return 0.5f * x * (1.0f + tanhf(c * (x + 0.044715f * x * x * x)));
}

__device__ __forceinline__ float gelu_grad_f(float x) {
  const float c = 0.7978845608028654f;
  const float th = tanhf(c * (x + 0.044715f * x * x * x));
  const float du = c * (1.0f + 3.0f * 0.044715f * x * x);
  return 0.5f * (1.0f + th) + 0.5f * x * (1.0f - th * th) * du;
}

template <typename T>
__device__ __forceinline__ T to_t(float v);
template <>
__device__ __forceinline__ __bf16 to_t<__bf16>(float v) {
  return __float2bfloat16(v);
}
template <>
__device__ __forceinline__ float to_t<float>(float v) {
  return v;
}
__device__ __forceinline__ float to_f(__bf16 v) { return __bfloat162float(v); }
__device__ __forceinline__ float to_f(float v) { return v; }

// Block-cooperative GEMM: D[m][n] = sum_k A[m][k] B[n][k] for an M x N
// output in 16 x 16 tiles spread over the block's wavefronts; `epi(m, n, v)`
// consumes every output. A, B are K-contiguous with row strides lda, ldb.
template <typename T, typename Epi>
__device__ __forceinline__ void block_gemm(const T *A, int lda, const T *B, int ldb, int M, int N,
                                           int K, Epi epi) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int tn = N >> 4, tiles = (M >> 4) * tn;
  const int row = lane & 15, kg = lane >> 4;
  for (int t = wave; t < tiles; t += nw) {
    const int m0 = (t / tn) << 4, n0 = (t % tn) << 4;
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (sizeof(T) == 2) {
      for (int k0 = 0; k0 < K; k0 += 32) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(A + (m0 + row) * lda + k0 + 8 * kg);
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(B + (n0 + row) * ldb + k0 + 8 * kg);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
      for (int k0 = 0; k0 < K; k0 += 4) {
        const float a = A[(m0 + row) * lda + k0 + kg];
        const float b = B[(n0 + row) * ldb + k0 + kg];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) epi(m0 + 4 * kg + j, n0 + row, acc[j]);
  }
}

// ---------------------------------------------------------------------------
// Weights in MFMA-ready form: W1 [128][64], W2 [128][128] and W2^T in the
// operand type, with rows padded to LDP = K + 8 elements (16 B) so that a
// lane's 8 consecutive K are 16-byte aligned.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void prepare_weights_kernel(const float *__restrict__ th, T *__restrict__ w1,
                                       T *__restrict__ w2, T *__restrict__ w2t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < kHidden * kIn) {
    const int o = k / kIn, i = k % kIn;
    w1[o * kLdIn + i] = to_t<T>(th[kOffW1 + k]);
  }
  if (k < kHidden * kHidden) {
    const int o = k / kHidden, i = k % kHidden;
    const T v = to_t<T>(th[kOffW2 + k]);
    w2[o * kLdH + i] = v;
    w2t[i * kLdH + o] = v;
  }
}

// ---------------------------------------------------------------------------
// Features of one window (entry order as stored; all entries present):
// centroid frame rotated so x runs along the chord a_0 - a_{W-1}.
// ---------------------------------------------------------------------------
constexpr int kMaxW = (kIn - 1) / 3;  // 21 entries fit the 64 inputs

__device__ __forceinline__ bool window_features(const float *w, int W, float (&x)[kIn],
                                                float (&frame)[5]) {
  // means taken over offsets from entry 0 (small numbers, so FP32 keeps them
  // accurate), then the centroid is entry 0 plus the mean offset
  const float x0 = w[0], y0 = w[1], r0 = w[2];
  float mx = 0.f, my = 0.f, mr = 0.f;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < kMaxW; ++k) {
    if (k < W) {
      mx += w[3 * k] - x0;
      my += w[3 * k + 1] - y0;
      const float r = w[3 * k + 2];
      ok = ok && (r == r);
      mr += r - r0;
    }
  }
  const float invw = 1.0f / (float)W;
  mx *= invw;
  my *= invw;
  mr *= invw;
  const float cx = w[0] - w[3 * (W - 1)], cy = w[1] - w[3 * (W - 1) + 1];
  const float len = sqrtf(fmaf(cx, cx, cy * cy));
  float c = 1.0f, s = 0.0f;
  if (len > 1e-6f) {
    c = cx / len;
    s = cy / len;
  }
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = 0.0f;
#pragma unroll
  for (int k = 0; k < kMaxW; ++k) {
    if (k < W) {
      const float dx = (w[3 * k] - x0) - mx, dy = (w[3 * k + 1] - y0) - my;
      x[3 * k] = fmaf(c, dx, s * dy) * 0.1f;
      x[3 * k + 1] = fmaf(-s, dx, c * dy) * 0.1f;
      x[3 * k + 2] = ((w[3 * k + 2] - r0) - mr) * 0.1f;
    } else if (k == W) {
      x[3 * k] = (r0 + mr) * 1e-3f;
    }
  }
  if (W == kMaxW) x[3 * kMaxW] = (r0 + mr) * 1e-3f;
  frame[0] = x0 + mx;
  frame[1] = y0 + my;
  frame[2] = c;
  frame[3] = s;
  frame[4] = r0 + mr;
  return ok;
}

__global__ void features_kernel(const float *__restrict__ win, int64_t N, int32_t W,
                                float *__restrict__ xout, float *__restrict__ frame) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float x[kIn], fr[5];
  window_features(win + n * W * 3, W, x, fr);
  float4 *xo = reinterpret_cast<float4 *>(xout + n * kIn);
#pragma unroll
  for (int q = 0; q < kIn / 4; ++q) xo[q] = make_float4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
#pragma unroll
  for (int q = 0; q < 5; ++q) frame[n * 5 + q] = fr[q];
}

// y_target = R(-theta)(p - abar) / rbar
__global__ void targets_kernel(const float *__restrict__ frame, const float *__restrict__ p,
                               int64_t N, float *__restrict__ y) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const float *fr = frame + n * 5;
  const float dx = p[2 * n] - fr[0], dy = p[2 * n + 1] - fr[1];
  y[2 * n] = (fr[2] * dx + fr[3] * dy) / fr[4];
  y[2 * n + 1] = (-fr[3] * dx + fr[2] * dy) / fr[4];
}

// ---------------------------------------------------------------------------
// Training step on a tile of S samples: forward, squared-error gradient,
// backward; writes this block's partial gradient (FP32) and loss.
// ---------------------------------------------------------------------------
template <typename T, int S>
struct TrainLds {
  T x[S][kIn + 8];           // X
  T xt[kIn][S + 8];          // X^T
  float z1[S][kHidden];      // pre-activations
  T h1[S][kHidden + 8];      // gelu(z1)
  T h1t[kHidden][S + 8];
  float z2[S][kHidden];
  T h2[S][kHidden + 8];      // gelu(z2), later dZ2
  T dz2t[kHidden][S + 8];
  T dz1t[kHidden][S + 8];
  float y[S][2];
  float dy[S][2];
};

template <typename T, int S>
__global__ void __launch_bounds__(256)
train_tile_kernel(int64_t N, const float *__restrict__ xin, const int64_t *__restrict__ index,
                  const float *__restrict__ target, const float *__restrict__ th,
                  const T *__restrict__ w1, const T *__restrict__ w2,
                  const T *__restrict__ w2t, float *__restrict__ partial,
                  float *__restrict__ loss_partial, float inv_n) {
  extern __shared__ __align__(16) unsigned char smem[];
  TrainLds<T, S> &L = *reinterpret_cast<TrainLds<T, S> *>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int64_t s0 = (int64_t)blockIdx.x * S;
  // ---- load X (and X^T) for the tile; rows past N are zero
  for (int e = tid; e < S * kIn; e += nthr) {
    const int s = e / kIn, i = e % kIn;
    float v = 0.0f;
    if (s0 + s < N) {
      const int64_t src = index ? index[s0 + s] : s0 + s;
      v = xin[src * kIn + i];
    }
    L.x[s][i] = to_t<T>(v);
    L.xt[i][s] = to_t<T>(v);
  }
  __syncthreads();
  // ---- layer 1
  block_gemm<T>(&L.x[0][0], kIn + 8, w1, kLdIn, S, kHidden, kIn, [&](int m, int n, float v) {
    const float z = v + th[kOffB1 + n];
    L.z1[m][n] = z;
    const T h = to_t<T>(gelu_f(z));
    L.h1[m][n] = h;
    L.h1t[n][m] = h;
  });
  __syncthreads();
  // ---- layer 2
  block_gemm<T>(&L.h1[0][0], kHidden + 8, w2, kLdH, S, kHidden, kHidden,
                [&](int m, int n, float v) {
                  const float z = v + th[kOffB2 + n];
                  L.z2[m][n] = z;
                  L.h2[m][n] = to_t<T>(gelu_f(z));
                });
  __syncthreads();
  // ---- layer 3 (two outputs) and the loss gradient
  if (tid < 2 * S) {
    const int s = tid >> 1, o = tid & 1;
    float acc = th[kOffB3 + o];
    for (int i = 0; i < kHidden; ++i) acc += th[kOffW3 + o * kHidden + i] * to_f(L.h2[s][i]);
    L.y[s][o] = acc;
    float d = 0.0f;
    if (s0 + s < N) {
      const int64_t src = index ? index[s0 + s] : s0 + s;
      d = acc - target[src * 2 + o];
    }
    L.dy[s][o] = 2.0f * d * inv_n;
    L.y[s][o] = d * d;  // reuse: squared error
  }
  __syncthreads();
  float *gp = partial + (int64_t)blockIdx.x * kNumParams;
  if (tid == 0) {
    float l = 0.0f;
    for (int s = 0; s < S; ++s) l += L.y[s][0] + L.y[s][1];
    loss_partial[blockIdx.x] = l;
  }
  // dW3, db3
  for (int e = tid; e < 2 * kHidden; e += nthr) {
    const int o = e / kHidden, i = e % kHidden;
    float acc = 0.0f;
    for (int s = 0; s < S; ++s) acc += L.dy[s][o] * to_f(L.h2[s][i]);
    gp[kOffW3 + e] = acc;
  }
  if (tid < 2) {
    float acc = 0.0f;
    for (int s = 0; s < S; ++s) acc += L.dy[s][tid];
    gp[kOffB3 + tid] = acc;
  }
  __syncthreads();
  // dZ2 = (dY W3) * gelu'(Z2), written over h2 and transposed into dz2t
  for (int e = tid; e < S * kHidden; e += nthr) {
    const int s = e / kHidden, i = e % kHidden;
    const float dh = L.dy[s][0] * th[kOffW3 + i] + L.dy[s][1] * th[kOffW3 + kHidden + i];
    const T d = to_t<T>(dh * gelu_grad_f(L.z2[s][i]));
    L.h2[s][i] = d;
    L.dz2t[i][s] = d;
  }
  __syncthreads();
  // db2
  for (int o = tid; o < kHidden; o += nthr) {
    float acc = 0.0f;
    for (int s = 0; s < S; ++s) acc += to_f(L.dz2t[o][s]);
    gp[kOffB2 + o] = acc;
  }
  // dW2[o][i] = sum_s dZ2[s][o] H1[s][i]
  block_gemm<T>(&L.dz2t[0][0], S + 8, &L.h1t[0][0], S + 8, kHidden, kHidden, S,
                [&](int m, int n, float v) { gp[kOffW2 + m * kHidden + n] = v; });
  // dH1 = dZ2 W2 (B operand = W2^T rows), dZ1 = dH1 * gelu'(Z1)
  block_gemm<T>(&L.h2[0][0], kHidden + 8, w2t, kLdH, S, kHidden, kHidden,
                [&](int m, int n, float v) { L.dz1t[n][m] = to_t<T>(v * gelu_grad_f(L.z1[m][n])); });
  __syncthreads();
  for (int o = tid; o < kHidden; o += nthr) {
    float acc = 0.0f;
    for (int s = 0; s < S; ++s) acc += to_f(L.dz1t[o][s]);
    gp[kOffB1 + o] = acc;
  }
  // dW1[o][i] = sum_s dZ1[s][o] X[s][i]
  block_gemm<T>(&L.dz1t[0][0], S + 8, &L.xt[0][0], S + 8, kHidden, kIn, S,
                [&](int m, int n, float v) { gp[kOffW1 + m * kIn + n] = v; });
}

// Deterministic sum of the per-block partial gradients and losses: a block
// takes 64 parameters; its four wavefronts each sum every fourth partial in
// order, and the four sums are added in a fixed order. Block 0 also sums the
// loss partials (fixed tree in FP64).
__global__ void __launch_bounds__(256)
reduce_grad_kernel(const float *__restrict__ partial, int nblocks, float *__restrict__ grad,
                   const float *__restrict__ loss_partial, float *__restrict__ loss, float inv_n) {
  __shared__ float part4[4][64];
  __shared__ double lred[256];
  const int pl = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + pl;
  float acc = 0.0f;
  if (p < kNumParams)
    for (int b = grp; b < nblocks; b += 4) acc += partial[(int64_t)b * kNumParams + p];
  part4[grp][pl] = acc;
  if (blockIdx.x == 0 && loss) {
    double l = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) l += loss_partial[b];
    lred[threadIdx.x] = l;
  }
  __syncthreads();
  if (grp == 0 && p < kNumParams)
    grad[p] = (part4[0][pl] + part4[1][pl]) + (part4[2][pl] + part4[3][pl]);
  if (blockIdx.x == 0 && loss) {
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) lred[threadIdx.x] += lred[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(lred[0] * inv_n);
  }
}

// Adam (Kingma and Ba) with bias correction; step counts from 1.
__global__ void adam_kernel(int64_t P, float *__restrict__ th, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Training step, BF16 operands, persistent form. G blocks of four wavefronts;
// block b takes the 32-sample tiles b, b + G, b + 2G, ... in that order and
// keeps the two hidden layers' weight gradients in its MFMA accumulators
// (registers) across its tiles, so that it writes one partial gradient per
// block instead of one per tile. Each wavefront owns fixed output tiles of
// every product, so its weight fragments are converted from the FP32 master
// copy once per launch (no separate preparation kernel). The partial is
// stored in accumulator order (one float4 per lane, coalesced); the
// reduction maps it back to the parameter layout.
//
// Products per tile (S = 32 samples, features 128, inputs 64):
//   Z1 = X W1^T, Z2 = H1 W2^T         weights as the MFMA's A operand, so a
//                                      lane holds 4 consecutive features of
//                                      one sample (bias, GELU, derivative)
//   dW2 += dZ2^T H1, dW1 += dZ1^T X    accumulated, K = the tile's samples
//   dH1 = dZ2 W2                       weights (W2^T rows) as the A operand
// GELU is the tanh form x sigma(2y) evaluated as x / (1 + 2^u) (the same
// function as the inference kernel's); its derivative, with s = sigma(2y),
// is s + x s (1 - s) (-ln 2) du/dx.
// ---------------------------------------------------------------------------
constexpr int kStepS = 32;
// partial vector: dW2 fragments, dW1 fragments, then b1, b2, W3, b3
constexpr int kPartW2 = 0;
constexpr int kPartW1 = kHidden * kHidden;
constexpr int kPartSmall = kPartW1 + kHidden * kIn;
constexpr int kPartFloats = ((kPartSmall + 2 * kHidden + kOut * kHidden + kOut) + 15) / 16 * 16;

struct StepLds {
  __bf16 x[kStepS][kIn + 8];         // X, sample-major
  __bf16 xt[kIn][kStepS + 8];        // X^T
  __bf16 h1[kStepS][kHidden + 8];    // H1 = gelu(Z1)
  __bf16 h1t[kHidden][kStepS + 8];   // H1^T
  union {
    struct {
      __bf16 h2[kStepS][kHidden + 8];    // H2 = gelu(Z2)
      __bf16 h2t[kHidden][kStepS + 8];   // H2^T
      __bf16 dz2[kStepS][kHidden + 8];   // dZ2, sample-major
      __bf16 dz2t[kHidden][kStepS + 8];  // dZ2^T
      __bf16 dz1t[kHidden][kStepS + 8];  // dZ1^T
    } t;
    __bf16 w2[kHidden][kHidden + 8];     // W2 staged for the fragments (set-up only)
  } u;
  float w3[kOut][kHidden];
  float tg[kStepS][kOut];            // targets
  float dyt[kOut][kStepS];           // dY^T
  float se[kStepS];                  // squared error per sample
};

__device__ __forceinline__ void gelu_and_grad(float z, float &h, float &g) {
  constexpr float a = -2.0f * 0.7978845608028654f * 1.4426950408889634f;
  constexpr float b = a * 0.044715f;
  constexpr float ln2 = 0.6931471805599453f;
  const float z2 = z * z;
  const float u = z * fmaf(b, z2, a);
  const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u));
  h = z * sg;
  g = fmaf(z * sg * (1.0f - sg) * (-ln2), fmaf(3.0f * b, z2, a), sg);
}

// 8 consecutive FP32 weights as one BF16 fragment
__device__ __forceinline__ bf16x8 frag8(const float *p) {
  const float4 lo = *reinterpret_cast<const float4 *>(p);
  const float4 hi = *reinterpret_cast<const float4 *>(p + 4);
  bf16x8 r;
  r[0] = __float2bfloat16(lo.x); r[1] = __float2bfloat16(lo.y);
  r[2] = __float2bfloat16(lo.z); r[3] = __float2bfloat16(lo.w);
  r[4] = __float2bfloat16(hi.x); r[5] = __float2bfloat16(hi.y);
  r[6] = __float2bfloat16(hi.z); r[7] = __float2bfloat16(hi.w);
  return r;
}

__device__ __forceinline__ float dot8(const bf16x8 h, const float4 a, const float4 b, float acc) {
  acc = fmaf(a.x, to_f(h[0]), acc);
  acc = fmaf(a.y, to_f(h[1]), acc);
  acc = fmaf(a.z, to_f(h[2]), acc);
  acc = fmaf(a.w, to_f(h[3]), acc);
  acc = fmaf(b.x, to_f(h[4]), acc);
  acc = fmaf(b.y, to_f(h[5]), acc);
  acc = fmaf(b.z, to_f(h[6]), acc);
  return fmaf(b.w, to_f(h[7]), acc);
}

__global__ void __launch_bounds__(256, 1)
train_accum_kernel(int64_t N, int64_t ntiles, const float *__restrict__ xin,
                   const int64_t *__restrict__ index, const float *__restrict__ target,
                   const float *__restrict__ th, float *__restrict__ partial,
                   float *__restrict__ loss_partial, float inv_n) {
  extern __shared__ __align__(16) unsigned char smem[];
  StepLds &L = *reinterpret_cast<StepLds *>(smem);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int row = lane & 15, kg = lane >> 4;
  // this thread's share of a tile's inputs: sample xs, inputs 8 xq .. 8 xq + 7
  // (and, for xq = 0, the sample's target); the first tile's rows are
  // requested before the weights
  const int xs = tid >> 3, xq = tid & 7;
  float4 xa = make_float4(0.f, 0.f, 0.f, 0.f), xb = xa;
  float2 tgv = make_float2(0.f, 0.f);
  auto fetch = [&](int64_t tile) {
    const int64_t s = tile * kStepS + xs;
    xa = make_float4(0.f, 0.f, 0.f, 0.f);
    xb = xa;
    tgv = make_float2(0.f, 0.f);
    if (tile < ntiles && s < N) {
      const int64_t src = index ? index[s] : s;
      const float4 *p = reinterpret_cast<const float4 *>(xin + src * kIn + 8 * xq);
      xa = p[0];
      xb = p[1];
      if (xq == 0) tgv = make_float2(target[src * 2], target[src * 2 + 1]);
    }
  };
  fetch(blockIdx.x);
  // ---- weight fragments (A operands) of W1, biases of this lane's
  // features, W2 staged in LDS as BF16 (coalesced reads: all loads issued
  // before the first store), W3
  bf16x8 w1f[2][2], w2f[2][4], w2tf[2][4];
  float b1r[2][4], b2r[2][4];
  {
    float4 w2raw[8][2];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = tid + 256 * k, o = e >> 4, i8 = (e & 15) << 3;
      const float4 *src = reinterpret_cast<const float4 *>(th + kOffW2 + o * kHidden + i8);
      w2raw[k][0] = src[0];
      w2raw[k][1] = src[1];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int n = ((wave + 4 * c) << 4) + row;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) w1f[c][ks] = frag8(th + kOffW1 + n * kIn + 32 * ks + 8 * kg);
      const int nf = ((wave + 4 * c) << 4) + 4 * kg;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        b1r[c][j] = th[kOffB1 + nf + j];
        b2r[c][j] = th[kOffB2 + nf + j];
      }
    }
    const float w3a = th[kOffW3 + tid];  // 256 threads = the 2 x 128 W3 entries
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = tid + 256 * k, o = e >> 4, i8 = (e & 15) << 3;
      bf16x8 r;
      r[0] = __float2bfloat16(w2raw[k][0].x); r[1] = __float2bfloat16(w2raw[k][0].y);
      r[2] = __float2bfloat16(w2raw[k][0].z); r[3] = __float2bfloat16(w2raw[k][0].w);
      r[4] = __float2bfloat16(w2raw[k][1].x); r[5] = __float2bfloat16(w2raw[k][1].y);
      r[6] = __float2bfloat16(w2raw[k][1].z); r[7] = __float2bfloat16(w2raw[k][1].w);
      *reinterpret_cast<bf16x8 *>(&L.u.w2[o][i8]) = r;
    }
    L.w3[tid / kHidden][tid % kHidden] = w3a;
  }
  __syncthreads();
  float w3r[2][4][2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int n = ((wave + 4 * c) << 4) + row;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      w2f[c][ks] = *reinterpret_cast<const bf16x8 *>(&L.u.w2[n][32 * ks + 8 * kg]);
      bf16x8 t;
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = L.u.w2[32 * ks + 8 * kg + q][n];
      w2tf[c][ks] = t;
    }
    const int nf = ((wave + 4 * c) << 4) + 4 * kg;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      w3r[c][j][0] = L.w3[0][nf + j];
      w3r[c][j][1] = L.w3[1][nf + j];
    }
  }
  // ---- accumulators: dW2 (o tiles 2w, 2w+1 x 8 i tiles), dW1 (x 4 i tiles)
  floatx4 acc2[2][8], acc1[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int b = 0; b < 8; ++b) acc2[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int b = 0; b < 4; ++b) acc1[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  float acc_w3 = 0.0f, acc_b3 = 0.0f, acc_b1 = 0.0f, acc_b2 = 0.0f, acc_loss = 0.0f;
  float b3v[2] = {th[kOffB3], th[kOffB3 + 1]};
  __syncthreads();  // the W2 staging area becomes the tile's buffers
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t s0 = tile * kStepS;
    // ---- X tile into LDS (the previous tile's last reads of x / xt are
    // behind the barrier that ends it), then fetch the next tile's rows
    {
      bf16x8 v;
      v[0] = __float2bfloat16(xa.x); v[1] = __float2bfloat16(xa.y);
      v[2] = __float2bfloat16(xa.z); v[3] = __float2bfloat16(xa.w);
      v[4] = __float2bfloat16(xb.x); v[5] = __float2bfloat16(xb.y);
      v[6] = __float2bfloat16(xb.z); v[7] = __float2bfloat16(xb.w);
      *reinterpret_cast<bf16x8 *>(&L.x[xs][8 * xq]) = v;
#pragma unroll
      for (int q = 0; q < 8; ++q) L.xt[8 * xq + q][xs] = v[q];
      if (xq == 0) {
        L.tg[xs][0] = tgv.x;
        L.tg[xs][1] = tgv.y;
      }
    }
    fetch(tile + gridDim.x);
    __syncthreads();
    // ---- layer 1: Z1 = X W1^T + b1 (lane: features nf..nf+3 of sample m);
    // gelu'(Z1) stays in this lane's registers for the backward pass
    float g1r[2][2][4], g2r[2][2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int m = (mt << 4) + row;
      bf16x8 xf[2];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
        xf[ks] = *reinterpret_cast<const bf16x8 *>(&L.x[m][32 * ks + 8 * kg]);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f[c][ks], xf[ks], acc, 0, 0, 0);
        const int nf = ((wave + 4 * c) << 4) + 4 * kg;
        bf16x4 hv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float h;
          gelu_and_grad(acc[j] + b1r[c][j], h, g1r[mt][c][j]);
          hv[j] = __float2bfloat16(h);
          L.h1t[nf + j][m] = hv[j];
        }
        *reinterpret_cast<bf16x4 *>(&L.h1[m][nf]) = hv;
      }
    }
    __syncthreads();
    // ---- layer 2: Z2 = H1 W2^T + b2
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int m = (mt << 4) + row;
      bf16x8 hf[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        hf[ks] = *reinterpret_cast<const bf16x8 *>(&L.h1[m][32 * ks + 8 * kg]);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2f[c][ks], hf[ks], acc, 0, 0, 0);
        const int nf = ((wave + 4 * c) << 4) + 4 * kg;
        bf16x4 hv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float h;
          gelu_and_grad(acc[j] + b2r[c][j], h, g2r[mt][c][j]);
          hv[j] = __float2bfloat16(h);
          L.u.t.h2t[nf + j][m] = hv[j];
        }
        *reinterpret_cast<bf16x4 *>(&L.u.t.h2[m][nf]) = hv;
      }
    }
    __syncthreads();
    // ---- output layer: four lanes per (sample, output), 32 features each,
    // quad sum; dY = 2 (Y - target) / N
    {
      const int d = tid >> 2, q = tid & 3, sm = d >> 1, o = d & 1;
      float a = 0.0f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bf16x8 h = *reinterpret_cast<const bf16x8 *>(&L.u.t.h2[sm][32 * q + 8 * k]);
        const float4 wa = *reinterpret_cast<const float4 *>(&L.w3[o][32 * q + 8 * k]);
        const float4 wb = *reinterpret_cast<const float4 *>(&L.w3[o][32 * q + 8 * k + 4]);
        a = dot8(h, wa, wb, a);
      }
      const float y = quad_sum(a) + b3v[o];
      const float dd = (s0 + sm < N) ? y - L.tg[sm][o] : 0.0f;
      const float sq = dd * dd;
      const float sq_other = __shfl_xor(sq, 4);  // the other output of the sample
      if (q == 0) {
        L.dyt[o][sm] = 2.0f * dd * inv_n;
        if (o == 0) L.se[sm] = sq + sq_other;
      }
    }
    __syncthreads();
    // ---- dW3 (thread: W3 entry o, i), db3, loss; dZ2 = (dY W3) * gelu'(Z2)
    // from this lane's own features
    {
      const int o = tid >> 7, i = tid & (kHidden - 1);
      float a = 0.0f;
#pragma unroll
      for (int k = 0; k < kStepS / 8; ++k) {
        const bf16x8 h = *reinterpret_cast<const bf16x8 *>(&L.u.t.h2t[i][8 * k]);
        const float4 da = *reinterpret_cast<const float4 *>(&L.dyt[o][8 * k]);
        const float4 db = *reinterpret_cast<const float4 *>(&L.dyt[o][8 * k + 4]);
        a = dot8(h, da, db, a);
      }
      acc_w3 += a;
      if (tid < kOut) {
        float bsum = 0.0f;
        for (int sm = 0; sm < kStepS; ++sm) bsum += L.dyt[tid][sm];
        acc_b3 += bsum;
      }
      if (tid == 0) {
        float l = 0.0f;
        for (int sm = 0; sm < kStepS; ++sm) l += L.se[sm];
        acc_loss += l;
      }
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int m = (mt << 4) + row;
      const float dy0 = L.dyt[0][m], dy1 = L.dyt[1][m];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int nf = ((wave + 4 * c) << 4) + 4 * kg;
        bf16x4 dv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float dh = fmaf(dy0, w3r[c][j][0], dy1 * w3r[c][j][1]);
          dv[j] = __float2bfloat16(dh * g2r[mt][c][j]);
          L.u.t.dz2t[nf + j][m] = dv[j];
        }
        *reinterpret_cast<bf16x4 *>(&L.u.t.dz2[m][nf]) = dv;
      }
    }
    __syncthreads();
    // ---- db2; dW2 += dZ2^T H1; dH1 = dZ2 W2 -> dZ1 = dH1 * gelu'(Z1)
    if (tid < kHidden) {
      float a = 0.0f;
#pragma unroll
      for (int k = 0; k < kStepS / 8; ++k) {
        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(&L.u.t.dz2t[tid][8 * k]);
#pragma unroll
        for (int q = 0; q < 8; ++q) a += to_f(v[q]);
      }
      acc_b2 += a;
    }
    {
      bf16x8 af[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        af[a] = *reinterpret_cast<const bf16x8 *>(&L.u.t.dz2t[((2 * wave + a) << 4) + row][8 * kg]);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bf16x8 bf = *reinterpret_cast<const bf16x8 *>(&L.h1t[(b << 4) + row][8 * kg]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
          acc2[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bf, acc2[a][b], 0, 0, 0);
      }
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int m = (mt << 4) + row;
      bf16x8 df[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        df[ks] = *reinterpret_cast<const bf16x8 *>(&L.u.t.dz2[m][32 * ks + 8 * kg]);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2tf[c][ks], df[ks], acc, 0, 0, 0);
        const int nf = ((wave + 4 * c) << 4) + 4 * kg;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          L.u.t.dz1t[nf + j][m] = __float2bfloat16(acc[j] * g1r[mt][c][j]);
      }
    }
    __syncthreads();
    // ---- db1; dW1 += dZ1^T X
    if (tid < kHidden) {
      float a = 0.0f;
#pragma unroll
      for (int k = 0; k < kStepS / 8; ++k) {
        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(&L.u.t.dz1t[tid][8 * k]);
#pragma unroll
        for (int q = 0; q < 8; ++q) a += to_f(v[q]);
      }
      acc_b1 += a;
    }
    {
      bf16x8 af[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        af[a] = *reinterpret_cast<const bf16x8 *>(&L.u.t.dz1t[((2 * wave + a) << 4) + row][8 * kg]);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const bf16x8 bf = *reinterpret_cast<const bf16x8 *>(&L.xt[(b << 4) + row][8 * kg]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
          acc1[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bf, acc1[a][b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // ---- this block's partial: accumulator fragments, then the small vectors
  float *gp = partial + (int64_t)blockIdx.x * kPartFloats;
  float4 *g4 = reinterpret_cast<float4 *>(gp);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b)
      g4[(kPartW2 >> 2) + (((wave * 16 + a * 8 + b) << 6) + lane)] =
          make_float4(acc2[a][b][0], acc2[a][b][1], acc2[a][b][2], acc2[a][b][3]);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      g4[(kPartW1 >> 2) + (((wave * 8 + a * 4 + b) << 6) + lane)] =
          make_float4(acc1[a][b][0], acc1[a][b][1], acc1[a][b][2], acc1[a][b][3]);
  if (tid < kHidden) {
    gp[kPartSmall + tid] = acc_b1;
    gp[kPartSmall + kHidden + tid] = acc_b2;
  }
  gp[kPartSmall + 2 * kHidden + tid] = acc_w3;  // 256 threads = the 2 x 128 W3 entries
  if (tid < kOut) gp[kPartSmall + 2 * kHidden + kOut * kHidden + tid] = acc_b3;
  if (tid == 0) loss_partial[blockIdx.x] = acc_loss;
}

// Parameter index of entry f of the partial vector (-1: padding).
__device__ __forceinline__ int partial_param(int f) {
  if (f < kPartW1) {  // dW2 fragment: tile (w, a, b), lane, element
    const int t = f >> 8, ln = (f >> 2) & 63, jj = f & 3;
    const int w = t >> 4, a = (t >> 3) & 1, b = t & 7;
    const int o = ((2 * w + a) << 4) + 4 * (ln >> 4) + jj, i = (b << 4) + (ln & 15);
    return kOffW2 + o * kHidden + i;
  }
  if (f < kPartSmall) {
    const int g = f - kPartW1;
    const int t = g >> 8, ln = (g >> 2) & 63, jj = g & 3;
    const int w = t >> 3, a = (t >> 2) & 1, b = t & 3;
    const int o = ((2 * w + a) << 4) + 4 * (ln >> 4) + jj, i = (b << 4) + (ln & 15);
    return kOffW1 + o * kIn + i;
  }
  const int g = f - kPartSmall;
  if (g < kHidden) return kOffB1 + g;
  if (g < 2 * kHidden) return kOffB2 + (g - kHidden);
  if (g < 2 * kHidden + kOut * kHidden) return kOffW3 + (g - 2 * kHidden);
  if (g < 2 * kHidden + kOut * kHidden + kOut) return kOffB3 + (g - 2 * kHidden - kOut * kHidden);
  return -1;
}

// Fixed-order sum of the G block partials and, with `adam`, the Adam update
// of the same parameters. A block takes 32 float4 columns of the partial
// vector; its eight wavefront-halves each sum every eighth partial in order,
// and the eight sums are added in a fixed order. Block 0 also sums the loss
// partials (fixed tree in FP64).
__global__ void __launch_bounds__(256)
reduce_step_kernel(const float *__restrict__ partial, int nblocks, float *__restrict__ grad,
                   const float *__restrict__ loss_partial, float *__restrict__ loss, float inv_n,
                   int adam, float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                   float lr, float b1, float b2, float eps, float c1, float c2) {
  __shared__ float4 red[8][32];
  __shared__ double lred[256];
  const int colw = threadIdx.x & 31, grp = threadIdx.x >> 5;
  const int col = blockIdx.x * 32 + colw;
  constexpr int ncol = kPartFloats / 4;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  if (col < ncol) {
    // partials grp, grp + 8, grp + 16, ... in order; four loads in flight
    const float4 *p4 = reinterpret_cast<const float4 *>(partial);
    for (int b0 = grp; b0 < nblocks; b0 += 32) {
      float4 q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + 8 * u;
        q[u] = b < nblocks ? p4[(int64_t)b * ncol + col] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (b0 + 8 * u < nblocks) {
          acc.x += q[u].x; acc.y += q[u].y; acc.z += q[u].z; acc.w += q[u].w;
        }
    }
  }
  red[grp][colw] = acc;
  if (blockIdx.x == 0 && loss) {
    double l = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) l += loss_partial[b];
    lred[threadIdx.x] = l;
  }
  __syncthreads();
  if (grp == 0 && col < ncol) {
    float4 t = red[0][colw];
#pragma unroll
    for (int g = 1; g < 8; ++g) {
      const float4 q = red[g][colw];
      t.x += q.x; t.y += q.y; t.z += q.z; t.w += q.w;
    }
    const float tv[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int pidx = partial_param(4 * col + j);
      if (pidx < 0) continue;
      const float gi = tv[j];
      if (grad) grad[pidx] = gi;
      if (adam) {
        const float mi = b1 * m[pidx] + (1.0f - b1) * gi;
        const float vi = b2 * v[pidx] + (1.0f - b2) * gi * gi;
        m[pidx] = mi;
        v[pidx] = vi;
        th[pidx] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
      }
    }
  }
  if (blockIdx.x == 0 && loss) {
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) lred[threadIdx.x] += lred[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(lred[0] * inv_n);
  }
}

// ---------------------------------------------------------------------------
// Forward only (training evaluation): tile of 64 samples per block.
// ---------------------------------------------------------------------------
template <typename T>
struct FwdLds {
  T x[64][kIn + 8];
  T h1[64][kHidden + 8];
  T h2[64][kHidden + 8];
  float b1[kHidden], b2[kHidden], w3[2][kHidden], b3[4];
};

template <typename T>
__global__ void __launch_bounds__(256)
forward_kernel(int64_t N, const float *__restrict__ xin, const float *__restrict__ th,
               const T *__restrict__ w1, const T *__restrict__ w2, float *__restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  FwdLds<T> &L = *reinterpret_cast<FwdLds<T> *>(smem);
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * 64;
  for (int e = tid; e < 64 * kIn; e += blockDim.x) {
    const int s = e / kIn, i = e % kIn;
    L.x[s][i] = to_t<T>(s0 + s < N ? xin[(s0 + s) * kIn + i] : 0.0f);
  }
  for (int e = tid; e < kHidden; e += blockDim.x) {
    L.b1[e] = th[kOffB1 + e];
    L.b2[e] = th[kOffB2 + e];
    L.w3[0][e] = th[kOffW3 + e];
    L.w3[1][e] = th[kOffW3 + kHidden + e];
  }
  if (tid < 2) L.b3[tid] = th[kOffB3 + tid];
  __syncthreads();
  if constexpr (sizeof(T) == 2) {
    // BF16 operands: the weight-stationary tile GEMM and the fast GELU (its
    // output is rounded to BF16 anyway)
    gemm_rs_bf16<kIn, kHidden>(&L.x[0][0], kIn + 8, w1, kLdIn, 64, [&](int m, int n, float v) {
      L.h1[m][n] = to_t<T>(gelu_tanh_fast(v + L.b1[n]));
    });
    __syncthreads();
    gemm_rs_bf16<kHidden, kHidden>(&L.h1[0][0], kHidden + 8, w2, kLdH, 64,
                          [&](int m, int n, float v) { L.h2[m][n] = to_t<T>(gelu_tanh_fast(v + L.b2[n])); });
  } else {
    block_gemm<T>(&L.x[0][0], kIn + 8, w1, kLdIn, 64, kHidden, kIn, [&](int m, int n, float v) {
      L.h1[m][n] = to_t<T>(gelu_f(v + L.b1[n]));
    });
    __syncthreads();
    block_gemm<T>(&L.h1[0][0], kHidden + 8, w2, kLdH, 64, kHidden, kHidden,
                  [&](int m, int n, float v) { L.h2[m][n] = to_t<T>(gelu_f(v + L.b2[n])); });
  }
  __syncthreads();
  {  // output layer: four threads per (sample, output), 32 inputs each, fixed sum order
    const int s = tid >> 2, part = tid & 3;
    float a0 = 0.0f, a1 = 0.0f;
    for (int i = part * 32; i < part * 32 + 32; ++i) {
      const float h = to_f(L.h2[s][i]);
      a0 += L.w3[0][i] * h;
      a1 += L.w3[1][i] * h;
    }
    a0 += __shfl_xor(a0, 1);
    a1 += __shfl_xor(a1, 1);
    a0 += __shfl_xor(a0, 2);
    a1 += __shfl_xor(a1, 2);
    if (part == 0 && s0 + s < N) {
      y[(s0 + s) * 2] = L.b3[0] + a0;
      y[(s0 + s) * 2 + 1] = L.b3[1] + a1;
    }
  }
}

// BF16 forward pass, persistent: the same layers as forward_kernel<bf16> with
// the structure of the inference kernel below (both hidden layers' weight
// fragments in registers for every tile, the next tile's features in
// registers while this one computes, the output layer fused into the second
// layer's epilogue: each lane's four BF16-rounded activations, then the four
// lanes of a row and the four wavefronts in a fixed order).
struct FwdBfLds {
  float w3[2][kHidden];
  float b1[kHidden], b2[kHidden], b3[4];
  __bf16 x[64][kIn + 8];
  __bf16 h1[64][kHidden + 8];
  float ypart[64][4][2];
};
static_assert(offsetof(FwdBfLds, x) % 16 == 0 && offsetof(FwdBfLds, h1) % 16 == 0 &&
                  offsetof(FwdBfLds, b1) % 16 == 0 && offsetof(FwdBfLds, b2) % 16 == 0,
              "MFMA operands and float4 parameter reads need 16-byte alignment");

__global__ void __launch_bounds__(256)
forward_bf16_kernel(int64_t N, const float *__restrict__ xin, const float *__restrict__ th,
                    const __bf16 *__restrict__ w1g, const __bf16 *__restrict__ w2g,
                    float *__restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  FwdBfLds &L = *reinterpret_cast<FwdBfLds *>(smem);
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * kHidden; e += blockDim.x) (&L.w3[0][0])[e] = th[kOffW3 + e];
  for (int e = tid; e < kHidden; e += blockDim.x) {
    L.b1[e] = th[kOffB1 + e];
    L.b2[e] = th[kOffB2 + e];
  }
  if (tid < 2) L.b3[tid] = th[kOffB3 + tid];
  BFrag<kIn, kHidden> f1;
  BFrag<kHidden, kHidden> f2;
  load_bfrag(f1, w1g, kLdIn);
  load_bfrag(f2, w2g, kLdH);
  const int64_t ntiles = (N + 63) / 64;
  constexpr int kPre = 64 * kIn / 256;
  float pre[kPre];
  auto fetch = [&](int64_t tile) {
    const int64_t t0 = tile * 64;
    const int nst = tile < ntiles ? ((N - t0) < 64 ? (int)(N - t0) : 64) : 0;
    const float *src = xin + t0 * kIn;
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
      const int e = tid + q * 256;
      pre[q] = e < nst * kIn ? src[e] : 0.0f;
    }
  };
  fetch(blockIdx.x);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t s0 = tile * 64;
    const int ns = (N - s0) < 64 ? (int)(N - s0) : 64;
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
      const int e = tid + q * 256;  // samples past the end stay zero
      L.x[e / kIn][e % kIn] = __float2bfloat16(pre[q]);
    }
    fetch(tile + gridDim.x);
    __syncthreads();
    gemm_rs_bf16_tf<kIn, kHidden>(&L.x[0][0], kIn + 8, f1, 64,
                                  [&](int m, int n, const floatx4 &v) {
                                    const float4 b = *reinterpret_cast<const float4 *>(&L.b1[n]);
                                    const bf16x4 h = {__float2bfloat16(gelu_tanh_fast(v[0] + b.x)),
                                                      __float2bfloat16(gelu_tanh_fast(v[1] + b.y)),
                                                      __float2bfloat16(gelu_tanh_fast(v[2] + b.z)),
                                                      __float2bfloat16(gelu_tanh_fast(v[3] + b.w))};
                                    *reinterpret_cast<bf16x4 *>(&L.h1[m][n]) = h;
                                  });
    __syncthreads();
    {
      const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kg = lane >> 4;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        bf16x8 a[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          a[ks] = *reinterpret_cast<const bf16x8 *>(&L.h1[16 * mt + row][ks * 32 + 8 * kg]);
        float y0 = 0.0f, y1 = 0.0f;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f2.v[c][ks], a[ks], acc, 0, 0, 0);
          const int n = ((wave + 4 * c) << 4) + 4 * kg;
          const float4 b = *reinterpret_cast<const float4 *>(&L.b2[n]);
          const float4 u0 = *reinterpret_cast<const float4 *>(&L.w3[0][n]);
          const float4 u1 = *reinterpret_cast<const float4 *>(&L.w3[1][n]);
          const float bb[4] = {b.x, b.y, b.z, b.w}, w0[4] = {u0.x, u0.y, u0.z, u0.w},
                      w1[4] = {u1.x, u1.y, u1.z, u1.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float h = __bfloat162float(__float2bfloat16(gelu_tanh_fast(acc[j] + bb[j])));
            y0 = fmaf(w0[j], h, y0);
            y1 = fmaf(w1[j], h, y1);
          }
        }
        y0 = col_sum4(y0);
        y1 = col_sum4(y1);
        if (kg == 0) {
          L.ypart[16 * mt + row][wave][0] = y0;
          L.ypart[16 * mt + row][wave][1] = y1;
        }
      }
    }
    __syncthreads();
    if (tid < 2 * ns) {
      const int s = tid >> 1, o = tid & 1;
      y[(s0 + s) * 2 + o] = L.b3[o] + ((L.ypart[s][0][o] + L.ypart[s][1][o]) +
                                       (L.ypart[s][2][o] + L.ypart[s][3][o]));
    }
    __syncthreads();  // before the next tile's features overwrite the stage
  }
}

// ---------------------------------------------------------------------------
// Inference: persistent blocks (as many as fit a CU) loop over tiles of 64 windows.
// The tile's windows (contiguous in memory) are staged in LDS with coalesced
// loads; features, the two hidden layers (MFMA; both layers' weight fragments
// are loaded into registers once per block), the output layer (fused into the
// second layer's epilogue), the decode (network bearing, distance fitted to
// the ranges) and the residual test all read that copy. Windows failing the test (or with
// missing entries) are appended, one atomic per wavefront, to a list that
// the fallback kernel solves exactly.
// ---------------------------------------------------------------------------
constexpr int kRefineIters = 3;  // distance-fit steps of the decode

struct InferLds {
  float win[64 * kMaxW * 3];
  float w3[2][kHidden];
  float b1[kHidden], b2[kHidden], b3[4];  // b3 padded: keeps x 16-byte aligned
  __bf16 x[64][kIn + 8];
  __bf16 h1[64][kHidden + 8];
  float frame[64][5];
  float ypart[64][4][2];  // output layer partial sums: [window][wavefront][output]
  int ok[64];
};

static_assert(offsetof(InferLds, x) % 16 == 0, "MFMA operands need 16-byte rows");
static_assert(offsetof(InferLds, h1) % 16 == 0 && offsetof(InferLds, b1) % 16 == 0 &&
                  offsetof(InferLds, b2) % 16 == 0 && offsetof(InferLds, w3) % 16 == 0,
              "MFMA operands and float4 parameter reads need 16-byte alignment");
static_assert(sizeof(InferLds) <= 52 * 1024, "three inference blocks per CU");

__global__ void __launch_bounds__(256)
infer_kernel(const float *__restrict__ win, int64_t N, int32_t W, const float *__restrict__ th,
             const __bf16 *__restrict__ w1g, const __bf16 *__restrict__ w2g,
             const float *__restrict__ sigma, float k_sigma, float *__restrict__ out,
             uint8_t *__restrict__ flag, int32_t *__restrict__ fb_count,
             int32_t *__restrict__ fb_list) {
  extern __shared__ __align__(16) unsigned char smem[];
  InferLds &L = *reinterpret_cast<InferLds *>(smem);
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * kHidden; e += blockDim.x) (&L.w3[0][0])[e] = th[kOffW3 + e];
  for (int e = tid; e < kHidden; e += blockDim.x) {
    L.b1[e] = th[kOffB1 + e];
    L.b2[e] = th[kOffB2 + e];
  }
  if (tid < 2) L.b3[tid] = th[kOffB3 + tid];
  // both hidden layers' weight fragments stay in registers for every tile
  BFrag<kIn, kHidden> f1;
  BFrag<kHidden, kHidden> f2;
  load_bfrag(f1, w1g, kLdIn);
  load_bfrag(f2, w2g, kLdH);
  const int64_t ntiles = (N + 63) / 64;
  const int wlen = W * 3;
  // the tile's windows (contiguous) are held in registers a tile ahead: each
  // thread's share of the next tile is in flight while this one computes
  constexpr int kPre = (64 * kMaxW * 3 + 255) / 256;
  float pre[kPre];
  auto fetch = [&](int64_t tile) {
    const int64_t t0 = tile * 64;
    const int nwt = tile < ntiles ? ((N - t0) < 64 ? (int)(N - t0) : 64) : 0;
    const float *src = win + t0 * wlen;
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
      const int e = tid + q * 256;
      pre[q] = e < nwt * wlen ? src[e] : 0.0f;
    }
  };
  fetch(blockIdx.x);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t s0 = tile * 64;
    const int nw = (N - s0) < 64 ? (int)(N - s0) : 64;  // windows in this tile
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
      const int e = tid + q * 256;
      if (e < nw * wlen) L.win[e] = pre[q];
    }
    fetch(tile + gridDim.x);
    __syncthreads();
    // features (the same quantities as window_features): four threads per
    // window, each taking entries part, part + 4, ...; the window's sums are
    // combined across the four threads
    {
      const int s = tid >> 2, part = tid & 3;
      const bool live = s < nw;
      const float *w = L.win + (live ? s : 0) * wlen;
      const float x0 = w[0], y0 = w[1], r0 = w[2];
      float mx = 0.f, my = 0.f, mr = 0.f, bad = 0.f;
      for (int k = part; k < W; k += 4) {
        mx += w[3 * k] - x0;
        my += w[3 * k + 1] - y0;
        const float r = w[3 * k + 2];
        bad += (r == r) ? 0.f : 1.f;
        mr += r - r0;
      }
      mx = quad_sum(mx);
      my = quad_sum(my);
      mr = quad_sum(mr);
      bad = quad_sum(bad);
      const float invw = 1.0f / (float)W;
      mx *= invw;
      my *= invw;
      mr *= invw;
      const float cx = w[0] - w[3 * (W - 1)], cy = w[1] - w[3 * (W - 1) + 1];
      const float len = sqrtf(fmaf(cx, cx, cy * cy));
      float c = 1.0f, sn = 0.0f;
      if (len > 1e-6f) {
        c = cx / len;
        sn = cy / len;
      }
      for (int k = part; k < W; k += 4) {
        const float dx = (w[3 * k] - x0) - mx, dy = (w[3 * k + 1] - y0) - my;
        L.x[s][3 * k] = __float2bfloat16(live ? fmaf(c, dx, sn * dy) * 0.1f : 0.0f);
        L.x[s][3 * k + 1] = __float2bfloat16(live ? fmaf(-sn, dx, c * dy) * 0.1f : 0.0f);
        L.x[s][3 * k + 2] = __float2bfloat16(live ? ((w[3 * k + 2] - r0) - mr) * 0.1f : 0.0f);
      }
      for (int i = 3 * W + part; i < kIn; i += 4)
        L.x[s][i] = __float2bfloat16((live && i == 3 * W) ? (r0 + mr) * 1e-3f : 0.0f);
      if (part == 0) {
        L.frame[s][0] = live ? x0 + mx : 0.0f;
        L.frame[s][1] = live ? y0 + my : 0.0f;
        L.frame[s][2] = live ? c : 1.0f;
        L.frame[s][3] = live ? sn : 0.0f;
        L.frame[s][4] = live ? r0 + mr : 1.0f;
        L.ok[s] = (live && bad == 0.f) ? 1 : 0;
      }
    }
    __syncthreads();
    gemm_rs_bf16_tf<kIn, kHidden>(&L.x[0][0], kIn + 8, f1, 64,
                                  [&](int m, int n, const floatx4 &v) {
                                    const float4 b = *reinterpret_cast<const float4 *>(&L.b1[n]);
                                    const bf16x4 h = {__float2bfloat16(gelu_tanh_fast(v[0] + b.x)),
                                                      __float2bfloat16(gelu_tanh_fast(v[1] + b.y)),
                                                      __float2bfloat16(gelu_tanh_fast(v[2] + b.z)),
                                                      __float2bfloat16(gelu_tanh_fast(v[3] + b.w))};
                                    *reinterpret_cast<bf16x4 *>(&L.h1[m][n]) = h;
                                  });
    __syncthreads();
    // second hidden layer and the output layer together: each lane rounds its
    // four GELU outputs to BF16 (the activation precision) and takes their
    // part of both output dot products; the four lanes of a row, then the four
    // wavefronts (fixed order, in the decode) complete them
    {
      const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kg = lane >> 4;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        bf16x8 a[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          a[ks] = *reinterpret_cast<const bf16x8 *>(&L.h1[16 * mt + row][ks * 32 + 8 * kg]);
        float y0 = 0.0f, y1 = 0.0f;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f2.v[c][ks], a[ks], acc, 0, 0, 0);
          const int n = ((wave + 4 * c) << 4) + 4 * kg;
          const float4 b = *reinterpret_cast<const float4 *>(&L.b2[n]);
          const float4 u0 = *reinterpret_cast<const float4 *>(&L.w3[0][n]);
          const float4 u1 = *reinterpret_cast<const float4 *>(&L.w3[1][n]);
          const float bb[4] = {b.x, b.y, b.z, b.w}, w0[4] = {u0.x, u0.y, u0.z, u0.w},
                      w1[4] = {u1.x, u1.y, u1.z, u1.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float h = __bfloat162float(__float2bfloat16(gelu_tanh_fast(acc[j] + bb[j])));
            y0 = fmaf(w0[j], h, y0);
            y1 = fmaf(w1[j], h, y1);
          }
        }
        y0 = col_sum4(y0);
        y1 = col_sum4(y1);
        if (kg == 0) {
          L.ypart[16 * mt + row][wave][0] = y0;
          L.ypart[16 * mt + row][wave][1] = y1;
        }
      }
    }
    __syncthreads();
    {  // decode, distance fit and residual test: four threads per window
      const int sw = tid >> 2, part = tid & 3;
      const bool live = sw < nw;
      const int64_t n = s0 + sw;
      const float *fr = L.frame[sw];
      const float *w = L.win + (live ? sw : 0) * wlen;
      auto sum4 = [](float v) { return quad_sum(v); };
      const float y0 = L.b3[0] + ((L.ypart[sw][0][0] + L.ypart[sw][1][0]) +
                                  (L.ypart[sw][2][0] + L.ypart[sw][3][0]));
      const float y1 = L.b3[1] + ((L.ypart[sw][0][1] + L.ypart[sw][1][1]) +
                                  (L.ypart[sw][2][1] + L.ypart[sw][3][1]));
      const float ux = fr[4] * y0, uy = fr[4] * y1;
      float px = fr[0] + fr[2] * ux - fr[3] * uy;
      float py = fr[1] + fr[3] * ux + fr[2] * uy;
      const bool ok = live && L.ok[sw];
      // the network fixes the bearing from the centroid; the distance along
      // it is fitted to the window's ranges (Gauss-Newton on d, a step kept
      // only if the squared residual falls). A rejected step would be
      // proposed again from the same point, so the fit stops there, and one
      // pass per point gives the residual, its derivative and the
      // curvature: the residual of the last kept point is the test's.
      float ex = px - fr[0], ey = py - fr[1];
      float d = __builtin_amdgcn_sqrtf(fmaf(ex, ex, ey * ey));
      const bool fit = ok && d > 0.0f;  // the same for the window's four threads
      if (fit) {
        const float inv = __builtin_amdgcn_rcpf(d);
        ex *= inv;
        ey *= inv;
      }
      // (sum of squared residuals, their derivative / 2, Gauss-Newton
      // curvature) at distance dd along the bearing, over the whole window
      auto eval = [&](float dd, float &j, float &g, float &h) {
        j = 0.0f;
        g = 0.0f;
        h = 0.0f;
        for (int k = part; k < W; k += 4) {
          const float dx = fmaf(dd, ex, fr[0]) - w[3 * k], dy = fmaf(dd, ey, fr[1]) - w[3 * k + 1];
          const float dist = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy));
          const float rho = dist - w[3 * k + 2];
          j = fmaf(rho, rho, j);
          if (dist > 0.0f) {
            const float jd = fmaf(dx, ex, dy * ey) * __builtin_amdgcn_rcpf(dist);
            g = fmaf(jd, rho, g);
            h = fmaf(jd, jd, h);
          }
        }
        j = sum4(j);
        g = sum4(g);
        h = sum4(h);
      };
      float acc = 0.0f;
      if (fit) {
        float j, g, h;
        eval(d, j, g, h);
        for (int it = 0; it < kRefineIters && h > 0.0f; ++it) {
          const float dn = d - g * __builtin_amdgcn_rcpf(h);
          float j1, g1, h1;
          eval(dn, j1, g1, h1);
          if (!(j1 < j)) break;
          d = dn;
          j = j1;
          g = g1;
          h = h1;
        }
        px = fmaf(d, ex, fr[0]);
        py = fmaf(d, ey, fr[1]);
        acc = j;
      } else if (ok) {  // the network's point at the centroid itself: no bearing
        for (int k = part; k < W; k += 4) {
          const float dx = px - w[3 * k], dy = py - w[3 * k + 1];
          const float res = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy)) - w[3 * k + 2];
          acc = fmaf(res, res, acc);
        }
        acc = sum4(acc);
      }
      bool accept = false, fail = false;
      if (live && part == 0) {
        accept = ok && __builtin_amdgcn_sqrtf(acc * (1.0f / (float)W)) <= k_sigma * sigma[n];
        if (accept) {
          out[2 * n] = px;
          out[2 * n + 1] = py;
          flag[n] = 1;
        }
        fail = !accept;
      }
      // wavefront-aggregated append to the fallback list
      const uint64_t m = __ballot(fail);
      const int lane = tid & 63;
      int base = 0;
      if (lane == 0 && m) base = atomicAdd(fb_count, __popcll(m));
      base = __shfl(base, 0);
      if (fail) {
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        fb_list[base + rank] = (int32_t)n;
      }
    }
    __syncthreads();
  }
}

template <int WC>
__global__ void fallback_kernel(const float *__restrict__ win, int32_t W,
                                const int32_t *__restrict__ fb_count,
                                const int32_t *__restrict__ fb_list, int32_t gn_iters, float tau,
                                float *__restrict__ out, uint8_t *__restrict__ flag) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= *fb_count) return;
  const int64_t n = fb_list[idx];
  const float *w = win + n * W * 3;
  float hx[WC], hy[WC], hr[WC];
#pragma unroll
  for (int k = 0; k < WC; ++k) {
    const bool in = k < W;
    hx[k] = in ? w[3 * k] : 0.f;
    hy[k] = in ? w[3 * k + 1] : 0.f;
    hr[k] = in ? w[3 * k + 2] : __int_as_float(0x7fc00000);
  }
  double px = 0.0, py = 0.0;
  const bool ok = ls_masked<WC>(hx, hy, hr, W, gn_iters, (double)tau, px, py);
  out[2 * n] = ok ? (float)px : 0.0f;
  out[2 * n + 1] = ok ? (float)py : 0.0f;
  flag[n] = ok ? 0 : 2;
}

__global__ void zero_i32_kernel(int32_t *p) { *p = 0; }

// Glorot-uniform init: weight (o, i) of a layer with fan_in + fan_out = f
// is a * (2u - 1), a = sqrt(6 / f), u from Philox(counter = (index, 0, 0,
// kPurposeMlpInit)); biases 0.
__global__ void init_kernel(float *th, uint32_t k0, uint32_t k1) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNumParams) return;
  float a = 0.0f;
  if (p < kOffB1) a = sqrtf(6.0f / (kIn + kHidden));
  else if (p >= kOffW2 && p < kOffB2) a = sqrtf(6.0f / (kHidden + kHidden));
  else if (p >= kOffW3 && p < kOffB3) a = sqrtf(6.0f / (kHidden + kOut));
  const u32x4 x = philox4x32_10((uint32_t)p, 0u, 0u, kPurposeMlpInit, k0, k1);
  th[p] = a * (2.0f * u01(x.x) - 1.0f);
}

int launch_init(float *th, uint64_t seed, void *stream) {
  hipLaunchKernelGGL(init_kernel, dim3((kNumParams + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, th, (uint32_t)seed, (uint32_t)(seed >> 32));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int ok_launch() { return hipGetLastError() == hipSuccess ? 0 : -1; }

// Dynamic LDS above 64 KB has to be requested per kernel (gfx950 has 160 KB).
static int allow_lds(const void *kernel, size_t bytes) {
  if (bytes <= 65536) return 0;
  return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
                 hipSuccess ? 0 : -1;
}

int launch_prepare(const float *th, int precision, void *prep, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int n = kHidden * kHidden, bs = 256;
  if (precision == 0) {
    __bf16 *w1 = (__bf16 *)prep, *w2 = w1 + kHidden * kLdIn, *w2t = w2 + kHidden * kLdH;
    hipLaunchKernelGGL(prepare_weights_kernel<__bf16>, dim3((n + bs - 1) / bs), dim3(bs), 0, st,
                       th, w1, w2, w2t);
  } else {
    float *w1 = (float *)prep, *w2 = w1 + kHidden * kLdIn, *w2t = w2 + kHidden * kLdH;
    hipLaunchKernelGGL(prepare_weights_kernel<float>, dim3((n + bs - 1) / bs), dim3(bs), 0, st,
                       th, w1, w2, w2t);
  }
  return ok_launch();
}

int launch_features(const float *win, int64_t N, int32_t W, float *x, float *frame, void *stream) {
  if (N <= 0) return 0;
  const int bs = 128;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((N + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, win, N, W, x, frame);
  return ok_launch();
}

int launch_targets(const float *frame, const float *p, int64_t N, float *y, void *stream) {
  if (N <= 0) return 0;
  const int bs = 256;
  hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((N + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, frame, p, N, y);
  return ok_launch();
}

int launch_forward(int64_t N, const float *x, const float *th, int precision, const void *prep,
                   float *y, void *stream) {
  if (N <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  const unsigned blocks = (unsigned)((N + 63) / 64);
  if (precision == 0) {
    const __bf16 *w1 = (const __bf16 *)prep, *w2 = w1 + kHidden * kLdIn;
    // persistent: as many blocks as fit the CUs, each looping over tiles
    static int per_cu = 0;  // resident blocks per CU (registers and LDS decide)
    if (per_cu == 0 &&
        (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)forward_bf16_kernel,
                                                      256, sizeof(FwdBfLds)) != hipSuccess ||
         per_cu < 1))
      per_cu = 1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    const int64_t slots = (int64_t)per_cu * cus;
    const unsigned grid = (unsigned)((int64_t)blocks < slots ? blocks : slots);
    hipLaunchKernelGGL(forward_bf16_kernel, dim3(grid), dim3(256), sizeof(FwdBfLds), st, N, x, th,
                       w1, w2, y);
  } else {
    const float *w1 = (const float *)prep, *w2 = w1 + kHidden * kLdIn;
    if (allow_lds((const void *)forward_kernel<float>, sizeof(FwdLds<float>))) return -1;
    hipLaunchKernelGGL(forward_kernel<float>, dim3(blocks), dim3(256), sizeof(FwdLds<float>), st,
                       N, x, th, w1, w2, y);
  }
  return ok_launch();
}

int64_t train_blocks(int64_t N, int precision) {
  if (precision == 0) {
    const int64_t tiles = (N + kStepS - 1) / kStepS;
    return tiles < kTrainBlocks ? tiles : kTrainBlocks;
  }
  return (N + kTileF32 - 1) / kTileF32;
}

int64_t train_partial_floats(int precision) {
  return precision == 0 ? kPartFloats : kNumParams;
}

// BF16: the persistent accumulation kernel, then the fixed-order reduction
// (with the Adam update of the same parameters when m and v are given).
static int launch_step_bf16(int64_t N, const float *x, const int64_t *index, const float *target,
                            float *th, float *partial, float *loss_partial, float *grad,
                            float *loss, float *m, float *v, float lr, float b1, float b2,
                            float eps, int32_t step, hipStream_t st) {
  const int64_t ntiles = (N + kStepS - 1) / kStepS;
  const int64_t nb = train_blocks(N, 0);
  const float inv_n = 1.0f / (float)N;
  if (allow_lds((const void *)train_accum_kernel, sizeof(StepLds))) return -1;
  hipLaunchKernelGGL(train_accum_kernel, dim3((unsigned)nb), dim3(256), sizeof(StepLds), st, N,
                     ntiles, x, index, target, th, partial, loss_partial, inv_n);
  if (ok_launch()) return -1;
  const bool adam = m && v;
  const float c1 = adam ? 1.0f - powf(b1, (float)step) : 1.0f;
  const float c2 = adam ? 1.0f - powf(b2, (float)step) : 1.0f;
  constexpr int ncol = kPartFloats / 4;
  hipLaunchKernelGGL(reduce_step_kernel, dim3((ncol + 31) / 32), dim3(256), 0, st, partial,
                     (int)nb, grad, loss_partial, loss, inv_n, adam ? 1 : 0, th, m, v, lr, b1, b2,
                     eps, c1, c2);
  return ok_launch();
}

int launch_train_step(int64_t N, const float *x, const int64_t *index, const float *target,
                      float *th, float *m, float *v, float lr, float b1, float b2, float eps,
                      int32_t step, float *partial, float *loss_partial, float *grad, float *loss,
                      void *stream) {
  if (N <= 0) return 0;
  return launch_step_bf16(N, x, index, target, th, partial, loss_partial, grad, loss, m, v, lr,
                          b1, b2, eps, step, (hipStream_t)stream);
}

int launch_train(int64_t N, const float *x, const int64_t *index, const float *target,
                 const float *th, int precision, const void *prep, float *partial,
                 float *loss_partial, float *grad, float *loss, void *stream) {
  if (N <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  const int64_t nb = train_blocks(N, precision);
  const float inv_n = 1.0f / (float)N;
  if (precision == 0) {
    return launch_step_bf16(N, x, index, target, const_cast<float *>(th), partial, loss_partial,
                            grad, loss, nullptr, nullptr, 0.f, 0.f, 0.f, 0.f, 1, st);
  } else {
    const float *w1 = (const float *)prep, *w2 = w1 + kHidden * kLdIn, *w2t = w2 + kHidden * kLdH;
    if (allow_lds((const void *)train_tile_kernel<float, kTileF32>, sizeof(TrainLds<float, kTileF32>)))
      return -1;
    hipLaunchKernelGGL((train_tile_kernel<float, kTileF32>), dim3((unsigned)nb), dim3(256),
                       sizeof(TrainLds<float, kTileF32>), st, N, x, index, target, th, w1, w2,
                       w2t, partial, loss_partial, inv_n);
  }
  if (ok_launch()) return -1;
  hipLaunchKernelGGL(reduce_grad_kernel, dim3((kNumParams + 63) / 64), dim3(256), 0, st,
                     partial, (int)nb, grad, loss_partial, loss, inv_n);
  return ok_launch();
}

int launch_adam(int64_t P, float *th, const float *g, float *m, float *v, float lr, float b1,
                float b2, float eps, int32_t step, void *stream) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  const int bs = 256;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((P + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, P, th, g, m, v, lr, b1, b2, eps, c1, c2);
  return ok_launch();
}

int launch_infer(const float *win, int64_t N, int32_t W, const float *th, const void *prep,
                 const float *sigma, float k_sigma, int32_t gn_iters, float tau, float *out,
                 uint8_t *flag, int32_t *fb_count, int32_t *fb_list, int num_cus, void *stream) {
  if (N <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  const __bf16 *w1 = (const __bf16 *)prep, *w2 = w1 + kHidden * kLdIn;
  if (W < 3 || W > kMaxW) return -1;
  if (allow_lds((const void *)infer_kernel, sizeof(InferLds))) return -1;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, st, fb_count);
  const int64_t ntiles = (N + 63) / 64;
  static int per_cu = 0;  // resident blocks per CU (registers and LDS decide)
  if (per_cu == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)infer_kernel, 256,
                                                     sizeof(InferLds)) != hipSuccess ||
        per_cu < 1)
      per_cu = 2;
  }
  const int64_t slots = (int64_t)per_cu * num_cus;
  const unsigned grid = (unsigned)(ntiles < slots ? ntiles : slots);
  hipLaunchKernelGGL(infer_kernel, dim3(grid), dim3(256), sizeof(InferLds), st, win, N, W, th, w1,
                     w2, sigma, k_sigma, out, flag, fb_count, fb_list);
  if (ok_launch()) return -1;
  const unsigned fb_blocks = (unsigned)((N + 255) / 256);
  if (W <= 16)
    hipLaunchKernelGGL(fallback_kernel<16>, dim3(fb_blocks), dim3(256), 0, st, win, W, fb_count,
                       fb_list, gn_iters, tau, out, flag);
  else
    hipLaunchKernelGGL(fallback_kernel<21>, dim3(fb_blocks), dim3(256), 0, st, win, W, fb_count,
                       fb_list, gn_iters, tau, out, flag);
  return ok_launch();
}

}  // namespace mil
