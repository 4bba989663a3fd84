// Training form of the attention networks (the learner's update: MAPPO's
// gradient step, Sec. III-B, through the TransfMAPPO actor and critic of
// Fig. 3): the per-row and per-(agent, head) parts of an FP32 forward pass
// that keeps every intermediate on a tape, and of its exact reverse pass,
// plus the weight gradients summed over all rows (FP32 matrix cores) and
// the bias / LayerNorm column sums. The other dense products (each layer's
// projections and their input gradients) are plain FP32 GEMMs issued by the
// host side (train_abi.cpp).
//
// Rows: an agent's n_tok rows are consecutive ([A][n_tok][64] residual
// stream); in the recurrent form its first row is the carried state and its
// n_tok - 1 observed tokens follow.
#include <hip/hip_runtime.h>
#include <math.h>

#include "policy_internal.h"
#include "train_internal.h"

namespace mil {
namespace {

constexpr int kTrThreads = 256;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ float gelu_tanh(float x) {
  const float c = 0.7978845608028654f;  // sqrt(2 / pi)
  return 0.5f * x * (1.0f + tanhf(c * (x + 0.044715f * x * x * x)));
}

__device__ __forceinline__ float gelu_tanh_grad(float x) {
  const float c = 0.7978845608028654f;
  const float t = tanhf(c * (x + 0.044715f * x * x * x));
  return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * x * x);
}

// Thread (row r, feature d): the row's embedding E x + e (or the carried
// state), its augmented input (x, 1) for the embedding gradient (zeros for
// the carried row) and its key mask.
__global__ void __launch_bounds__(kTrThreads)
embed_kernel(const float *__restrict__ obs, const uint8_t *__restrict__ mask, int64_t R, int nt,
             int rec, const float *__restrict__ hidden, const float *__restrict__ prm,
             float *__restrict__ h, float *__restrict__ xaug, uint8_t *__restrict__ mrow) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * kPolD) return;
  const int64_t r = i / kPolD;
  const int d = (int)(i - r * kPolD);
  const int64_t a = r / nt;
  const int k = (int)(r - a * nt);
  const float *E = prm + kPolOffEmbW, *e = prm + kPolOffEmbB;
  if (rec && k == 0) {
    h[i] = hidden ? hidden[a * kPolD + d] : 0.0f;
    if (d < 8) xaug[r * 8 + d] = 0.0f;
    if (d == 0) mrow[r] = 1;
    return;
  }
  const int64_t orow = rec ? a * (nt - 1) + (k - 1) : r;
  const float *x = obs + orow * 6;
  float acc = e[d];
#pragma unroll
  for (int c = 0; c < 6; ++c) acc = fmaf(E[d * 6 + c], x[c], acc);
  h[i] = acc;
  if (d < 6) xaug[r * 8 + d] = x[d];
  if (d == 6) xaug[r * 8 + 6] = 1.0f;
  if (d == 7) xaug[r * 8 + 7] = 0.0f;
  if (d == 0) mrow[r] = mask[orow];
}

// One wavefront per row, lane d = feature d.
__global__ void __launch_bounds__(kTrThreads)
layernorm_kernel(const float *__restrict__ x, const float *__restrict__ g,
                 const float *__restrict__ b, float *__restrict__ y, int64_t R) {
  const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int d = threadIdx.x & 63;
  if (r >= R) return;
  const float v = x[r * kPolD + d];
  const float m = wave_sum(v) * (1.0f / kPolD);
  const float c = v - m;
  const float rs = rsqrtf(wave_sum(c * c) * (1.0f / kPolD) + 1e-5f);
  y[r * kPolD + d] = fmaf(c * rs, g[d], b[d]);
}

// out[r][n] = base[r][n] (or 0) + bias[n]: a GEMM then adds its product.
__global__ void __launch_bounds__(kTrThreads)
bias_rows_kernel(const float *__restrict__ base, const float *__restrict__ bias, int64_t R, int N,
                 float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * N) return;
  const int n = (int)(i % N);
  out[i] = (base ? base[i] : 0.0f) + bias[n];
}

// Feed-forward up-projection fused with its bias and GELU: z = X W1^T + b1
// and f = GELU(z) for X [R][64], W1 [256][64], both written (the tape keeps
// z for the derivative and f for W2's weight gradient). FP32 matrix cores,
// v_mfma_f32_16x16x4f32 on the transposed product z^T = W1 X^T; persistent
// blocks of eight wavefronts share W1 (rows padded to 68 floats) and b1 in
// LDS, each wavefront takes 16-row tiles across all 256 outputs (16 n-blocks).
// Lane l = (m, kk) = (l%16, l/16) holds row m's inputs 16kk..16kk+15 as four
// float4s; virtual k-step (g, c) pairs A[i][kk] = W1[i][16kk + 4g + c] with
// B[kk][m] = X[m][16kk + 4g + c], so the 16 steps sum over all 64 inputs.
// Lane l receives D[4(l/16)+v][l%16] = z[row m][column 4kk + v of the
// n-block]: four consecutive outputs of one row, stored as a float4.
constexpr int kFfnThreads = 512, kFfnLd = kPolD + 4;
typedef float ffn_f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kFfnThreads, 4)  // 4 waves per SIMD: two blocks per CU
ffn_up_kernel(const float *__restrict__ X, const float *__restrict__ W1,
              const float *__restrict__ b1, float *__restrict__ z, float *__restrict__ f,
              int64_t R) {
  extern __shared__ float ffn_w[];  // [256][kFfnLd], then b1 [256]
  float *ffn_b = ffn_w + kPolF * kFfnLd;
  for (int e = threadIdx.x; e < kPolF * kPolD; e += kFfnThreads)
    ffn_w[(e / kPolD) * kFfnLd + (e % kPolD)] = W1[e];
  for (int e = threadIdx.x; e < kPolF; e += kFfnThreads) ffn_b[e] = b1[e];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, kk = lane >> 4;
  const int64_t tiles = (R + 15) / 16;
  const int64_t nw = (int64_t)gridDim.x * (kFfnThreads / 64);
  const ffn_f32x4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t tile = (int64_t)blockIdx.x * (kFfnThreads / 64) + (threadIdx.x >> 6); tile < tiles;
       tile += nw) {
    const int64_t row = tile * 16 + m;
    const bool in = row < R;
    ffn_f32x4 xa[4];
    const ffn_f32x4 *xr = reinterpret_cast<const ffn_f32x4 *>(X + row * kPolD + 16 * kk);
#pragma unroll
    for (int g = 0; g < 4; ++g) xa[g] = in ? xr[g] : zero4;
    // two n-blocks at a time (independent accumulator chains), each finished
    // and stored before the next pair, so few accumulators are live
#pragma unroll 1
    for (int nb = 0; nb < kPolF / 16; nb += 2) {
      ffn_f32x4 acc0 = zero4, acc1 = zero4;
      const float *wr0 = ffn_w + (nb * 16 + m) * kFfnLd + 16 * kk;  // lane (i = m, kk)
      const float *wr1 = wr0 + 16 * kFfnLd;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const ffn_f32x4 wa0 = *reinterpret_cast<const ffn_f32x4 *>(wr0 + 4 * g);
        const ffn_f32x4 wa1 = *reinterpret_cast<const ffn_f32x4 *>(wr1 + 4 * g);
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa0[cc], xa[g][cc], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa1[cc], xa[g][cc], acc1, 0, 0, 0);
        }
      }
      if (in) {
        const int n0 = nb * 16 + 4 * kk;
        const ffn_f32x4 z0 = acc0 + *reinterpret_cast<const ffn_f32x4 *>(ffn_b + n0);
        const ffn_f32x4 z1 = acc1 + *reinterpret_cast<const ffn_f32x4 *>(ffn_b + n0 + 16);
        *reinterpret_cast<ffn_f32x4 *>(z + row * kPolF + n0) = z0;
        *reinterpret_cast<ffn_f32x4 *>(z + row * kPolF + n0 + 16) = z1;
        *reinterpret_cast<ffn_f32x4 *>(f + row * kPolF + n0) =
            ffn_f32x4{gelu_tanh(z0[0]), gelu_tanh(z0[1]), gelu_tanh(z0[2]), gelu_tanh(z0[3])};
        *reinterpret_cast<ffn_f32x4 *>(f + row * kPolF + n0 + 16) =
            ffn_f32x4{gelu_tanh(z1[0]), gelu_tanh(z1[1]), gelu_tanh(z1[2]), gelu_tanh(z1[3])};
      }
    }
  }
}

// LayerNorm on float4s: 16 lanes per row (lane q: features 4q..4q+3), four
// rows per wavefront; row sums over the 16 lanes by a fixed butterfly.
__device__ __forceinline__ float row16_sum(float v) {
#pragma unroll
  for (int m = 8; m >= 1; m >>= 1) v += __shfl_xor(v, m, 16);
  return v;
}

__global__ void __launch_bounds__(kTrThreads)
layernorm4_kernel(const float4 *__restrict__ x, const float *__restrict__ g,
                  const float *__restrict__ b, float4 *__restrict__ y, int64_t R) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = t >> 4;
  const int q = (int)(t & 15);
  if (r >= R) return;  // whole 16-lane groups leave together
  const float4 v = x[r * (kPolD / 4) + q];
  const float m = row16_sum((v.x + v.y) + (v.z + v.w)) * (1.0f / kPolD);
  const float c0 = v.x - m, c1 = v.y - m, c2 = v.z - m, c3 = v.w - m;
  const float var = row16_sum((c0 * c0 + c1 * c1) + (c2 * c2 + c3 * c3)) * (1.0f / kPolD);
  const float rs = rsqrtf(var + 1e-5f);
  const int d = 4 * q;
  y[r * (kPolD / 4) + q] = make_float4(fmaf(c0 * rs, g[d], b[d]), fmaf(c1 * rs, g[d + 1], b[d + 1]),
                                       fmaf(c2 * rs, g[d + 2], b[d + 2]),
                                       fmaf(c3 * rs, g[d + 3], b[d + 3]));
}

// Reverse passes fused with the column sums of what they produce (bias and
// LayerNorm gradients), so that the tape is not read again for those: rows
// split into kCsBlocks blocks of `per` rows, each block's FP64 sums combined
// in a fixed order into part[block], the partials then added by
// colsum_final_kernel / sums3_final_kernel.
constexpr int kCsBlocks = 1024;

// dz *= GELU'(z) in place (rows of F = 256), and the column sums of the
// result (the first feed-forward bias's gradient). Thread (row slot s,
// quad q) = (tid / 64, tid % 64): four row slots, four rows in flight each;
// kGbBlocks blocks.
constexpr int kGbBlocks = 2048;
__global__ void __launch_bounds__(256)
gelu_back_sums_kernel(float4 *__restrict__ dz, const float4 *__restrict__ z, int64_t R,
                      int64_t per, double *__restrict__ part) {
  __shared__ double red[4][kPolF];
  const int s = threadIdx.x >> 6, q = threadIdx.x & 63;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < R ? r0 + per : R;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r = r0 + s; r < r1; r += 16) {  // rows r, r + 4, r + 8, r + 12 in flight
    float4 v[4], d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t ru = r + 4 * u < r1 ? r + 4 * u : r;  // past the end: reread row r
      v[u] = z[ru * (kPolF / 4) + q];
      d[u] = dz[ru * (kPolF / 4) + q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (r + 4 * u < r1) {
        d[u].x *= gelu_tanh_grad(v[u].x);
        d[u].y *= gelu_tanh_grad(v[u].y);
        d[u].z *= gelu_tanh_grad(v[u].z);
        d[u].w *= gelu_tanh_grad(v[u].w);
        dz[(r + 4 * u) * (kPolF / 4) + q] = d[u];
        a[0] += (double)d[u].x;
        a[1] += (double)d[u].y;
        a[2] += (double)d[u].z;
        a[3] += (double)d[u].w;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) red[s][4 * q + k] = a[k];
  __syncthreads();
  const int col = threadIdx.x;  // 256 threads = 256 columns
  part[(int64_t)blockIdx.x * kPolF + col] =
      ((red[0][col] + red[1][col]) + red[2][col]) + red[3][col];
}

// LayerNorm's reverse pass on float4s (16 lanes per row as in the forward;
// dx added to dxacc) and the column sums of dy * xhat (the gain's gradient),
// dy (the bias's) and the updated dxacc (the gradient of the bias whose sum
// this LayerNorm normalised). Thread (row slot s, quad q) = (tid / 16,
// tid % 16): 16 row slots.
__global__ void __launch_bounds__(256)
layernorm_back_sums_kernel(const float4 *__restrict__ x, const float *__restrict__ g,
                           const float4 *__restrict__ dy, float4 *__restrict__ dxacc, int64_t R,
                           int64_t per, double *__restrict__ part) {
  __shared__ double red[16][3 * kPolD];
  const int s = threadIdx.x >> 4, q = threadIdx.x & 15;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < R ? r0 + per : R;
  float gq[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) gq[k] = g[4 * q + k];
  double sg[4] = {0.0, 0.0, 0.0, 0.0}, sb[4] = {0.0, 0.0, 0.0, 0.0}, sh[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r = r0 + s; r < r1; r += 16) {  // a row's 16 lanes share every trip
    const int64_t i = r * (kPolD / 4) + q;
    const float4 v = x[i];
    const float m = row16_sum((v.x + v.y) + (v.z + v.w)) * (1.0f / kPolD);
    const float c[4] = {v.x - m, v.y - m, v.z - m, v.w - m};
    const float var = row16_sum((c[0] * c[0] + c[1] * c[1]) + (c[2] * c[2] + c[3] * c[3])) *
                      (1.0f / kPolD);
    const float rs = rsqrtf(var + 1e-5f);
    const float4 gy4 = dy[i];
    const float gy[4] = {gy4.x, gy4.y, gy4.z, gy4.w};
    float xh[4], dxh[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      xh[k] = c[k] * rs;
      dxh[k] = gy[k] * gq[k];
    }
    const float s1 = row16_sum((dxh[0] + dxh[1]) + (dxh[2] + dxh[3])) * (1.0f / kPolD);
    const float s2 =
        row16_sum((dxh[0] * xh[0] + dxh[1] * xh[1]) + (dxh[2] * xh[2] + dxh[3] * xh[3])) *
        (1.0f / kPolD);
    const float4 a0 = dxacc[i];
    const float a[4] = {a0.x + rs * (dxh[0] - s1 - xh[0] * s2), a0.y + rs * (dxh[1] - s1 - xh[1] * s2),
                        a0.z + rs * (dxh[2] - s1 - xh[2] * s2), a0.w + rs * (dxh[3] - s1 - xh[3] * s2)};
    dxacc[i] = make_float4(a[0], a[1], a[2], a[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sg[k] += (double)(gy[k] * xh[k]);
      sb[k] += (double)gy[k];
      sh[k] += (double)a[k];
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    red[s][4 * q + k] = sg[k];
    red[s][kPolD + 4 * q + k] = sb[k];
    red[s][2 * kPolD + 4 * q + k] = sh[k];
  }
  __syncthreads();
  if (threadIdx.x < 3 * kPolD) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) t += red[k][threadIdx.x];
    part[(int64_t)blockIdx.x * 3 * kPolD + threadIdx.x] = t;
  }
}

// Partials [nb][192] of layernorm_back_sums_kernel -> three 64-wide outputs
// (out2 may be NULL), one wavefront per column as in colsum_final_kernel.
__global__ void __launch_bounds__(256)
sums3_final_kernel(const double *__restrict__ part, int nb, int acc, float *__restrict__ out0,
                   float *__restrict__ out1, float *__restrict__ out2) {
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  float *out = col < kPolD ? out0 : (col < 2 * kPolD ? out1 : out2);
  if (col >= 3 * kPolD || !out) return;  // wavefront-uniform
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += part[(int64_t)b * 3 * kPolD + col];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
  const int d = col % kPolD;
  if (lane == 0) out[d] = acc ? out[d] + (float)s : (float)s;
}

// Attention of one agent per wavefront (a block of 64 threads): the agent's
// rows are staged in LDS with coalesced float4 loads, then lane (head h,
// query t) = (lane / 16, lane % 16) does that query's work; lanes t >= nt
// only help with the staging. Rows of Q/K/V hold [Q | K | V], 64 each, head h
// in columns 16h..16h+15.
constexpr int kAtThreads = 64;

__device__ __forceinline__ void lds_row16(const float *src, float (&v)[kPolDh]) {
#pragma unroll
  for (int c4 = 0; c4 < kPolDh / 4; ++c4) {
    const float4 x = reinterpret_cast<const float4 *>(src)[c4];
    v[4 * c4] = x.x;
    v[4 * c4 + 1] = x.y;
    v[4 * c4 + 2] = x.z;
    v[4 * c4 + 3] = x.w;
  }
}

// Copy n 16-byte words (1 <= n <= 64 * MAXV) from global memory to LDS,
// every load of the lane issued before its first LDS write (lanes past the
// end re-read word n - 1 and write nothing).
typedef float at_f32x4 __attribute__((ext_vector_type(4)));
template <int MAXV>
__device__ __forceinline__ void stage_lds(void *dst, const void *__restrict__ src, int n,
                                          int lane) {
  const at_f32x4 *s = reinterpret_cast<const at_f32x4 *>(src);
  at_f32x4 *d = reinterpret_cast<at_f32x4 *>(dst);
  at_f32x4 v[MAXV];
#pragma unroll
  for (int k = 0; k < MAXV; ++k) {
    const int e = lane + k * kAtThreads;
    v[k] = s[e < n ? e : n - 1];
  }
#pragma unroll
  for (int k = 0; k < MAXV; ++k) {
    const int e = lane + k * kAtThreads;
    if (e < n) d[e] = v[k];
  }
}

__device__ __forceinline__ void store_row16(float *dst, const float (&v)[kPolDh]) {
#pragma unroll
  for (int c4 = 0; c4 < kPolDh / 4; ++c4)
    reinterpret_cast<float4 *>(dst)[c4] =
        make_float4(v[4 * c4], v[4 * c4 + 1], v[4 * c4 + 2], v[4 * c4 + 3]);
}

// Forward: scores q.k / 4 over the agent's unmasked keys, softmax (kept in
// P [agent][head][query][key]), and the head's output o = P V.
__global__ void __launch_bounds__(kAtThreads)
attention_kernel(const float *__restrict__ qkv, const uint8_t *__restrict__ mrow, int nt,
                 float *__restrict__ P, float *__restrict__ o) {
  extern __shared__ float4 at_lds[];  // [nt][48]: the agent's Q/K/V rows
  const int64_t a = blockIdx.x;
  const int64_t r0 = a * nt;
  const int lane = threadIdx.x;
  constexpr int kQkv4 = kPolMaxTok * 3 * kPolD / 4 / kAtThreads;  // float4s per lane, at most
  stage_lds<kQkv4>(at_lds, qkv + r0 * 3 * kPolD, nt * 3 * kPolD / 4, lane);
  __syncthreads();
  const int hd = lane >> 4, t = lane & 15;
  if (t >= nt) return;  // no barrier follows
  const float *sq = reinterpret_cast<const float *>(at_lds);
  float q[kPolDh];
  lds_row16(sq + t * 3 * kPolD + hd * kPolDh, q);
  float s[kPolMaxTok];
  float mx = -INFINITY;
#pragma unroll
  for (int u = 0; u < kPolMaxTok; ++u) {
    s[u] = -INFINITY;
    if (u < nt && mrow[r0 + u]) {
      float k[kPolDh];
      lds_row16(sq + u * 3 * kPolD + kPolD + hd * kPolDh, k);
      float acc = 0.0f;
#pragma unroll
      for (int c = 0; c < kPolDh; ++c) acc = fmaf(q[c], k[c], acc);
      s[u] = acc * 0.25f;
      mx = fmaxf(mx, s[u]);
    }
  }
  float z = 0.0f;
#pragma unroll
  for (int u = 0; u < kPolMaxTok; ++u) {
    if (u < nt) {
      s[u] = mrow[r0 + u] ? expf(s[u] - mx) : 0.0f;
      z += s[u];
    }
  }
  const float iz = 1.0f / z;
  float *pr = P + ((a * kPolHeads + hd) * nt + t) * nt;
  float acc[kPolDh];
#pragma unroll
  for (int c = 0; c < kPolDh; ++c) acc[c] = 0.0f;
#pragma unroll
  for (int u = 0; u < kPolMaxTok; ++u) {
    if (u < nt) {
      const float p = s[u] * iz;
      pr[u] = p;
      float v[kPolDh];
      lds_row16(sq + u * 3 * kPolD + 2 * kPolD + hd * kPolDh, v);
#pragma unroll
      for (int c = 0; c < kPolDh; ++c) acc[c] = fmaf(p, v[c], acc[c]);
    }
  }
  store_row16(o + (r0 + t) * kPolD + hd * kPolDh, acc);
}

// Reverse pass of attention_kernel, same layout (LDS: the agent's Q/K/V
// rows, output gradients dO, probabilities P and score gradients dS).
// Lane (h, t): dP[u] = dO[t] . V[u], dS[t][u] = P (dP - sum_u P dP) / 4,
// dQ[t] = dS[t] K; after the block's barrier, as lane (h, x) with x = t:
// dK[x] = sum_t dS[t][x] Q[t], dV[x] = sum_t P[t][x] dO[t].
__global__ void __launch_bounds__(kAtThreads)
attention_back_kernel(const float *__restrict__ qkv, const float *__restrict__ P,
                      const uint8_t *__restrict__ mrow, const float *__restrict__ dout, int nt,
                      float *__restrict__ dqkv) {
  extern __shared__ float4 ab_lds[];  // [nt][48] Q/K/V | [nt][16] dO | [4 nt nt / 4] P | dS
  const int64_t a = blockIdx.x;
  const int64_t r0 = a * nt;
  const int lane = threadIdx.x;
  const int nqkv = nt * 3 * kPolD / 4, ndo = nt * kPolD / 4, np = kPolHeads * nt * nt / 4;
  {
    // all three copies as one: every load in flight before the first LDS write
    constexpr int kAll4 = (kPolMaxTok * 3 * kPolD / 4 + kPolMaxTok * kPolD / 4 +
                           kPolHeads * kPolMaxTok * kPolMaxTok / 4) / kAtThreads;
    const at_f32x4 *s1 = reinterpret_cast<const at_f32x4 *>(qkv + r0 * 3 * kPolD);
    const at_f32x4 *s2 = reinterpret_cast<const at_f32x4 *>(dout + r0 * kPolD);
    const at_f32x4 *s3 = reinterpret_cast<const at_f32x4 *>(P + a * kPolHeads * nt * nt);
    at_f32x4 *d = reinterpret_cast<at_f32x4 *>(ab_lds);
    const int n = nqkv + ndo + np;
    at_f32x4 v[kAll4];
#pragma unroll
    for (int k = 0; k < kAll4; ++k) {
      const int e0 = lane + k * kAtThreads, e = e0 < n ? e0 : n - 1;
      v[k] = e < nqkv ? s1[e] : (e < nqkv + ndo ? s2[e - nqkv] : s3[e - nqkv - ndo]);
    }
#pragma unroll
    for (int k = 0; k < kAll4; ++k)
      if (lane + k * kAtThreads < n) d[lane + k * kAtThreads] = v[k];
  }
  __syncthreads();
  float *const base = reinterpret_cast<float *>(ab_lds);
  const float *sq = base, *so = base + 4 * nqkv, *sp = so + 4 * ndo;
  float *sd = base + 4 * (nqkv + ndo + np);
  const int hd = lane >> 4, t = lane & 15;
  const bool live = t < nt;
  float dq[kPolDh];
#pragma unroll
  for (int c = 0; c < kPolDh; ++c) dq[c] = 0.0f;
  if (live) {
    float dot[kPolDh];
    lds_row16(so + t * kPolD + hd * kPolDh, dot);
    const float *prow = sp + (hd * nt + t) * nt;
    float dp[kPolMaxTok];
    float ssum = 0.0f;
#pragma unroll
    for (int u = 0; u < kPolMaxTok; ++u) {
      dp[u] = 0.0f;
      if (u < nt) {
        float v[kPolDh];
        lds_row16(sq + u * 3 * kPolD + 2 * kPolD + hd * kPolDh, v);
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < kPolDh; ++c) acc = fmaf(dot[c], v[c], acc);
        dp[u] = acc;
      }
    }
#pragma unroll
    for (int u = 0; u < kPolMaxTok; ++u)
      if (u < nt) ssum = fmaf(prow[u], dp[u], ssum);
    float *drow = sd + (hd * nt + t) * nt;
#pragma unroll
    for (int u = 0; u < kPolMaxTok; ++u) {
      if (u < nt) {
        // a masked key has probability 0 and takes no gradient
        const float ds = mrow[r0 + u] ? prow[u] * (dp[u] - ssum) * 0.25f : 0.0f;
        drow[u] = ds;
        float k[kPolDh];
        lds_row16(sq + u * 3 * kPolD + kPolD + hd * kPolDh, k);
#pragma unroll
        for (int c = 0; c < kPolDh; ++c) dq[c] = fmaf(ds, k[c], dq[c]);
      }
    }
  }
  __syncthreads();  // every lane's dS row is in LDS
  if (!live) return;
  const int x = t;
  float dk[kPolDh], dv[kPolDh];
#pragma unroll
  for (int c = 0; c < kPolDh; ++c) {
    dk[c] = 0.0f;
    dv[c] = 0.0f;
  }
#pragma unroll
  for (int tq = 0; tq < kPolMaxTok; ++tq) {
    if (tq < nt) {
      const float ds = sd[(hd * nt + tq) * nt + x], p = sp[(hd * nt + tq) * nt + x];
      float qv[kPolDh], ov[kPolDh];
      lds_row16(sq + tq * 3 * kPolD + hd * kPolDh, qv);
      lds_row16(so + tq * kPolD + hd * kPolDh, ov);
#pragma unroll
      for (int c = 0; c < kPolDh; ++c) {
        dk[c] = fmaf(ds, qv[c], dk[c]);
        dv[c] = fmaf(p, ov[c], dv[c]);
      }
    }
  }
  float *row = dqkv + (r0 + x) * 3 * kPolD + hd * kPolDh;
  store_row16(row, dq);
  store_row16(row + kPolD, dk);
  store_row16(row + 2 * kPolD, dv);
}

// Weight-gradient partials on the FP32 matrix cores: dW [N][K] = sum over
// rows r of dY[r][n] X[r][k], as v_mfma_f32_16x16x4f32 products with
// A = dY^T (16 n x 4 rows) and B = X (4 rows x 16 k), four rows of the sum
// per instruction. Block b (four wavefronts) takes rows [b per, (b+1) per)
// and writes its sums to part[b]; wavefront w holds the n-blocks
// [w NBW, (w+1) NBW) against every 16-wide k-block. Lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and receives D[4(l/16)+v][l%16] in accumulator v. Rows
// past the block's end are read as 0. Each block's sum runs over its rows in
// order, so the result does not depend on the run.
typedef float wg_floatx4 __attribute__((ext_vector_type(4)));
constexpr int kWgThreads = 256;

template <int NBW, int K>
__global__ void __launch_bounds__(kWgThreads)
wgrad_kernel(const float *__restrict__ dY, const float *__restrict__ X, int64_t R, int64_t per,
             float *__restrict__ part) {
  constexpr int N = NBW * 64, KB = (K + 15) / 16;  // K < 16: lanes past K read 0, write nothing
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rl = lane >> 4, cl = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < R ? r0 + per : R;
  wg_floatx4 acc[NBW][KB];
#pragma unroll
  for (int i = 0; i < NBW; ++i)
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[i][j] = wg_floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  const float *ya = dY + w * NBW * 16 + cl;
  const float *xb = X + cl;
  for (int64_t r = r0; r < r1; r += 16) {
    float a[4][NBW], b[4][KB];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t row = r + 4 * s + rl;
      const bool in = row < r1;
#pragma unroll
      for (int i = 0; i < NBW; ++i) a[s][i] = in ? ya[row * N + i * 16] : 0.0f;
#pragma unroll
      for (int j = 0; j < KB; ++j) b[s][j] = (in && j * 16 + cl < K) ? xb[row * K + j * 16] : 0.0f;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < NBW; ++i)
#pragma unroll
        for (int j = 0; j < KB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s][i], b[s][j], acc[i][j], 0, 0, 0);
  }
  float *pb = part + (int64_t)blockIdx.x * N * K;
#pragma unroll
  for (int i = 0; i < NBW; ++i)
#pragma unroll
    for (int j = 0; j < KB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (j * 16 + cl < K) pb[((w * NBW + i) * 16 + 4 * rl + v) * K + j * 16 + cl] = acc[i][j][v];
}

// The same sums with float4 loads, one 64 x 64 output tile per wavefront
// (block = TN x TK wavefronts, wavefront w the tile (w / TK, w % TK)): lane l
// reads columns 4(l%16)..4(l%16)+3 of the tile's 64 in row l/16 of a 4-row
// slab, for dY and for X, and component i of each is the fragment of
// virtual 16-column block i. So virtual block i of the tile holds columns
// 4c + i (c = 0..15), and D_ij[m][c] is dW[tile n0 + 4m + i][tile k0 + 4c + j];
// lane l, accumulator v holds m = 4(l/16) + v, so its four j values are
// four consecutive k and leave as one float4.
typedef float wg4_f32x4 __attribute__((ext_vector_type(4)));
template <int TN, int TK>
__global__ void __launch_bounds__(64 * TN * TK)
wgrad4_kernel(const float *__restrict__ dY, const float *__restrict__ X, int64_t R, int64_t per,
              float *__restrict__ part) {
  constexpr int N = TN * 64, K = TK * 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tn = w / TK, tk = w - tn * TK;
  const int rl = lane >> 4, cl = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < R ? r0 + per : R;
  wg4_f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = wg4_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const wg4_f32x4 *ya = reinterpret_cast<const wg4_f32x4 *>(dY + tn * 64) + cl;
  const wg4_f32x4 *xb = reinterpret_cast<const wg4_f32x4 *>(X + tk * 64) + cl;
  const wg4_f32x4 zero4 = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t r = r0; r < r1; r += 16) {
    wg4_f32x4 a[4], b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t row = r + 4 * s + rl;
      const bool in = row < r1;
      a[s] = in ? ya[row * (N / 4)] : zero4;
      b[s] = in ? xb[row * (K / 4)] : zero4;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s][i], b[s][j], acc[i][j], 0, 0, 0);
  }
  float *pb = part + (int64_t)blockIdx.x * N * K;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = tn * 64 + 4 * (4 * rl + v) + i;
      *reinterpret_cast<wg4_f32x4 *>(pb + (int64_t)n * K + tk * 64 + 4 * cl) =
          wg4_f32x4{acc[i][0][v], acc[i][1][v], acc[i][2][v], acc[i][3][v]};
    }
}

// out [n] (+)= sum over b < nb of part[b][n]: block = 64 outputs, wavefront
// w adds partials [w q, (w+1) q) in order (FP64), then the four sums are
// added in order.
__global__ void __launch_bounds__(kWgThreads)
wgrad_sum_kernel(const float *__restrict__ part, int nb, int64_t n, int acc,
                 float *__restrict__ out) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const int q = (nb + 3) / 4;
  const int b0 = w * q, b1 = b0 + q < nb ? b0 + q : nb;
  double s = 0.0;
  if (i < n) {
    int b = b0;
    for (; b + 7 < b1; b += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + u) * n + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; b < b1; ++b) s += (double)part[(int64_t)b * n + i];
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && i < n) {
    const double t = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    out[i] = acc ? out[i] + (float)t : (float)t;
  }
}

// Column sums of Y [R][N] (N <= 256) in two fixed-order passes: block b adds
// rows [b * per, (b + 1) * per) in FP64 (thread (group, column) with four
// running sums over its rows, groups combined in order), then one wavefront
// per column adds the blocks' partials (lane j: partials j, j + 64, ...;
// then a fixed butterfly). With N a multiple of 4 and Y 16-byte aligned the
// first pass reads float4s instead (thread (group, column quad), one running
// sum per column, four row loads in flight), which keeps enough bytes in
// flight to stream Y at close to HBM rate.

__global__ void __launch_bounds__(256)
colsum_partial4_kernel(const float4 *__restrict__ Y, int64_t R, int N, int64_t per,
                       double *__restrict__ part) {
  __shared__ double red[1024];
  const int nq = N >> 2;
  const int groups = 256 / nq;
  const int g = threadIdx.x / nq, q = threadIdx.x - g * nq;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < R ? r0 + per : R;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (g < groups) {
    int64_t r = r0 + g;
    for (; r + 3 * groups < r1; r += 4 * groups) {
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = Y[(r + u * groups) * nq + q];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        s0 += (double)v[u].x;
        s1 += (double)v[u].y;
        s2 += (double)v[u].z;
        s3 += (double)v[u].w;
      }
    }
    for (; r < r1; r += groups) {
      const float4 v = Y[r * nq + q];
      s0 += (double)v.x;
      s1 += (double)v.y;
      s2 += (double)v.z;
      s3 += (double)v.w;
    }
    double *o = red + g * N + 4 * q;  // groups * N <= 1024
    o[0] = s0;
    o[1] = s1;
    o[2] = s2;
    o[3] = s3;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0.0;
    for (int k = 0; k < groups; ++k) s += red[k * N + threadIdx.x];
    part[(int64_t)blockIdx.x * N + threadIdx.x] = s;
  }
}
__global__ void __launch_bounds__(256)
colsum_partial_kernel(const float *__restrict__ Y, int64_t R, int N, int64_t per,
                      double *__restrict__ part) {
  __shared__ double red[256];
  const int groups = 256 / N;
  const int g = threadIdx.x / N, col = threadIdx.x - g * N;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < R ? r0 + per : R;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (g < groups) {
    int64_t r = r0 + g;
    for (; r + 3 * groups < r1; r += 4 * groups) {
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += (double)Y[(r + q * groups) * N + col];
    }
    for (; r < r1; r += groups) acc[0] += (double)Y[r * N + col];
  }
  red[threadIdx.x] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0.0;
    for (int q = 0; q < groups; ++q) s += red[q * N + threadIdx.x];
    part[(int64_t)blockIdx.x * N + threadIdx.x] = s;
  }
}

__global__ void __launch_bounds__(256)
colsum_final_kernel(const double *__restrict__ part, int nb, int N, int acc,
                    float *__restrict__ out) {
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col >= N) return;  // wavefront-uniform
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += part[(int64_t)b * N + col];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
  if (lane == 0) out[col] = acc ? out[col] + (float)s : (float)s;
}

// Sum of nb partial matrices of n floats each, in order.
__global__ void __launch_bounds__(256)
sum_partials_kernel(const float *__restrict__ part, int nb, int64_t n, int acc,
                    float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += (double)part[(int64_t)b * n + i];
  out[i] = acc ? out[i] + (float)s : (float)s;
}

// One wavefront per agent: final LayerNorm of its first row and the head.
__global__ void __launch_bounds__(kTrThreads)
head_kernel(const float *__restrict__ h, int64_t A, int nt, const float *__restrict__ prm,
            float *__restrict__ logits, float *__restrict__ feat) {
  const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int d = threadIdx.x & 63;
  if (a >= A) return;
  const float *fp = prm + kPolOffFinal;
  const float v = h[a * nt * kPolD + d];
  const float m = wave_sum(v) * (1.0f / kPolD);
  const float c = v - m;
  const float rs = rsqrtf(wave_sum(c * c) * (1.0f / kPolD) + 1e-5f);
  const float s = fmaf(c * rs, fp[kPolLnfG + d], fp[kPolLnfB + d]);
  feat[a * kPolD + d] = s;
#pragma unroll
  for (int k = 0; k < kPolActions; ++k) {
    const float y = wave_sum(fp[kPolWh + k * kPolD + d] * s);
    if (d == 0 && logits) logits[a * kPolActions + k] = y + fp[kPolBh + k];
  }
}

// One wavefront per agent: the head's and the final LayerNorm's reverse
// pass. dl8 [A][8] = the output gradients padded with zeros (for the head's
// weight gradient), dh row 0 of the agent = the LayerNorm's input gradient
// (dh zero elsewhere beforehand), gfa / bfa [A][64] the per-agent terms of
// the final LayerNorm's gain and offset gradients. dnext [A][64] (may be
// null): an extra gradient at the LayerNorm's output.
__global__ void __launch_bounds__(kTrThreads)
head_back_kernel(const float *__restrict__ h, int64_t A, int nt, const float *__restrict__ prm,
                 const float *__restrict__ dout, int ld, int n_out, const float *__restrict__ dnext,
                 float *__restrict__ dl8, float *__restrict__ dh, float *__restrict__ gfa,
                 float *__restrict__ bfa) {
  const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int d = threadIdx.x & 63;
  if (a >= A) return;
  const float *fp = prm + kPolOffFinal;
  // the gradient at the head's input: from the outputs, plus (recurrent form)
  // the loss gradient at the state passed on to the next step
  float ds = dnext ? dnext[a * kPolD + d] : 0.0f;
#pragma unroll
  for (int k = 0; k < kPolActions; ++k) {
    const float gk = k < n_out ? dout[a * ld + k] : 0.0f;
    if (d == k) dl8[a * kPolActions + k] = gk;
    ds = fmaf(gk, fp[kPolWh + k * kPolD + d], ds);
  }
  const int64_t i = a * nt * kPolD + d;
  const float v = h[i];
  const float m = wave_sum(v) * (1.0f / kPolD);
  const float c = v - m;
  const float rs = rsqrtf(wave_sum(c * c) * (1.0f / kPolD) + 1e-5f);
  const float xh = c * rs;
  const float dxh = ds * fp[kPolLnfG + d];
  const float s1 = wave_sum(dxh) * (1.0f / kPolD), s2 = wave_sum(dxh * xh) * (1.0f / kPolD);
  dh[i] = rs * (dxh - s1 - xh * s2);
  gfa[a * kPolD + d] = ds * xh;
  bfa[a * kPolD + d] = ds;
}

// Embedding gradient [64][8] (E's six columns, e, padding) into the
// parameter layout.
__global__ void embed_grad_scatter_kernel(const float *__restrict__ gaug, int acc,
                                          float *__restrict__ grad) {
  const int i = threadIdx.x + blockIdx.x * blockDim.x;
  if (i >= kPolD * 7) return;
  const int d = i / 7, c = i - d * 7;
  float *dst = c < 6 ? grad + kPolOffEmbW + d * 6 + c : grad + kPolOffEmbB + d;
  const float v = gaug[d * 8 + c];
  *dst = acc ? *dst + v : v;
}

// The gradient at each agent's carried state (its first row).
__global__ void __launch_bounds__(kTrThreads)
first_rows_kernel(const float *__restrict__ dh, int64_t A, int nt, float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A * kPolD) return;
  const int64_t a = i / kPolD;
  out[i] = dh[a * nt * kPolD + (i - a * kPolD)];
}

__global__ void __launch_bounds__(kTrThreads)
fill_kernel(float *__restrict__ p, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

int check() { return hipGetLastError() == hipSuccess ? 0 : -1; }

dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kTrThreads - 1) / kTrThreads)); }

}  // namespace

int tr_embed(const float *obs, const uint8_t *mask, int64_t R, int nt, int rec,
             const float *hidden, const float *prm, float *h, float *xaug, uint8_t *mrow,
             void *stream) {
  if (R == 0) return 0;
  hipLaunchKernelGGL(embed_kernel, grid_for(R * kPolD), dim3(kTrThreads), 0, (hipStream_t)stream,
                     obs, mask, R, nt, rec, hidden, prm, h, xaug, mrow);
  return check();
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

int tr_layernorm(const float *x, const float *g, const float *b, float *y, int64_t R, void *stream) {
  if (R == 0) return 0;
  if (aligned16(x) && aligned16(y))
    hipLaunchKernelGGL(layernorm4_kernel, grid_for(R * 16), dim3(kTrThreads), 0,
                       (hipStream_t)stream, reinterpret_cast<const float4 *>(x), g, b,
                       reinterpret_cast<float4 *>(y), R);
  else
    hipLaunchKernelGGL(layernorm_kernel, grid_for(R * 64), dim3(kTrThreads), 0,
                       (hipStream_t)stream, x, g, b, y, R);
  return check();
}

int tr_bias_rows(const float *base, const float *bias, int64_t R, int N, float *out, void *stream) {
  if (R == 0) return 0;
  hipLaunchKernelGGL(bias_rows_kernel, grid_for(R * N), dim3(kTrThreads), 0, (hipStream_t)stream,
                     base, bias, R, N, out);
  return check();
}

int tr_ffn_up(const float *x, const float *w1, const float *b1, float *z, float *f, int64_t R,
              void *stream) {
  if (R == 0) return 0;
  if (!aligned16(x) || !aligned16(z) || !aligned16(f)) return -1;
  static int blocks[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  const size_t lds = (size_t)kPolF * (kFfnLd + 1) * sizeof(float);  // 69 KB: above the 64 KB default
  if (!blocks[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0 ||
        hipFuncSetAttribute((const void *)ffn_up_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return -1;
    blocks[dev] = 2 * cus;  // two blocks of W1 per CU
  }
  const int64_t tiles = (R + 15) / 16, waves = tiles < INT32_MAX ? tiles : INT32_MAX;
  const int64_t need = (waves + kFfnThreads / 64 - 1) / (kFfnThreads / 64);
  const unsigned nb = (unsigned)(need < blocks[dev] ? need : blocks[dev]);
  hipLaunchKernelGGL(ffn_up_kernel, dim3(nb), dim3(kFfnThreads), lds, (hipStream_t)stream, x, w1,
                     b1, z, f, R);
  return check();
}

int tr_gelu_back_sums(float *dz, const float *z, int64_t R, double *scratch, int acc,
                      float *bias_grad, void *stream) {
  if (R == 0) return 0;
  if (!aligned16(dz) || !aligned16(z)) return -1;
  hipStream_t st = (hipStream_t)stream;
  const int64_t per = (R + kGbBlocks - 1) / kGbBlocks;
  const int64_t nb = (R + per - 1) / per;
  hipLaunchKernelGGL(gelu_back_sums_kernel, dim3((unsigned)nb), dim3(256), 0, st,
                     reinterpret_cast<float4 *>(dz), reinterpret_cast<const float4 *>(z), R, per,
                     scratch);
  if (check()) return -1;
  hipLaunchKernelGGL(colsum_final_kernel, dim3(kPolF / 4), dim3(256), 0, st, scratch, (int)nb,
                     kPolF, acc, bias_grad);
  return check();
}

int tr_attention(const float *qkv, const uint8_t *mrow, int64_t A, int nt, float *P, float *o,
                 void *stream) {
  if (A == 0) return 0;
  if (nt < 1 || nt > kPolMaxTok || A > INT32_MAX || !aligned16(qkv) || !aligned16(o)) return -1;
  const size_t lds = (size_t)nt * 3 * kPolD * 4;
  hipLaunchKernelGGL(attention_kernel, dim3((unsigned)A), dim3(kAtThreads), lds,
                     (hipStream_t)stream, qkv, mrow, nt, P, o);
  return check();
}

int tr_attention_back(const float *qkv, const float *P, const uint8_t *mrow, const float *dout,
                      int64_t A, int nt, float *dqkv, void *stream) {
  if (A == 0) return 0;
  if (nt < 1 || nt > kPolMaxTok || A > INT32_MAX || !aligned16(qkv) || !aligned16(P) ||
      !aligned16(dout) || !aligned16(dqkv))
    return -1;
  const size_t lds = ((size_t)nt * 3 * kPolD + (size_t)nt * kPolD + 2 * kPolHeads * nt * nt) * 4;
  hipLaunchKernelGGL(attention_back_kernel, dim3((unsigned)A), dim3(kAtThreads), lds,
                     (hipStream_t)stream, qkv, P, mrow, dout, nt, dqkv);
  return check();
}

int64_t tr_colsum_scratch_doubles() {
  return (int64_t)(kCsBlocks > kGbBlocks ? kCsBlocks : kGbBlocks) * 256;
}

int tr_colsum(const float *Y, int64_t R, int N, double *scratch, int acc, float *out,
              void *stream) {
  if (N < 1 || N > 256) return -1;
  hipStream_t st = (hipStream_t)stream;
  const int64_t per = R > 0 ? (R + kCsBlocks - 1) / kCsBlocks : 1;
  if (N % 4 == 0 && ((uintptr_t)Y & 15) == 0)
    hipLaunchKernelGGL(colsum_partial4_kernel, dim3(kCsBlocks), dim3(256), 0, st,
                       reinterpret_cast<const float4 *>(Y), R, N, per, scratch);
  else
    hipLaunchKernelGGL(colsum_partial_kernel, dim3(kCsBlocks), dim3(256), 0, st, Y, R, N, per,
                       scratch);
  if (check()) return -1;
  hipLaunchKernelGGL(colsum_final_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, scratch,
                     kCsBlocks, N, acc, out);
  return check();
}

int tr_wgrad(const float *dY, const float *X, int64_t R, int N, int K, float *part, int acc,
             float *out, void *stream) {
  if (R < 1) return -2;
  int64_t per = (R + kWgMaxBlocks - 1) / kWgMaxBlocks;
  per = (per + 15) / 16 * 16;
  const int64_t nb = (R + per - 1) / per;
  hipStream_t st = (hipStream_t)stream;
  const dim3 g((unsigned)nb), b(kWgThreads);
  const bool vec = aligned16(dY) && aligned16(X);
  if (N == 64 && K == 64)
    hipLaunchKernelGGL((wgrad_kernel<1, 64>), g, b, 0, st, dY, X, R, per, part);
  else if (N == 64 && K == 256 && vec)
    hipLaunchKernelGGL((wgrad4_kernel<1, 4>), g, b, 0, st, dY, X, R, per, part);
  else if (N == 64 && K == 256)
    hipLaunchKernelGGL((wgrad_kernel<1, 256>), g, b, 0, st, dY, X, R, per, part);
  else if (N == 192 && K == 64)  // three-wavefront float4 blocks measured slower here
    hipLaunchKernelGGL((wgrad_kernel<3, 64>), g, b, 0, st, dY, X, R, per, part);
  else if (N == 256 && K == 64 && vec)
    hipLaunchKernelGGL((wgrad4_kernel<4, 1>), g, b, 0, st, dY, X, R, per, part);
  else if (N == 256 && K == 64)
    hipLaunchKernelGGL((wgrad_kernel<4, 64>), g, b, 0, st, dY, X, R, per, part);
  else if (N == 64 && K == 8)
    hipLaunchKernelGGL((wgrad_kernel<1, 8>), g, b, 0, st, dY, X, R, per, part);
  else
    return -2;
  if (check()) return -1;
  const int64_t n = (int64_t)N * K;
  hipLaunchKernelGGL(wgrad_sum_kernel, dim3((unsigned)((n + 63) / 64)), b, 0, st, part, (int)nb,
                     n, acc, out);
  return check();
}

int tr_sum_partials(const float *part, int nb, int64_t n, int acc, float *out, void *stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(sum_partials_kernel, grid_for(n), dim3(kTrThreads), 0, (hipStream_t)stream,
                     part, nb, n, acc, out);
  return check();
}

int tr_layernorm_back_sums(const float *x, const float *g, const float *dy, float *dxacc,
                           int64_t R, double *scratch, int acc, float *gain_grad,
                           float *bias_grad, float *next_grad, void *stream) {
  if (R == 0) return 0;
  if (!aligned16(x) || !aligned16(dy) || !aligned16(dxacc)) return -1;
  hipStream_t st = (hipStream_t)stream;
  const int64_t per = (R + kCsBlocks - 1) / kCsBlocks;
  const int64_t nb = (R + per - 1) / per;
  hipLaunchKernelGGL(layernorm_back_sums_kernel, dim3((unsigned)nb), dim3(256), 0, st,
                     reinterpret_cast<const float4 *>(x), g, reinterpret_cast<const float4 *>(dy),
                     reinterpret_cast<float4 *>(dxacc), R, per, scratch);
  if (check()) return -1;
  hipLaunchKernelGGL(sums3_final_kernel, dim3(3 * kPolD / 4), dim3(256), 0, st, scratch, (int)nb,
                     acc, gain_grad, bias_grad, next_grad);
  return check();
}

int tr_head(const float *h, int64_t A, int nt, const float *prm, float *logits, float *feat,
            void *stream) {
  if (A == 0) return 0;
  hipLaunchKernelGGL(head_kernel, grid_for(A * 64), dim3(kTrThreads), 0, (hipStream_t)stream, h, A,
                     nt, prm, logits, feat);
  return check();
}

int tr_head_back(const float *h, int64_t A, int nt, const float *prm, const float *dout, int ld,
                 int n_out, const float *dnext, float *dl8, float *dh, float *gfa, float *bfa,
                 void *stream) {
  if (A == 0) return 0;
  hipLaunchKernelGGL(head_back_kernel, grid_for(A * 64), dim3(kTrThreads), 0, (hipStream_t)stream,
                     h, A, nt, prm, dout, ld, n_out, dnext, dl8, dh, gfa, bfa);
  return check();
}

int tr_embed_grad_scatter(const float *gaug, int acc, float *grad, void *stream) {
  hipLaunchKernelGGL(embed_grad_scatter_kernel, dim3(2), dim3(kTrThreads), 0, (hipStream_t)stream,
                     gaug, acc, grad);
  return check();
}

int tr_first_rows(const float *dh, int64_t A, int nt, float *out, void *stream) {
  if (A == 0) return 0;
  hipLaunchKernelGGL(first_rows_kernel, grid_for(A * kPolD), dim3(kTrThreads), 0,
                     (hipStream_t)stream, dh, A, nt, out);
  return check();
}

int tr_fill(float *p, float v, int64_t n, void *stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(fill_kernel, grid_for(n), dim3(kTrThreads), 0, (hipStream_t)stream, p, v, n);
  return check();
}

}  // namespace mil
