// Attention policy of the full-rollout workload on gfx950: the per-agent
// transformer actor of arXiv 2505.08222, Sec. III-B (TransfMAPPO, entity
// tokens, LayerNorm throughout), without its recurrent token; forward only.
//
// A persistent block takes tiles of agents (at most 160 token rows): tokens
// are embedded on VALU, every dense layer (QKV, output projection, FFN) runs
// as BF16 MFMA with FP32 accumulation over the tile's stacked token rows, and
// attention (n_tok <= 16 keys per agent, 4 heads of 16) runs on VALU with
// keys whose observation mask is 0 excluded. The residual stream stays in
// LDS in FP32. The self token's final LayerNorm feeds the action head; the
// action is an inverse-CDF draw from Philox (purpose 4).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <math.h>

#include "policy_internal.h"
#include "rng.h"

namespace mil {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ float gelu_tanh(float x) {
  const float c = 0.7978845608028654f;
  return 0.5f * x * (1.0f + tanhf(c * (x + 0.044715f * x * x * x)));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// D[m][n] = sum_k A[m][k] B[n][k] over 16x16 tiles; both operands K-contiguous
// BF16 (lane l: row l%16, 8 consecutive K at 8*(l/16); D rows 4*(l/16)+j).
// Column-stationary: a wavefront takes a 16-wide block of output columns,
// keeps that block's weight fragments (B, from global memory / L2) in
// registers, and sweeps every row tile of A (LDS) with them.
template <int K, typename Epi>
__device__ __forceinline__ void gemm_bf16(const __bf16 *A, int lda, const __bf16 *B, int ldb, int M,
                                          int N, Epi epi) {
  constexpr int KS = K / 32;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int tm = M >> 4, tn = N >> 4;
  const int row = lane & 15, kg = lane >> 4;
  for (int ct = wave; ct < tn; ct += nw) {
    const int n0 = ct << 4;
    bf16x8 b[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      b[ks] = *reinterpret_cast<const bf16x8 *>(B + (n0 + row) * ldb + ks * 32 + 8 * kg);
    for (int mt = 0; mt < tm; ++mt) {
      const int m0 = mt << 4;
      floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const bf16x8 a =
            *reinterpret_cast<const bf16x8 *>(A + (m0 + row) * lda + ks * 32 + 8 * kg);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[ks], acc, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) epi(m0 + 4 * kg + j, n0 + row, acc[j]);
    }
  }
}

}  // namespace

struct PolicyLds {
  float h[kPolRows][kPolD];               // residual stream
  __bf16 xn[kPolRows][kPolD + 8];         // LayerNorm output / attention output
  __bf16 buf[kPolRows][3 * kPolD + 8];    // QKV, or one half of the FFN hidden layer
  uint8_t mask[kPolRows];
  float logits[kPolMaxAgents][kPolActions];
};
static_assert(sizeof(PolicyLds) <= 160 * 1024, "policy LDS");
static_assert(offsetof(PolicyLds, xn) % 16 == 0 && offsetof(PolicyLds, buf) % 16 == 0, "align");

// LayerNorm of every row (one wavefront per row, lane = feature) into xn.
__device__ __forceinline__ void layer_norm_rows(PolicyLds &L, int rows, const float *g,
                                                const float *b) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int r = wave; r < rows; r += nw) {
    const float x = L.h[r][lane];
    const float mean = wave_sum(x) * (1.0f / kPolD);
    const float d = x - mean;
    const float var = wave_sum(d * d) * (1.0f / kPolD);
    L.xn[r][lane] = __float2bfloat16(d * rsqrtf(var + 1e-5f) * g[lane] + b[lane]);
  }
}

__global__ void __launch_bounds__(256)
policy_kernel(PolicyArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  PolicyLds &L = *reinterpret_cast<PolicyLds *>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nt = a.n_tok;
  const int at = a.agents_per_tile;
  const int rows_used = at * nt;
  const int rows = (rows_used + 15) & ~15;
  const float *th = a.params;
  const int64_t ntiles = (a.A + at - 1) / at;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t ag0 = tile * at;
    // ---- tokens: embed 6 -> 64 (VALU), masks
    for (int e = tid; e < rows * kPolD; e += nthr) {
      const int r = e / kPolD, d = e % kPolD;
      const int al = r / nt;
      float acc = 0.0f;
      if (r < rows_used && ag0 + al < a.A) {
        const float *x = a.obs + ((ag0 + al) * nt + (r % nt)) * 6;
        acc = th[kPolOffEmbB + d];
#pragma unroll
        for (int c = 0; c < 6; ++c) acc = fmaf(th[kPolOffEmbW + d * 6 + c], x[c], acc);
      }
      L.h[r][d] = acc;
    }
    for (int r = tid; r < rows; r += nthr) {
      const int al = r / nt;
      L.mask[r] = (r < rows_used && ag0 + al < a.A) ? a.mask[(ag0 + al) * nt + (r % nt)] : 0;
    }
    __syncthreads();
    for (int l = 0; l < kPolLayers; ++l) {
      const float *lp = th + kPolOffLayer0 + l * kPolLayerParams;
      const __bf16 *wq = a.wqkv + l * (3 * kPolD) * kPolLdD;
      const __bf16 *wo = a.wo + l * kPolD * kPolLdD;
      const __bf16 *w1 = a.w1 + l * kPolF * kPolLdD;
      const __bf16 *w2 = a.w2 + l * kPolD * kPolLdF;
      // ---- attention block
      layer_norm_rows(L, rows, lp + kPolLn1G, lp + kPolLn1B);
      __syncthreads();
      gemm_bf16<kPolD>(&L.xn[0][0], kPolD + 8, wq, kPolLdD, rows, 3 * kPolD,
                [&](int m, int n, float v) { L.buf[m][n] = __float2bfloat16(v + lp[kPolBqkv + n]); });
      __syncthreads();
      for (int e = tid; e < at * kPolHeads * nt; e += nthr) {
        const int al = e / (kPolHeads * nt), rem = e % (kPolHeads * nt);
        const int hd = rem / nt, tq = rem % nt;
        const int r0 = al * nt, rq = r0 + tq;
        float q[kPolDh];
#pragma unroll
        for (int c = 0; c < kPolDh; ++c) q[c] = __bfloat162float(L.buf[rq][hd * kPolDh + c]);
        float s[kPolMaxTok];
        float mx = -INFINITY;
        for (int u = 0; u < nt; ++u) {
          float acc = 0.0f;
#pragma unroll
          for (int c = 0; c < kPolDh; ++c)
            acc = fmaf(q[c], __bfloat162float(L.buf[r0 + u][kPolD + hd * kPolDh + c]), acc);
          s[u] = L.mask[r0 + u] ? acc * 0.25f : -INFINITY;
          mx = fmaxf(mx, s[u]);
        }
        float z = 0.0f;
        for (int u = 0; u < nt; ++u) {
          s[u] = L.mask[r0 + u] ? __expf(s[u] - mx) : 0.0f;
          z += s[u];
        }
        const float iz = z > 0.0f ? 1.0f / z : 0.0f;  // rows of absent agents have no keys
#pragma unroll
        for (int c = 0; c < kPolDh; ++c) {
          float acc = 0.0f;
          for (int u = 0; u < nt; ++u)
            acc = fmaf(s[u], __bfloat162float(L.buf[r0 + u][2 * kPolD + hd * kPolDh + c]), acc);
          L.xn[rq][hd * kPolDh + c] = __float2bfloat16(acc * iz);
        }
      }
      __syncthreads();
      gemm_bf16<kPolD>(&L.xn[0][0], kPolD + 8, wo, kPolLdD, rows, kPolD,
                [&](int m, int n, float v) { L.h[m][n] += v + lp[kPolBo + n]; });
      __syncthreads();
      // ---- feed-forward block, hidden layer in two halves of 128
      layer_norm_rows(L, rows, lp + kPolLn2G, lp + kPolLn2B);
      __syncthreads();
      for (int half = 0; half < 2; ++half) {
        gemm_bf16<kPolD>(&L.xn[0][0], kPolD + 8, w1 + half * 128 * kPolLdD, kPolLdD, rows, 128,
                  [&](int m, int n, float v) {
                    L.buf[m][n] = __float2bfloat16(gelu_tanh(v + lp[kPolB1 + half * 128 + n]));
                  });
        __syncthreads();
        gemm_bf16<128>(&L.buf[0][0], 3 * kPolD + 8, w2 + half * 128, kPolLdF, rows, kPolD,
                  [&](int m, int n, float v) { L.h[m][n] += v + (half == 0 ? lp[kPolB2 + n] : 0.0f); });
        __syncthreads();
      }
    }
    // ---- head on the self token of each agent: final LayerNorm, logits
    {
      const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
      const float *fp = th + kPolOffFinal;
      for (int al = wave; al < at; al += nw) {
        const float x = L.h[al * nt][lane];
        const float mean = wave_sum(x) * (1.0f / kPolD);
        const float d = x - mean;
        const float var = wave_sum(d * d) * (1.0f / kPolD);
        const float sv = d * rsqrtf(var + 1e-5f) * fp[kPolLnfG + lane] + fp[kPolLnfB + lane];
        for (int k = 0; k < kPolActions; ++k) {
          const float v = wave_sum(fp[kPolWh + k * kPolD + lane] * sv);
          if (lane == 0) L.logits[al][k] = v + fp[kPolBh + k];
        }
      }
    }
    __syncthreads();
    // ---- actions: inverse-CDF draw from softmax over the first n_actions logits
    for (int al = tid; al < at; al += nthr) {
      const int64_t ag = ag0 + al;
      if (ag >= a.A) continue;
      if (a.logits)
        for (int k = 0; k < kPolActions; ++k) a.logits[ag * kPolActions + k] = L.logits[al][k];
      if (a.actions) {
        const int64_t env = ag / a.n_agents;
        const uint32_t i = (uint32_t)(ag - env * a.n_agents);
        const u32x4 x = philox4x32_10(a.t, a.env_ids ? a.env_ids[env] : (uint32_t)env, i,
                                      (a.episode << 4) | kPurposePolicy, a.key0, a.key1);
        const float u = u01(x.x);
        float mx = -INFINITY;
        for (int k = 0; k < a.n_actions; ++k) mx = fmaxf(mx, L.logits[al][k]);
        float z = 0.0f;
        for (int k = 0; k < a.n_actions; ++k) z += __expf(L.logits[al][k] - mx);
        float c = 0.0f;
        int act = a.n_actions - 1;
        for (int k = 0; k < a.n_actions; ++k) {
          c += __expf(L.logits[al][k] - mx) / z;
          if (u < c) {
            act = k;
            break;
          }
        }
        a.actions[ag] = act;
      }
    }
    __syncthreads();
  }
}

// MFMA-ready BF16 copies of the dense weights (rows K-contiguous, padded).
__global__ void policy_prepare_kernel(const float *__restrict__ th, __bf16 *wqkv, __bf16 *wo,
                                      __bf16 *w1, __bf16 *w2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  for (int l = 0; l < kPolLayers; ++l) {
    const float *lp = th + kPolOffLayer0 + l * kPolLayerParams;
    if (k < 3 * kPolD * kPolD) {
      const int o = k / kPolD, i = k % kPolD;
      wqkv[l * 3 * kPolD * kPolLdD + o * kPolLdD + i] = __float2bfloat16(lp[kPolWqkv + k]);
    }
    if (k < kPolD * kPolD) {
      const int o = k / kPolD, i = k % kPolD;
      wo[l * kPolD * kPolLdD + o * kPolLdD + i] = __float2bfloat16(lp[kPolWo + k]);
    }
    if (k < kPolF * kPolD) {
      const int o = k / kPolD, i = k % kPolD;
      w1[l * kPolF * kPolLdD + o * kPolLdD + i] = __float2bfloat16(lp[kPolW1 + k]);
      const int o2 = k / kPolF, i2 = k % kPolF;  // W2 is [64][256]
      w2[l * kPolD * kPolLdF + o2 * kPolLdF + i2] = __float2bfloat16(lp[kPolW2 + k]);
    }
  }
}

// Glorot-uniform dense weights (Philox keyed by seed, purpose 6), LayerNorm
// gains 1, every bias and LayerNorm offset 0.
__global__ void policy_init_kernel(float *th, uint32_t k0, uint32_t k1) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kPolNumParams) return;
  float a = 0.0f, one = 0.0f;
  int q = p;
  if (q < kPolOffEmbB) {
    a = sqrtf(6.0f / (6 + kPolD));
  } else if (q < kPolOffLayer0) {
    a = 0.0f;
  } else if (q < kPolOffFinal) {
    const int r = (q - kPolOffLayer0) % kPolLayerParams;
    if (r < kPolLn1B || (r >= kPolLn2G && r < kPolLn2B)) one = 1.0f;
    else if (r >= kPolWqkv && r < kPolBqkv) a = sqrtf(6.0f / (kPolD + kPolD));
    else if (r >= kPolWo && r < kPolBo) a = sqrtf(6.0f / (kPolD + kPolD));
    else if (r >= kPolW1 && r < kPolB1) a = sqrtf(6.0f / (kPolD + kPolF));
    else if (r >= kPolW2 && r < kPolB2) a = sqrtf(6.0f / (kPolF + kPolD));
  } else {
    const int r = q - kPolOffFinal;
    if (r < kPolLnfB) one = 1.0f;
    else if (r >= kPolWh && r < kPolBh) a = sqrtf(6.0f / (kPolD + kPolActions));
  }
  const u32x4 x = philox4x32_10((uint32_t)p, 0u, 0u, kPurposePolicyInit, k0, k1);
  th[p] = one + a * (2.0f * u01(x.x) - 1.0f);
}

int launch_policy_init(float *th, uint64_t seed, void *stream) {
  hipLaunchKernelGGL(policy_init_kernel, dim3((kPolNumParams + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, th, (uint32_t)seed, (uint32_t)(seed >> 32));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_policy_prepare(const float *th, __bf16 *wqkv, __bf16 *wo, __bf16 *w1, __bf16 *w2,
                          void *stream) {
  const int n = kPolF * kPolD;
  hipLaunchKernelGGL(policy_prepare_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, th, wqkv, wo, w1, w2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_policy(const PolicyArgs &args, int num_cus, void *stream) {
  static bool lds_set = false;
  if (!lds_set) {
    if (hipFuncSetAttribute((const void *)policy_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sizeof(PolicyLds)) != hipSuccess)
      return -1;
    lds_set = true;
  }
  const int64_t ntiles = (args.A + args.agents_per_tile - 1) / args.agents_per_tile;
  const int64_t grid = ntiles < (int64_t)num_cus ? ntiles : (int64_t)num_cus;
  if (grid <= 0) return 0;
  hipLaunchKernelGGL(policy_kernel, dim3((unsigned)grid), dim3(256), sizeof(PolicyLds),
                     (hipStream_t)stream, args);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mil
