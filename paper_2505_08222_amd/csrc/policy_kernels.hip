// Attention policy of the full-rollout workload on gfx950: the per-agent
// transformer actor of arXiv 2505.08222, Sec. III-B (TransfMAPPO, entity
// tokens, LayerNorm throughout), without its recurrent token; forward only.
//
// A persistent block (two per CU) takes tiles of agents (at most 80 token
// rows); the small FP32 parameters (embedding, LayerNorms, biases, head) are
// staged in LDS once per block. Tokens are embedded on VALU, every dense
// layer (QKV, output projection, FFN) runs as BF16 MFMA with FP32
// accumulation over the tile's stacked token rows, and
// attention (n_tok <= 16 keys per agent, 4 heads of 16) runs on VALU with
// keys whose observation mask is 0 excluded. The residual stream stays in
// LDS in FP32. The self token's final LayerNorm feeds the action head; the
// action is an inverse-CDF draw from Philox (purpose 4).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <math.h>

#include "mfma_tile.h"
#include "policy_internal.h"
#include "rng.h"

namespace mil {

namespace {

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Position in the parameter vector of entry i of the LDS copy of the small
// FP32 parameters (embedding, LayerNorms, biases, head).
__device__ __forceinline__ int small_param_src(int i) {
  if (i < kSmLayer0) return i;  // embedding W, b: the vector's first entries
  if (i < kSmFinal) {
    const int l = (i - kSmLayer0) / kSmLayer, r = (i - kSmLayer0) % kSmLayer;
    const int lp = kPolOffLayer0 + l * kPolLayerParams;
    if (r < kSmBqkv) return lp + kPolLn1G + r;                    // ln1 gain, offset
    if (r < kSmBo) return lp + kPolBqkv + (r - kSmBqkv);
    if (r < kSmLn2G) return lp + kPolBo + (r - kSmBo);
    if (r < kSmB1) return lp + kPolLn2G + (r - kSmLn2G);           // ln2 gain, offset
    if (r < kSmB2) return lp + kPolB1 + (r - kSmB1);
    return lp + kPolB2 + (r - kSmB2);
  }
  return kPolOffFinal + (i - kSmFinal);  // final LayerNorm and head
}

}  // namespace

struct PolicyLds {
  float prm[kSmTotal];                    // small FP32 parameters
  float h[kPolRows][kPolD];               // residual stream
  __bf16 xn[kPolRows][kPolD + 8];         // LayerNorm output / attention output
  __bf16 buf[kPolRows][3 * kPolD + 8];    // QKV, or one half of the FFN hidden layer, or raw tokens
  uint8_t mask[kPolRows];
  float logits[kPolMaxAgents][kPolActions];
};
static_assert(sizeof(PolicyLds) <= 80 * 1024, "two policy blocks per CU");
static_assert(offsetof(PolicyLds, h) % 16 == 0 && offsetof(PolicyLds, xn) % 16 == 0 &&
                  offsetof(PolicyLds, buf) % 16 == 0,
              "align");

// LayerNorm of every row (one wavefront per row, lane = feature) into xn.
__device__ __forceinline__ void layer_norm_rows(PolicyLds &L, int rows, const float *g,
                                                const float *b) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const float gl = g[lane], bl = b[lane];
  for (int r = wave; r < rows; r += nw) {
    const float x = L.h[r][lane];
    const float mean = wave_sum(x) * (1.0f / kPolD);
    const float d = x - mean;
    const float var = wave_sum(d * d) * (1.0f / kPolD);
    L.xn[r][lane] = __float2bfloat16(fmaf(d * rsqrtf(var + 1e-5f), gl, bl));
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
  const int64_t ntiles = (a.A + at - 1) / at;
  for (int i = tid; i < kSmTotal; i += nthr) L.prm[i] = a.params[small_param_src(i)];
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t ag0 = tile * at;
    const int64_t nag = (a.A - ag0) < at ? (a.A - ag0) : at;  // agents in this tile
    const int nrow = (int)nag * nt;
    // ---- raw tokens of the tile (contiguous in memory) staged through LDS
    float *x_raw = reinterpret_cast<float *>(&L.buf[0][0]);
    const float *src = a.obs + ag0 * nt * 6;
    for (int e = tid; e < rows * 6; e += nthr) x_raw[e] = e < nrow * 6 ? src[e] : 0.0f;
    for (int r = tid; r < rows; r += nthr) L.mask[r] = r < nrow ? a.mask[ag0 * nt + r] : 0;
    __syncthreads();
    // ---- embed 6 -> 64 (VALU)
    for (int e = tid; e < rows * kPolD; e += nthr) {
      const int r = e >> 6, d = e & (kPolD - 1);
      float acc = L.prm[kSmEmbB + d];
#pragma unroll
      for (int c = 0; c < 6; ++c) acc = fmaf(L.prm[kSmEmbW + d * 6 + c], x_raw[r * 6 + c], acc);
      L.h[r][d] = r < nrow ? acc : 0.0f;
    }
    __syncthreads();
    for (int l = 0; l < kPolLayers; ++l) {
      const float *lp = L.prm + kSmLayer0 + l * kSmLayer;
      const __bf16 *wq = a.wqkv + l * (3 * kPolD) * kPolLdD;
      const __bf16 *wo = a.wo + l * kPolD * kPolLdD;
      const __bf16 *w1 = a.w1 + l * kPolF * kPolLdD;
      const __bf16 *w2 = a.w2 + l * kPolD * kPolLdF;
      // ---- attention block
      layer_norm_rows(L, rows, lp + kSmLn1G, lp + kSmLn1B);
      __syncthreads();
      gemm_cs_bf16<kPolD>(&L.xn[0][0], kPolD + 8, wq, kPolLdD, rows, 3 * kPolD,
                       [&](int m, int n, float v) { L.buf[m][n] = __float2bfloat16(v + lp[kSmBqkv + n]); });
      __syncthreads();
      for (int e = tid; e < at * kPolHeads * nt; e += nthr) {
        const int al = e / (kPolHeads * nt), rem = e % (kPolHeads * nt);
        const int hd = rem / nt, tq = rem % nt;
        const int r0 = al * nt, rq = r0 + tq;
        const bf16x8 *qp = reinterpret_cast<const bf16x8 *>(&L.buf[rq][hd * kPolDh]);
        const bf16x8 q0 = qp[0], q1 = qp[1];
        float s[kPolMaxTok];
        float mx = -INFINITY;
#pragma unroll
        for (int u = 0; u < kPolMaxTok; ++u) {
          s[u] = -INFINITY;
          if (u < nt && L.mask[r0 + u]) {
            const bf16x8 *kp = reinterpret_cast<const bf16x8 *>(&L.buf[r0 + u][kPolD + hd * kPolDh]);
            const bf16x8 k0 = kp[0], k1 = kp[1];
            float acc = 0.0f;
#pragma unroll
            for (int c = 0; c < 8; ++c) acc = fmaf((float)q0[c], (float)k0[c], acc);
#pragma unroll
            for (int c = 0; c < 8; ++c) acc = fmaf((float)q1[c], (float)k1[c], acc);
            s[u] = acc * 0.25f;
          }
          mx = fmaxf(mx, s[u]);
        }
        float z = 0.0f;
#pragma unroll
        for (int u = 0; u < kPolMaxTok; ++u) {
          s[u] = s[u] > -INFINITY ? __expf(s[u] - mx) : 0.0f;
          z += s[u];
        }
        const float iz = z > 0.0f ? 1.0f / z : 0.0f;  // rows of absent agents have no keys
        float o[kPolDh];
#pragma unroll
        for (int c = 0; c < kPolDh; ++c) o[c] = 0.0f;
#pragma unroll
        for (int u = 0; u < kPolMaxTok; ++u) {
          if (u < nt && s[u] > 0.0f) {
            const bf16x8 *vp =
                reinterpret_cast<const bf16x8 *>(&L.buf[r0 + u][2 * kPolD + hd * kPolDh]);
            const bf16x8 v0 = vp[0], v1 = vp[1];
#pragma unroll
            for (int c = 0; c < 8; ++c) o[c] = fmaf(s[u], (float)v0[c], o[c]);
#pragma unroll
            for (int c = 0; c < 8; ++c) o[8 + c] = fmaf(s[u], (float)v1[c], o[8 + c]);
          }
        }
        bf16x8 w0, w1v;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          w0[c] = __float2bfloat16(o[c] * iz);
          w1v[c] = __float2bfloat16(o[8 + c] * iz);
        }
        bf16x8 *op = reinterpret_cast<bf16x8 *>(&L.xn[rq][hd * kPolDh]);
        op[0] = w0;
        op[1] = w1v;
      }
      __syncthreads();
      gemm_cs_bf16<kPolD>(&L.xn[0][0], kPolD + 8, wo, kPolLdD, rows, kPolD,
                       [&](int m, int n, float v) { L.h[m][n] += v + lp[kSmBo + n]; });
      __syncthreads();
      // ---- feed-forward block, hidden layer in two halves of 128
      layer_norm_rows(L, rows, lp + kSmLn2G, lp + kSmLn2B);
      __syncthreads();
      for (int half = 0; half < 2; ++half) {
        gemm_cs_bf16<kPolD>(&L.xn[0][0], kPolD + 8, w1 + half * 128 * kPolLdD, kPolLdD, rows, 128,
                         [&](int m, int n, float v) {
                           L.buf[m][n] = __float2bfloat16(gelu_tanh_fast(v + lp[kSmB1 + half * 128 + n]));
                         });
        __syncthreads();
        gemm_cs_bf16<128>(&L.buf[0][0], 3 * kPolD + 8, w2 + half * 128, kPolLdF, rows, kPolD,
                       [&](int m, int n, float v) { L.h[m][n] += v + (half == 0 ? lp[kSmB2 + n] : 0.0f); });
        __syncthreads();
      }
    }
    // ---- head on the self token of each agent: final LayerNorm, logits
    {
      const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
      const float *fp = L.prm + kSmFinal;
      for (int al = wave; al < at; al += nw) {
        const float x = L.h[al * nt][lane];
        const float mean = wave_sum(x) * (1.0f / kPolD);
        const float d = x - mean;
        const float var = wave_sum(d * d) * (1.0f / kPolD);
        const float sv = fmaf(d * rsqrtf(var + 1e-5f), fp[kPolLnfG + lane], fp[kPolLnfB + lane]);
        for (int k = 0; k < kPolActions; ++k) {
          const float v = wave_sum(fp[kPolWh + k * kPolD + lane] * sv);
          if (lane == 0) L.logits[al][k] = v + fp[kPolBh + k];
        }
      }
    }
    __syncthreads();
    // ---- actions: inverse-CDF draw from softmax over the first n_actions logits
    for (int al = tid; al < nag; al += nthr) {
      const int64_t ag = ag0 + al;
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
  const int64_t slots = 2 * (int64_t)num_cus;  // two resident blocks per CU
  const int64_t grid = ntiles < slots ? ntiles : slots;
  if (grid <= 0) return 0;
  hipLaunchKernelGGL(policy_kernel, dim3((unsigned)grid), dim3(256), sizeof(PolicyLds),
                     (hipStream_t)stream, args);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mil
