// Attention policy of the full-rollout workload on gfx950: the per-agent
// transformer actor of arXiv 2505.08222, Sec. IV-B-1 (TransfMAPPO, entity
// tokens, LayerNorm throughout), plain or with its recurrent token (Fig. 3: a
// carried 64-wide state as an unmasked first row, not embedded, whose final
// LayerNorm is the head's input and the next state); forward only.
//
// A persistent block (two per CU) takes tiles of agents (at most 80 token
// rows); the small FP32 parameters (embedding, LayerNorms, biases, head) are
// staged in LDS once per block. Tokens are embedded on VALU, every dense
// layer (QKV, output projection, FFN) runs as BF16 MFMA with FP32
// accumulation over the tile's stacked token rows, and attention (n_tok <= 16
// keys per agent, 4 heads of 16) runs as two 16x16x16 MFMA products per
// (agent, head) with keys whose observation mask is 0 excluded. The residual
// stream stays in LDS in FP32. The first row's final LayerNorm (the self
// token, or the recurrent row) feeds the action head; the action is an
// inverse-CDF draw from Philox (purpose 4).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <math.h>

#include "mfma_tile.h"
#include "policy_internal.h"
#include "rng.h"

namespace mil {

typedef int int2v __attribute__((ext_vector_type(2)));

namespace {

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

constexpr int kPlane = kPolRows * (kPolD + 8);  // one Q / K / V plane (elements)
constexpr int kLdQ = kPolD + 8;                  // row stride of a plane
constexpr int kLdVt = kPolRows + 8;              // row stride of V^T
constexpr int kLdHid = 128 + 8;                  // row stride of the FFN hidden half
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// the staging buffer: Q and K planes then V^T; or one half of the FFN hidden
// layer; or the raw tokens; or the head's scratch. The last agent of a tile
// reads 16 keys from its first row on: up to row (at - 1) * n_tok + 15, which
// passes the V^T row stride (kPolRows + 8) for n_tok = 5 (16 agents, row 90),
// so spare elements follow the plane
constexpr int kVtSpare = 16;
constexpr int kBufElems =
    cmax(cmax(2 * kPlane + kPolD * kLdVt + kVtSpare, kPolRows * kLdHid),
         cmax(kPolMaxAgents * (kPolD + 4) * 2, kPolRows * 6 * 2));

struct PolicyLds {
  float prm[kSmTotal];                    // small FP32 parameters
  float h[kPolRows][kPolD + 4];           // residual stream (rows padded: conflict-free row reads)
  __bf16 xn[kPolRows][kPolD + 8];         // LayerNorm output / attention output
  __bf16 buf[kBufElems];
  uint8_t mask[kPolRows];
  uint32_t mbits[kPolMaxAgents];          // per agent: bit k = observation mask of token k
  float logits[kPolMaxAgents][kPolActions];
};
static_assert(sizeof(PolicyLds) <= 160 * 1024 / kPolBlocksPerCU, "resident policy blocks per CU");
static_assert((kPlane * 2) % 16 == 0, "plane alignment");
static_assert(offsetof(PolicyLds, h) % 16 == 0 && offsetof(PolicyLds, xn) % 16 == 0 &&
                  offsetof(PolicyLds, buf) % 16 == 0,
              "align");

// Sum over a lane pair (DPP, lanes xor 1); both lanes end with the same value.
__device__ __forceinline__ float pair_sum(float v) {
  return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// LayerNorm (eps 1e-5) of every row of the residual stream into xn (BF16):
// two lanes per row, 32 features each held in registers, pair sums for the
// mean and the variance; 128 rows per pass of the block's 256 threads (one
// pass for a full tile).
__device__ __forceinline__ void layer_norm_rows(PolicyLds &L, int rows, const float *g,
                                                const float *b) {
  const int q = threadIdx.x & 1;
  const float4 *gp = reinterpret_cast<const float4 *>(g + 32 * q);
  const float4 *bp = reinterpret_cast<const float4 *>(b + 32 * q);
  for (int r0 = 0; r0 < rows; r0 += 128) {
    const int r = r0 + (threadIdx.x >> 1);
    const int rr = r < rows ? r : rows - 1;  // whole pairs stay active
    const float4 *xp = reinterpret_cast<const float4 *>(&L.h[rr][32 * q]);
    float x[32];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float4 v = xp[i];
      x[4 * i] = v.x;
      x[4 * i + 1] = v.y;
      x[4 * i + 2] = v.z;
      x[4 * i + 3] = v.w;
    }
    float s8[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) s8[i] = (x[4 * i] + x[4 * i + 1]) + (x[4 * i + 2] + x[4 * i + 3]);
    const float mean =
        pair_sum(((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]))) *
        (1.0f / kPolD);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float t = 0.0f;
#pragma unroll
      for (int c = 0; c < 4; ++c) t = fmaf(x[4 * i + c] - mean, x[4 * i + c] - mean, t);
      s8[i] = t;
    }
    const float var =
        pair_sum(((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]))) *
        (1.0f / kPolD);
    const float inv = rsqrtf(var + 1e-5f);
    bf16x8 w[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float4 gv = gp[i], bv = bp[i];
      const float gg[4] = {gv.x, gv.y, gv.z, gv.w}, bb[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
      for (int c = 0; c < 4; ++c)
        w[i >> 1][4 * (i & 1) + c] = __float2bfloat16(fmaf((x[4 * i + c] - mean) * inv, gg[c], bb[c]));
    }
    if (r < rows) {
      bf16x8 *o = reinterpret_cast<bf16x8 *>(&L.xn[r][32 * q]);
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] = w[i];
    }
  }
}

// Bias of four consecutive features (FP32, LDS) added to an MFMA result.
__device__ __forceinline__ floatx4 add4(const floatx4 &v, const float *bias) {
  const float4 b = *reinterpret_cast<const float4 *>(bias);
  return floatx4{v[0] + b.x, v[1] + b.y, v[2] + b.z, v[3] + b.w};
}

__device__ __forceinline__ bf16x4 to_bf16x4(const floatx4 &v) {
  return bf16x4{__float2bfloat16(v[0]), __float2bfloat16(v[1]), __float2bfloat16(v[2]),
                __float2bfloat16(v[3])};
}

// h[m][n..n+3] += v (+ bias)
__device__ __forceinline__ void residual4(float *h, const floatx4 &v) {
  float4 *p = reinterpret_cast<float4 *>(h);
  float4 x = *p;
  x.x += v[0];
  x.y += v[1];
  x.z += v[2];
  x.w += v[3];
  *p = x;
}

// kPolBlocksPerCU resident blocks of four wavefronts per CU
__global__ void __launch_bounds__(256, kPolBlocksPerCU)
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
  // the V^T plane's padding columns, and with five tokens per agent the
  // spare elements after the plane, are read in attention (and multiplied by
  // a zero probability, which leaves a NaN or Inf in stale LDS standing) but
  // never written: start them at zero
  for (int i = tid; i < kPolD * kLdVt + kVtSpare; i += nthr) L.buf[2 * kPlane + i] = __bf16{};
  // raw tokens and masks of a tile are contiguous in memory; each thread
  // holds its share of the next tile's in registers while this one computes
  constexpr int kTokRegs = (kPolRows * 6 + 255) / 256;
  static_assert(kTokRegs * 256 >= kPolRows * 6 && kPolRows <= 256, "token prefetch");
  float tok[kTokRegs];
  uint8_t msk = 0;
  uint32_t eid_next = 0;
  const int ot = nt - a.rec;  // observed tokens per agent (the recurrent row is not in obs)
  auto fetch = [&](int64_t tile) {
    const int64_t ag0 = tile * at;
    const int64_t nag = (a.A - ag0) < at ? (a.A - ag0) : at;
    const int nrow = (int)nag * nt;
    const float *src = a.obs + ag0 * ot * 6;
#pragma unroll
    for (int q = 0; q < kTokRegs; ++q) {
      const int e = tid + q * nthr;
      tok[q] = (tile < ntiles && e < (int)nag * ot * 6) ? src[e] : 0.0f;
    }
    if (a.rec) {  // row k of agent al: the carried state (never masked) or token k - 1
      const int al = tid / nt, k = tid - al * nt;
      msk = (tile < ntiles && tid < nrow) ? (k == 0 ? 1 : a.mask[(ag0 + al) * ot + k - 1]) : 0;
    } else {
      msk = (tile < ntiles && tid < nrow) ? a.mask[ag0 * nt + tid] : 0;
    }
    // the global env id of agent tid of the tile, for its action draw
    const int64_t env = (ag0 + tid) / a.n_agents;
    eid_next = (tile < ntiles && tid < nag) ? (a.env_ids ? a.env_ids[env] : (uint32_t)env) : 0u;
  };
  fetch(blockIdx.x);
  // weight fragments are loaded one GEMM ahead (the first layer's QKV here)
  BFrag<kPolD, 3 * kPolD> fq;
  load_bfrag(fq, a.wqkv, kPolLdD);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t ag0 = tile * at;
    const int64_t nag = (a.A - ag0) < at ? (a.A - ag0) : at;  // agents in this tile
    const int nrow = (int)nag * nt;
    // ---- raw tokens of the tile staged through LDS, the next tile's fetched
    float *x_raw = reinterpret_cast<float *>(&L.buf[0]);
#pragma unroll
    for (int q = 0; q < kTokRegs; ++q) {
      const int e = tid + q * nthr;
      if (e < rows * 6) x_raw[e] = tok[q];
    }
    if (tid < rows) L.mask[tid] = msk;
    const uint32_t eid = eid_next;  // this tile's, fetched a tile ahead
    fetch(tile + gridDim.x);
    __syncthreads();
    // ---- embed 6 -> 64 (VALU)
    {  // thread (feature d, row group): the feature's weights stay in registers
      const int d = tid & (kPolD - 1);
      float wv[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) wv[c] = L.prm[kSmEmbW + d * 6 + c];
      const float bd = L.prm[kSmEmbB + d];
      for (int r = tid >> 6; r < rows; r += nthr >> 6) {
        // the staged row of row r: r itself, or with the recurrent row first,
        // token k - 1 of agent al (row-uniform across the wavefront)
        int xrow = r;
        bool carried = false;
        if (a.rec) {
          const int al = r / nt, k = r - al * nt;
          carried = k == 0;
          xrow = al * ot + (carried ? 0 : k - 1);
        }
        // the row's six inputs as three 8-byte reads (rows start 24 bytes apart)
        const float2 *xr = reinterpret_cast<const float2 *>(x_raw + xrow * 6);
        const float2 x01 = xr[0], x23 = xr[1], x45 = xr[2];
        float acc = bd;
        acc = fmaf(wv[0], x01.x, acc);
        acc = fmaf(wv[1], x01.y, acc);
        acc = fmaf(wv[2], x23.x, acc);
        acc = fmaf(wv[3], x23.y, acc);
        acc = fmaf(wv[4], x45.x, acc);
        acc = fmaf(wv[5], x45.y, acc);
        if (carried)  // (rows past the tile's last agent stay zero)
          acc = (a.hidden_in && r < nrow) ? a.hidden_in[(ag0 + r / nt) * kPolD + d] : 0.0f;
        L.h[r][d] = r < nrow ? acc : 0.0f;
      }
      if (tid < at) {
        uint32_t bits = 0;
        for (int k = 0; k < nt; ++k) bits |= (uint32_t)(L.mask[tid * nt + k] != 0) << k;
        L.mbits[tid] = bits;
      }
    }
    __syncthreads();
    for (int l = 0; l < kPolLayers; ++l) {
      const float *lp = L.prm + kSmLayer0 + l * kSmLayer;
      const __bf16 *wo = a.wo + l * kPolD * kPolLdD;
      const __bf16 *w1 = a.w1 + l * kPolF * kPolLdD;
      const __bf16 *w2 = a.w2 + l * kPolD * kPolLdF;
      // ---- attention block
      layer_norm_rows(L, rows, lp + kSmLn1G, lp + kSmLn1B);
      __syncthreads();
      __bf16 *Qp = L.buf, *Kp = L.buf + kPlane, *Vt = L.buf + 2 * kPlane;
      BFrag<kPolD, kPolD> fo;
      load_bfrag(fo, wo, kPolLdD);
      gemm_rs_bf16_tf<kPolD, 3 * kPolD>(&L.xn[0][0], kPolD + 8, fq, rows,
                                       [&](int m, int n, const floatx4 &v) {
                                         const bf16x4 x = to_bf16x4(add4(v, lp + kSmBqkv + n));
                                         if (n < 2 * kPolD) {
                                           *reinterpret_cast<bf16x4 *>(
                                               &L.buf[(n >> 6) * kPlane + m * kLdQ + (n & 63)]) = x;
                                         } else {
#pragma unroll
                                           for (int j = 0; j < 4; ++j)
                                             Vt[(n - 2 * kPolD + j) * kLdVt + m] = x[j];
                                         }
                                       });
      __syncthreads();
      // attention on the matrix cores, per (agent, head): S^T = K Q^T and
      // O^T = V^T P^T are single 16x16x16 products (tokens padded to 16, the
      // head dimension is the instruction's K), so each lane holds four keys
      // of one query, exactly the four that the second product takes from it:
      // the softmax needs only two cross-lane steps and P never moves
      {
        const int wave = tid >> 6, lane = tid & 63, nw = nthr >> 6;
        const int row = lane & 15, kg = lane >> 4;
        constexpr int NP = 8;  // (agent, head) pairs in flight per wavefront
        for (int pr0 = wave * NP; pr0 < at * kPolHeads; pr0 += nw * NP) {
          int r0[NP], hd[NP], ag[NP];
          bool live[NP];
          floatx4 st[NP];
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            const int pr = pr0 + i;
            live[i] = pr < at * kPolHeads;
            ag[i] = live[i] ? pr / kPolHeads : 0;
            r0[i] = ag[i] * nt;
            hd[i] = pr % kPolHeads;
            // A = K (row = key), B = Q (column = query); rows past the
            // agent's tokens hold finite values of other rows: their keys are
            // masked below and their queries' outputs are not written
            const bf16x4 ka =
                *reinterpret_cast<const bf16x4 *>(Kp + (r0[i] + row) * kLdQ + hd[i] * kPolDh + 4 * kg);
            const bf16x4 qb =
                *reinterpret_cast<const bf16x4 *>(Qp + (r0[i] + row) * kLdQ + hd[i] * kPolDh + 4 * kg);
            st[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ka, qb, floatx4{0.0f, 0.0f, 0.0f, 0.0f},
                                                             0, 0, 0);
          }
          // st[i][j] = S[query row][key 4 kg + j]; keys without a mask bit
          // (masked, or at or beyond nt) are excluded
          float x[NP][4], m[NP], z[NP];
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            m[i] = -INFINITY;
            const uint32_t mb = L.mbits[ag[i]] >> (4 * kg);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              x[i][j] = ((mb >> j) & 1u) ? st[i][j] * 0.25f : -INFINITY;
              m[i] = fmaxf(m[i], x[i][j]);
            }
          }
          // max and sum over the four lane groups of a query: each swap
          // leaves a lane's own value in one result and its partner's in the
          // other, and both operations are symmetric
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(m[i]), __float_as_int(m[i]),
                                                            false, false);
            m[i] = fmaxf(__int_as_float(r[0]), __int_as_float(r[1]));
          }
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(m[i]), __float_as_int(m[i]),
                                                            false, false);
            m[i] = fmaxf(__int_as_float(r[0]), __int_as_float(r[1]));
          }
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            z[i] = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              x[i][j] = x[i][j] > -INFINITY ? __expf(x[i][j] - m[i]) : 0.0f;
              z[i] += x[i][j];
            }
          }
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(z[i]), __float_as_int(z[i]),
                                                            false, false);
            z[i] = __int_as_float(r[0]) + __int_as_float(r[1]);
          }
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(z[i]), __float_as_int(z[i]),
                                                            false, false);
            z[i] = __int_as_float(r[0]) + __int_as_float(r[1]);
          }
          // A = V^T (row = head dimension, K = key), B = P^T (column =
          // query, K = key): this lane's own four probabilities. Keys at or
          // beyond nt meet P = 0 and read finite V^T values (written by the
          // QKV epilogue, or the plane's zeroed padding).
          floatx4 ot[NP];
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            const bf16x4 pb = bf16x4{__float2bfloat16(x[i][0]), __float2bfloat16(x[i][1]),
                                     __float2bfloat16(x[i][2]), __float2bfloat16(x[i][3])};
            const __bf16 *vr = Vt + (hd[i] * kPolDh + row) * kLdVt + r0[i] + 4 * kg;
            bf16x4 va;
            if ((r0[i] & 1) == 0) {  // 4-byte aligned key pairs
              const uint32_t *v32 = reinterpret_cast<const uint32_t *>(vr);
              va = __builtin_bit_cast(bf16x4, int2v{(int)v32[0], (int)v32[1]});
            } else {
#pragma unroll
              for (int t = 0; t < 4; ++t) va[t] = vr[t];
            }
            ot[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(va, pb, floatx4{0.0f, 0.0f, 0.0f, 0.0f},
                                                             0, 0, 0);
          }
          // ot[i][j] = O[query row][head dim 4 kg + j]
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            if (live[i] && row < nt) {
              const float iz = z[i] > 0.0f ? __builtin_amdgcn_rcpf(z[i]) : 0.0f;  // no keys: zero output
              bf16x4 o4;
#pragma unroll
              for (int j = 0; j < 4; ++j) o4[j] = __float2bfloat16(ot[i][j] * iz);
              *reinterpret_cast<bf16x4 *>(&L.xn[r0[i] + row][hd[i] * kPolDh + 4 * kg]) = o4;
            }
          }
        }
      }
      __syncthreads();
      BFrag<kPolD, 128> f1;
      load_bfrag(f1, w1, kPolLdD);
      gemm_rs_bf16_tf<kPolD, kPolD>(&L.xn[0][0], kPolD + 8, fo, rows,
                                   [&](int m, int n, const floatx4 &v) {
                                     residual4(&L.h[m][n], add4(v, lp + kSmBo + n));
                                   });
      __syncthreads();
      // ---- feed-forward block, hidden layer in two halves of 128
      layer_norm_rows(L, rows, lp + kSmLn2G, lp + kSmLn2B);
      __syncthreads();
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        BFrag<128, kPolD> f2;
        load_bfrag(f2, w2 + half * 128, kPolLdF);
        gemm_rs_bf16_tf<kPolD, 128>(&L.xn[0][0], kPolD + 8, f1,
                                   rows, [&](int m, int n, const floatx4 &v) {
                                     const floatx4 y = add4(v, lp + kSmB1 + half * 128 + n);
                                     *reinterpret_cast<bf16x4 *>(&L.buf[m * kLdHid + n]) =
                                         to_bf16x4(floatx4{gelu_tanh_fast(y[0]), gelu_tanh_fast(y[1]),
                                                           gelu_tanh_fast(y[2]), gelu_tanh_fast(y[3])});
                                   });
        __syncthreads();
        if (half == 0)
          load_bfrag(f1, w1 + 128 * kPolLdD, kPolLdD);  // the second half's W1
        else  // the next layer's QKV, or the first layer's for the next tile
          load_bfrag(fq, a.wqkv + (l + 1 < kPolLayers ? l + 1 : 0) * (3 * kPolD) * kPolLdD, kPolLdD);
        gemm_rs_bf16_tf<128, kPolD>(L.buf, kLdHid, f2, rows,
                                   [&](int m, int n, const floatx4 &v) {
                                     residual4(&L.h[m][n], half == 0 ? add4(v, lp + kSmB2 + n) : v);
                                   });
        __syncthreads();
      }
    }
    // ---- head on the self token of each agent: final LayerNorm (four lanes
    // per agent, into a scratch copy in the QKV buffer), then four lanes per
    // (agent, logit), each a 16-feature partial dot product
    {
      const float *fp = L.prm + kSmFinal;
      float(*sv)[kPolD + 4] = reinterpret_cast<float(*)[kPolD + 4]>(L.buf);
      const int q = tid & 3;
      for (int al = tid >> 2; al < at; al += nthr >> 2) {  // al is uniform on a quad
        const float4 *xp = reinterpret_cast<const float4 *>(&L.h[al * nt][16 * q]);
        float x[16];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float4 v = xp[i];
          x[4 * i] = v.x;
          x[4 * i + 1] = v.y;
          x[4 * i + 2] = v.z;
          x[4 * i + 3] = v.w;
        }
        float sum = 0.0f;
#pragma unroll
        for (int c = 0; c < 16; ++c) sum += x[c];
        const float mean = quad_sum(sum) * (1.0f / kPolD);
        float sq = 0.0f;
#pragma unroll
        for (int c = 0; c < 16; ++c) sq = fmaf(x[c] - mean, x[c] - mean, sq);
        const float inv = rsqrtf(quad_sum(sq) * (1.0f / kPolD) + 1e-5f);
#pragma unroll
        for (int c = 0; c < 16; ++c)
          sv[al][16 * q + c] =
              fmaf((x[c] - mean) * inv, fp[kPolLnfG + 16 * q + c], fp[kPolLnfB + 16 * q + c]);
      }
      __syncthreads();
      if (a.feat) {  // the head's input features of each agent, for its gradient
        for (int e = tid; e < nag * kPolD; e += nthr) {
          const int al = e / kPolD, d = e - al * kPolD;
          a.feat[(ag0 + al) * kPolD + d] = sv[al][d];
        }
      }
      for (int e = tid >> 2; e < at * kPolActions; e += nthr >> 2) {
        const int al = e / kPolActions, k = e % kPolActions;
        const float4 *w = reinterpret_cast<const float4 *>(fp + kPolWh + k * kPolD + 16 * q);
        const float4 *v = reinterpret_cast<const float4 *>(&sv[al][16 * q]);
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float4 wv = w[i], xv = v[i];
          acc = fmaf(wv.x, xv.x, acc);
          acc = fmaf(wv.y, xv.y, acc);
          acc = fmaf(wv.z, xv.z, acc);
          acc = fmaf(wv.w, xv.w, acc);
        }
        acc = quad_sum(acc);
        if (q == 0) L.logits[al][k] = acc + fp[kPolBh + k];
      }
    }
    __syncthreads();
    // ---- actions: inverse-CDF draw from softmax over the first n_actions logits
    if (tid < nag) {  // nag <= kPolMaxAgents: one thread per agent
      const int al = tid;
      const int64_t ag = ag0 + al;
      if (a.logits)
        for (int k = 0; k < kPolActions; ++k) a.logits[ag * kPolActions + k] = L.logits[al][k];
      if (a.actions) {
        const int64_t env = ag / a.n_agents;
        const uint32_t i = (uint32_t)(ag - env * a.n_agents);
        const u32x4 x = philox4x32_10(a.t, eid, i, (a.episode << 4) | kPurposePolicy, a.key0,
                                      a.key1);
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
  const int64_t slots = (int64_t)kPolBlocksPerCU * num_cus;  // resident blocks
  const int64_t grid = ntiles < slots ? ntiles : slots;
  if (grid <= 0) return 0;
  hipLaunchKernelGGL(policy_kernel, dim3((unsigned)grid), dim3(256), sizeof(PolicyLds),
                     (hipStream_t)stream, args);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mil
