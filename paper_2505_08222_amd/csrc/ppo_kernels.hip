// The learner's forward half (Sec. III-B: MAPPO's clipped surrogate for the
// actors and one centralised critic V(S) of the global state; Sec. IV-B-1:
// the TransformerCritic): the critic's entity tokens, generalised advantage
// estimation and the clipped PPO objective with its gradients in the logits
// and values. The critic network itself is the attention kernel of
// policy_kernels.hip run on these tokens (its head's first output is V).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "policy_internal.h"

namespace mil {
namespace {

constexpr int kPpoThreads = 256;

// One thread per (state, token): with lead = 1, token 0 is the critic's own
// value token (all-zero features: its embedding is the embedding bias) and
// tokens 1.. the state's agents and targets; with lead = 0 (the recurrent
// critic, whose carried state takes the first row inside the attention
// kernel) only the entities. An entity token is (x / s, y / s, v cos psi,
// v sin psi, is_agent, is_target) from the global-state row (x, y, z, speed,
// heading, is_target).
__global__ void __launch_bounds__(kPpoThreads)
critic_tokens_kernel(const float *__restrict__ gstate, int64_t N, int M, int lead,
                     float inv_scale, float *__restrict__ tokens, uint8_t *__restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nt = M + lead;
  if (i >= N * nt) return;
  const int64_t n = i / nt;
  const int k = (int)(i - n * nt) - lead;  // entity, or -1 for the value token
  float f[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (k >= 0) {
    const float *g = gstate + (n * M + k) * 6;
    const float x = g[0], y = g[1], v = g[3], psi = g[4], is_t = g[5];
    // hardware sin / cos take revolutions
    const float rev = psi * 0.15915494309189535f;
    const float s = __builtin_amdgcn_sinf(rev), c = __builtin_amdgcn_cosf(rev);
    f[0] = x * inv_scale;
    f[1] = y * inv_scale;
    f[2] = v * c;
    f[3] = v * s;
    f[4] = 1.0f - is_t;
    f[5] = is_t;
  }
  float2 *dst = reinterpret_cast<float2 *>(tokens + i * 6);
  dst[0] = make_float2(f[0], f[1]);
  dst[1] = make_float2(f[2], f[3]);
  dst[2] = make_float2(f[4], f[5]);
  mask[i] = 1;
}

__global__ void __launch_bounds__(kPpoThreads)
first_column_kernel(const float *__restrict__ logits, int64_t N, float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[i] = logits[i * kPolActions];
}

// One thread per env, backwards in time, FP64 recurrence:
// delta_t = r_t + gamma V_{t+1} (1 - d_t) - V_t,
// A_t = delta_t + gamma lambda (1 - d_t) A_{t+1}, R_t = A_t + V_t.
__global__ void __launch_bounds__(kPpoThreads)
gae_kernel(const float *__restrict__ rewards, const uint8_t *__restrict__ dones,
           const float *__restrict__ values, int32_t T, int64_t E, double gamma, double gl,
           float *__restrict__ adv, float *__restrict__ ret) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double nxt = 0.0;
  double v_next = (double)values[(int64_t)T * E + e];
  for (int32_t t = T - 1; t >= 0; --t) {
    const int64_t i = (int64_t)t * E + e;
    const double v = (double)values[i];
    const double cont = dones[i] ? 0.0 : 1.0;
    const double delta = fma(gamma * cont, v_next, (double)rewards[i] - v);
    nxt = fma(gl * cont, nxt, delta);
    adv[i] = (float)nxt;
    ret[i] = (float)(nxt + v);
    v_next = v;
  }
}

// Fixed-order block sums of doubles: lane strided partial, then a tree in LDS.
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double *out) {
  __shared__ double red[NV][kPpoThreads];
#pragma unroll
  for (int q = 0; q < NV; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int s = kPpoThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int q = 0; q < NV; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = red[q][0];
  }
}

// Per agent-sample (t, a): log-softmax of the new and old logits over the
// first n_actions, rho = exp(lp_new(k) - lp_old(k)), the clipped surrogate
// min(rho A, clip(rho) A), the entropy of the new policy, and (dlogits set)
// d(-mean surrogate)/d logits = -(A rho / N)(onehot(k) - p) where the
// unclipped term is the minimum, 0 where the clipped one is strictly smaller.
// Block partials: surrogate sum, entropy sum, clipped count.
__global__ void __launch_bounds__(kPpoThreads)
ppo_policy_kernel(const float *__restrict__ lnew, const float *__restrict__ lold,
                  const int32_t *__restrict__ actions, const float *__restrict__ adv, int64_t S,
                  int64_t A, int32_t n_agents, int32_t n_actions, float clip_eps, float inv_n,
                  float *__restrict__ dlogits, double *__restrict__ part, int64_t per_block) {
  double acc[3] = {0.0, 0.0, 0.0};
  const int64_t s0 = (int64_t)blockIdx.x * per_block;
  const int64_t s1 = s0 + per_block < S ? s0 + per_block : S;
  for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
    const int64_t t = s / A, a = s - t * A;
    const float *zn = lnew + s * kPolActions;
    const float *zo = lold + s * kPolActions;
    float vn[kPolActions], vo[kPolActions];
    float mn = -INFINITY, mo = -INFINITY;
#pragma unroll
    for (int j = 0; j < kPolActions; ++j) {
      vn[j] = zn[j];
      vo[j] = zo[j];
      if (j < n_actions) {
        mn = fmaxf(mn, vn[j]);
        mo = fmaxf(mo, vo[j]);
      }
    }
    float sn = 0.0f, so = 0.0f;
    float p[kPolActions];
#pragma unroll
    for (int j = 0; j < kPolActions; ++j) {
      p[j] = 0.0f;
      if (j < n_actions) {
        p[j] = __expf(vn[j] - mn);
        sn += p[j];
        so += __expf(vo[j] - mo);
      }
    }
    const float lsn = __logf(sn), lso = __logf(so);
    int k = actions[s];
    k = k < 0 ? 0 : (k >= n_actions ? n_actions - 1 : k);
    float zk = 0.0f, zok = 0.0f;
#pragma unroll
    for (int j = 0; j < kPolActions; ++j)
      if (j == k) {
        zk = vn[j];
        zok = vo[j];
      }
    const float lpn = zk - mn - lsn, lpo = zok - mo - lso;
    const float rho = __expf(lpn - lpo);
    const float Av = adv[t * (A / n_agents) + a / n_agents];
    const float unc = rho * Av;
    const float clp = fminf(fmaxf(rho, 1.0f - clip_eps), 1.0f + clip_eps) * Av;
    float ent = 0.0f;
    const float inv_sn = 1.0f / sn;
#pragma unroll
    for (int j = 0; j < kPolActions; ++j) {
      if (j < n_actions) {
        p[j] *= inv_sn;
        ent -= p[j] * (vn[j] - mn - lsn);
      }
    }
    const bool clipped = clp < unc;
    acc[0] += (double)(clipped ? clp : unc);
    acc[1] += (double)ent;
    acc[2] += clipped ? 1.0 : 0.0;
    if (dlogits) {
      const float g = clipped ? 0.0f : -Av * rho * inv_n;
      float *d = dlogits + s * kPolActions;
#pragma unroll
      for (int j = 0; j < kPolActions; ++j)
        d[j] = (j < n_actions) ? g * ((j == k ? 1.0f : 0.0f) - p[j]) : 0.0f;
    }
  }
  double out[3];
  block_sums<3>(acc, out);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) part[blockIdx.x * 4 + q] = out[q];
  }
}

// Per env-step: squared value error and (dvalues set) its gradient 2 (V - R) / n.
__global__ void __launch_bounds__(kPpoThreads)
ppo_value_kernel(const float *__restrict__ values, const float *__restrict__ returns, int64_t n,
                 float inv_n, float *__restrict__ dvalues, double *__restrict__ part,
                 int64_t per_block) {
  double acc[1] = {0.0};
  const int64_t s0 = (int64_t)blockIdx.x * per_block;
  const int64_t s1 = s0 + per_block < n ? s0 + per_block : n;
  for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
    const float d = values[i] - returns[i];
    acc[0] += (double)d * (double)d;
    if (dvalues) dvalues[i] = 2.0f * d * inv_n;
  }
  double out[1];
  block_sums<1>(acc, out);
  if (threadIdx.x == 0) part[blockIdx.x * 4 + 3] = out[0];
}

// Partials in block order -> (policy loss, value loss, entropy, clip fraction).
__global__ void ppo_final_kernel(const double *__restrict__ part, int nb, double inv_s,
                                 double inv_v, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < nb; ++b)
    for (int q = 0; q < 4; ++q) s[q] += part[b * 4 + q];
  out[0] = -s[0] * inv_s;
  out[1] = s[3] * inv_v;
  out[2] = s[1] * inv_s;
  out[3] = s[2] * inv_s;
}

// Head gradient partials: block b sums samples [b * per, (b + 1) * per).
// Wavefront w of the block takes rows w, w + 16, ... of its range, lane d
// feature d of each row (coalesced 256-byte row reads; the row's output
// gradients are wavefront-uniform, scalar loads); each lane keeps FP64 sums
// for every output, its rows in increasing order, four rows in flight. The
// 16 wavefronts' sums are then added in a fixed order through LDS.
constexpr int kHgThreads = 1024, kHgGroups = kHgThreads / kPolD;
__global__ void __launch_bounds__(kHgThreads)
head_grad_partial_kernel(const float *__restrict__ feat, const float *__restrict__ dout, int64_t N,
                         int ld, int n_out, int64_t per, double *__restrict__ part) {
  __shared__ double red[kHgGroups / 2][kPolActions][kPolD + 1];
  const int d = threadIdx.x & (kPolD - 1);
  const int rg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t n0 = (int64_t)blockIdx.x * per;
  const int64_t n1 = n0 + per < N ? n0 + per : N;
  double acc[kPolActions], accb[kPolActions];
#pragma unroll
  for (int o = 0; o < kPolActions; ++o) acc[o] = accb[o] = 0.0;
  auto add_row = [&](int64_t n, float f) {
    const float *g = dout + n * ld;
#pragma unroll
    for (int o = 0; o < kPolActions; ++o)
      if (o < n_out) {
        const float go = g[o];
        acc[o] += (double)(go * f);
        accb[o] += (double)go;
      }
  };
  int64_t n = n0 + rg;
  for (; n + 3 * kHgGroups < n1; n += 4 * kHgGroups) {
    const float f0 = feat[n * kPolD + d];
    const float f1 = feat[(n + kHgGroups) * kPolD + d];
    const float f2 = feat[(n + 2 * kHgGroups) * kPolD + d];
    const float f3 = feat[(n + 3 * kHgGroups) * kPolD + d];
    add_row(n, f0);
    add_row(n + kHgGroups, f1);
    add_row(n + 2 * kHgGroups, f2);
    add_row(n + 3 * kHgGroups, f3);
  }
  for (; n < n1; n += kHgGroups) add_row(n, feat[n * kPolD + d]);
  // wavefronts 8..15 store, 0..7 add theirs (fixed pairs), then eight in order
  const int half = kHgGroups / 2;
  if (rg >= half) {
#pragma unroll
    for (int o = 0; o < kPolActions; ++o) {
      red[rg - half][o][d] = acc[o];
      if (d == 0) red[rg - half][o][kPolD] = accb[o];
    }
  }
  __syncthreads();
  if (rg < half) {
#pragma unroll
    for (int o = 0; o < kPolActions; ++o) {
      red[rg][o][d] += acc[o];
      if (d == 0) red[rg][o][kPolD] += accb[o];
    }
  }
  __syncthreads();
  const int ne = n_out * (kPolD + 1);
  for (int j = threadIdx.x; j < ne; j += blockDim.x) {
    const int o = j / (kPolD + 1), i = j - o * (kPolD + 1);
    double s = 0.0;
    for (int r = 0; r < half; ++r) s += red[r][o][i];
    part[(int64_t)blockIdx.x * ne + j] = s;
  }
}

// Partials in block order -> grad in the head's parameter layout: weights
// [8][64], then biases [8]; rows n_out..7 are 0.
__global__ void __launch_bounds__(kPpoThreads)
head_grad_final_kernel(const double *__restrict__ part, int nb, int n_out,
                       float *__restrict__ grad) {
  const int ne = n_out * (kPolD + 1);
  for (int j = threadIdx.x; j < kPolActions * (kPolD + 1); j += blockDim.x) {
    const int o = j / (kPolD + 1), i = j - o * (kPolD + 1);
    double s = 0.0;
    if (j < ne)
      for (int b = 0; b < nb; ++b) s += part[(int64_t)b * ne + j];
    if (i < kPolD)
      grad[o * kPolD + i] = (float)s;
    else
      grad[kPolActions * kPolD + o] = (float)s;
  }
}

int check() { return hipGetLastError() == hipSuccess ? 0 : -1; }

}  // namespace

int launch_critic_tokens(const float *gstate, int64_t N, int M, int lead, float pos_scale,
                         float *tokens, uint8_t *mask, void *stream) {
  const int64_t n = N * (M + lead);
  if (n == 0) return 0;
  hipLaunchKernelGGL(critic_tokens_kernel, dim3((unsigned)((n + kPpoThreads - 1) / kPpoThreads)),
                     dim3(kPpoThreads), 0, (hipStream_t)stream, gstate, N, M, lead,
                     1.0f / pos_scale, tokens, mask);
  return check();
}

int launch_first_column(const float *logits, int64_t N, float *out, void *stream) {
  if (N == 0) return 0;
  hipLaunchKernelGGL(first_column_kernel, dim3((unsigned)((N + kPpoThreads - 1) / kPpoThreads)),
                     dim3(kPpoThreads), 0, (hipStream_t)stream, logits, N, out);
  return check();
}

int launch_head_grad(const float *feat, const float *dout, int64_t N, int ld, int n_out,
                     float *grad, double *part, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (N > 0) {
    const int64_t per = (N + kPpoBlocks - 1) / kPpoBlocks;
    hipLaunchKernelGGL(head_grad_partial_kernel, dim3(kPpoBlocks), dim3(kHgThreads), 0, st, feat,
                       dout, N, ld, n_out, per, part);
    if (check()) return -1;
  }
  // no samples: no partials, a zero gradient
  hipLaunchKernelGGL(head_grad_final_kernel, dim3(1), dim3(kPpoThreads), 0, st, part,
                     N > 0 ? kPpoBlocks : 0, n_out, grad);
  return check();
}

int launch_gae(const float *rewards, const uint8_t *dones, const float *values, int32_t T, int64_t E,
               float gamma, float lambda, float *adv, float *ret, void *stream) {
  if (E == 0 || T == 0) return 0;
  hipLaunchKernelGGL(gae_kernel, dim3((unsigned)((E + kPpoThreads - 1) / kPpoThreads)),
                     dim3(kPpoThreads), 0, (hipStream_t)stream, rewards, dones, values, T, E,
                     (double)gamma, (double)gamma * (double)lambda, adv, ret);
  return check();
}

int launch_ppo_objective(const float *lnew, const float *lold, const int32_t *actions,
                         const float *adv, const float *values, const float *returns, int32_t T,
                         int64_t A, int32_t n_agents, int32_t n_actions, float clip_eps,
                         double *out, float *dlogits, float *dvalues, double *part, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t S = (int64_t)T * A, V = (int64_t)T * (A / n_agents);
  const int64_t ps = (S + kPpoBlocks - 1) / kPpoBlocks, pv = (V + kPpoBlocks - 1) / kPpoBlocks;
  hipLaunchKernelGGL(ppo_policy_kernel, dim3(kPpoBlocks), dim3(kPpoThreads), 0, st, lnew, lold,
                     actions, adv, S, A, n_agents, n_actions, clip_eps, (float)(1.0 / (double)S),
                     dlogits, part, ps > 0 ? ps : 1);
  if (check()) return -1;
  hipLaunchKernelGGL(ppo_value_kernel, dim3(kPpoBlocks), dim3(kPpoThreads), 0, st, values, returns,
                     V, (float)(1.0 / (double)V), dvalues, part, pv > 0 ? pv : 1);
  if (check()) return -1;
  hipLaunchKernelGGL(ppo_final_kernel, dim3(1), dim3(64), 0, st, part, kPpoBlocks,
                     1.0 / (double)S, 1.0 / (double)V, out);
  return check();
}

}  // namespace mil
