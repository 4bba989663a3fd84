// Environment kernels for gfx950: reset, the persistent multi-step rollout
// (which is also the one-step kernel, with T = 1), the metrics reduction and
// a state copy.
//
// Mapping. One lane per (agent, lane-of-agent): an environment with n_a
// agents occupies n_a * G consecutive lanes of one wavefront (G = lanes per
// agent, 1 or 2; with G = 2 the agent's targets are split between its two
// lanes by parity). Environments are packed by shape, so every lane of a
// wavefront has the same (n_a, n_t) and all loops over entities have
// wave-uniform trip counts. Per-lane state (the agent, the targets the lane
// owns, its trackers' range histories and estimates) stays in registers for
// the whole rollout; target positions are broadcast through a per-wavefront
// LDS slab, agent positions and tracking errors through ds_bpermute (2x2
// batches: targets advanced in every lane of the env, broadcasts by DPP
// quad permutations). Large batches may run under a dynamic schedule that
// hands chunks of steps between wavefronts (see take_unit).
//
// Step semantics (arXiv 2505.08222): kinematic surrogate with heading noise
// (Sec. IV-A-3), noisy ranges after the move, one range-only least-squares
// tracker per (agent, target) over the last W ranges (Sec. III-A, IV-A-2),
// tracking reward Eq. (1) normalised by the number of targets with the crash
// penalty (text after Eq. 2), entity-token observation (Sec. IV-A-2 and the
// TransfMAPPO caption), termination at the step limit only.
#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>

#include "env_internal.h"
#include "learned_internal.h"
#include "ls_device.h"
#include "rng.h"

namespace mil {

constexpr uint32_t kStatusBadAction = 0x1u;
constexpr uint32_t kStatusNonFinite = 0x2u;

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Eq. (1): 1 below eps_min, exp(-2t/(1-t)) with t = (e-eps_min)/(eps_max-eps_min)
// up to eps_max, 0 from eps_max on (the limit of the exponential there).
__device__ __forceinline__ float tracking_reward(float e, float emin, float emax, float inv_span) {
  if (e < emin) return 1.0f;
  if (!(e < emax)) return 0.0f;
  const float t = (e - emin) * inv_span;  // inv_span = 1 / (emax - emin)
  return __expf(-2.0f * t * __builtin_amdgcn_rcpf(1.0f - t));
}

// A heading is an angle: kept in [-pi, pi] after every update.
__device__ __forceinline__ float wrap_angle(float a) {
  const float pi = 3.14159265358979f, two_pi = 6.28318530717959f;
  if (a > pi) return a - two_pi;
  if (a < -pi) return a + two_pi;
  return a;
}

__device__ __forceinline__ float norm2(float dx, float dy) { return fast_sqrt(fmaf(dx, dx, dy * dy)); }
// |(dx, dy)|^2, for comparisons against a squared radius (no square root)
__device__ __forceinline__ float sqnorm(float dx, float dy) { return fmaf(dx, dx, dy * dy); }

// 1/d for finite d > 0: the hardware estimate refined by two Newton steps
// (each doubles the number of correct bits), instead of the long IEEE divide
// sequence.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// sin and cos of an angle in radians via the revolution-based hardware ops.
__device__ __forceinline__ void sincos_rad(float a, float &s, float &c) {
  sincos_rev(a * 0.15915494309189535f, s, c);
}

__device__ __forceinline__ void store_token(float *dst, float dx, float dy, float is_self,
                                            float is_agent, float is_target) {
  float2 *d = reinterpret_cast<float2 *>(dst);
  d[0] = make_float2(dx, dy);
  d[1] = make_float2(0.0f, is_self);
  d[2] = make_float2(is_agent, is_target);
}

// A Philox draw whose key schedule is rebuilt at the call (a few scalar adds)
// instead of being held in 20 scalar registers across the step loop.
__device__ __forceinline__ u32x4 draw(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                      uint32_t key0, uint32_t key1) {
  asm volatile("" : "+s"(key0), "+s"(key1));
  return philox4x32_10(c0, c1, c2, c3, key0, key1);
}

// Environments of at most two targets keep them in registers in every lane
// (one draw block: no owner has to broadcast them through LDS).
template <int S>
constexpr bool kRegTargets = (S == 2);

// Observation tokens a wavefront can stage: 64 agents (lanes) of at most
// 2S tokens each. Only a token's offset word and mask are staged; the type
// columns follow from the token's position and are rebuilt while copying.
template <int S>
constexpr int kStageTok = 64 * 2 * S;

// Dynamic schedule of the rollout. A unit is (chunk c, wave group w): the
// steps [c*span, (c+1)*span) of the environments that the static mapping
// gives to wavefront w. Units are numbered chunk-major, u = c*groups + w, and
// handed out by an atomic counter in queue[0]; queue[1 + w] counts the chunks
// of group w that are complete (their state is back in memory). Unit (c, w)
// waits for queue[1 + w] >= c; unit (c-1, w) has a smaller number, so it was
// taken earlier by a wavefront that is running, and the wait ends.
//
// Hand-over. The state a group carries from one chunk to the next is written
// and read with device-coherent accesses (relaxed atomics at agent scope: the
// stores write through and the loads miss in the per-XCD L2 caches, so a
// wavefront on another XCD sees the memory copy). Publishing therefore needs
// only the completion of those stores before the flag store, and taking over
// only the flag load before the state loads; no cache-wide write-back or
// invalidation is involved.
constexpr uint32_t kStatusSchedule = 0x4u;  // a chunk wait gave up (never expected)
constexpr int kMaxPolls = 1 << 22;

// (global address space spelled out: a generic pointer would become a flat
// access, which also counts against the LDS wait counter)
template <typename T>
__device__ __forceinline__ T ld_dc(const T *p) {
  using GT = __attribute__((address_space(1))) T;
  return __hip_atomic_load((GT *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dc(T *p, T v) {
  using GT = __attribute__((address_space(1))) T;
  __hip_atomic_store((GT *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Carried state: device-coherent under the dynamic schedule (dc, uniform),
// ordinary cached accesses under the static one.
template <typename T>
__device__ __forceinline__ T ld_st(const T *p, bool dc) {
  using GT = __attribute__((address_space(1))) T;
  return dc ? ld_dc(p) : *(const GT *)p;
}
template <typename T>
__device__ __forceinline__ void st_st(T *p, T v, bool dc) {
  using GT = __attribute__((address_space(1))) T;
  if (dc)
    st_dc(p, v);
  else
    *(GT *)p = v;
}

__device__ __forceinline__ int take_unit(int32_t *queue, int lane) {
  int u = 0;
  if (lane == 0)
    u = __hip_atomic_fetch_add((__attribute__((address_space(1))) int32_t *)queue, 1,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_amdgcn_readlane(u, 0);
}

// Wait (lane 0 polls) until the group has `need` chunks complete. False if
// the poll limit ran out.
__device__ __forceinline__ bool wait_chunks(int32_t *flag, int need, int lane) {
  int ok = 1;
  if (lane == 0) {
    for (int polls = 0; ld_dc(flag) < need; ++polls) {
      if (polls >= kMaxPolls) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
  }
  ok = __builtin_amdgcn_readlane(ok, 0);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // state loads stay after the poll
  return ok != 0;
}

// Publish that the group's state for `done` chunks is in memory: every store
// of this wavefront has completed before the flag is written.
__device__ __forceinline__ void publish_chunks(int32_t *flag, int done, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  if (lane == 0) st_dc(flag, done);
}

__global__ void queue_init_kernel(int32_t *queue, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) queue[i] = 0;
}

// Broadcast inside an environment of the 2x2 kernels, by DPP (no LDS round
// trip). With S = 2 an environment spans lpe = n_a * G lanes (1, 2 or 4)
// starting at a multiple of lpe, so it never leaves an aligned quad: the
// value of lane base + OFF reaches every lane of the environment through one
// quad permutation, whose pattern depends only on OFF and lpe. Whole quads
// are active.
template <int OFF>
__device__ __forceinline__ int env_bcast_q(int v, int lpe) {
  constexpr int p4 = (OFF & 3) * 0x55;  // lpe 4: every lane takes OFF
  constexpr int p2 = (OFF & 1) | ((OFF & 1) << 2) | ((2 + (OFF & 1)) << 4) | ((2 + (OFF & 1)) << 6);
  const int w4 = __builtin_amdgcn_mov_dpp(v, p4, 0xF, 0xF, false);
  const int w2 = __builtin_amdgcn_mov_dpp(v, p2, 0xF, 0xF, false);
  return lpe == 4 ? w4 : (lpe == 2 ? w2 : v);  // lpe 1: OFF is 0, the lane itself
}

// Value of lane base_lane + off of the wavefront (off < lpe, a compile-time
// constant after unrolling): DPP for S = 2, ds_bpermute for larger envs.
template <int S, typename T>
__device__ __forceinline__ T env_shfl(T v, int base_lane, int off, int lpe) {
  if constexpr (S == 2) {
    int w = 0;
    const int x = __builtin_bit_cast(int, v);
    switch (off) {
      case 0: w = env_bcast_q<0>(x, lpe); break;
      case 1: w = env_bcast_q<1>(x, lpe); break;
      case 2: w = env_bcast_q<2>(x, lpe); break;
      default: w = env_bcast_q<3>(x, lpe); break;
    }
    return __builtin_bit_cast(T, w);
  } else {
    return __shfl(v, base_lane + off);
  }
}

// Element (g + G*sl) of a per-env array held with compile-time indices.
template <int G, int N>
__device__ __forceinline__ float pick(const float (&arr)[N], int g, int sl) {
  if constexpr (G == 1) {
    return arr[sl];
  } else {
    const int j0 = G * sl;
    const float a = arr[j0 < N ? j0 : N - 1];
    const float b = arr[j0 + 1 < N ? j0 + 1 : N - 1];
    return g ? b : a;
  }
}

// ---------------------------------------------------------------------------
// Pairwise spawn (Sec. IV-A-2: every entity 50-200 m from every other), by
// the env's reset thread: entities take distinct sites of a hexagonal patch
// about the centre (the centre, six sites at distance sp, six at sp sqrt(3)
// between them), in a Fisher-Yates order, the patch rotated by a uniform
// angle and each entity moved by a uniform offset in the square of half-side
// h; sp = spawn_min + 2 sqrt(2) h and 2 sqrt(3) sp + 2 sqrt(2) h <= spawn_max
// keep every pair within the bounds (h at 0.9 of its largest value). Words
// of Philox(1 + k, env, env entity, reset), k = 0..9, in order: 12 swap
// choices, the rotation, then two offset words per entity (agents first).
// ---------------------------------------------------------------------------
__device__ void spawn_pairwise(const DevParams &p, const DevState &s, int64_t e, uint32_t id,
                               uint32_t c3, int na, int nt) {
  const float r2 = 1.41421356237310f, r3 = 1.73205080756888f;
  const float h = 0.9f * (p.spawn_max - 2.0f * r3 * p.spawn_min) / (2.0f * r2 * (2.0f * r3 + 1.0f));
  const float sp = p.spawn_min + 2.0f * r2 * h;
  uint32_t w[40];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    const u32x4 x = philox4x32_10(1u + (uint32_t)k, id, kEntEnv, c3, p.key0, p.key1);
    w[4 * k] = x.x;
    w[4 * k + 1] = x.y;
    w[4 * k + 2] = x.z;
    w[4 * k + 3] = x.w;
  }
  int perm[13];
#pragma unroll
  for (int k = 0; k < 13; ++k) perm[k] = k;
  for (int k = 12; k >= 1; --k) {
    const int j = (int)choice(w[12 - k], (uint32_t)(k + 1));
    const int tmp = perm[k];
    perm[k] = perm[j];
    perm[j] = tmp;
  }
  const float rot = u01(w[12]);  // revolutions
  const int n = na + nt;
  for (int m = 0; m < n; ++m) {
    const int site = perm[m];
    float rad = 0.0f, rev = 0.0f;
    if (site >= 1 && site <= 6) {
      rad = sp;
      rev = (float)(site - 1) / 6.0f;
    } else if (site >= 7) {
      rad = sp * r3;
      rev = 1.0f / 12.0f + (float)(site - 7) / 6.0f;
    }
    float sn, cs;
    sincos_rev(rev + rot, sn, cs);
    const float x = fmaf(rad, cs, h * (2.0f * u01(w[13 + 2 * m]) - 1.0f));
    const float y = fmaf(rad, sn, h * (2.0f * u01(w[14 + 2 * m]) - 1.0f));
    if (m < na) {
      s.ax[s.aoff[e] + m] = x;
      s.ay[s.aoff[e] + m] = y;
    } else {
      s.tx[s.toff[e] + (m - na)] = x;
      s.ty[s.toff[e] + (m - na)] = y;
    }
  }
}

// ---------------------------------------------------------------------------
// Reset: one thread per (env, slot); slots 0..7 agents, 8..15 targets, 16 env.
// ---------------------------------------------------------------------------
__global__ void reset_kernel(DevParams p, DevState s, uint32_t episode) {
  constexpr int kSlots = 17;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t e = tid / kSlots;
  const int slot = (int)(tid - e * kSlots);
  if (e >= s.E) return;
  const uint32_t id = s.env_id[e];
  const int na = s.cnt_a[e], nt = s.cnt_t[e];
  const uint32_t c3 = (episode << 4) | kPurposeReset;
  if (slot < 8) {
    const int i = slot;
    if (i >= na) return;
    const u32x4 x = philox4x32_10(0u, id, (uint32_t)i, c3, p.key0, p.key1);
    const int64_t a = s.aoff[e] + i;
    if (p.spawn_mode == 0) {
      const float rad = p.spawn_r * sqrtf(u01(x.x));
      float sn, cs;
      sincospif(2.0f * u01(x.y), &sn, &cs);
      s.ax[a] = rad * cs;
      s.ay[a] = rad * sn;
    }
    s.apsi[a] = -3.14159265358979f + 6.28318530717959f * u01(x.z);
    s.arud[a] = (p.n_rudder - 1) / 2;  // rudder at the middle angle
    const int64_t pb = s.poff[e] + (int64_t)i * nt;
    for (int j = 0; j < nt; ++j) s.ev[pb + j] = 0;
  } else if (slot < 16) {
    const int j = slot - 8;
    if (j >= nt) return;
    const u32x4 x = philox4x32_10(0u, id, kEntTargetBlock + (uint32_t)j, c3, p.key0, p.key1);
    const int64_t q = s.toff[e] + j;
    if (p.spawn_mode == 0) {
      s.tx[q] = -0.5f * p.area + p.area * u01(x.x);
      s.ty[q] = -0.5f * p.area + p.area * u01(x.y);
    }
    s.tpsi[q] = -3.14159265358979f + 6.28318530717959f * u01(x.z);
    s.tv[q] = p.tv_lo + (p.tv_hi - p.tv_lo) * u01(x.w);
  } else {
    const u32x4 x = philox4x32_10(0u, id, kEntEnv, c3, p.key0, p.key1);
    s.sigma[e] = p.sr_lo + (p.sr_hi - p.sr_lo) * u01(x.x);
    if (p.spawn_mode == 1) spawn_pairwise(p, s, e, id, c3, na, nt);
    s.macc[3 * e] = 0.0;
    s.macc[3 * e + 1] = 0.0;
    s.macc[3 * e + 2] = 0.0;
    s.miacc[2 * e] = 0;
    s.miacc[2 * e + 1] = 0;
  }
}

// Initial observation and global state after reset: one thread per (env,
// slot); agents write their tokens (no tracker has an estimate yet, every
// broadcast is received within the comm range), both write global state.
__global__ void reset_obs_kernel(DevParams p, DevState s, DevOut o) {
  constexpr int kSlots = 16;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t e = tid / kSlots;
  const int slot = (int)(tid - e * kSlots);
  if (e >= s.E) return;
  const int na = s.cnt_a[e], nt = s.cnt_t[e];
  const int64_t ab = s.aoff[e], tb = s.toff[e];
  const int64_t gb = ab + tb;
  if (slot < 8) {
    const int i = slot;
    if (i >= na) return;
    const float ax = s.ax[ab + i], ay = s.ay[ab + i];
    if (o.gstate) {
      float *gs = o.gstate + (gb + i) * 6;
      gs[0] = ax; gs[1] = ay; gs[2] = 0.0f; gs[3] = p.agent_speed; gs[4] = s.apsi[ab + i]; gs[5] = 0.0f;
    }
    const int64_t kb = s.koff[e] + (int64_t)i * (na + nt);
    int m = 0;
    if (o.obs) store_token(o.obs + (kb + m) * 6, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f);
    if (o.obs_mask) o.obs_mask[kb + m] = 1;
    ++m;
    for (int k = 0; k < na; ++k) {
      if (k == i) continue;
      const float dx = s.ax[ab + k] - ax, dy = s.ay[ab + k] - ay;
      const bool ok = sqnorm(dx, dy) <= p.comm_range * p.comm_range;
      if (o.obs) store_token(o.obs + (kb + m) * 6, ok ? dx : 0.0f, ok ? dy : 0.0f, 0.0f, 1.0f, 0.0f);
      if (o.obs_mask) o.obs_mask[kb + m] = ok;
      ++m;
    }
    for (int j = 0; j < nt; ++j) {
      if (o.obs) store_token(o.obs + (kb + m) * 6, 0.0f, 0.0f, 0.0f, 0.0f, 1.0f);
      if (o.obs_mask) o.obs_mask[kb + m] = 0;
      ++m;
    }
  } else {
    const int j = slot - 8;
    if (j >= nt || !o.gstate) return;
    float *gs = o.gstate + (gb + na + j) * 6;
    gs[0] = s.tx[tb + j]; gs[1] = s.ty[tb + j]; gs[2] = 0.0f; gs[3] = s.tv[tb + j];
    gs[4] = s.tpsi[tb + j]; gs[5] = 1.0f;
  }
}

// ---------------------------------------------------------------------------
// Rollout: T steps per launch. S = largest supported entity count per env
// (agents and targets), WC = register window capacity (W <= WC), G = lanes
// per agent. FULL = false is the lean form for the common case: actions
// drawn in-kernel, only obs / obs_mask / reward / done recorded, no
// detection cut, no dropped broadcasts, no Gauss-Newton refinement. It gives
// the same bits as the full form on those outputs and carries none of the
// other paths' pointers and registers.
// ---------------------------------------------------------------------------
template <int S, int WC, int G, bool FULL, bool STAGE>
__global__ void __launch_bounds__(256, (!FULL && WC == 10 && S <= 5) ? 2 : ((FULL && WC == 1) ? (S == 2 ? 3 : 2) : 1))
rollout_kernel(DevParams p, const DevState *sp, int32_t num_waves, int32_t t0, int32_t T,
               uint32_t episode, const int32_t *__restrict__ actions, DevOut o, DevExt ext,
               int32_t chunk) {
  constexpr bool stage = STAGE && !FULL;
  // split step (full form only): phase 1 moves, phase 2 observes; phase 3
  // observes the launch's first step and moves its second
  const bool move_all = !FULL || ext.phase != 2;
  const bool observe_all = !FULL || ext.phase != 1;
  constexpr int MA = S, MT = S;
  constexpr int NPL = (MT + G - 1) / G;  // (agent, target) pairs per lane
  constexpr int NQ = (MT + 3) / 4;       // range-noise draws per agent
  // per wavefront: the targets of its envs, (x, y, heading, speed); then
  // (lean form) the staging area of the wavefront's observation block
  extern __shared__ float4 lds_targets[];
  __shared__ float lds_dpsi[4][8];  // per wavefront: the action table

  const int lane = threadIdx.x & 63;
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (lane < 8) lds_dpsi[wib][lane] = p.dpsi[lane];
  wave_lds_fence();

  // static schedule (chunk 0): wavefront = group, all T steps; dynamic: units
  // from the queue (see take_unit)
  const bool dyn = chunk > 0;
  const int span = dyn ? chunk : T;
  const int units = dyn ? num_waves * ((T + span - 1) / span) : num_waves;
  int unit = dyn ? take_unit(sp->queue, lane)
                 : ext.wave0 + __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + wib);
  while (unit < units) {
    const int cix = unit / num_waves;
    const int wave = unit - cix * num_waves;
    uint32_t status = 0;
    if (cix > 0 && !wait_chunks(sp->queue + 1 + wave, cix, lane) && lane == 0)
      status |= kStatusSchedule;
    const int s_begin = cix * span;
    const int s_end = min(T, s_begin + span);
    // prologue and epilogue only (reloaded after the loop); a copy, so that the
    // device-coherent accesses below do not make the compiler re-read each field
    const DevState s = *sp;
    const ClassInfo C = s.classes[s.wave_class[wave]];
    const int na = C.na, nt = C.nt;
    const int lpe = na * G;
    const int epw = 64 / lpe;
    const int el = lane / lpe;
    const int r = lane - el * lpe;
    const int i = r / G;
    const int g = r - i * G;
    const int64_t ce_raw = (int64_t)(wave - C.wave0) * epw + el;
    const bool active = (el < epw) && (ce_raw < C.nenv);
    const int64_t ce = active ? ce_raw : 0;
    const int64_t e = C.env0 + ce;
    const int64_t aidx = C.aoff0 + ce * na + i;
    const int64_t tbase = C.toff0 + ce * nt;
    const int64_t pbase = C.poff0 + ce * na * nt + (int64_t)i * nt;
    const int64_t kbase = C.koff0 + ce * na * (na + nt) + (int64_t)i * (na + nt);
    const int64_t gbase = C.aoff0 + C.toff0 + ce * (na + nt);
    const int base_lane = el * lpe;
    const uint32_t env_id = s.env_id[e];
    const float sig_r = s.sigma[e];
    const int W = p.window;
    const uint32_t c3dyn = (episode << 4) | kPurposeDynamics;
    const uint32_t c3meas = (episode << 4) | kPurposeMeasure;
    const float vdt = p.agent_speed * p.dt;
    const int nB = (nt + 1) >> 1;
    const double tau = (double)p.tau;
    const double invW = 1.0 / (double)W;
    const float inv_span = 1.0f / (p.eps_max - p.eps_min);
    const float comm2 = p.comm_range * p.comm_range, dsafe2 = p.d_safe * p.d_safe;
    const float inv_nt = 1.0f / (float)nt;
    const float kInf = __int_as_float(0x7f800000);
    const float kNaN = __int_as_float(0x7fc00000);
    float4 *tl = lds_targets + (wib * 64 + (el < 64 ? el : 63)) * MT;  // this env's targets
    // staging of the wavefront's observation tokens (offsets only; the type
    // columns follow from the token's position) and masks, in output order
    float2 *const st_base =
        reinterpret_cast<float2 *>(lds_targets + (size_t)(blockDim.x >> 6) * 64 * MT);
    float2 *st_xy = st_base + (size_t)wib * kStageTok<S>;
    uint8_t *st_m = reinterpret_cast<uint8_t *>(st_base + (size_t)(blockDim.x >> 6) * kStageTok<S>) +
                    (size_t)wib * kStageTok<S>;
    const int ntok = na + nt;
    const int agent_w = el * na + i;  // agent index inside the wavefront
    const int64_t env_left = C.nenv - (int64_t)(wave - C.wave0) * epw;  // >= 1 for a live wave
    const int64_t nenv_w = env_left < epw ? env_left : epw;
    const int ntok_w = (int)nenv_w * na * ntok;  // tokens of the wavefront's active agents
    const int64_t kbase_w = C.koff0 + (int64_t)(wave - C.wave0) * epw * na * ntok;
    const int m_lane0 = lane % ntok, m_step = 64 % ntok;  // token positions for the block copy

    // ---- load state: targets of the env into LDS (each lane its own blocks);
    // with at most two targets (one draw block), every lane of the env keeps
    // them in registers and advances them itself (the same draws and
    // arithmetic in each lane), so no LDS round trip is needed
    float4 treg[kRegTargets<S> ? 2 : 1];
    if constexpr (kRegTargets<S>) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        treg[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (j < nt) {
          const int64_t idx = tbase + j;
          treg[j] = make_float4(ld_st(&s.tx[idx], dyn), ld_st(&s.ty[idx], dyn),
                                ld_st(&s.tpsi[idx], dyn), s.tv[idx]);
        }
      }
    } else {
      for (int q = r; q < nB; q += lpe) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const int j = 2 * q + m;
          if (j < nt) {
            const int64_t idx = tbase + j;
            tl[j] = make_float4(ld_st(&s.tx[idx], dyn), ld_st(&s.ty[idx], dyn),
                                ld_st(&s.tpsi[idx], dyn), s.tv[idx]);
          }
        }
      }
    }
    float ax = ld_st(&s.ax[aidx], dyn), ay = ld_st(&s.ay[aidx], dyn);
    float apsi = ld_st(&s.apsi[aidx], dyn);
    int rud = (FULL && p.action_mode == 1) ? ld_st(&s.arud[aidx], dyn) : 0;
    float hx[WC], hy[WC], hr[NPL][WC], ex[NPL], ey[NPL];
    uint32_t evb = 0;
    // pooled tracker: which agents' broadcasts of each window entry this
    // agent received (bit k = agent k; its own bit always set)
    uint32_t recm[FULL ? WC : 1];
#pragma unroll
    for (int k = 0; k < WC; ++k) {
      hx[k] = (k < W) ? ld_st(&s.hx[(int64_t)k * s.A + aidx], dyn) : 0.0f;
      hy[k] = (k < W) ? ld_st(&s.hy[(int64_t)k * s.A + aidx], dyn) : 0.0f;
      if constexpr (FULL)
        recm[k] = (p.pooled && k < W) ? (uint32_t)ld_st(&s.hrec[(int64_t)k * s.A + aidx], dyn) : 0u;
    }
#pragma unroll
    for (int sl = 0; sl < NPL; ++sl) {
      const int j = g + G * sl;
      const int64_t pidx = pbase + (j < nt ? j : 0);
#pragma unroll
      for (int k = 0; k < WC; ++k)
        hr[sl][k] = (k < W) ? ld_st(&s.hr[(int64_t)k * s.P + pidx], dyn) : 0.0f;
      ex[sl] = ld_st(&s.ex[pidx], dyn);
      ey[sl] = ld_st(&s.ey[pidx], dyn);
      if (j < nt && ld_st(&s.ev[pidx], dyn)) evb |= 1u << sl;
    }
    double acc_rew = 0.0, acc_err = 0.0, acc_err2 = 0.0;
    int acc_cnt = 0, acc_crash = 0;
    if (active && r == 0) {
      acc_rew = ld_st(&s.macc[3 * e], dyn);
      acc_err = ld_st(&s.macc[3 * e + 1], dyn);
      acc_err2 = ld_st(&s.macc[3 * e + 2], dyn);
      acc_cnt = ld_st(&s.miacc[2 * e], dyn);
      acc_crash = ld_st(&s.miacc[2 * e + 1], dyn);
    }
    wave_lds_fence();  // the target slab is complete

    for (int step = s_begin; step < s_end; ++step) {
      const uint32_t t = (uint32_t)(t0 + step);
      const bool move = (FULL && ext.phase == 3) ? step > 0 : move_all;
      const bool observe = (FULL && ext.phase == 3) ? step == 0 : observe_all;

      // ---- agent: action, heading noise, turn then move (Sec. IV-A-3)
      const u32x4 xa = draw(t, env_id, (uint32_t)i, c3dyn, p.key0, p.key1);
      int act;
      if (FULL && actions) {
        act = actions[(int64_t)step * o.A + aidx];
        if (act < 0 || act >= p.n_actions) {
          act = -1;
          if (active) status |= kStatusBadAction;
        }
      } else {
        act = (int)choice(xa.x, (uint32_t)p.n_actions);
      }
      if (move) {
        float za, zb;
        normal2(xa.y, xa.z, za, zb);
        float dpsi;
        if (FULL && p.action_mode == 1) {
          // rudder: one angle down / keep / one up (Sec. IV-A-2), then the
          // heading change theta(gamma) of the rudder angle
          if (act >= 0) rud = min(max(rud + act - 1, 0), p.n_rudder - 1);
          dpsi = lds_dpsi[wib][rud];
        } else {
          dpsi = act >= 0 ? lds_dpsi[wib][act] : 0.0f;
        }
        apsi = wrap_angle((apsi + dpsi) + p.sig_a * za);
        float sn, cs;
        sincos_rad(apsi, sn, cs);
        ax = fmaf(vdt, cs, ax);
        ay = fmaf(vdt, sn, ay);
      }
      const bool comm_ok = FULL ? !(u01(xa.w) < p.comm_loss_p) : true;

      // ---- targets (blocks of two, each owned by one lane, or by every lane
      // of the env when they stay in registers): heading random walk
      auto walk = [&](float4 &tg, float z) {
        tg.z = wrap_angle(tg.z + p.sig_t * z);
        float sn, cs;
        sincos_rad(tg.z, sn, cs);
        const float step_len = tg.w * p.dt;
        tg.x = fmaf(step_len, cs, tg.x);
        tg.y = fmaf(step_len, sn, tg.y);
      };
      float tpx[MT], tpy[MT];
      if constexpr (kRegTargets<S>) {
        if (move) {
          const u32x4 xt = draw(t, env_id, kEntTargetBlock, c3dyn, p.key0, p.key1);
          float zt[2];
          normal2(xt.x, xt.y, zt[0], zt[1]);
#pragma unroll
          for (int j = 0; j < 2; ++j)
            if (j < nt) walk(treg[j], zt[j]);
        }
#pragma unroll
        for (int j = 0; j < MT; ++j) {
          tpx[j] = j < nt ? treg[j].x : 0.0f;
          tpy[j] = j < nt ? treg[j].y : 0.0f;
        }
      } else {
        for (int q = r; move && q < nB; q += lpe) {
          const u32x4 xt =
              draw(t, env_id, kEntTargetBlock + (uint32_t)q, c3dyn, p.key0, p.key1);
          float zt[2];
          normal2(xt.x, xt.y, zt[0], zt[1]);
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            const int j = 2 * q + m;
            if (j < nt) {
              float4 tg = tl[j];
              walk(tg, zt[m]);
              tl[j] = tg;
            }
          }
        }
        wave_lds_fence();
#pragma unroll
        for (int j = 0; j < MT; ++j) {
          tpx[j] = 0.0f;
          tpy[j] = 0.0f;
          if (j < nt) {
            const float4 v = tl[j];
            tpx[j] = v.x;
            tpy[j] = v.y;
          }
        }
        wave_lds_fence();  // every lane has read before next step's owners write
      }

      if (move) {
      // ---- noisy ranges after the move; missing beyond the detection range
        float rnew[NPL];
#pragma unroll
        for (int sl = 0; sl < NPL; ++sl) rnew[sl] = kNaN;
#pragma unroll
        for (int q4 = 0; q4 < NQ; ++q4) {
          if (4 * q4 < nt) {
            const u32x4 xr = draw(t, env_id, kEntRangeRow + 8u * (uint32_t)i + (uint32_t)q4, c3meas,
                                  p.key0, p.key1);
            float zr[4];
            normal2(xr.x, xr.y, zr[0], zr[1]);
            normal2(xr.z, xr.w, zr[2], zr[3]);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const int j = 4 * q4 + m;
              if (j < MT && j < nt && (j % G) == g) {
                const float dist = norm2(ax - tpx[j], ay - tpy[j]);
                const float rr = fmaf(sig_r, zr[m], dist);
                rnew[j / G] = (!FULL || dist <= p.det_range) ? rr : kNaN;
              }
            }
          }
        }
  
        // ---- range history: entry 0 is the newest
#pragma unroll
        for (int k = WC - 1; k > 0; --k) {
          hx[k] = hx[k - 1];
          hy[k] = hy[k - 1];
#pragma unroll
          for (int sl = 0; sl < NPL; ++sl) hr[sl][k] = hr[sl][k - 1];
        }
        hx[0] = ax;
        hy[0] = ay;
#pragma unroll
        for (int sl = 0; sl < NPL; ++sl) hr[sl][0] = rnew[sl];
        if constexpr (FULL) {
          if (p.pooled) {
            // what this agent receives this step: the observation's rule (a
            // broadcast not dropped, within comm_range), its own entry always
#pragma unroll
            for (int k = WC - 1; k > 0; --k) recm[k] = recm[k - 1];
            uint32_t bits = 0;
#pragma unroll
            for (int k = 0; k < MA; ++k) {
              if (k < na) {
                const float ox = env_shfl<S>(ax, base_lane, k * G, lpe);
                const float oy = env_shfl<S>(ay, base_lane, k * G, lpe);
                const int oc = env_shfl<S>((int)comm_ok, base_lane, k * G, lpe);
                if (k == i || (oc && sqnorm(ox - ax, oy - ay) <= comm2)) bits |= 1u << k;
              }
            }
            recm[0] = bits;
          }
        }
      }
      if (FULL && ext.win && move && active) {
        // phase 1 hands the windows to the estimator (entry 0 newest)
#pragma unroll
        for (int sl = 0; sl < NPL; ++sl) {
          const int j = g + G * sl;
          if (j < nt) {
            const int64_t pidx = pbase + j;
            float *dst = ext.win + pidx * (int64_t)(3 * W);
            if (WC % 4 == 0 && W == WC) {  // 16-byte aligned windows: 12-float groups
              float4 *d4 = reinterpret_cast<float4 *>(dst);
#pragma unroll
              for (int k = 0; k < WC; k += 4) {
                d4[3 * (k / 4)] = make_float4(hx[k], hy[k], hr[sl][k], hx[k + 1]);
                d4[3 * (k / 4) + 1] = make_float4(hy[k + 1], hr[sl][k + 1], hx[k + 2], hy[k + 2]);
                d4[3 * (k / 4) + 2] = make_float4(hr[sl][k + 2], hx[k + 3], hy[k + 3], hr[sl][k + 3]);
              }
            } else {
#pragma unroll
              for (int k = 0; k < WC; ++k)
                if (k < W) {
                  dst[3 * k] = hx[k];
                  dst[3 * k + 1] = hy[k];
                  dst[3 * k + 2] = hr[sl][k];
                }
            }
            if (ext.wsig) ext.wsig[pidx] = sig_r;
          }
        }
      }
      if (FULL && ext.meas && move && active) {
        // phase 1 hands each tracker's newest entry to the particle filter
#pragma unroll
        for (int sl = 0; sl < NPL; ++sl) {
          const int j = g + G * sl;
          if (j < nt)
            reinterpret_cast<float4 *>(ext.meas)[pbase + j] = make_float4(ax, ay, hr[sl][0], 0.0f);
        }
      }
      if (!observe) continue;  // phase 1 ends here: the estimator runs next
      const int filled = min((int)t + 1, W);

      // ---- trackers (Sec. III-A): linearised LS about the centroid of the
      // agent's window, FP64. With every entry present and no refinement the
      // agent's 2x2 matrix S = sum u u^T and G = sum u |u|^2 are shared by its
      // trackers and each tracker only adds g = G - sum u_k r_k^2 (the r-bar^2
      // term of the centred form vanishes because sum u_k = 0). Other trackers
      // take the general path below.
      uint32_t pending = 0;
      if (FULL && ext.phase >= 2 && !ext.est) {
        // the particle filter has written this step's estimates into the state
      } else if (FULL && p.pooled) {
        // ---- pooled tracker: the agent's own entries and those of every
        // agent whose broadcast of that entry it received; each lane's window
        // goes to LDS, then a two-pass centred LS over the received rows (FP64)
        constexpr int WS = WC * (2 + NPL);  // floats of one lane's window
        float *pw = reinterpret_cast<float *>(lds_targets + (size_t)(blockDim.x >> 6) * 64 * MT) +
                    (size_t)wib * 64 * WS;
        {
          float *mine = pw + lane * WS;
#pragma unroll
          for (int k = 0; k < WC; ++k) {
            mine[k] = hx[k];
            mine[WC + k] = hy[k];
#pragma unroll
            for (int sl = 0; sl < NPL; ++sl) mine[(2 + sl) * WC + k] = hr[sl][k];
          }
        }
        wave_lds_fence();
#pragma unroll
        for (int sl = 0; sl < NPL; ++sl) {
          const int j = g + G * sl;
          if (j < nt) {
            int n = 0;
            double mx = 0.0, my = 0.0, mr = 0.0;
            for (int k = 0; k < na; ++k) {
              const float *src = pw + (base_lane + k * G + g) * WS;
#pragma unroll
              for (int e = 0; e < WC; ++e) {
                const float rk = src[(2 + sl) * WC + e];
                if (e < filled && ((recm[e] >> k) & 1u) && rk == rk) {
                  mx += (double)src[e];
                  my += (double)src[WC + e];
                  mr += (double)rk;
                  ++n;
                }
              }
            }
            if (n >= 3) {
              const double inv = 1.0 / (double)n;
              mx *= inv;
              my *= inv;
              mr *= inv;
              double sxx = 0.0, sxy = 0.0, syy = 0.0, gx = 0.0, gy = 0.0;
              for (int k = 0; k < na; ++k) {
                const float *src = pw + (base_lane + k * G + g) * WS;
#pragma unroll
                for (int e = 0; e < WC; ++e) {
                  const float rk = src[(2 + sl) * WC + e];
                  if (e < filled && ((recm[e] >> k) & 1u) && rk == rk) {
                    const double ux = (double)src[e] - mx, uy = (double)src[WC + e] - my;
                    const double d = (double)rk - mr;
                    const double c = fma(ux, ux, uy * uy) - d * fma(2.0, mr, d);
                    sxx = fma(ux, ux, sxx);
                    sxy = fma(ux, uy, sxy);
                    syy = fma(uy, uy, syy);
                    gx = fma(ux, c, gx);
                    gy = fma(uy, c, gy);
                  }
                }
              }
              const double det = fma(sxx, syy, -sxy * sxy), tr = sxx + syy;
              if (det > tau * tr * tr) {
                const double hd = 0.5 / det;
                const float nx = (float)fma(hd, fma(syy, gx, -sxy * gy), mx);
                const float ny = (float)fma(hd, fma(sxx, gy, -sxy * gx), my);
                if (nx == nx && ny == ny) {
                  ex[sl] = nx;
                  ey[sl] = ny;
                  evb |= 1u << sl;
                }
              }
            }
          }
        }
        wave_lds_fence();  // every lane has read before the next step's writes
      } else if (FULL && ext.phase == 2 && filled == W) {
        // estimates from the external estimator (window full)
#pragma unroll
        for (int sl = 0; sl < NPL; ++sl) {
          const int j = g + G * sl;
          if (j < nt) {
            const int64_t pidx = pbase + j;
            if (ext.flag[pidx] != 2) {
              ex[sl] = ext.est[2 * pidx];
              ey[sl] = ext.est[2 * pidx + 1];
              evb |= 1u << sl;
            }
          }
        }
      } else if (filled >= 3) {
        double mx = 0.0, my = 0.0;
#pragma unroll
        for (int k = 0; k < WC; ++k)
          if (k < filled) {
            mx += (double)hx[k];
            my += (double)hy[k];
          }
        const double invn = (filled == W) ? invW : 1.0 / (double)filled;  // filled is uniform
        mx *= invn;
        my *= invn;
        bool full[NPL];
#pragma unroll
        for (int sl = 0; sl < NPL; ++sl) full[sl] = (g + G * sl) < nt;
        double sxx = 0.0, sxy = 0.0, syy = 0.0, gx[NPL], gy[NPL];
#pragma unroll
        for (int sl = 0; sl < NPL; ++sl) {
          gx[sl] = 0.0;
          gy[sl] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < WC; ++k) {
          if (k < filled) {
            const double ux = (double)hx[k] - mx, uy = (double)hy[k] - my;
            const double nu = fma(ux, ux, uy * uy);
            sxx = fma(ux, ux, sxx);
            sxy = fma(ux, uy, sxy);
            syy = fma(uy, uy, syy);
#pragma unroll
            for (int sl = 0; sl < NPL; ++sl) {
              const float rk = hr[sl][k];
              // lean form: every range is finite while the state is (checked
              // on the estimate below instead of on each entry)
              if constexpr (FULL) full[sl] = full[sl] && (rk == rk);
              const double rr = (double)rk;
              const double c = fma(-rr, rr, nu);
              gx[sl] = fma(ux, c, gx[sl]);
              gy[sl] = fma(uy, c, gy[sl]);
            }
          }
        }
        const double det = fma(sxx, syy, -sxy * sxy), tr = sxx + syy;
        const bool agent_ok = det > tau * tr * tr;
        const double hdet = agent_ok ? 0.5 * recip(det) : 0.0;
#pragma unroll
        for (int sl = 0; sl < NPL; ++sl) {
          const int j = g + G * sl;
          if (j < nt) {
            if (full[sl] && (!FULL || p.gn_iters == 0)) {
              if (agent_ok) {
                const float nx = (float)fma(hdet, fma(syy, gx[sl], -sxy * gy[sl]), mx);
                const float ny = (float)fma(hdet, fma(sxx, gy[sl], -sxy * gx[sl]), my);
                if (FULL || (nx == nx && ny == ny)) {
                  ex[sl] = nx;
                  ey[sl] = ny;
                  evb |= 1u << sl;
                } else if (active) {
                  status |= kStatusNonFinite;  // lean form: hold, flag the broken state
                }
              }
            } else if (FULL) {
              pending |= 1u << sl;
            } else if (active) {
              status |= kStatusNonFinite;  // lean form: every range is finite unless the state is not
            }
          }
        }
      }
      // general path: missing entries or Gauss-Newton refinement (one copy of
      // the solver, the tracker's history selected into a scratch row)
      while (FULL && pending) {
        const int sl = __builtin_ctz(pending);
        pending &= pending - 1;
        float row[WC];
#pragma unroll
        for (int k = 0; k < WC; ++k) {
          float v = hr[0][k];
#pragma unroll
          for (int q = 1; q < NPL; ++q) v = (sl == q) ? hr[q][k] : v;
          row[k] = v;
        }
        double px, py;
        if (ls_masked<WC>(hx, hy, row, filled, p.gn_iters, tau, px, py)) {
#pragma unroll
          for (int q = 0; q < NPL; ++q)
            if (sl == q) {
              ex[q] = (float)px;
              ey[q] = (float)py;
            }
          evb |= 1u << sl;
        }
      }

      // ---- tracking error of this lane's trackers
      float errp[NPL];
#pragma unroll
      for (int sl = 0; sl < NPL; ++sl) {
        const int j = g + G * sl;
        errp[sl] = kInf;
        if (j < nt && ((evb >> sl) & 1u)) {
          errp[sl] = norm2(ex[sl] - pick<G>(tpx, g, sl), ey[sl] - pick<G>(tpy, g, sl));
        }
      }
      // ---- team error per target (best tracker), Eq. (1), normalisation
      float ej[MT];
      float rsum = 0.0f;
#pragma unroll
      for (int j = 0; j < MT; ++j) {
        float v = kInf;
        if (j < nt) {
#pragma unroll
          for (int k = 0; k < MA; ++k) {
            if (k < na) v = fminf(v, env_shfl<S>(errp[j / G], base_lane, k * G + (j % G), lpe));
          }
          rsum += tracking_reward(v, p.eps_min, p.eps_max, inv_span);
        }
        ej[j] = v;
      }
      float rew = rsum * inv_nt;
      // ---- agents' positions and broadcasts; crash penalty
      float agx[MA], agy[MA];
      int agc[MA];
#pragma unroll
      for (int k = 0; k < MA; ++k) {
        agx[k] = 0.0f;
        agy[k] = 0.0f;
        agc[k] = 0;
        if (k < na) {
          agx[k] = env_shfl<S>(ax, base_lane, k * G, lpe);
          agy[k] = env_shfl<S>(ay, base_lane, k * G, lpe);
          agc[k] = FULL ? env_shfl<S>((int)comm_ok, base_lane, k * G, lpe) : 1;
        }
      }
      if (FULL && p.reward_mode == 1) {
        // Eq. (2): a target scores 1 when its nearest agent is within d_follow
        const float dfol2 = p.d_follow * p.d_follow;
        float fsum = 0.0f;
#pragma unroll
        for (int j = 0; j < MT; ++j) {
          if (j < nt) {
            float dmin2 = kInf;
#pragma unroll
            for (int k = 0; k < MA; ++k)
              if (k < na) dmin2 = fminf(dmin2, sqnorm(agx[k] - tpx[j], agy[k] - tpy[j]));
            fsum += (dmin2 <= dfol2) ? 1.0f : 0.0f;
          }
        }
        rew = fsum * inv_nt;
      }
      bool crash = false;
#pragma unroll
      for (int k = 0; k < MA; ++k)
#pragma unroll
        for (int k2 = k + 1; k2 < MA; ++k2)
          if (k2 < na) {
            crash = crash || (sqnorm(agx[k] - agx[k2], agy[k] - agy[k2]) < dsafe2);
          }
      if (crash) rew = -1.0f;
      const bool done = (t + 1u == (uint32_t)p.episode_len);

      // ---- outputs
      if constexpr (!FULL) {
        if (active) {
          if (r == 0) {
            acc_rew += (double)rew;
            acc_crash += crash ? 1 : 0;
#pragma unroll
            for (int j = 0; j < MT; ++j)
              if (j < nt && ej[j] < kInf) {
                acc_err += (double)ej[j];
                acc_err2 += (double)ej[j] * (double)ej[j];
                acc_cnt += 1;
              }
            if (o.reward) o.reward[(int64_t)step * o.E + e] = rew;
            if (o.done) o.done[(int64_t)step * o.E + e] = done ? 1 : 0;
          }
          // this lane's tokens: into the staging area (position = output order)
          // for a large batch, else straight to the output
          const int tb = agent_w * ntok;
          const int64_t kb = (int64_t)step * o.K + kbase;
          float *ob = o.obs ? o.obs + kb * 6 : nullptr;
          uint8_t *om = o.obs_mask ? o.obs_mask + kb : nullptr;
          auto emit = [&](int m, float dx, float dy, bool ok, float is_self, float is_agent,
                          float is_target) {
            if constexpr (stage) {
              st_xy[tb + m] = make_float2(dx, dy);
              st_m[tb + m] = ok ? 1 : 0;
            } else {
              if (ob) store_token(ob + m * 6, dx, dy, is_self, is_agent, is_target);
              if (om) om[m] = ok ? 1 : 0;
            }
          };
          if (g == 0) emit(0, 0.0f, 0.0f, true, 1.0f, 0.0f, 0.0f);
#pragma unroll
          for (int m = 1; m < MA; ++m) {
            if (m < na && (m % G) == g) {
              const bool before = (m - 1) < i;  // other agent k = m-1 if m-1 < i else m
              const float ox = before ? agx[m - 1] : agx[m];
              const float oy = before ? agy[m - 1] : agy[m];
              const float dx = ox - ax, dy = oy - ay;
              const bool ok = sqnorm(dx, dy) <= comm2;
              emit(m, ok ? dx : 0.0f, ok ? dy : 0.0f, ok, 0.0f, 1.0f, 0.0f);
            }
          }
#pragma unroll
          for (int j = 0; j < MT; ++j) {
            if (j < nt && (j % G) == g) {
              const int sl = j / G;
              const bool ok = (evb >> sl) & 1u;
              emit(na + j, ok ? ex[sl] - ax : 0.0f, ok ? ey[sl] - ay : 0.0f, ok, 0.0f, 0.0f, 1.0f);
            }
          }
          if (!(fabsf(ax) < kInf) || !(fabsf(ay) < kInf) || !(fabsf(apsi) < kInf))
            status |= kStatusNonFinite;
        }
        // the wavefront's token block is contiguous in the output: one lane per
        // token, consecutive lanes on consecutive tokens
        if constexpr (stage) {
          wave_lds_fence();
          const int64_t kw = (int64_t)step * o.K + kbase_w;
          float2 *ob = o.obs ? reinterpret_cast<float2 *>(o.obs + kw * 6) : nullptr;
          uint8_t *om = o.obs_mask ? o.obs_mask + kw : nullptr;
          int m = m_lane0;  // position of token `t` inside its agent's token list
          for (int t = lane; t < ntok_w; t += 64) {
            if (ob) {
              ob[3 * t] = st_xy[t];
              ob[3 * t + 1] = make_float2(0.0f, m == 0 ? 1.0f : 0.0f);
              ob[3 * t + 2] = make_float2((m >= 1 && m < na) ? 1.0f : 0.0f, m >= na ? 1.0f : 0.0f);
            }
            if (om) om[t] = st_m[t];
            m += m_step;
            if (m >= ntok) m -= ntok;
          }
          wave_lds_fence();  // the staging area is rewritten next step
        }
      } else if (active) {
        if (r == 0) {
          acc_rew += (double)rew;
          acc_crash += crash ? 1 : 0;
#pragma unroll
          for (int j = 0; j < MT; ++j)
            if (j < nt && ej[j] < kInf) {
              acc_err += (double)ej[j];
              acc_err2 += (double)ej[j] * (double)ej[j];
              acc_cnt += 1;
            }
          if (o.reward) o.reward[(int64_t)step * o.E + e] = rew;
          if (o.done) o.done[(int64_t)step * o.E + e] = done ? 1 : 0;
          if (o.err) {
#pragma unroll
            for (int j = 0; j < MT; ++j)
              if (j < nt) o.err[(int64_t)step * o.Tt + tbase + j] = ej[j];
          }
        }
        const int64_t kb = (int64_t)step * o.K + kbase;
        if (o.obs) {
          float *ob = o.obs + kb * 6;
          if (g == 0) store_token(ob, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f);
#pragma unroll
          for (int m = 1; m < MA; ++m) {
            if (m < na && (m % G) == g) {
              const bool before = (m - 1) < i;  // other agent k = m-1 if m-1 < i else m
              const float ox = before ? agx[m - 1] : agx[m];
              const float oy = before ? agy[m - 1] : agy[m];
              const int oc = before ? agc[m - 1] : agc[m];
              const float dx = ox - ax, dy = oy - ay;
              const bool ok = oc && (sqnorm(dx, dy) <= comm2);
              store_token(ob + m * 6, ok ? dx : 0.0f, ok ? dy : 0.0f, 0.0f, 1.0f, 0.0f);
              if (o.obs_mask) o.obs_mask[kb + m] = ok ? 1 : 0;
            }
          }
#pragma unroll
          for (int j = 0; j < MT; ++j) {
            if (j < nt && (j % G) == g) {
              const int sl = j / G;
              const bool ok = (evb >> sl) & 1u;
              store_token(ob + (na + j) * 6, ok ? ex[sl] - ax : 0.0f, ok ? ey[sl] - ay : 0.0f, 0.0f,
                          0.0f, 1.0f);
              if (o.obs_mask) o.obs_mask[kb + na + j] = ok ? 1 : 0;
            }
          }
          if (o.obs_mask && g == 0) o.obs_mask[kb] = 1;
        } else if (o.obs_mask) {
          if (g == 0) o.obs_mask[kb] = 1;
#pragma unroll
          for (int m = 1; m < MA; ++m) {
            if (m < na && (m % G) == g) {
              const bool before = (m - 1) < i;
              const float ox = before ? agx[m - 1] : agx[m];
              const float oy = before ? agy[m - 1] : agy[m];
              const int oc = before ? agc[m - 1] : agc[m];
              o.obs_mask[kb + m] = (oc && (sqnorm(ox - ax, oy - ay) <= comm2)) ? 1 : 0;
            }
          }
#pragma unroll
          for (int j = 0; j < MT; ++j)
            if (j < nt && (j % G) == g) o.obs_mask[kb + na + j] = ((evb >> (j / G)) & 1u) ? 1 : 0;
        }
        if (g == 0) {
          if (o.actions) o.actions[(int64_t)step * o.A + aidx] = act;
          if (o.gstate) {
            float *gs = o.gstate + ((int64_t)step * (o.A + o.Tt) + gbase + i) * 6;
            gs[0] = ax; gs[1] = ay; gs[2] = 0.0f; gs[3] = p.agent_speed; gs[4] = apsi; gs[5] = 0.0f;
          }
        }
        if (o.gstate) {
          for (int q = r; q < nB; q += lpe) {
#pragma unroll
            for (int m = 0; m < 2; ++m) {
              const int j = 2 * q + m;
              if (j < nt) {
                const float4 tg = kRegTargets<S> ? treg[m] : tl[j];
                float *gs = o.gstate + ((int64_t)step * (o.A + o.Tt) + gbase + na + j) * 6;
                gs[0] = tg.x; gs[1] = tg.y; gs[2] = 0.0f; gs[3] = tg.w; gs[4] = tg.z; gs[5] = 1.0f;
              }
            }
          }
        }
#pragma unroll
        for (int sl = 0; sl < NPL; ++sl) {
          const int j = g + G * sl;
          if (j < nt) {
            const int64_t pidx = (int64_t)step * o.P + pbase + j;
            const bool ok = (evb >> sl) & 1u;
            if (o.est) {
              o.est[2 * pidx] = ok ? ex[sl] : 0.0f;
              o.est[2 * pidx + 1] = ok ? ey[sl] : 0.0f;
            }
            if (o.est_valid) o.est_valid[pidx] = ok ? 1 : 0;
            if (o.ranges) o.ranges[pidx] = hr[sl][0];
          }
        }
        if (!(fabsf(ax) < kInf) || !(fabsf(ay) < kInf) || !(fabsf(apsi) < kInf))
          status |= kStatusNonFinite;
      }
    }

    // ---- store state back (state pointers re-read from the device copy)
    if (active) {
      const DevState s = *sp;
      if (g == 0) {
        st_st(&s.ax[aidx], ax, dyn);
        st_st(&s.ay[aidx], ay, dyn);
        st_st(&s.apsi[aidx], apsi, dyn);
        if (FULL && p.action_mode == 1) st_st(&s.arud[aidx], rud, dyn);
        if constexpr (FULL) {
          if (p.pooled) {
#pragma unroll
            for (int k = 0; k < WC; ++k)
              if (k < W) st_st(&s.hrec[(int64_t)k * s.A + aidx], (uint8_t)recm[k], dyn);
          }
        }
#pragma unroll
        for (int k = 0; k < WC; ++k) {
          if (k < W) {
            st_st(&s.hx[(int64_t)k * s.A + aidx], hx[k], dyn);
            st_st(&s.hy[(int64_t)k * s.A + aidx], hy[k], dyn);
          }
        }
      }
      for (int q = r; q < nB; q += lpe) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const int j = 2 * q + m;
          if (j < nt) {
            const float4 tg = kRegTargets<S> ? treg[m] : tl[j];
            st_st(&s.tx[tbase + j], tg.x, dyn);
            st_st(&s.ty[tbase + j], tg.y, dyn);
            st_st(&s.tpsi[tbase + j], tg.z, dyn);
          }
        }
      }
#pragma unroll
      for (int sl = 0; sl < NPL; ++sl) {
        const int j = g + G * sl;
        if (j < nt) {
          const int64_t pidx = pbase + j;
#pragma unroll
          for (int k = 0; k < WC; ++k)
            if (k < W) st_st(&s.hr[(int64_t)k * s.P + pidx], hr[sl][k], dyn);
          st_st(&s.ex[pidx], ex[sl], dyn);
          st_st(&s.ey[pidx], ey[sl], dyn);
          st_st(&s.ev[pidx], (uint8_t)((evb >> sl) & 1u), dyn);
        }
      }
      if (r == 0) {
        st_st(&s.macc[3 * e], acc_rew, dyn);
        st_st(&s.macc[3 * e + 1], acc_err, dyn);
        st_st(&s.macc[3 * e + 2], acc_err2, dyn);
        st_st(&s.miacc[2 * e], acc_cnt, dyn);
        st_st(&s.miacc[2 * e + 1], acc_crash, dyn);
      }
    }
    if (status) atomicOr(sp->status, status);
    wave_lds_fence();  // the next unit rewrites the target slab
    if (!dyn) break;
    if (s_end < T) publish_chunks(sp->queue + 1 + wave, cix + 1, lane);
    unit = take_unit(sp->queue, lane);
  }
}

// ---------------------------------------------------------------------------
// Metrics: each block sums a fixed range of envs (thread t takes envs t,
// t + 256, ... of its range, then a fixed tree), a second one-block kernel
// sums the block partials in block order: reproducible run to run.
// ---------------------------------------------------------------------------
constexpr int kMetricThreads = 256;

__device__ __forceinline__ void block_sum6(double (&v)[6], double (*red)[6]) {
  for (int c = 0; c < 6; ++c) red[threadIdx.x][c] = v[c];
  __syncthreads();
  for (int w = kMetricThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 6; ++c) red[threadIdx.x][c] += red[threadIdx.x + w][c];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kMetricThreads) metrics_partial_kernel(DevParams p, DevState s,
                                                                         int64_t per_block) {
  __shared__ double red[kMetricThreads][6];
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int64_t e0 = (int64_t)blockIdx.x * per_block;
  const int64_t e1 = min(s.E, e0 + per_block);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kMetricThreads) {
    v[0] += s.macc[3 * e];
    v[1] += s.macc[3 * e + 1];
    v[2] += s.macc[3 * e + 2];
    v[3] += (double)s.miacc[2 * e];
    v[4] += (double)s.miacc[2 * e + 1];
    const int64_t ab = s.aoff[e], tb = s.toff[e];
    const int na = s.cnt_a[e], nt = s.cnt_t[e];
    for (int j = 0; j < nt; ++j) {
      float dmin = __int_as_float(0x7f800000);
      for (int i = 0; i < na; ++i) {
        dmin = fminf(dmin, norm2(s.ax[ab + i] - s.tx[tb + j], s.ay[ab + i] - s.ty[tb + j]));
      }
      if (dmin > p.lost_range) v[5] += 1.0;
    }
  }
  block_sum6(v, red);
  if (threadIdx.x == 0)
    for (int c = 0; c < 6; ++c) s.mpart[6 * blockIdx.x + c] = red[0][c];
}

__global__ void __launch_bounds__(kMetricThreads) metrics_final_kernel(DevState s, int32_t steps,
                                                                       int32_t nblocks,
                                                                       double *out) {
  __shared__ double red[kMetricThreads][6];
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kMetricThreads)
    for (int c = 0; c < 6; ++c) v[c] += s.mpart[6 * b + c];
  block_sum6(v, red);
  if (threadIdx.x == 0) {
    for (int c = 0; c < 6; ++c) out[c] = red[0][c];
    out[6] = (double)s.E * (double)steps;
    out[7] = (double)s.A * (double)steps;
  }
}

__global__ void get_state_kernel(DevState s, float *agent, float *target) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (agent && k < s.A) {
    agent[3 * k] = s.ax[k];
    agent[3 * k + 1] = s.ay[k];
    agent[3 * k + 2] = s.apsi[k];
  }
  if (target && k < s.Tt) {
    target[4 * k] = s.tx[k];
    target[4 * k + 1] = s.ty[k];
    target[4 * k + 2] = s.tpsi[k];
    target[4 * k + 3] = s.tv[k];
  }
}

// Every tracker's window (entry 0 = newest) with its env's range-noise std
// and the true target position: one thread per (env, pair slot, window
// entry), the entry index fastest, so consecutive threads write consecutive
// 12-byte entries of the output.
__global__ void env_windows_kernel(DevState s, int32_t W, int32_t slots, float *win, float *sigma,
                                   float *truth) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t q = tid / W;
  const int k = (int)(tid - q * W);
  const int64_t e = q / slots;
  const int slot = (int)(q - e * slots);
  if (e >= s.E) return;
  const int na = s.cnt_a[e], nt = s.cnt_t[e];
  if (slot >= na * nt) return;
  const int i = slot / nt, j = slot - i * nt;
  const int64_t a = s.aoff[e] + i;
  const int64_t p = s.poff[e] + slot;
  float *w = win + (p * W + k) * 3;
  w[0] = s.hx[(int64_t)k * s.A + a];
  w[1] = s.hy[(int64_t)k * s.A + a];
  w[2] = s.hr[(int64_t)k * s.P + p];
  if (k == 0) {
    if (sigma) sigma[p] = s.sigma[e];
    if (truth) {
      truth[2 * p] = s.tx[s.toff[e] + j];
      truth[2 * p + 1] = s.ty[s.toff[e] + j];
    }
  }
}

int launch_env_windows(const DevState &s, int32_t W, int32_t slots, float *win, float *sigma,
                       float *truth, void *stream) {
  const int bs = 256;
  const int64_t n = s.E * (int64_t)slots * W;
  hipLaunchKernelGGL(env_windows_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, s, W, slots, win, sigma, truth);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static int check_launch() { return hipGetLastError() == hipSuccess ? 0 : -1; }

static int device_cus() {
  int dev = 0, n = 0;
  hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
    n = 256;
  return n;
}

int launch_reset(const DevParams &p, const DevState &s, uint32_t episode, const DevOut &o,
                 void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = s.E * 17;
  const int bs = 256;
  hipLaunchKernelGGL(reset_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, p, s,
                     episode);
  if (check_launch()) return -1;
  if (o.obs || o.obs_mask || o.gstate) {
    const int64_t n2 = s.E * 16;
    hipLaunchKernelGGL(reset_obs_kernel, dim3((unsigned)((n2 + bs - 1) / bs)), dim3(bs), 0, st,
                       p, s, o);
    if (check_launch()) return -1;
  }
  return 0;
}

// Wavefronts of one rollout instantiation the GPU holds at once, for blocks
// of `waves_per_block` wavefronts (cached per instantiation and block size).
template <int S, int WC, int G, bool FULL, bool STAGE>
static int resident_waves(int waves_per_block, size_t lds) {
  static int cached[5] = {0, 0, 0, 0, 0};
  int &c = cached[waves_per_block];
  if (c == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&rollout_kernel<S, WC, G, FULL, STAGE>),
            64 * waves_per_block, lds) != hipSuccess ||
        nb < 1)
      nb = 1;
    c = nb * device_cus() * waves_per_block;
  }
  return c;
}

// Steps per chunk of the automatic dynamic schedule: about 128, evenly split.
static int auto_chunk(int32_t T) {
  const int n = (T + 64) / 128;
  return n <= 1 ? T : (T + n - 1) / n;
}

template <int S, int WC, int G, bool FULL, bool STAGE>
static int launch_rollout_t(int waves_per_block, int num_waves, const DevParams &p,
                            const DevState &hs, const DevState *s, int32_t t0, int32_t T,
                            uint32_t episode, const int32_t *actions, const DevOut &o,
                            hipStream_t st, const DevExt &ext, int32_t sched) {
  // per wavefront: target slab, then (lean form) token offsets and masks, or
  // (full form, pooled tracker) every lane's window; the pooled form runs
  // one wavefront per block to keep the block's LDS small
  const bool pooled_ls = FULL && p.pooled && p.est_kind == 0;
  if (pooled_ls) waves_per_block = 1;
  constexpr int NPLT = (S + G - 1) / G;
  const size_t lds = (size_t)waves_per_block *
                     (64 * S * sizeof(float4) + (STAGE ? kStageTok<S> * (sizeof(float2) + 1) : 0) +
                      (pooled_ls ? 64 * WC * (2 + NPLT) * sizeof(float) : 0));
  int blocks = (num_waves - ext.wave0 + waves_per_block - 1) / waves_per_block;
  int32_t chunk = 0;
  if ((sched >= 0 || sched == kSchedProbe) && hs.queue && ext.wave0 == 0) {
    const int resident = resident_waves<S, WC, G, FULL, STAGE>(waves_per_block, lds);
    if (sched > 0) {
      chunk = sched < T ? sched : T;
    } else if (num_waves > resident && num_waves < 8 * resident) {
      // a few rounds of wavefronts: the last round would run part-empty;
      // with many rounds the hardware's own dispatch leaves little idle
      chunk = sched == kSchedProbe ? (T + 1) / 2 : auto_chunk(T);
      if (chunk >= T) chunk = 0;  // one chunk: nothing to rebalance
    }
    if (chunk > 0) {
      const int64_t units = (int64_t)num_waves * ((T + chunk - 1) / chunk);
      if (units + resident >= (int64_t)INT32_MAX) {
        chunk = 0;  // beyond the counter's range: static schedule
      } else {
        const int64_t want = (units + waves_per_block - 1) / waves_per_block;
        const int64_t cap = resident / waves_per_block;
        blocks = (int)(want < cap ? want : cap);
        const int32_t nq = num_waves + 1;
        hipLaunchKernelGGL(queue_init_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0,
                           st, hs.queue, nq);
        if (check_launch()) return -1;
      }
    }
  }
  hipLaunchKernelGGL((rollout_kernel<S, WC, G, FULL, STAGE>), dim3(blocks),
                     dim3(64 * waves_per_block), lds, st, p, s, num_waves, t0, T, episode, actions, o,
                     ext, chunk);
  return check_launch();
}

int launch_rollout(int size_class, int wcap, int G, int waves_per_block, int num_waves,
                   const DevParams &p, const DevState &hs, const DevState *s, int32_t t0,
                   int32_t T, uint32_t episode, const int32_t *actions, const DevOut &o_in,
                   void *stream, const DevExt &ext, int32_t sched) {
  hipStream_t st = (hipStream_t)stream;
  if (num_waves - ext.wave0 <= 0 || T <= 0) return 0;
  DevOut o = o_in;
  o.E = hs.E;
  o.A = hs.A;
  o.Tt = hs.Tt;
  o.P = hs.P;
  o.K = hs.K;
  // the lean form applies when none of the full form's extra paths is asked for
  const bool lean = !actions && !o.est && !o.est_valid && !o.gstate && !o.actions && !o.ranges &&
                    !o.err && std::isinf(p.det_range) && p.det_range > 0.0f &&
                    p.comm_loss_p == 0.0f && p.gn_iters == 0 && ext.phase == 0 &&
                    p.action_mode == 0 && p.reward_mode == 0 && p.pooled == 0 && p.est_kind == 0;
  // the lean form stages its observation block for a coalesced write once at
  // least two wavefronts per SIMD take turns on the store path (large
  // batches); small batches are latency-bound and write directly
  const bool stage = lean && num_waves >= 8 * device_cus();
#define MIL_ROLL(SC, WCV, GV)                                                                \
  if (size_class == SC && wcap == WCV && G == GV) {                                         \
    if (!lean)                                                                               \
      return launch_rollout_t<SC, WCV, GV, true, false>(waves_per_block, num_waves, p, hs, s, \
                                                        t0, T, episode, actions, o, st, ext, \
                                                        sched);                              \
    return stage ? launch_rollout_t<SC, WCV, GV, false, true>(waves_per_block, num_waves, p, \
                                                              hs, s, t0, T, episode, actions, \
                                                              o, st, ext, sched)             \
                 : launch_rollout_t<SC, WCV, GV, false, false>(waves_per_block, num_waves, p, \
                                                               hs, s, t0, T, episode, actions, \
                                                               o, st, ext, sched);           \
  }
  MIL_ROLL(2, 10, 1)
  MIL_ROLL(2, 10, 2)
  MIL_ROLL(2, 16, 1)
  MIL_ROLL(2, 16, 2)
  MIL_ROLL(5, 10, 1)
  MIL_ROLL(5, 10, 2)
  MIL_ROLL(5, 16, 1)
  MIL_ROLL(5, 16, 2)
  MIL_ROLL(8, 16, 1)
  MIL_ROLL(8, 16, 2)
#undef MIL_ROLL
  // the particle filter's halves: full form with a window of one entry
#define MIL_ROLL_PF(SC, GV)                                                                 \
  if (size_class == SC && wcap == 1 && G == GV && !lean)                                    \
    return launch_rollout_t<SC, 1, GV, true, false>(waves_per_block, num_waves, p, hs, s, t0, \
                                                    T, episode, actions, o, st, ext, sched);
  MIL_ROLL_PF(2, 1)
  MIL_ROLL_PF(2, 2)
  MIL_ROLL_PF(5, 1)
  MIL_ROLL_PF(5, 2)
  MIL_ROLL_PF(8, 1)
  MIL_ROLL_PF(8, 2)
#undef MIL_ROLL_PF
  return -2;
}

int launch_metrics(const DevParams &p, const DevState &s, int32_t steps, double *d_metrics,
                   void *stream) {
  hipStream_t st = (hipStream_t)stream;
  int64_t nb = (s.E + kMetricThreads - 1) / kMetricThreads;
  if (nb > kMetricBlocks) nb = kMetricBlocks;
  if (nb < 1) nb = 1;
  const int64_t per_block = (s.E + nb - 1) / nb;
  hipLaunchKernelGGL(metrics_partial_kernel, dim3((unsigned)nb), dim3(kMetricThreads), 0, st, p, s,
                     per_block);
  if (check_launch()) return -1;
  hipLaunchKernelGGL(metrics_final_kernel, dim3(1), dim3(kMetricThreads), 0, st, s, steps,
                     (int32_t)nb, d_metrics);
  return check_launch();
}

int launch_get_state(const DevState &s, float *d_agent, float *d_target, void *stream) {
  const int64_t n = s.A > s.Tt ? s.A : s.Tt;
  const int bs = 256;
  hipLaunchKernelGGL(get_state_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, s, d_agent, d_target);
  return check_launch();
}

}  // namespace mil
