// Particle-filter tracker (Sec. II: each target's position as a cloud of
// particles moved by a motion model and resampled by the likelihood of the
// measured ranges; Sec. IV-A-2: one model per (agent, target)).
//
// Two trackers per wavefront, 32 lanes each, two consecutive particles per
// lane: the lane's particles 2l and 2l + 1 are one 16-byte access, a tracker's
// set 512 contiguous bytes, and one Philox block per lane gives both
// particles' normals (four words). The scans the filter needs (largest
// log-weight, cumulative weights, the mean) run over 32-lane halves: DPP
// inside each 16-lane row, then row_bcast:15 into the half's second row; the
// resampling search and gather are ds_bpermute reads. Per step and tracker:
//   seed     (no belief, first row a, r): particle k on the ring about a,
//            radius r + sigma_l z_k, angle 2 pi (k + u_k) / 64;
//   move     (belief): x_k += q (z_k, z'_k);
//   weight   (rows not used to seed): log w_k = -sum (|x_k - a| - r)^2 /
//            (2 sigma_l^2), taken relative to the largest;
//   resample (systematic): with C the inclusive cumulative weights and U one
//            offset, particle k copies min{m : C_m > (k + U) / 64 * C_63};
//   estimate the mean of the particles.
// Draws: particle pair h = k / 2 of tracker (agent i, target j) takes
// Philox(step, env id, (8 i + j) * 32 + h, 7 | episode << 4): words 0, 1 are
// particle 2h's Box-Muller pair (z, z'), words 2, 3 particle 2h + 1's; the
// same counter with purpose 8 gives the seeding angles u (words 0 and 2); U is
// word 0 of Philox(step, env id, 2048 + 8 i + j, 7 | episode << 4), the same
// for the whole tracker (computed from uniform inputs). Rows: the agent's own
// range of the step, and with pooling the ranges it received from the other
// agents (own first, then agent order), each kept when present.
#include <hip/hip_runtime.h>

#include "env_internal.h"
#include "rng.h"

namespace mil {
namespace {

constexpr uint32_t kPurposePf = 7;
constexpr uint32_t kPurposePfSeed = 8;
constexpr uint32_t kEntPfOffset = 2048;
constexpr int kPfWaves = 4;  // wavefronts per block, two trackers each
constexpr int kPairs = kPfParticles / 2;

// Value of the lane a DPP control selects inside each row of 16 lanes
// (quad_perm 0xB1: lanes 1,0,3,2 of each quad; 0x4E: 2,3,0,1; row_ror:n =
// 0x120 + n rotates the row), for patterns where every lane has a source.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// v shifted by a DPP control with 0 wherever no value arrives: lanes whose
// source is outside the pattern and rows the row mask leaves out keep the
// `old` operand, 0 (and a zero-filled out-of-bounds read is 0 as well), so
// the add below it folds into one DPP add.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp0(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xF, true));
}

// Inclusive prefix sum over each 32-lane half: Hillis-Steele inside each row
// (row_shr 1, 2, 4, 8), then row_bcast:15 carries row 0's total into row 1
// and row 2's into row 3 (row mask 0xA).
__device__ __forceinline__ float half_scan_add(float v) {
  v += dpp0<0x111, 0xF>(v);
  v += dpp0<0x112, 0xF>(v);
  v += dpp0<0x114, 0xF>(v);
  v += dpp0<0x118, 0xF>(v);
  v += dpp0<0x142, 0xA>(v);
  return v;
}

__device__ __forceinline__ float lane_value(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Every lane of a 16-lane row ends with the row's maximum (or sum): a
// butterfly of quad swaps and row rotations, every lane having a source.
__device__ __forceinline__ float row_max(float v) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x124>(v));
  return fmaxf(v, dpp<0x128>(v));
}
__device__ __forceinline__ float row_sum(float v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x124>(v);
  return v + dpp<0x128>(v);
}

struct PfArgs {
  const uint32_t *env_id;
  const float *sigma;
  const uint8_t *hrec;  // entry 0: the first A bytes
  const uint4 *pmeta;
  float4 *pfxy;  // [P][32]: particles 2l and 2l + 1 of lane l
  uint8_t *pfb;
  const float4 *pfm;
  float *ex, *ey;
  uint8_t *ev;
  int64_t p0, P;  // trackers p0 .. P - 1
  uint32_t t, c3, c3seed, key0, key1;
  float q, lik2;
};

// Byte `idx` of a byte array read through a scalar load of its aligned
// 32-bit word (the arrays are allocated in 256-byte units, so the word never
// leaves the allocation); idx is uniform over the wavefront.
__device__ __forceinline__ uint32_t uniform_byte(const uint8_t *base, int64_t idx) {
  const uint32_t word = *reinterpret_cast<const uint32_t *>(base + (idx & ~(int64_t)3));
  return (word >> (8 * (uint32_t)(idx & 3))) & 0xFFu;
}

// The lane's tracker's rows of this step in slot order (slot 0 the agent's
// own range, then with pooling the other agents in index order, each when
// its broadcast was received): returns the mask of slots holding a range.
// Without pooling the two trackers' rows come through scalar loads and are
// selected per half; with pooling each lane loads its tracker's rows (the 32
// lanes of a half read the same addresses).
template <bool POOLED, int MR>
__device__ __forceinline__ uint32_t lane_rows(const PfArgs &a, int half, int64_t wa, int64_t wb,
                                              const uint4 &meta_a, const uint4 &meta_b,
                                              float (&rx)[MR], float (&ry)[MR], float (&rr)[MR]) {
  uint32_t valid = 0;
  if constexpr (POOLED) {
    const uint4 meta = half ? meta_b : meta_a;
    const int64_t w = half ? wb : wa;
    const uint32_t code = meta.y & 0xFFu;
    const int i = (int)(code >> 3), j = (int)(code & 7u);
    const int na = (int)((meta.y >> 8) & 15u), nt = (int)((meta.y >> 12) & 15u);
    const int64_t p0 = w - (int64_t)(i * nt + j);  // the env's first pair
    const uint32_t bits = (uint32_t)a.hrec[meta.z] | (1u << i);
#pragma unroll
    for (int k2 = 0; k2 < MR; ++k2) {
      rx[k2] = ry[k2] = rr[k2] = 0.0f;
      const int ag = (k2 == 0) ? i : (k2 <= i ? k2 - 1 : k2);  // own row first
      if (k2 < na && ((bits >> ag) & 1u)) {
        const float4 v = a.pfm[p0 + (int64_t)ag * nt + j];
        rx[k2] = v.x;
        ry[k2] = v.y;
        rr[k2] = v.z;
        if (v.z == v.z) valid |= 1u << k2;
      }
    }
  } else {
    const float4 va = a.pfm[wa], vb = a.pfm[wb];
    rx[0] = half ? vb.x : va.x;
    ry[0] = half ? vb.y : va.y;
    rr[0] = half ? vb.z : va.z;
    valid = (rr[0] == rr[0]) ? 1u : 0u;
  }
  return valid;
}

template <bool POOLED>
__global__ void __launch_bounds__(64 * kPfWaves) pf_kernel(PfArgs a) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;  // which tracker of the wavefront's two
  const int hl = lane & 31;    // this lane holds particles 2 hl and 2 hl + 1
  const int64_t wa = a.p0 + 2 * ((int64_t)blockIdx.x * kPfWaves +
                                 __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)));
  if (wa >= a.P) return;  // uniform over the wavefront
  const bool has_b = wa + 1 < a.P;
  const int64_t wb = has_b ? wa + 1 : wa;  // a lone tracker: the upper half repeats it, unstored
  const int64_t w = half ? wb : wa;
  // the particles first: their load overlaps everything up to the move
  const float4 prev = a.pfxy[w * kPairs + hl];

  // both trackers' uniform values, then each lane's
  const uint4 meta_a = a.pmeta[wa], meta_b = a.pmeta[wb];
  constexpr int MR = POOLED ? 8 : 1;
  float rx[MR], ry[MR], rr[MR];
  const uint32_t valid = lane_rows<POOLED, MR>(a, half, wa, wb, meta_a, meta_b, rx, ry, rr);
  const uint32_t va = (uint32_t)__builtin_amdgcn_readlane((int)valid, 0);
  const uint32_t vb = (uint32_t)__builtin_amdgcn_readlane((int)valid, 32);
  const bool bel_a = a.t > 0u && uniform_byte(a.pfb, wa) != 0;
  const bool bel_b = a.t > 0u && uniform_byte(a.pfb, wb) != 0;
  const bool act_a = bel_a || va != 0, act_b = has_b && (bel_b || vb != 0);
  if (!act_a && !act_b) {
    // no belief and no range: nothing to estimate (a new episode starts
    // without a belief)
    if (lane == 0) a.pfb[wa] = 0;
    if (lane == 32 && has_b) a.pfb[wb] = 0;
    return;
  }
  const uint32_t env_a = a.env_id[meta_a.x], env_b = a.env_id[meta_b.x];
  const uint32_t code_a = meta_a.y & 0xFFu, code_b = meta_b.y & 0xFFu;
  const float sr_a = a.sigma[meta_a.x], sr_b = a.sigma[meta_b.x];
  // the resampling offsets (uniform inputs: scalar arithmetic)
  const float U_a = u01(philox4x32_10(a.t, env_a, kEntPfOffset + code_a, a.c3, a.key0, a.key1).x);
  const float U_b = u01(philox4x32_10(a.t, env_b, kEntPfOffset + code_b, a.c3, a.key0, a.key1).x);

  const uint32_t env = half ? env_b : env_a, code = half ? code_b : code_a;
  const float sr = half ? sr_b : sr_a;
  const float sl2 = fmaf(sr, sr, a.lik2);
  const bool belief = half ? bel_b : bel_a;
  const float U = half ? U_b : U_a;
  // the rows that weight: all present ones, less the one that seeds a
  // tracker without a belief (its first)
  const uint32_t wt_a = bel_a ? va : (va & (va - 1)), wt_b = bel_b ? vb : (vb & (vb - 1));
  const uint32_t wmask = half ? wt_b : wt_a;

  const u32x4 x = philox4x32_10(a.t, env, code * (uint32_t)kPairs + (uint32_t)hl, a.c3, a.key0,
                                a.key1);
  float z0, z1, z2, z3;
  normal2(x.x, x.y, z0, z1);  // particle 2 hl
  normal2(x.z, x.w, z2, z3);  // particle 2 hl + 1
  float pxa = fmaf(a.q, z0, prev.x), pya = fmaf(a.q, z1, prev.y);
  float pxb = fmaf(a.q, z2, prev.z), pyb = fmaf(a.q, z3, prev.w);
  if (!bel_a || !bel_b) {
    // a tracker without a belief seeds on its first row's ring, one particle
    // per sector
    const u32x4 xs = philox4x32_10(a.t, env, code * (uint32_t)kPairs + (uint32_t)hl, a.c3seed,
                                   a.key0, a.key1);
    // the seeding row: the lane's first present slot
    float r0 = rr[0], ax0 = rx[0], ay0 = ry[0];
#pragma unroll
    for (int s = MR - 1; s > 0; --s) {
      if (((valid >> s) & 1u) && !(valid & ((1u << s) - 1u))) {
        r0 = rr[s];
        ax0 = rx[s];
        ay0 = ry[s];
      }
    }
    const float sl = fast_sqrt(sl2);
    const float k0 = (float)(2 * hl);
    float s, c, s2, c2;
    sincos_rev((k0 + u01(xs.x)) * (1.0f / (float)kPfParticles), s, c);
    sincos_rev((k0 + 1.0f + u01(xs.z)) * (1.0f / (float)kPfParticles), s2, c2);
    const float rad_a = fmaf(sl, z0, r0), rad_b = fmaf(sl, z2, r0);
    if (!belief) {
      pxa = fmaf(rad_a, c, ax0);
      pya = fmaf(rad_a, s, ay0);
      pxb = fmaf(rad_b, c2, ax0);
      pyb = fmaf(rad_b, s2, ay0);
    }
  }
  const bool res_a = wt_a != 0, res_b = wt_b != 0;
  if (res_a || res_b) {
    const float inv2s2 = 0.5f * __builtin_amdgcn_rcpf(sl2);
    float lwa = 0.0f, lwb = 0.0f;
    const uint32_t wany = wt_a | wt_b;
#pragma unroll
    for (int s = 0; s < MR; ++s) {
      if ((wany >> s) & 1u) {
        if ((wmask >> s) & 1u) {
          float dx = pxa - rx[s], dy = pya - ry[s];
          const float ea = fast_sqrt(fmaf(dx, dx, dy * dy)) - rr[s];
          lwa = fmaf(-ea * ea, inv2s2, lwa);
          dx = pxb - rx[s];
          dy = pyb - ry[s];
          const float eb = fast_sqrt(fmaf(dx, dx, dy * dy)) - rr[s];
          lwb = fmaf(-eb * eb, inv2s2, lwb);
        }
      }
    }
    // largest log-weight of each half, then the cumulative weights
    // (lane reads are taken for both halves, then selected: a lane read under
    // a branch on the half would run once per half)
    const float rm = row_max(fmaxf(lwa, lwb));
    const float top_a = fmaxf(lane_value(rm, 0), lane_value(rm, 16));
    const float top_b = fmaxf(lane_value(rm, 32), lane_value(rm, 48));
    const float top = half ? top_b : top_a;
    const float wta = __expf(lwa - top), wtb = __expf(lwb - top);
    const float cum_b = half_scan_add(wta + wtb);  // C of particle 2 hl + 1
    const float cum_a = cum_b - wtb;                // C of particle 2 hl
    const float tot_a = lane_value(cum_b, 31), tot_b = lane_value(cum_b, 63);
    const float total = half ? tot_b : tot_a;
    const int base = half << 5;
    float ox[2], oy[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      const float point = ((float)(2 * hl + o) + U) * (1.0f / (float)kPfParticles) * total;
      // the pair holding the first cumulative weight above the point: the
      // number of pairs whose upper cumulative weight is <= point (at most 31)
      int L = 0;
#pragma unroll
      for (int step = 16; step >= 1; step >>= 1) {
        const float cv = __shfl(cum_b, base + L + step - 1);
        if (cv <= point) L += step;
      }
      const int src_lane = base + L;
      const bool upper = __shfl(cum_a, src_lane) <= point;
      const float sxa = __shfl(pxa, src_lane), sxb = __shfl(pxb, src_lane);
      const float sya = __shfl(pya, src_lane), syb = __shfl(pyb, src_lane);
      ox[o] = upper ? sxb : sxa;
      oy[o] = upper ? syb : sya;
    }
    const bool res = half ? res_b : res_a;
    if (res) {
      pxa = ox[0];
      pya = oy[0];
      pxb = ox[1];
      pyb = oy[1];
    }
  }
  const bool act = half ? act_b : act_a;
  if (act) a.pfxy[w * kPairs + hl] = make_float4(pxa, pya, pxb, pyb);
  const float sx = row_sum(pxa + pxb), sy = row_sum(pya + pyb);
  const float mx_a = lane_value(sx, 0) + lane_value(sx, 16);
  const float mx_b = lane_value(sx, 32) + lane_value(sx, 48);
  const float my_a = lane_value(sy, 0) + lane_value(sy, 16);
  const float my_b = lane_value(sy, 32) + lane_value(sy, 48);
  const float mx = (half ? mx_b : mx_a) * (1.0f / (float)kPfParticles);
  const float my = (half ? my_b : my_a) * (1.0f / (float)kPfParticles);
  if (hl == 0 && (half == 0 || has_b)) {
    if (act) {
      a.pfb[w] = 1;
      a.ex[w] = mx;
      a.ey[w] = my;
      a.ev[w] = 1;
    } else {
      a.pfb[w] = 0;
    }
  }
}

}  // namespace

int launch_pf(const DevParams &p, const DevState &s, int32_t t, uint32_t episode, void *stream,
              int64_t p_begin, int64_t p_end) {
  if (p_end < 0 || p_end > s.P) p_end = s.P;
  if (p_begin < 0) p_begin = 0;
  if (p_end <= p_begin) return 0;
  if (!s.pmeta || !s.pfxy || !s.pfb || !s.pfm) return -1;
  PfArgs a{};
  a.env_id = s.env_id;
  a.sigma = s.sigma;
  a.hrec = s.hrec;
  a.pmeta = reinterpret_cast<const uint4 *>(s.pmeta);
  a.pfxy = reinterpret_cast<float4 *>(s.pfxy);
  a.pfb = s.pfb;
  a.pfm = reinterpret_cast<const float4 *>(s.pfm);
  a.ex = s.ex;
  a.ey = s.ey;
  a.ev = s.ev;
  a.p0 = p_begin;
  a.P = p_end;
  a.t = (uint32_t)t;
  a.c3 = (episode << 4) | kPurposePf;
  a.c3seed = (episode << 4) | kPurposePfSeed;
  a.key0 = p.key0;
  a.key1 = p.key1;
  a.q = p.pf_q;
  a.lik2 = p.pf_lik_sigma * p.pf_lik_sigma;
  const int64_t pairs = (p_end - p_begin + 1) / 2;
  const int64_t blocks = (pairs + kPfWaves - 1) / kPfWaves;
  hipStream_t st = (hipStream_t)stream;
  if (p.pooled)
    hipLaunchKernelGGL(pf_kernel<true>, dim3((unsigned)blocks), dim3(64 * kPfWaves), 0, st, a);
  else
    hipLaunchKernelGGL(pf_kernel<false>, dim3((unsigned)blocks), dim3(64 * kPfWaves), 0, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mil
