// Particle-filter tracker (Sec. II: each target's position as a cloud of
// particles moved by a motion model and resampled by the likelihood of the
// measured ranges; Sec. IV-A-2: one model per (agent, target)).
//
// One wavefront per tracker, one particle per lane: the particle set of a
// tracker is 64 float2 = 512 contiguous bytes, read and written with one
// coalesced access per lane; the scans the filter needs (largest log-weight,
// cumulative weights, the mean) are DPP row shifts and row broadcasts, and
// the resampling search and gather are ds_bpermute reads. Per step and tracker:
//   seed     (no belief, first row a, r): particle k on the ring about a,
//            radius r + sigma_l z_k, angle 2 pi (k + u_k) / 64;
//   move     (belief): x_k += q (z_k, z'_k);
//   weight   (rows not used to seed): log w_k = -sum (|x_k - a| - r)^2 /
//            (2 sigma_l^2), taken relative to the largest;
//   resample (systematic): with C the inclusive cumulative weights and U one
//            offset, particle k copies min{m : C_m > (k + U) / 64 * C_63};
//   estimate the mean of the particles.
// z, z' (Box-Muller of words 0, 1), u (word 2) and U (word 3 of particle 0)
// come from Philox(step, env id, (8 agent + target) * 64 + k, 7 | episode << 4).
// Rows: the agent's own range of the step, and with pooling the ranges it
// received from the other agents (own first, then agent order), each kept
// when present.
#include <hip/hip_runtime.h>

#include "env_internal.h"
#include "rng.h"

namespace mil {
namespace {

constexpr uint32_t kPurposePf = 7;
constexpr int kPfWaves = 4;  // wavefronts (trackers) per block

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

// Wavefront-wide inclusive scans: Hillis-Steele inside each row, then the row
// broadcasts carry the totals across rows (row_bcast:15 into rows 1 and 3,
// row_bcast:31 into rows 2 and 3).
__device__ __forceinline__ float wave_scan_add(float v, int) {
  v += dpp0<0x111, 0xF>(v);
  v += dpp0<0x112, 0xF>(v);
  v += dpp0<0x114, 0xF>(v);
  v += dpp0<0x118, 0xF>(v);
  v += dpp0<0x142, 0xA>(v);
  v += dpp0<0x143, 0xC>(v);
  return v;
}

__device__ __forceinline__ float lane_value(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Sum over the wavefront, the same value in every lane (the scan's last lane).
__device__ __forceinline__ float wave_sum(float v, int lane) { return lane_value(wave_scan_add(v, lane), 63); }

// Maximum over the wavefront, the same value in every lane: a butterfly
// inside each row (quad_perm swaps of neighbours and pairs, then row_ror by 4
// and 8; every lane has a source, so no lane needs a select), then the four
// row maxima.
__device__ __forceinline__ float wave_max(float v, int) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x124>(v));
  v = fmaxf(v, dpp<0x128>(v));
  return fmaxf(fmaxf(lane_value(v, 0), lane_value(v, 16)),
               fmaxf(lane_value(v, 32), lane_value(v, 48)));
}

struct PfArgs {
  const uint32_t *env_id;
  const float *sigma;
  const uint8_t *hrec;  // entry 0: the first A bytes
  const uint4 *pmeta;
  float2 *pfxy;
  uint8_t *pfb;
  const float4 *pfm;
  float *ex, *ey;
  uint8_t *ev;
  int64_t p0, P;  // trackers p0 .. P - 1
  uint32_t t, c3, key0, key1;
  float q, lik2;
};

// Byte `idx` of a byte array read through a scalar load of its aligned
// 32-bit word (the arrays are allocated in 256-byte units, so the word never
// leaves the allocation); idx is uniform over the wavefront.
__device__ __forceinline__ uint32_t uniform_byte(const uint8_t *base, int64_t idx) {
  const uint32_t word = *reinterpret_cast<const uint32_t *>(base + (idx & ~(int64_t)3));
  return (word >> (8 * (uint32_t)(idx & 3))) & 0xFFu;
}

template <bool POOLED>
__global__ void __launch_bounds__(64 * kPfWaves) pf_kernel(PfArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t w = a.p0 + (int64_t)blockIdx.x * kPfWaves +
                    __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (w >= a.P) return;  // uniform over the wavefront
  // the particles first: their load overlaps everything up to the move
  const float2 prev = a.pfxy[w * kPfParticles + lane];
  const uint4 meta = a.pmeta[w];
  const uint32_t e = meta.x, code = meta.y & 0xFFu;
  const int i = (int)(code >> 3), j = (int)(code & 7u);
  const float sr = a.sigma[e];
  const float sl2 = fmaf(sr, sr, a.lik2);
  const bool belief = a.t > 0u && uniform_byte(a.pfb, w) != 0;

  // this step's rows (uniform over the wavefront)
  constexpr int MR = POOLED ? 8 : 1;
  float rx[MR], ry[MR], rr[MR];
  int m = 0;
  if constexpr (POOLED) {
    const int na = (int)((meta.y >> 8) & 15u), nt = (int)((meta.y >> 12) & 15u);
    const int64_t p0 = w - (int64_t)(i * nt + j);  // the env's first pair
    const uint32_t bits = uniform_byte(a.hrec, (int64_t)meta.z) | (1u << i);
#pragma unroll
    for (int k2 = 0; k2 < MR; ++k2) {
      rx[k2] = ry[k2] = rr[k2] = 0.0f;
      if (k2 < na) {
        const int ag = (k2 == 0) ? i : (k2 <= i ? k2 - 1 : k2);  // own row first
        if ((bits >> ag) & 1u) {
          const float4 v = a.pfm[p0 + (int64_t)ag * nt + j];
          if (v.z == v.z) {
            // compacted: rows present go to the front (m is uniform)
#pragma unroll
            for (int s = 0; s < MR; ++s)
              if (s == m) {
                rx[s] = v.x;
                ry[s] = v.y;
                rr[s] = v.z;
              }
            ++m;
          }
        }
      }
    }
  } else {
    const float4 v = a.pfm[w];
    rx[0] = v.x;
    ry[0] = v.y;
    rr[0] = v.z;
    m = (v.z == v.z) ? 1 : 0;
  }

  if (!belief && m == 0) {
    if (lane == 0) a.pfb[w] = 0;  // a new episode starts without a belief
    return;
  }
  const u32x4 x = philox4x32_10(a.t, a.env_id[e], code * (uint32_t)kPfParticles + (uint32_t)lane,
                                a.c3, a.key0, a.key1);
  float z0, z1;
  normal2(x.x, x.y, z0, z1);
  float px, py;
  int first = 0;
  if (!belief) {
    // seed on the first row's ring, one particle per sector
    float s, c;
    sincos_rev(((float)lane + u01(x.z)) * (1.0f / (float)kPfParticles), s, c);
    const float rad = fmaf(fast_sqrt(sl2), z0, rr[0]);
    px = fmaf(rad, c, rx[0]);
    py = fmaf(rad, s, ry[0]);
    first = 1;
  } else {
    px = fmaf(a.q, z0, prev.x);
    py = fmaf(a.q, z1, prev.y);
  }
  if (m > first) {
    const float inv2s2 = 0.5f * __builtin_amdgcn_rcpf(sl2);
    float lw = 0.0f;
#pragma unroll
    for (int s = 0; s < MR; ++s) {
      if (s >= first && s < m) {
        const float dx = px - rx[s], dy = py - ry[s];
        const float res = fast_sqrt(fmaf(dx, dx, dy * dy)) - rr[s];
        lw = fmaf(-res * res, inv2s2, lw);
      }
    }
    const float top = wave_max(lw, lane);
    const float wt = __expf(lw - top);
    const float cum = wave_scan_add(wt, lane);
    const float total = lane_value(cum, 63);
    const float U = u01(__builtin_amdgcn_readfirstlane(x.w));
    const float point = ((float)lane + U) * (1.0f / (float)kPfParticles) * total;
    // first index whose cumulative weight exceeds the point: the number of
    // cumulative weights <= point (at most 63)
    int src = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
      const float cv = __shfl(cum, src + step - 1);
      if (cv <= point) src += step;
    }
    px = __shfl(px, src);
    py = __shfl(py, src);
  }
  a.pfxy[w * kPfParticles + lane] = make_float2(px, py);
  const float mx = wave_sum(px, lane) * (1.0f / (float)kPfParticles);
  const float my = wave_sum(py, lane) * (1.0f / (float)kPfParticles);
  if (lane == 0) {
    a.pfb[w] = 1;
    a.ex[w] = mx;
    a.ey[w] = my;
    a.ev[w] = 1;
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
  a.pfxy = reinterpret_cast<float2 *>(s.pfxy);
  a.pfb = s.pfb;
  a.pfm = reinterpret_cast<const float4 *>(s.pfm);
  a.ex = s.ex;
  a.ey = s.ey;
  a.ev = s.ev;
  a.p0 = p_begin;
  a.P = p_end;
  a.t = (uint32_t)t;
  a.c3 = (episode << 4) | kPurposePf;
  a.key0 = p.key0;
  a.key1 = p.key1;
  a.q = p.pf_q;
  a.lik2 = p.pf_lik_sigma * p.pf_lik_sigma;
  const int64_t blocks = (p_end - p_begin + kPfWaves - 1) / kPfWaves;
  hipStream_t st = (hipStream_t)stream;
  if (p.pooled)
    hipLaunchKernelGGL(pf_kernel<true>, dim3((unsigned)blocks), dim3(64 * kPfWaves), 0, st, a);
  else
    hipLaunchKernelGGL(pf_kernel<false>, dim3((unsigned)blocks), dim3(64 * kPfWaves), 0, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mil
