// Batched range-only estimator over independent windows, and the RNG check
// kernel.
//
// est_exact: one thread per window. A block stages its windows through LDS
// with coalesced 16-byte loads (the [N][W][3] layout is contiguous per
// block), then every thread solves its own window in registers: linearised
// least squares about the window centroid (arXiv 2505.08222, Sec. III-A) in
// FP64 (or FP32 on request), optionally refined by Gauss-Newton.
#include <hip/hip_runtime.h>

#include "env_internal.h"
#include "ls_device.h"
#include "rng.h"

namespace mil {

// FP32 variant of the linearised solve, centred form c_k = |u_k|^2 - d_k (2 rbar + d_k).
template <int WC>
__device__ __forceinline__ bool ls_fp32(const float (&hx)[WC], const float (&hy)[WC],
                                        const float (&hr)[WC], int W, float tau, float &px,
                                        float &py) {
  int n = 0;
  float mx = 0.f, my = 0.f, mr = 0.f;
#pragma unroll
  for (int k = 0; k < WC; ++k)
    if (k < W && hr[k] == hr[k]) {
      ++n;
      mx += hx[k];
      my += hy[k];
      mr += hr[k];
    }
  if (n < 3) return false;
  const float invn = 1.0f / (float)n;
  mx *= invn;
  my *= invn;
  mr *= invn;
  float sxx = 0.f, sxy = 0.f, syy = 0.f, gx = 0.f, gy = 0.f;
#pragma unroll
  for (int k = 0; k < WC; ++k)
    if (k < W && hr[k] == hr[k]) {
      const float ux = hx[k] - mx, uy = hy[k] - my, d = hr[k] - mr;
      const float c = ux * ux + uy * uy - d * (2.0f * mr + d);
      sxx += ux * ux;
      sxy += ux * uy;
      syy += uy * uy;
      gx += ux * c;
      gy += uy * c;
    }
  const float det = sxx * syy - sxy * sxy, tr = sxx + syy;
  if (!(det > tau * tr * tr)) return false;
  const float h = 0.5f / det;
  px = mx + h * (syy * gx - sxy * gy);
  py = my + h * (sxx * gy - sxy * gx);
  return true;
}

template <int WC, int BLOCK>
__global__ void __launch_bounds__(BLOCK)
est_exact_kernel(const float *__restrict__ win, int64_t N, int32_t W, int32_t gn_iters,
                 float tau, int32_t accum, float *__restrict__ out, uint8_t *__restrict__ valid) {
  extern __shared__ float stage[];  // BLOCK * W * 3 floats
  const int64_t first = (int64_t)blockIdx.x * BLOCK;
  const int64_t nwin = (N - first) < BLOCK ? (N - first) : BLOCK;
  const int64_t nfl = nwin * W * 3;
  const float *src = win + first * W * 3;
  // the block's slab is contiguous: copy it with 16-byte loads when aligned
  if ((((uintptr_t)src) & 15) == 0) {
    const int64_t n4 = nfl / 4;
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
    float4 *d4 = reinterpret_cast<float4 *>(stage);
    for (int64_t k = threadIdx.x; k < n4; k += BLOCK) d4[k] = s4[k];
    for (int64_t k = n4 * 4 + threadIdx.x; k < nfl; k += BLOCK) stage[k] = src[k];
  } else {
    for (int64_t k = threadIdx.x; k < nfl; k += BLOCK) stage[k] = src[k];
  }
  __syncthreads();
  if (threadIdx.x >= nwin) return;
  float hx[WC], hy[WC], hr[WC];
  const float *mine = stage + (int64_t)threadIdx.x * W * 3;
#pragma unroll
  for (int k = 0; k < WC; ++k) {
    const bool in = k < W;
    hx[k] = in ? mine[3 * k] : 0.f;
    hy[k] = in ? mine[3 * k + 1] : 0.f;
    hr[k] = in ? mine[3 * k + 2] : __int_as_float(0x7fc00000);
  }
  const int64_t w = first + threadIdx.x;
  bool ok;
  float px = 0.f, py = 0.f;
  if (accum == 1 && gn_iters == 0) {
    ok = ls_fp32<WC>(hx, hy, hr, W, tau, px, py);
  } else {
    double dx = 0.0, dy = 0.0;
    ok = ls_masked<WC>(hx, hy, hr, W, gn_iters, (double)tau, dx, dy);
    px = (float)dx;
    py = (float)dy;
  }
  out[2 * w] = ok ? px : 0.f;
  out[2 * w + 1] = ok ? py : 0.f;
  valid[w] = ok ? 1 : 0;
}

template <int WC, int BLOCK>
static int launch_est_t(const float *d_win, int64_t N, int32_t W, int32_t gn_iters, float tau,
                        int32_t accum, float *d_out, uint8_t *d_valid, hipStream_t st) {
  const int64_t blocks = (N + BLOCK - 1) / BLOCK;
  const size_t lds = (size_t)BLOCK * W * 3 * sizeof(float);
  hipLaunchKernelGGL((est_exact_kernel<WC, BLOCK>), dim3((unsigned)blocks), dim3(BLOCK), lds, st,
                     d_win, N, W, gn_iters, tau, accum, d_out, d_valid);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_est_exact(const float *d_win, int64_t N, int32_t W, int32_t gn_iters, float tau,
                     int32_t accum, float *d_out, uint8_t *d_valid, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (N <= 0) return 0;
  if (W <= 16) return launch_est_t<16, 256>(d_win, N, W, gn_iters, tau, accum, d_out, d_valid, st);
  if (W <= 32) return launch_est_t<32, 128>(d_win, N, W, gn_iters, tau, accum, d_out, d_valid, st);
  return launch_est_t<64, 64>(d_win, N, W, gn_iters, tau, accum, d_out, d_valid, st);
}

__global__ void rng_kernel(const uint32_t *__restrict__ ctr, int64_t n, uint32_t key0,
                           uint32_t key1, uint32_t *__restrict__ out, float *__restrict__ uo,
                           float *__restrict__ no) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const u32x4 x = philox4x32_10(ctr[4 * k], ctr[4 * k + 1], ctr[4 * k + 2], ctr[4 * k + 3], key0,
                                key1);
  if (out) {
    out[4 * k] = x.x;
    out[4 * k + 1] = x.y;
    out[4 * k + 2] = x.z;
    out[4 * k + 3] = x.w;
  }
  if (uo) {
    uo[4 * k] = u01(x.x);
    uo[4 * k + 1] = u01(x.y);
    uo[4 * k + 2] = u01(x.z);
    uo[4 * k + 3] = u01(x.w);
  }
  if (no) {
    float a, b, c, d;
    normal2(x.x, x.y, a, b);
    normal2(x.z, x.w, c, d);
    no[4 * k] = a;
    no[4 * k + 1] = b;
    no[4 * k + 2] = c;
    no[4 * k + 3] = d;
  }
}

int launch_rng(const uint32_t *d_ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t *d_out,
               float *d_u01, float *d_normal, void *stream) {
  if (n <= 0) return 0;
  const int bs = 256;
  hipLaunchKernelGGL(rng_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, d_ctr, n, key0, key1, d_out, d_u01, d_normal);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mil
