// Block-level BF16 GEMM on gfx950 matrix cores, shared by the policy and the
// learned-estimator inference kernels.
//
// D[m][n] = sum_k A[m][k] B[n][k] over 16x16 output tiles with
// v_mfma_f32_16x16x32_bf16 (FP32 accumulation). Both operands are
// K-contiguous BF16 with 16-byte aligned rows; lane l of a wavefront feeds
// row l%16 and the 8 consecutive K at 8*(l/16), and receives D rows
// 4*(l/16)+j, column l%16. Column-stationary: a wavefront takes a 16-wide
// block of output columns, keeps that block's weight fragments (B, read
// once from global memory / L2, the next block's fetched while this one is
// used) in registers, and sweeps the row tiles of A
// (LDS) two at a time so that the LDS reads of one pair overlap the MFMAs of
// the other. epi(m, n, value) consumes every output element.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

namespace mil {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int K, typename Epi>
__device__ __forceinline__ void gemm_cs_bf16(const __bf16 *A, int lda, const __bf16 *B, int ldb,
                                             int M, int N, Epi epi) {
  constexpr int KS = K / 32;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int tm = M >> 4, tn = N >> 4;
  const int row = lane & 15, kg = lane >> 4;
  bf16x8 bn[KS];  // fragments of the next column block, loaded one block ahead
  if (wave < tn) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      bn[ks] = *reinterpret_cast<const bf16x8 *>(B + ((wave << 4) + row) * ldb + ks * 32 + 8 * kg);
  }
  for (int ct = wave; ct < tn; ct += nw) {
    const int n0 = ct << 4;
    bf16x8 b[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) b[ks] = bn[ks];
    if (ct + nw < tn) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        bn[ks] = *reinterpret_cast<const bf16x8 *>(B + (((ct + nw) << 4) + row) * ldb + ks * 32 + 8 * kg);
    }
    for (int mt = 0; mt < tm; mt += 2) {
      const bool two = mt + 1 < tm;  // uniform
      const int m0 = mt << 4, m1 = two ? m0 + 16 : m0;
      bf16x8 a0[KS], a1[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        a0[ks] = *reinterpret_cast<const bf16x8 *>(A + (m0 + row) * lda + ks * 32 + 8 * kg);
        a1[ks] = *reinterpret_cast<const bf16x8 *>(A + (m1 + row) * lda + ks * 32 + 8 * kg);
      }
      floatx4 c0 = {0.0f, 0.0f, 0.0f, 0.0f}, c1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[ks], b[ks], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[ks], b[ks], c1, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) epi(m0 + 4 * kg + j, n0 + row, c0[j]);
      if (two) {
#pragma unroll
        for (int j = 0; j < 4; ++j) epi(m1 + 4 * kg + j, n0 + row, c1[j]);
      }
    }
  }
}

// The same product for a block of four wavefronts with N a multiple of 64:
// row-stationary. Wavefront w owns column blocks w, w + 4, ... (N / 64 of
// them) and loads all their weight fragments once; it then walks the row
// tiles of A, fetching the next tile's A fragments while the current one's
// MFMAs (independent across its column blocks) and epilogue run.
template <int K, int N, typename Epi>
__device__ __forceinline__ void gemm_rs_bf16(const __bf16 *A, int lda, const __bf16 *B, int ldb,
                                             int M, Epi epi) {
  constexpr int KS = K / 32, NW = 4, NCT = N / (16 * NW);
  static_assert(N % (16 * NW) == 0 && K % 32 == 0, "shape");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = lane & 15, kg = lane >> 4;
  const int tm = M >> 4;
  bf16x8 b[NCT][KS];
#pragma unroll
  for (int c = 0; c < NCT; ++c)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      b[c][ks] = *reinterpret_cast<const bf16x8 *>(B + (((wave + c * NW) << 4) + row) * ldb + ks * 32 + 8 * kg);
  bf16x8 a[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) a[ks] = *reinterpret_cast<const bf16x8 *>(A + row * lda + ks * 32 + 8 * kg);
  for (int mt = 0; mt < tm; ++mt) {
    const int m0 = mt << 4;
    bf16x8 an[KS];
    const int mn = (mt + 1 < tm ? m0 + 16 : m0);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) an[ks] = *reinterpret_cast<const bf16x8 *>(A + (mn + row) * lda + ks * 32 + 8 * kg);
    floatx4 acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      acc[c] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks], b[c][ks], acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) epi(m0 + 4 * kg + j, ((wave + c * NW) << 4) + row, acc[c][j]);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[ks] = an[ks];
  }
}

// GELU, tanh form (Hendrycks & Gimpel), for activations that are rounded to
// BF16 next: tanh(y) = 1 - 2 / (1 + e^{2y}) with the hardware exponential and
// reciprocal.
__device__ __forceinline__ float gelu_tanh_fast(float x) {
  const float y = 0.7978845608028654f * fmaf(0.044715f * x, x * x, x);
  const float th = 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * y));
  return 0.5f * x * (1.0f + th);
}

}  // namespace mil
