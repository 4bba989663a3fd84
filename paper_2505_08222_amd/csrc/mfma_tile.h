// Block-level BF16 GEMM on gfx950 matrix cores, shared by the policy and the
// learned-estimator inference kernels.
//
// D[m][n] = sum_k A[m][k] B[n][k] over 16x16 output tiles with
// v_mfma_f32_16x16x32_bf16 (FP32 accumulation). Both operands are
// K-contiguous BF16 with 16-byte aligned rows; lane l of a wavefront feeds
// row l%16 and the 8 consecutive K at 8*(l/16), and receives D rows
// 4*(l/16)+j, column l%16. epi(m, n, value) consumes every output element.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

namespace mil {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Block of four wavefronts, N a multiple of 64, row-stationary: wavefront w
// owns column blocks w, w + 4, ... (N / 64 of them) and loads all their
// weight fragments (B, from global memory / L2) once; it then walks the row
// tiles of A (LDS), fetching the next tile's A fragments while the current
// one's MFMAs (independent across its column blocks) and epilogue run.
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
      b[c][ks] = *reinterpret_cast<const bf16x8 *>(B + (((wave + c * NW) << 4) + row) * ldb +
                                                   ks * 32 + 8 * kg);
  bf16x8 a[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
    a[ks] = *reinterpret_cast<const bf16x8 *>(A + row * lda + ks * 32 + 8 * kg);
  for (int mt = 0; mt < tm; ++mt) {
    const int m0 = mt << 4;
    bf16x8 an[KS];
    const int mn = (mt + 1 < tm ? m0 + 16 : m0);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      an[ks] = *reinterpret_cast<const bf16x8 *>(A + (mn + row) * lda + ks * 32 + 8 * kg);
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

// A wavefront's weight fragments for a K x N layer: column blocks w, w + 4,
// ... of B, every K slice. Loaded ahead of the GEMM that uses them, so that
// their latency overlaps the work before it.
template <int K, int N>
struct BFrag {
  static constexpr int KS = K / 32, NCT = N / 64;
  bf16x8 v[NCT][KS];
};
template <int K, int N>
__device__ __forceinline__ void load_bfrag(BFrag<K, N> &f, const __bf16 *B, int ldb) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = lane & 15, kg = lane >> 4;
#pragma unroll
  for (int c = 0; c < BFrag<K, N>::NCT; ++c)
#pragma unroll
    for (int ks = 0; ks < BFrag<K, N>::KS; ++ks)
      f.v[c][ks] = *reinterpret_cast<const bf16x8 *>(B + (((wave + c * 4) << 4) + row) * ldb +
                                                     ks * 32 + 8 * kg);
}

// The same walk with the operands' roles swapped in the instruction (weights
// as its A, activations as its B) and the weight fragments already in
// registers. The 16x16 result comes out transposed: lane l receives row
// m0 + l%16 and the four consecutive columns n0 + 4*(l/16) + j, and epi4(m,
// n, v) consumes v[j] = D[m][n + j], so that the epilogue reads and writes
// four neighbouring features at once.
template <int K, int N, typename Epi4>
__device__ __forceinline__ void gemm_rs_bf16_tf(const __bf16 *A, int lda, const BFrag<K, N> &f,
                                                int M, Epi4 epi4) {
  constexpr int KS = K / 32, NW = 4, NCT = N / (16 * NW);
  static_assert(N % (16 * NW) == 0 && K % 32 == 0, "shape");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = lane & 15, kg = lane >> 4;
  const int tm = M >> 4;
  bf16x8 a[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
    a[ks] = *reinterpret_cast<const bf16x8 *>(A + row * lda + ks * 32 + 8 * kg);
  for (int mt = 0; mt < tm; ++mt) {
    const int m0 = mt << 4;
    bf16x8 an[KS];
    const int mn = (mt + 1 < tm ? m0 + 16 : m0);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      an[ks] = *reinterpret_cast<const bf16x8 *>(A + (mn + row) * lda + ks * 32 + 8 * kg);
    floatx4 acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      acc[c] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.v[c][ks], a[ks], acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < NCT; ++c) epi4(m0 + row, ((wave + c * NW) << 4) + 4 * kg, acc[c]);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[ks] = an[ks];
  }
}

// Sum over the four lanes of a quad (DPP butterfly, lanes xor 1 then xor 2);
// every lane of the quad ends with the same value. The whole quad must be
// active.
__device__ __forceinline__ float quad_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  return v;
}

// Sum over the four lanes l % 16 + 16 g (g = 0..3) of a wavefront: each
// cross-row swap leaves a lane's own value in one result and its partner's in
// the other, and the sum is symmetric.
__device__ __forceinline__ float col_sum4(float v) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
  v = __int_as_float(r[0]) + __int_as_float(r[1]);
  r = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}

// GELU, tanh form (Hendrycks & Gimpel), for activations that are rounded to
// BF16 next: 0.5 x (1 + tanh(y)) with y = sqrt(2/pi) (x + 0.044715 x^3) is
// the same function as x * sigma(2y) = x / (1 + 2^u), u = -2 y log2(e),
// evaluated with the hardware base-2 exponential and reciprocal.
__device__ __forceinline__ float gelu_tanh_fast(float x) {
  constexpr float a = -2.0f * 0.7978845608028654f * 1.4426950408889634f;
  constexpr float b = a * 0.044715f;
  const float u = x * fmaf(b, x * x, a);
  return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u));
}

}  // namespace mil
