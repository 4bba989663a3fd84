// Device-side counter-based random numbers for gfx950.
//
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): a 128-bit counter, a 64-bit key,
// each round multiplies words 0 and 2 by two fixed odd constants, mixes the
// product halves with words 1 and 3 and the key, and bumps the key by two
// Weyl constants. The key is the user seed, so on a wavefront it is uniform
// and the key schedule lives in scalar registers.
//
// Every draw of the environment is a pure function of
// (step, global env id, entity code, purpose | episode << 4): results do not
// depend on which lane or launch computes them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mil {

struct u32x4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    // one 32x32->64 multiply-add per product (both halves at once)
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return u32x4{c0, c1, c2, c3};
}

// Uniform in (0,1): ((x >> 9) + 1/2) / 2^23, exact in binary32.
__device__ __forceinline__ float u01(uint32_t x) {
  return __uint2float_rn(x >> 9) * 0x1p-23f + 0x1p-24f;
}

// Native transcendental instructions of gfx950 (about 1-2 ulp): log2, sqrt,
// and sin/cos of an angle given in revolutions (v_sin_f32(x) = sin(2 pi x)).
__device__ __forceinline__ float fast_ln(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ void sincos_rev(float rev, float &s, float &c) {
  s = __builtin_amdgcn_sinf(rev);
  c = __builtin_amdgcn_cosf(rev);
}

// Box-Muller (1958): z0 = sqrt(-2 ln u0) cos(2 pi u1), z1 = ... sin(2 pi u1);
// the angle 2 pi u1 is passed to the hardware as u1 revolutions, exactly.
__device__ __forceinline__ void normal2(uint32_t x0, uint32_t x1, float &z0, float &z1) {
  const float u0 = u01(x0);
  const float u1 = u01(x1);
  const float rad = fast_sqrt(-2.0f * fast_ln(u0));
  float s, c;
  sincos_rev(u1, s, c);
  z0 = rad * c;
  z1 = rad * s;
}

// Uniform choice in 0..n-1: floor(n * x / 2^32).
__device__ __forceinline__ uint32_t choice(uint32_t x, uint32_t n) { return __umulhi(x, n); }

// Counter layout of the environment's draws.
enum : uint32_t {
  kPurposeDynamics = 0,
  kPurposeMeasure = 1,
  kPurposeReset = 2,
  kPurposeConfig = 3,
  kPurposePolicy = 4,
  kPurposeMlpInit = 5,
  kPurposePolicyInit = 6,
};
enum : uint32_t {
  kEntTargetBlock = 16,  // + j/2 for step draws, + j for reset draws
  kEntRangeRow = 64,     // + 8 * agent + j/4
  kEntEnv = 127,
};

}  // namespace mil
