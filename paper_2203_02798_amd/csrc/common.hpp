// Shared device helpers of libpsk (gfx950): Philox4x32-10, the CountSketch
// hash, Box-Muller normals, wave-level primitives, and error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace psk {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);

#define PSK_HIP_TRY(expr)                                                     \
  do {                                                                        \
    hipError_t _e = (expr);                                                   \
    if (_e != hipSuccess)                                                     \
      return ::psk::fail(-4, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): four 32-bit words of
// state, two of key; each round multiplies words 0 and 2 by fixed odd
// constants, crosses the high halves with words 1/3 and the key, and the key
// advances by the Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct u32x4 {
  uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1,
                                               uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    // one 32x32->64 multiply (v_mad_u64_u32) gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return u32x4{c0, c1, c2, c3};
}

// CountSketch hash of global row i: bucket in [0, r), sign bit (1 = -1).
__device__ __forceinline__ void cs_hash_row(uint64_t i, uint32_t r, uint64_t seed,
                                            uint32_t &h, uint32_t &neg) {
  const u32x4 x = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), 0u, 0u,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t X = ((uint64_t)x.x1 << 32) | x.x0;
  h = (uint32_t)__umul64hi(X, (uint64_t)r);
  neg = x.x2 & 1u;
}

// Four unscaled standard normals z0..z3 for buckets 4q .. 4q+3 of Gaussian
// row a (Box-Muller on two pairs of uniforms in (0,1)), FP64.
__device__ __forceinline__ void gauss4_f64(uint64_t q, uint32_t a, uint64_t seed,
                                           double z[4]) {
  const u32x4 x = philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), a, 1u,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  const double s = 2.3283064365386963e-10;  // 2^-32
  const double u0 = ((double)x.x0 + 0.5) * s;
  const double u1 = ((double)x.x1 + 0.5) * s;
  const double u2 = ((double)x.x2 + 0.5) * s;
  const double u3 = ((double)x.x3 + 0.5) * s;
  const double r0 = sqrt(-2.0 * log(u0));
  const double r2 = sqrt(-2.0 * log(u2));
  double s1, c1, s3, c3;
  sincospi(2.0 * u1, &s1, &c1);
  sincospi(2.0 * u3, &s3, &c3);
  z[0] = r0 * c1;
  z[1] = r0 * s1;
  z[2] = r2 * c3;
  z[3] = r2 * s3;
}

// Same normals computed in FP32 (for the reduced-precision GEMM, where the
// values are rounded to bfloat16 afterwards).  Uniforms keep the top 24 bits
// of each word: u = (floor(x / 2^8) + 1/2) * 2^-24.
__device__ __forceinline__ void gauss4_f32(uint64_t q, uint32_t a, uint64_t seed,
                                           float z[4]) {
  const u32x4 x = philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), a, 1u,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  const float s = 5.9604644775390625e-08f;  // 2^-24
  const float u0 = ((float)(x.x0 >> 8) + 0.5f) * s;
  const float u1 = ((float)(x.x1 >> 8) + 0.5f) * s;
  const float u2 = ((float)(x.x2 >> 8) + 0.5f) * s;
  const float u3 = ((float)(x.x3 >> 8) + 0.5f) * s;
  const float r0 = sqrtf(-2.0f * __logf(u0));
  const float r2 = sqrtf(-2.0f * __logf(u2));
  float s1, c1, s3, c3;
  sincospif(2.0f * u1, &s1, &c1);
  sincospif(2.0f * u3, &s3, &c3);
  z[0] = r0 * c1;
  z[1] = r0 * s1;
  z[2] = r2 * c3;
  z[3] = r2 * s3;
}

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) {
  return (a + b - 1) / b;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ int wave_uniform(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace psk
