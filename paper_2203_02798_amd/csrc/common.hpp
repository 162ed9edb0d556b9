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

__host__ __device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1,
                                               uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    // one 32x32->64 multiply (v_mad_u64_u32) gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
#if defined(__HIP_DEVICE_COMPILE__)
    // three-input XOR in one instruction (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
#else
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
#endif
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
__host__ __device__ __forceinline__ void cs_hash_row(uint64_t i, uint32_t r, uint64_t seed,
                                            uint32_t &h, uint32_t &neg) {
  const u32x4 x = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), 0u, 0u,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t X = ((uint64_t)x.x1 << 32) | x.x0;
  h = (uint32_t)(((unsigned __int128)X * (uint64_t)r) >> 64);
  neg = x.x2 & 1u;
}

// ---------------------------------------------------------------------------
// Lean FP64 elementary functions for Box-Muller, on the ranges it needs.
// Accuracy about 1e-16 relative; no branches.
// ---------------------------------------------------------------------------
// ln(x) for x in (0, 1]: x = f 2^e with f in [1/sqrt2, sqrt2),
// ln f = 2 atanh(s), s = (f-1)/(f+1), |s| <= 0.1716, atanh by its power
// series s + s^3/3 + ... + s^19/19 (truncation below 1e-17); ln 2 is split so
// that e * ln2_hi is exact.
__host__ __device__ __forceinline__ double bm_log(double x) {
  int e;
  double f = frexp(x, &e);  // f in [1/2, 1)
  const bool lo = f < 0.70710678118654752440;
  f = lo ? 2.0 * f : f;
  e = lo ? e - 1 : e;
  const double s = (f - 1.0) / (f + 1.0);
  const double s2 = s * s;
  double p = 1.0 / 19.0;
  p = fma(p, s2, 1.0 / 17.0);
  p = fma(p, s2, 1.0 / 15.0);
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  const double lnf = fma(2.0 * s * s2, p, 2.0 * s);
  const double ln2_hi = 0.6931467056274414;       // ln 2 to 21 bits
  const double ln2_lo = 4.7493250390316726e-07;   // ln 2 - ln2_hi
  return fma((double)e, ln2_hi, fma((double)e, ln2_lo, lnf));
}

// sin(pi z) and cos(pi z) for z in [0, 2]: z = k/2 + y with |y| <= 1/4 (exact
// split), Taylor series of sin(pi y) (9 terms) and cos(pi y) (10 terms),
// truncation below 1e-19, then the quarter-turn k mod 4 picks and signs.
__host__ __device__ __forceinline__ void bm_sincospi(double z, double &sn, double &cs) {
  const double k = rint(2.0 * z);
  const double y = fma(-0.5, k, z);
  const double y2 = y * y;
  double ps = 7.952054001475513e-07;
  ps = fma(ps, y2, -2.1915353447830217e-05);
  ps = fma(ps, y2, 0.00046630280576761255);
  ps = fma(ps, y2, -0.0073704309457143504);
  ps = fma(ps, y2, 0.08214588661112823);
  ps = fma(ps, y2, -0.5992645293207921);
  ps = fma(ps, y2, 2.5501640398773455);
  ps = fma(ps, y2, -5.16771278004997);
  ps = fma(ps, y2, 3.141592653589793);
  const double sp = ps * y;
  double pc = -1.3878952462213771e-07;
  pc = fma(pc, y2, 4.303069587032947e-06);
  pc = fma(pc, y2, -0.0001046381049248457);
  pc = fma(pc, y2, 0.0019295743094039231);
  pc = fma(pc, y2, -0.02580689139001406);
  pc = fma(pc, y2, 0.2353306303588932);
  pc = fma(pc, y2, -1.3352627688545895);
  pc = fma(pc, y2, 4.0587121264167685);
  pc = fma(pc, y2, -4.934802200544679);
  const double cp = fma(pc, y2, 1.0);
  const int q = ((int)k) & 3;
  // sin(pi(k/2 + y)) = sp, cp, -sp, -cp ; cos(...) = cp, -sp, -cp, sp
  const double a = (q & 1) ? cp : sp;
  const double b = (q & 1) ? sp : cp;
  sn = (q & 2) ? -a : a;
  cs = ((q + 1) & 2) ? -b : b;
}

// Four unscaled standard normals z0..z3 for buckets 4q .. 4q+3 of Gaussian
// row a (Box-Muller on two pairs of uniforms in (0,1)), FP64.  Counter word 3
// is the stream: 1 for G, 2 for the JL matrix of the leverage estimate (the
// hash uses 0).
__host__ __device__ __forceinline__ void gauss4_f64(uint64_t q, uint32_t a, uint64_t seed,
                                           double z[4], uint32_t stream = 1u) {
  const u32x4 x = philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), a, stream,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  const double s = 2.3283064365386963e-10;  // 2^-32
  const double u0 = ((double)x.x0 + 0.5) * s;
  const double u1 = ((double)x.x1 + 0.5) * s;
  const double u2 = ((double)x.x2 + 0.5) * s;
  const double u3 = ((double)x.x3 + 0.5) * s;
  const double r0 = sqrt(-2.0 * bm_log(u0));
  const double r2 = sqrt(-2.0 * bm_log(u2));
  double s1, c1, s3, c3;
  bm_sincospi(2.0 * u1, s1, c1);
  bm_sincospi(2.0 * u3, s3, c3);
  z[0] = r0 * c1;
  z[1] = r0 * s1;
  z[2] = r2 * c3;
  z[3] = r2 * s3;
}

// sin(2 pi u) and cos(2 pi u) in FP32 for u in [0, 1]: u = k/4 + y with
// |y| <= 1/8 (exact split), Taylor series in y of sin(2 pi y) to y^9 and of
// cos(2 pi y) to y^10 (truncation below 2e-9), quarter turn k mod 4.
__device__ __forceinline__ void sincos_turns_f32(float u, float &sn, float &cs) {
  const float k = rintf(4.0f * u);
  const float y = fmaf(-0.25f, k, u);
  const float y2 = y * y;
  float ps = 42.058693944897634f;
  ps = fmaf(ps, y2, -76.70585975306136f);
  ps = fmaf(ps, y2, 81.60524927607504f);
  ps = fmaf(ps, y2, -41.341702240399755f);
  ps = fmaf(ps, y2, 6.283185307179586f);
  const float sp = ps * y;
  float pc = -26.426256783374388f;
  pc = fmaf(pc, y2, 60.24464137187664f);
  pc = fmaf(pc, y2, -85.45681720669371f);
  pc = fmaf(pc, y2, 64.93939402266828f);
  pc = fmaf(pc, y2, -19.739208802178716f);
  const float cp = fmaf(pc, y2, 1.0f);
  const int q = ((int)k) & 3;
  const float a = (q & 1) ? cp : sp;
  const float b = (q & 1) ? sp : cp;
  sn = (q & 2) ? -a : a;
  cs = ((q + 1) & 2) ? -b : b;
}

// The same four normals as gauss4_f64 evaluated in FP32 (for the bfloat16
// GEMM, which rounds them to 8 significant bits afterwards): u = x 2^-32 +
// 2^-33 in FP32 (exact for small x, so the tail is kept), ln u through the
// hardware base-2 logarithm, sin/cos by sincos_turns_f32.  Error a few FP32
// ulps against the FP64 values.
__device__ __forceinline__ void gauss4_f32(uint64_t q, uint32_t a, uint64_t seed,
                                           float z[4]) {
  const u32x4 x = philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), a, 1u,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  const float s = 2.3283064365386963e-10f;  // 2^-32
  const float h = 1.1641532182693481e-10f;  // 2^-33
  const float u0 = fmaf((float)x.x0, s, h);
  const float u1 = fmaf((float)x.x1, s, h);
  const float u2 = fmaf((float)x.x2, s, h);
  const float u3 = fmaf((float)x.x3, s, h);
  const float m2ln2 = -1.3862943611198906f;  // -2 ln 2
  const float r0 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u0));
  const float r2 = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u2));
  float s1, c1, s3, c3;
  sincos_turns_f32(u1, s1, c1);
  sincos_turns_f32(u3, s3, c3);
  z[0] = r0 * c1;
  z[1] = r0 * s1;
  z[2] = r2 * c3;
  z[3] = r2 * s3;
}

// ---------------------------------------------------------------------------
// CountSketch bucket sum of CSR rows into an LDS row (one wavefront)
// ---------------------------------------------------------------------------
// acc[col] += sign * A[row, col] for the rows of bin-list entries j0 .. j1-1
// (perm[j] = row | sign << 31), rows applied in list order, a row's entries
// in any order (they touch distinct columns), so the sums have one fixed
// order.  The row pointers and the first kBucketEnt entries of up to 64 rows
// are loaded at once, one row per lane, and the rows are then applied one
// after another from registers; rows with more entries are spread over the
// wavefront.  The accumulators have type AT (FP64 for every S*A of this
// library: FP32 entries are widened exactly and summed in FP64).
constexpr int kBucketEnt = 4;

template <typename T, typename AT>
__device__ __forceinline__ void bucket_rows_add(const T *__restrict__ vals,
                                                const int64_t *__restrict__ indptr,
                                                const int32_t *__restrict__ indices,
                                                const uint32_t *__restrict__ perm, uint32_t j0,
                                                uint32_t j1, AT *acc) {
  const int lane = (int)(threadIdx.x & 63u);
  for (uint32_t base = j0; base < j1; base += 64) {
    const uint32_t j = base + (uint32_t)lane;
    int64_t p0 = 0, p1 = 0;
    int ng = 0;
    if (j < j1) {
      const uint32_t pv = perm[j];
      const int64_t row = (int64_t)(pv & 0x7fffffffu);
      ng = (int)(pv >> 31);
      p0 = indptr[row];
      p1 = indptr[row + 1];
    }
    const int64_t len = p1 - p0;
    const bool lng = len > kBucketEnt;
    int ci[kBucketEnt];
    AT xv[kBucketEnt];
#pragma unroll
    for (int e = 0; e < kBucketEnt; ++e) {
      ci[e] = 0;
      xv[e] = AT(0);
      if (!lng && e < len) {
        ci[e] = indices[p0 + e];
        const AT v = (AT)vals[p0 + e];
        xv[e] = ng ? -v : v;
      }
    }
    const uint64_t longmask = __ballot(lng);
    const int cnt = (j1 - base) < 64u ? (int)(j1 - base) : 64;
    for (int i = 0; i < cnt; ++i) {
      if ((longmask >> i) & 1u) {
        const int64_t q0 = __shfl(p0, i, 64);
        const int64_t q1 = __shfl(p1, i, 64);
        const int ngi = __shfl(ng, i, 64);
        for (int64_t p = q0 + lane; p < q1; p += 64) {
          const AT v = (AT)vals[p];
          atomicAdd(&acc[indices[p]], ngi ? -v : v);
        }
      } else if (lane == i) {
#pragma unroll
        for (int e = 0; e < kBucketEnt; ++e)
          if (e < len) atomicAdd(&acc[ci[e]], xv[e]);
      }
    }
  }
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
