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

// Non-zero k (0 <= k < s) of column i of an OSNAP with s blocks of rb rows
// (block construction): the CountSketch hash with k in counter word 2, its
// range reduced to the block, offset to block k.  k = 0 with rb = r is
// cs_hash_row.
__host__ __device__ __forceinline__ void osnap_hash_nz(uint64_t i, uint32_t k, uint32_t rb,
                                                       uint64_t seed, uint32_t &row,
                                                       uint32_t &neg) {
  const u32x4 x = philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), k, 0u, (uint32_t)seed,
                                (uint32_t)(seed >> 32));
  const uint64_t X = ((uint64_t)x.x1 << 32) | x.x0;
  row = k * rb + (uint32_t)(((unsigned __int128)X * (uint64_t)rb) >> 64);
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
__host__ __device__ __forceinline__ void box_muller_f64(const u32x4 &x, double z[4]) {
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

__host__ __device__ __forceinline__ void gauss4_f64(uint64_t q, uint32_t a, uint64_t seed,
                                           double z[4], uint32_t stream = 1u) {
  const u32x4 x = philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), a, stream,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  box_muller_f64(x, z);
}

// sin(2 pi u) and cos(2 pi u) in FP32 for u = (x + 1/2) 2^-32, reduced to a
// quarter turn on the integer: u = k/4 + y with k = round(4 u) and the
// offset y = (x - k 2^30 + 1/2) 2^-32 in [-1/8, 1/8] formed exactly before
// its one rounding to FP32 (so y keeps its relative accuracy even where u
// is close to 1); Taylor series in y of sin(2 pi y) to y^9 and of
// cos(2 pi y) to y^10 (truncation below 2e-9), then the quarter turn.
__device__ __forceinline__ void sincos_turns_u32(uint32_t x, float &sn, float &cs) {
  const uint32_t k = (x + 0x20000000u) >> 30;          // 0 .. 4
  const int32_t yi = (int32_t)(x - (k << 30));          // [-2^29, 2^29)
  const float y = fmaf((float)yi, 2.3283064365386963e-10f, 1.1641532182693481e-10f);
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
  const uint32_t q = k & 3u;
  // sin(2 pi (k/4 + y)) = sp, cp, -sp, -cp ; cos(...) = cp, -sp, -cp, sp
  const float a = (q & 1u) ? cp : sp;
  const float b = (q & 1u) ? sp : cp;
  sn = (q & 2u) ? -a : a;
  cs = ((q + 1u) & 2u) ? -b : b;
}

// -2 ln(u) in FP32 for u = (x + 1/2) 2^-32.  For u < 3/4 from u itself
// (exact to one rounding) through the hardware base-2 logarithm.  For
// u >= 3/4 from v = 1 - u = (~x + 1/2) 2^-32, formed exactly from the
// complement of x before its one rounding: -ln(1 - v) = v (1 + v/2 + v^2/3
// + ... + v^11/12) (v <= 1/4: truncation below 2^-26 relative), which
// keeps the relative accuracy that u itself, rounded to FP32 next to 1,
// has lost.
__device__ __forceinline__ float m2ln_unit_f32(uint32_t x) {
  const float s = 2.3283064365386963e-10f;  // 2^-32
  const float h = 1.1641532182693481e-10f;  // 2^-33
  const float u = fmaf((float)x, s, h);
  const float v = fmaf((float)(~x), s, h);
  const float lg = -1.3862943611198906f * __builtin_amdgcn_logf(u);  // -2 ln 2 log2(u)
  float p = 1.0f / 12.0f;
  p = fmaf(p, v, 1.0f / 11.0f);
  p = fmaf(p, v, 1.0f / 10.0f);
  p = fmaf(p, v, 1.0f / 9.0f);
  p = fmaf(p, v, 1.0f / 8.0f);
  p = fmaf(p, v, 1.0f / 7.0f);
  p = fmaf(p, v, 1.0f / 6.0f);
  p = fmaf(p, v, 1.0f / 5.0f);
  p = fmaf(p, v, 1.0f / 4.0f);
  p = fmaf(p, v, 1.0f / 3.0f);
  p = fmaf(p, v, 0.5f);
  p = fmaf(p, v, 1.0f);
  const float ls = 2.0f * v * p;
  return x >= 0xC0000000u ? ls : lg;
}

// The same four normals as gauss4_f64 evaluated in FP32 (for the bfloat16
// and FP8 products, which round them to 8 or 4 significant bits afterwards):
// the radius from m2ln_unit_f32 and the hardware square root, the angle from
// sincos_turns_u32.  Measured against the FP64 values on 2^30 blocks: see
// kNormalF32Ulps.
__device__ __forceinline__ void box_muller_f32(const u32x4 &x, float z[4]) {
  const float r0 = __builtin_amdgcn_sqrtf(m2ln_unit_f32(x.x0));
  const float r2 = __builtin_amdgcn_sqrtf(m2ln_unit_f32(x.x2));
  float s1, c1, s3, c3;
  sincos_turns_u32(x.x1, s1, c1);
  sincos_turns_u32(x.x3, s3, c3);
  z[0] = r0 * c1;
  z[1] = r0 * s1;
  z[2] = r2 * c3;
  z[3] = r2 * s3;
}

__device__ __forceinline__ void gauss4_f32(uint64_t q, uint32_t a, uint64_t seed,
                                           float z[4]) {
  const u32x4 x = philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), a, 1u,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  box_muller_f32(x, z);
}

// ---------------------------------------------------------------------------
// G rounded to bfloat16 or FP8 e4m3 with every rounding decided as for the
// FP64 normal.  An FP32 normal lies within kNormalF32Ulps FP32 ulps of the
// FP64 one (measured maximum 5.2 over 4.3e9 normals, all seeds tested); its
// rounding can differ from the FP64 value's only when it lies within that
// distance of a rounding midpoint.  Such values (about 1 in 4000 for
// bfloat16, 1 in 5000 for e4m3 counting its subnormal range) are recomputed
// in FP64 from the same Philox words and rounded once from FP64; the FP32
// rounding is kept for all others.  The window is counted in ulps of the
// FP32 value: 2 kNormalF32Ulps + 2 covers a binade change between the two.
// ---------------------------------------------------------------------------
constexpr uint32_t kNormalF32Ulps = 8;
constexpr uint32_t kTieWindow = 2 * kNormalF32Ulps + 2;

// bits of x below bfloat16's 7 fraction bits within kTieWindow of the
// half-way pattern (also true for NaN/Inf patterns, which do not occur)
__device__ __forceinline__ bool bf16_near_tie(float x) {
  const uint32_t dbits = __float_as_uint(x) & 0xFFFFu;
  return dbits - (0x8000u - kTieWindow) <= 2u * kTieWindow;
}

// e4m3 of x (x = z 2^6, |x| < 448): on e4m3's normal range (|x| >= 2^-6)
// the 20 bits of x below e4m3's 3 fraction bits within kTieWindow of the
// half-way pattern; below it (quantum 2^-9) |x| 2^9 within kTieWindow of
// its ulps from a half-integer
__device__ __forceinline__ bool e4m3_near_tie(float x) {
  const uint32_t b = __float_as_uint(x) & 0x7FFFFFFFu;
  if (b >= 0x3C800000u) {
    const uint32_t dbits = b & 0xFFFFFu;
    return dbits - (0x80000u - kTieWindow) <= 2u * kTieWindow;
  }
  const float t = __uint_as_float(b) * 512.0f;                 // exact, < 8
  const float ulp = __uint_as_float((__float_as_uint(t) & 0x7F800000u)) * 1.1920928955078125e-7f;
  return fabsf((t - truncf(t)) - 0.5f) <= (float)kTieWindow * ulp;
}

// FP32 of a double by round-to-odd: a later rounding to a narrower format
// (bfloat16, e4m3) is then a single correct rounding of the double
__device__ __forceinline__ float f32_round_odd(double v) {
  float f = (float)v;
  if ((double)f != v && v == v) {
    uint32_t b = __float_as_uint(f);
    if (fabs((double)f) > fabs(v)) b -= 1;
    b |= 1u;
    f = __uint_as_float(b);
  }
  return f;
}

// e4m3 byte (RNE) of an FP32 value
__device__ __forceinline__ uint32_t e4m3_byte(float x) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFFu;
}

// exponent of G's fixed FP8 scale: |z| < 6.77 for every normal of this
// generator and 448 2^-6 = 7, so no value saturates
constexpr int kGFp8Exp = -6;

// The Philox words of G's block (q, a): stream 1.
__device__ __forceinline__ u32x4 philox_g(uint64_t q, uint32_t a, uint64_t seed) {
  return philox4x32_10((uint32_t)q, (uint32_t)(q >> 32), a, 1u, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
}

// Four normals from Philox words x rounded to bfloat16 (RNE) through FP32,
// returned as FP32 values; bit k of the result is set where normal k lies
// within the window of a rounding midpoint and needs gauss4_bf16_fix.
__device__ __forceinline__ uint32_t gauss4_bf16_fast(const u32x4 &x, float out[4]) {
  float z[4];
  box_muller_f32(x, z);
  uint32_t near = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    out[k] = (float)(__bf16)z[k];
    near |= (uint32_t)bf16_near_tie(z[k]) << k;
  }
  return near;
}

// Normal k (0 .. 3) of Philox words x in FP64, alone (as box_muller_f64)
__device__ __forceinline__ double normal_f64_k(const u32x4 &x, int k) {
  const double s = 2.3283064365386963e-10;  // 2^-32
  const uint32_t xr = k < 2 ? x.x0 : x.x2, xa = k < 2 ? x.x1 : x.x3;
  const double rad = sqrt(-2.0 * bm_log(((double)xr + 0.5) * s));
  double sn, cs;
  bm_sincospi(2.0 * (((double)xa + 0.5) * s), sn, cs);
  return rad * ((k & 1) ? sn : cs);
}

// out[k] for the set bits k of `near`: the rounding of the FP64 normal
// (one normal at a time, called out of line: the path is rare and its FP64
// temporaries stay out of the callers' registers)
__device__ __noinline__ void gauss4_bf16_fix(const u32x4 &x, uint32_t near, float out[4]) {
#pragma unroll 1
  for (int k = 0; k < 4; ++k)
    if ((near >> k) & 1u) out[k] = (float)(__bf16)f32_round_odd(normal_f64_k(x, k));
}

// Four normals of Philox block (q, a) rounded to bfloat16 (RNE), returned
// as FP32 values, each equal to the rounding of the FP64 normal.
__device__ __forceinline__ void gauss4_bf16(uint64_t q, uint32_t a, uint64_t seed,
                                            float out[4]) {
  const u32x4 x = philox_g(q, a, seed);
  const uint32_t near = gauss4_bf16_fast(x, out);
  if (__builtin_expect(near != 0u, 0)) gauss4_bf16_fix(x, near, out);
}

// The same four normals as e4m3 bytes of z 2^6 (G's fixed scale), byte k in
// bits 8k .. 8k+7, rounded through FP32; *near as for gauss4_bf16_fast.
__device__ __forceinline__ uint32_t gauss4_e4m3_fast(const u32x4 &x, uint32_t *near) {
  float z[4];
  box_muller_f32(x, z);
  uint32_t bytes = 0, nr = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float xs = ldexpf(z[k], -kGFp8Exp);
    bytes |= e4m3_byte(xs) << (8 * k);
    nr |= (uint32_t)e4m3_near_tie(xs) << k;
  }
  *near = nr;
  return bytes;
}

// `bytes` with byte k replaced, for the set bits k of `near`, by the
// rounding of the FP64 normal
__device__ __noinline__ uint32_t gauss4_e4m3_fix(const u32x4 &x, uint32_t near, uint32_t bytes) {
#pragma unroll 1
  for (int k = 0; k < 4; ++k)
    if ((near >> k) & 1u) {
      const uint32_t bk = e4m3_byte(f32_round_odd(ldexp(normal_f64_k(x, k), -kGFp8Exp)));
      bytes = (bytes & ~(0xFFu << (8 * k))) | (bk << (8 * k));
    }
  return bytes;
}

__device__ __forceinline__ uint32_t gauss4_e4m3(uint64_t q, uint32_t a, uint64_t seed) {
  const u32x4 x = philox_g(q, a, seed);
  uint32_t near;
  const uint32_t bytes = gauss4_e4m3_fast(x, &near);
  return __builtin_expect(near != 0u, 0) ? gauss4_e4m3_fix(x, near, bytes) : bytes;
}

// the value of e4m3 byte k of `bytes` times G's scale, as FP32
__device__ __forceinline__ float e4m3_g_value(uint32_t bytes, int k) {
  const int b = (int)((bytes >> (8 * k)) & 0xFFu);
  return ldexpf(__builtin_amdgcn_cvt_f32_fp8(b, 0), kGFp8Exp);
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
