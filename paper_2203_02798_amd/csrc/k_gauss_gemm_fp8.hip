// C = G * (S*A) with FP8 e4m3 operands and power-of-two block scales on the
// gfx950 matrix cores (v_mfma_scale_f32_16x16x128_f8f6f4, FP32 accumulation).
//
// Paper mapping (arXiv 2203.02798): Algorithm countgauss_multiply's batched
// C += G_i * B with both operands quantised to OCP e4m3: every block of 128
// buckets of a row of G, and of a column of S*A, shares one scale 2^e with
// e = ceil(log2(amax / 448)) (E8M0), so the block's largest magnitude maps
// into (224, 448].  The matrix instruction applies the two scales itself
// (its scale operands are E8M0 exponents, one per row of G and per column
// of S*A for each 32 values of K; the four of a 128-bucket chunk are equal
// here).  K-split partial products are summed in FP64 by a second kernel,
// which applies 1/sqrt(m).
//
// Operand layout.  For one 128-bucket chunk, lane l of the instruction
// (row or column l % 16, lane group g = l / 16) supplies 32 bytes; byte j of
// group g is taken here to be bucket 32 g + j for both G and S*A, so each
// product pairs a normal with the S*A entry of the same bucket.  Quantised
// S*A is stored as [chunk][g][half][column][16 bytes] (written by
// k_sa_fp8, or for CSR A by k_scatter_csr_fp8 from the binned rows), so
// the 16 lanes of a group read 256 contiguous bytes per load;
// its scale bytes as [chunk][512-column tile][column % 16][column / 16 % 32]
// so that each lane reads the 32 scales of its 32 column blocks as 8 dwords
// and selects the byte with the instruction's opsel.
//
// Tiling as in the BF16 kernel: 512 threads, 128 rows x 512 columns per
// workgroup, 16 rows x 512 columns (32 blocks) per wavefront, the chunk of
// quantised S*A and its scales copied into double-buffered LDS by buffer
// loads one chunk ahead while the next chunk of G is drawn in registers.
#include "internal.hpp"

namespace psk {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void *lds_ptr_t;

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kBM = 16 * kWaves;  // 128
constexpr int kBN = 512;
constexpr int kNB = kBN / 16;     // 32 blocks per wavefront
constexpr int kBK = 128;          // buckets per chunk = one scale block
constexpr int kPartBytes = kBN * 16;           // one (g, half) slab: 8 KiB
constexpr int kDataBytes = 8 * kPartBytes;     // 64 KiB per chunk tile
constexpr int kScaleBytes = kBN;               // 512 scale bytes per chunk tile
constexpr int kBufBytes = kDataBytes + kScaleBytes;

// exponent e of the block scale: smallest integer with 448 * 2^e >= amax
// (amax = f 2^x, f in [1/2, 1); 448 = 0.875 2^9), 0 for amax == 0 and for
// an infinite amax (the block then carries a NaN, see e4m3x2)
__device__ __forceinline__ int scale_exp_f32(float amax) {
  int x;
  const float f = frexpf(amax, &x);
  const int e = (f <= 0.875f) ? x - 9 : x - 8;
  return (amax > 0.0f && amax <= 3.4028234663852886e38f) ? e : 0;
}
__device__ __forceinline__ int scale_exp_f64(double amax) {
  int x;
  const double f = frexp(amax, &x);
  const int e = (f <= 0.875) ? x - 9 : x - 8;
  return (amax > 0.0 && amax <= 1.7976931348623157e308) ? e : 0;
}

// FP32 of a double by round-to-odd (then a later RNE to e4m3 is a single
// correct rounding)
__device__ __forceinline__ float f32_odd(double v) {
  float f = (float)v;
  if ((double)f != v && v == v) {
    uint32_t b = __float_as_uint(f);
    if (fabs((double)f) > fabs(v)) b -= 1;
    b |= 1u;
    f = __uint_as_float(b);
  }
  return f;
}

// two e4m3 bytes (RNE) packed in the low 16 bits; a NaN or an infinity
// becomes the e4m3 NaN, so a non-finite S*A entry reaches the product
__device__ __forceinline__ uint32_t e4m3x2(float a, float b) {
  a = fabsf(a) <= 3.4028234663852886e38f ? a : __builtin_nanf("");
  b = fabsf(b) <= 3.4028234663852886e38f ? b : __builtin_nanf("");
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xFFFFu;
}

// Quantise S*A (r x d, dtype T) per column in 128-bucket blocks.  One thread
// per (chunk, padded column).
template <typename T>
__global__ __launch_bounds__(256) void k_sa_fp8(const T *__restrict__ SA, int64_t r, int64_t d,
                                                int64_t npad, int64_t nkc,
                                                unsigned char *__restrict__ q,
                                                unsigned char *__restrict__ sc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nkc * npad) return;
  const int64_t n = t % npad;
  const int64_t kc = t / npad;
  const int64_t k0 = kc * kBK;
  double amax = 0.0;
  if (n < d)
    for (int i = 0; i < kBK; ++i)
      if (k0 + i < r) amax = fmax(amax, fabs((double)SA[(k0 + i) * d + n]));
  int e = scale_exp_f64(amax);
  e = e < -127 ? -127 : (e > 127 ? 127 : e);
  const double inv = ldexp(1.0, -e);
  for (int gh = 0; gh < 8; ++gh) {  // (g, half): buckets 16 gh .. 16 gh + 15
    uint32_t w[4];
    for (int p = 0; p < 4; ++p) {
      float f[4];
      for (int u = 0; u < 4; ++u) {
        const int64_t k = k0 + 16 * gh + 4 * p + u;
        const double v = (n < d && k < r) ? (double)SA[k * d + n] : 0.0;
        f[u] = f32_odd(v * inv);
      }
      w[p] = e4m3x2(f[0], f[1]) | (e4m3x2(f[2], f[3]) << 16);
    }
    reinterpret_cast<uint4 *>(q)[(kc * 8 + gh) * npad + n] = uint4{w[0], w[1], w[2], w[3]};
  }
  // scale byte at [kc][tile][n % 16][(n / 16) % 32]
  const int64_t tile = n / kBN, nn = n % kBN;
  sc[(kc * (npad / kBN) + tile) * kBN + (nn % 16) * kNB + nn / 16] = (unsigned char)(e + 127);
}

// S*A of CSR A straight into the quantised layout, without the r x d array.
// Workgroup (kc, y) owns the 128 buckets of chunk kc and the 64-column
// slices s = kSlices y .. kSlices y + kSlices - 1, taken one after another
// through one LDS tile of 128 x 64 accumulators (dtype of A).  Wavefront w
// (of 8) owns buckets 16 w .. 16 w + 15, one run of the bin list: the row
// pointers and first kBucketEnt entries of its first 64 rows are loaded
// once, one row per lane (a lane finds its row's bucket among the 17 bucket
// pointers, held one per lane), and kept in registers for all slices; later
// batches of a longer run are reloaded per slice.  Per slice the rows are
// applied bucket-parallel, each bucket's rows in list order (apply_batch),
// keeping the entries of the slice's columns, so every sum has the order of
// the CountSketch scatter.  Then thread (w, l)
// takes column 64 s + l, buckets 16 w .. 16 w + 15 (one e4m3 group): the
// column's amax over the chunk gives the scale exponent, and the values are
// rounded to e4m3 as k_sa_fp8 does.
constexpr int kSlices = 8;

template <typename T>
struct RowBatch {
  int64_t p0, p1;
  int ng, lb;
  int rank;   // position of the row among its bucket's rows in the batch, -1 past the run
  int nrank;  // 1 + the largest rank in the batch
  uint64_t longmask;
  int ci[kBucketEnt];
  double xv[kBucketEnt];  // FP64: every S*A sum is formed in FP64
};

template <typename T>
__device__ __forceinline__ void load_batch(RowBatch<T> &B, uint32_t base, uint32_t j1,
                                           uint32_t bpl, const T *__restrict__ vals,
                                           const int64_t *__restrict__ indptr,
                                           const int32_t *__restrict__ indices,
                                           const uint32_t *__restrict__ perm) {
  const int lane = (int)(threadIdx.x & 63u);
  const uint32_t j = base + (uint32_t)lane;
  B.p0 = 0;
  B.p1 = 0;
  B.ng = 0;
  if (j < j1) {
    const uint32_t pv = perm[j];
    const int64_t row = (int64_t)(pv & 0x7fffffffu);
    B.ng = (int)(pv >> 31);
    B.p0 = indptr[row];
    B.p1 = indptr[row + 1];
  }
  // bucket of list entry j: the last b in 0..15 with bp[b] <= j
  B.lb = 0;
#pragma unroll
  for (int step = 8; step >= 1; step >>= 1) {
    const uint32_t v = (uint32_t)__shfl((int)bpl, B.lb + step, 64);
    if (v <= j) B.lb += step;
  }
  const int64_t len = B.p1 - B.p0;
  const bool lng = len > kBucketEnt;
#pragma unroll
  for (int e = 0; e < kBucketEnt; ++e) {
    B.ci[e] = -1;
    B.xv[e] = 0.0;
    if (!lng && e < len) {
      B.ci[e] = indices[B.p0 + e];
      const double v = (double)vals[B.p0 + e];
      B.xv[e] = B.ng ? -v : v;
    }
  }
  B.longmask = __ballot(lng);
  // rank counted from the bucket's first row in this batch
  uint32_t start = (uint32_t)__shfl((int)bpl, B.lb, 64);
  if (start < base) start = base;
  B.rank = j < j1 ? (int)(j - start) : -1;
  int mr = B.rank;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mr = max(mr, __shfl_xor(mr, off, 64));
  B.nrank = mr + 1;
}

// Round t applies the t-th row (in list order) of every bucket of the
// batch: rows of different buckets write different LDS rows, and a bucket's
// rows keep their order, so each sum is formed in list order.
template <typename T>
__device__ __forceinline__ void apply_batch(const RowBatch<T> &B, int64_t c0,
                                            const T *__restrict__ vals,
                                            const int32_t *__restrict__ indices, double *myacc) {
  const int lane = (int)(threadIdx.x & 63u);
  const int64_t len = B.p1 - B.p0;
  const bool lng = (B.longmask >> lane) & 1u;
  for (int t = 0; t < B.nrank; ++t) {
    if (B.rank == t && !lng) {
#pragma unroll
      for (int e = 0; e < kBucketEnt; ++e) {
        const int64_t cl = (int64_t)B.ci[e] - c0;
        if (e < len && cl >= 0 && cl < 64) atomicAdd(&myacc[B.lb * 64 + cl], B.xv[e]);
      }
    }
    uint64_t lm = __ballot(B.rank == t && lng);
    while (lm) {
      const int i = __ffsll((unsigned long long)lm) - 1;
      lm &= lm - 1;
      const int64_t q0 = __shfl(B.p0, i, 64);
      const int64_t q1 = __shfl(B.p1, i, 64);
      const int ngi = __shfl(B.ng, i, 64);
      const int lbi = __shfl(B.lb, i, 64);
      for (int64_t p = q0 + lane; p < q1; p += 64) {
        const int64_t cl = (int64_t)indices[p] - c0;
        if (cl >= 0 && cl < 64) {
          const double v = (double)vals[p];
          atomicAdd(&myacc[lbi * 64 + cl], ngi ? -v : v);
        }
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(512) void k_scatter_csr_fp8(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, int64_t npad, int64_t r,
    const uint32_t *__restrict__ perm, const uint32_t *__restrict__ bptr,
    unsigned char *__restrict__ q, unsigned char *__restrict__ sc) {
  __shared__ __align__(16) double acc[kBK * 64];  // FP64 bucket sums
  __shared__ double amax_s[2][8][64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t kc = blockIdx.x;
  const int64_t k0 = kc * kBK;
  const int b0 = 16 * wave;  // first bucket of this wavefront (in the chunk)
  // bucket pointers b0 .. b0 + 16, one per lane
  const int64_t kb = k0 + b0 + (lane <= 16 ? lane : 16);
  const uint32_t bpl = bptr[kb < r ? kb : r];
  const uint32_t j0 = (uint32_t)__shfl((int)bpl, 0, 64);
  const uint32_t j1 = (uint32_t)__shfl((int)bpl, 16, 64);
  RowBatch<T> first;
  load_batch(first, j0, j1, bpl, vals, indptr, indices, perm);
  double *myacc = acc + b0 * 64;
  const int nsl = (int)(npad / 64);
  const int s0 = (int)blockIdx.y * kSlices;
  const int s1 = (s0 + kSlices) < nsl ? (s0 + kSlices) : nsl;
  for (int sl = s0; sl < s1; ++sl) {
    const int64_t c0 = (int64_t)sl * 64;
    for (int i = lane; i < 16 * 64; i += 64) myacc[i] = 0.0;
    if (j0 < j1) apply_batch(first, c0, vals, indices, myacc);
    for (uint32_t base = j0 + 64; base < j1; base += 64) {
      RowBatch<T> more;
      load_batch(more, base, j1, bpl, vals, indptr, indices, perm);
      apply_batch(more, c0, vals, indices, myacc);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    double am = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) am = fmax(am, fabs(myacc[i * 64 + lane]));
    double(*ams)[64] = amax_s[sl & 1];
    ams[wave][lane] = am;
    __syncthreads();
    double amax = ams[0][lane];
#pragma unroll
    for (int w = 1; w < 8; ++w) amax = fmax(amax, ams[w][lane]);
    int e = scale_exp_f64(amax);
    e = e < -127 ? -127 : (e > 127 ? 127 : e);
    const double inv = ldexp(1.0, -e);
    const int64_t n = c0 + lane;
    // this wavefront's 16 buckets are e4m3 group gh = wave
    uint32_t w4[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      float f[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) f[u] = f32_odd(myacc[(4 * p + u) * 64 + lane] * inv);
      w4[p] = e4m3x2(f[0], f[1]) | (e4m3x2(f[2], f[3]) << 16);
    }
    reinterpret_cast<uint4 *>(q)[(kc * 8 + wave) * npad + n] =
        uint4{w4[0], w4[1], w4[2], w4[3]};
    if (wave == 0) {
      const int64_t tile = n / kBN, nn = n % kBN;
      sc[(kc * (npad / kBN) + tile) * kBN + (nn % 16) * kNB + nn / 16] =
          (unsigned char)(e + 127);
    }
  }
}

// G's FP8 operand, drawn once: thread (chunk c, row a, lane group g) writes
// the e4m3 bytes (G's fixed scale, each the rounding of the FP64 normal) of
// buckets 128 c + 32 g .. + 31 of row a, 32 contiguous bytes at
// gq[((c m_pad + a) 4 + g) 32], the A fragment of MFMA lane (a % 16, g);
// rows past m and buckets past r are zero.
__global__ __launch_bounds__(256) void k_draw_g_e4m3(int64_t m, int64_t m_pad, int64_t r,
                                                     int64_t kchunks, uint64_t seed,
                                                     unsigned char *__restrict__ gq) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= kchunks * m_pad * 4) return;
  const int g = (int)(t & 3);
  const int64_t a = (t >> 2) % m_pad;
  const int64_t c = (t >> 2) / m_pad;
  uint32_t w[8];
  const uint64_t qb = (uint64_t)c * 32u + 8u * (uint64_t)g;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    uint32_t by = a < m ? gauss4_e4m3(qb + u, (uint32_t)a, seed) : 0u;
    const int64_t valid = r - (int64_t)(4 * (qb + u));
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k >= valid) by &= ~(0xFFu << (8 * k));
    w[u] = by;
  }
  uint4 *o = reinterpret_cast<uint4 *>(gq + t * 32);
  o[0] = uint4{w[0], w[1], w[2], w[3]};
  o[1] = uint4{w[4], w[5], w[6], w[7]};
}

template <bool TAIL>
__global__ __launch_bounds__(kThreads) void k_gauss_gemm_fp8(
    int64_t m, int64_t d, int64_t r, int64_t npad, const unsigned char *__restrict__ gq,
    int64_t m_pad, int64_t kchunks,
    const unsigned char *__restrict__ q, const unsigned char *__restrict__ sc, int tiles_m,
    int tiles_n, int64_t c0, int64_t kend, int64_t cper, int ks0,
    float *__restrict__ out /* [splits][m][d] */) {
  // the two chunk buffers as separate objects: the compiler can then tell a
  // copy into one from the reads of the other and need not wait for the
  // copy before reading
  __shared__ __align__(16) unsigned char smem0[kBufBytes];
  __shared__ __align__(16) unsigned char smem1[kBufBytes];

  const int64_t nblk = (int64_t)gridDim.x;
  int64_t lin = blockIdx.x;
  if ((nblk & 7) == 0) lin = (lin & 7) * (nblk >> 3) + (lin >> 3);
  const int mt = (int)(lin % tiles_m);
  const int64_t rest = lin / tiles_m;
  const int nt = (int)(rest % tiles_n);
  const int ks = (int)(rest / tiles_n);
  const int64_t m0 = (int64_t)mt * kBM;
  const int64_t n0 = (int64_t)nt * kBN;
  const int64_t cb = c0 + (int64_t)ks * cper;
  int64_t ce = cb + cper;
  if (ce > kend) ce = kend;
  const int64_t nch = ce > cb ? ce - cb : 0;

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int g = lane >> 4;
  const int li = lane & 15;

  v4f acc[kNB];
#pragma unroll
  for (int b = 0; b < kNB; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};

  // descriptors over this split's chunks: data and scales
  const int64_t chunk_data = 8 * npad * 16;  // bytes per chunk (all columns)
  const int64_t chunk_sc = npad;             // scale bytes per chunk
  const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(q + cb * chunk_data), (short)0, (int)(nch * chunk_data), 0x00020000);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(sc + cb * chunk_sc), (short)0, (int)(nch * chunk_sc), 0x00020000);
  auto copy_chunk = [&](int64_t crel, unsigned char *base) __attribute__((always_inline)) {
    // 64 KiB of data: 64 pieces of 1 KiB, wave w takes pieces w, w+8, ...
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int piece = wave + kWaves * p;  // 0..63
      const int gh = piece >> 3;            // (g, half) slab
      const int off = (piece & 7) * 1024;
      const int gsrc = (int)(crel * chunk_data + ((int64_t)gh * npad + n0) * 16) + off +
                       lane * 16;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rq, (lds_ptr_t)(base + gh * kPartBytes + off),
                                               16, gsrc, 0, 0, 0);
    }
    // 512 scale bytes: wave 0, two loads of 64 lanes x 4 bytes
    if (wave == 0) {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int gsrc = (int)(crel * chunk_sc + (int64_t)nt * kBN) + p * 256 + lane * 4;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (lds_ptr_t)(base + kDataBytes + p * 256), 4, gsrc, 0, 0, 0);
      }
    }
  };

  const uint32_t row_a = (uint32_t)(m0 + wave * 16 + li);
  // this lane's A fragment of chunk c: the 32 e4m3 bytes of G (buckets
  // 128 c + 32 g + j of its row) drawn by k_draw_g_e4m3, and the E8M0 byte
  // of G's fixed scale (chunks past the last read the last, unused)
  (void)r;
  auto make_a = [&](int64_t c_abs, int &sbyte) {
    const int64_t cc = c_abs < kchunks ? c_abs : kchunks - 1;
    const uint4 *p = reinterpret_cast<const uint4 *>(gq + ((cc * m_pad + row_a) * 4 + g) * 32);
    const uint4 x0 = p[0], x1 = p[1];
    const v8i a = {(int)x0.x, (int)x0.y, (int)x0.z, (int)x0.w,
                   (int)x1.x, (int)x1.y, (int)x1.z, (int)x1.w};
    sbyte = 127 + kGFp8Exp;
    return a;
  };

  // G's fragments are read once (L2 misses): they are fetched two chunks
  // ahead, S*A's (shared by the row tiles of the split, on one XCD) one
  // chunk ahead into the other LDS buffer
  v8i a_cur, a_n1;
  int sa_cur = 127, sa_n1 = 127;
  if (nch > 0) {
    copy_chunk(0, smem0);
    a_cur = make_a(cb, sa_cur);
    a_n1 = make_a(cb + 1, sa_n1);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  // chunk c from cur while chunk c + 1 is copied into nxt
  auto chunk = [&](int64_t c, const unsigned char *bb, unsigned char *nxt)
                   __attribute__((always_inline)) {
    copy_chunk(c + 1, nxt);  // past the split: range check reads zeros
    // the two fragment loads of chunk c + 2 are issued after the copies,
    // so that the wait below can leave them in flight
    __builtin_amdgcn_sched_barrier(0);
    int sa_n2;
    const v8i a_n2 = make_a(cb + c + 2, sa_n2);
    __builtin_amdgcn_sched_barrier(0);
    const unsigned char *lo = bb + (2 * g) * kPartBytes + li * 16;      // bytes 0..15
    const unsigned char *hi = bb + (2 * g + 1) * kPartBytes + li * 16;  // bytes 16..31
    const uint4 *scp = reinterpret_cast<const uint4 *>(bb + kDataBytes + li * kNB);
    const uint4 s03 = scp[0], s47 = scp[1];
    const uint32_t sw[8] = {s03.x, s03.y, s03.z, s03.w, s47.x, s47.y, s47.z, s47.w};
#pragma unroll
    for (int nb = 0; nb < kNB; ++nb) {
      const uint4 b0 = *reinterpret_cast<const uint4 *>(lo + nb * 256);
      const uint4 b1 = *reinterpret_cast<const uint4 *>(hi + nb * 256);
      const v8i bf = {(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w,
                      (int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
      const int sbw = (int)sw[nb >> 2];
      switch (nb & 3) {
        case 0:
          acc[nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a_cur, bf, acc[nb], 0, 0,
                                                                     0, sa_cur, 0, sbw);
          break;
        case 1:
          acc[nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a_cur, bf, acc[nb], 0, 0,
                                                                     0, sa_cur, 1, sbw);
          break;
        case 2:
          acc[nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a_cur, bf, acc[nb], 0, 0,
                                                                     0, sa_cur, 2, sbw);
          break;
        default:
          acc[nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a_cur, bf, acc[nb], 0, 0,
                                                                     0, sa_cur, 3, sbw);
          break;
      }
    }
    // this wave's copies of chunk c + 1 have landed: vmcnt(2) (expcnt and
    // lgkmcnt not waited for), only chunk c + 2's two fragment loads remain
    __builtin_amdgcn_s_waitcnt(0x0F72);
    __syncthreads();
    a_cur = a_n1;
    sa_cur = sa_n1;
    a_n1 = a_n2;
    sa_n1 = sa_n2;
  };
  for (int64_t c = 0; c < nch; c += 2) {
    chunk(c, smem0, smem1);
    if (c + 1 < nch) chunk(c + 1, smem1, smem0);
  }

  // accumulator element e of block nb: row 4 g + e, column li
  float *o = out + (int64_t)(ks0 + ks) * m * d;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t row = m0 + wave * 16 + 4 * g + e;
    if (row >= m) continue;
#pragma unroll
    for (int nb = 0; nb < kNB; ++nb) {
      const int64_t col = n0 + nb * 16 + li;
      if (col < d) o[row * d + col] = acc[nb][e];
    }
  }
}

// C[i] = scale * sum_s part[s][i] (FP32 partials summed in FP64, fixed order)
__global__ __launch_bounds__(256) void k_reduce_fp8(const float *__restrict__ part, int64_t len,
                                                    int splits, double scale,
                                                    double *__restrict__ C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double acc = (double)part[i];
  for (int s = 1; s < splits; ++s) acc += (double)part[(int64_t)s * len + i];
  C[i] = acc * scale;
}

}  // namespace

namespace {

// Tiling, K split and workspace of one FP8 product (bytes, scales, partials).
// K is cut into kfull whole 128-bucket chunks, split splits_main ways, and,
// when 128 does not divide r, the tail chunk as one more split of its own
// (the one launch that masks G past bucket r).
struct Fp8Plan {
  int tiles_m, tiles_n;
  int64_t r, npad, kchunks, kfull, tiles, splits, splits_main, cper, m_pad;
  unsigned char *q, *sc, *gq;
  float *part;
};

int fp8_plan(int64_t m, int64_t r, int64_t d, Arena &ws, Fp8Plan &P) {
  P.r = r;
  P.tiles_m = (int)ceil_div(m, kBM);
  P.tiles_n = (int)ceil_div(d, kBN);
  P.npad = (int64_t)P.tiles_n * kBN;
  P.kchunks = ceil_div(r, kBK);
  P.kfull = r / kBK;
  P.tiles = (int64_t)P.tiles_m * P.tiles_n;
  int64_t splits = ceil_div(512, P.tiles);
  const int64_t max_splits = P.kfull / 8 > 0 ? P.kfull / 8 : 1;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  P.cper = P.kfull > 0 ? ceil_div(P.kfull, splits) : 1;
  P.splits_main = P.kfull > 0 ? ceil_div(P.kfull, P.cper) : 0;
  P.splits = P.splits_main + (P.kfull < P.kchunks ? 1 : 0);
  if ((P.cper + 1) * 8 * P.npad * 16 + 65536 >= ((int64_t)1 << 31))
    return fail(PSK_EUNSUPPORTED, "FP8 Gaussian GEMM: K slice too large for one descriptor");
  P.q = ws.take<unsigned char>((size_t)(P.kchunks * 8 * P.npad * 16));
  P.sc = ws.take<unsigned char>((size_t)(P.kchunks * P.npad));
  P.part = ws.take<float>((size_t)P.splits * m * d);
  P.m_pad = (int64_t)P.tiles_m * kBM;
  P.gq = ws.take<unsigned char>((size_t)(P.kchunks * P.m_pad * kBK));
  if (!ws.dry() && !ws.ok())
    return fail(PSK_ENOMEM, "workspace too small for the FP8 Gaussian GEMM");
  return 0;
}

int fp8_run(const Fp8Plan &P, int64_t m, int64_t d, uint64_t seed, double *C,
            hipStream_t st) {
  {
    KTimer t("g_draw", st);
    const int64_t thr = P.kchunks * P.m_pad * 4;
    k_draw_g_e4m3<<<(unsigned)ceil_div(thr, (int64_t)256), 256, 0, st>>>(m, P.m_pad, P.r,
                                                                        P.kchunks, seed, P.gq);
  }
  {
    KTimer t("gauss_gemm", st);
    if (P.splits_main > 0)
      k_gauss_gemm_fp8<false><<<(unsigned)(P.tiles * P.splits_main), kThreads, 0, st>>>(
          m, d, P.r, P.npad, P.gq, P.m_pad, P.kchunks, P.q, P.sc, P.tiles_m, P.tiles_n, 0,
          P.kfull, P.cper, 0, P.part);
    if (P.kfull < P.kchunks)
      k_gauss_gemm_fp8<true><<<(unsigned)P.tiles, kThreads, 0, st>>>(
          m, d, P.r, P.npad, P.gq, P.m_pad, P.kchunks, P.q, P.sc, P.tiles_m, P.tiles_n, P.kfull,
          P.kchunks, 1, (int)P.splits_main, P.part);
  }
  {
    KTimer t("gemm_reduce", st);
    const int64_t len = m * d;
    k_reduce_fp8<<<(unsigned)ceil_div(len, 256), 256, 0, st>>>(P.part, len, (int)P.splits,
                                                                 1.0 / sqrt((double)m), C);
  }
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace

int gauss_gemm_fp8(int64_t m, int64_t r, int64_t d, uint64_t seed, const void *SA,
                   int sa_dtype, double *C, Arena &ws, hipStream_t st) {
  Fp8Plan P;
  int rc = fp8_plan(m, r, d, ws, P);
  if (rc || ws.dry()) return rc;
  {
    KTimer t("sa_quant", st);
    const int64_t threads = P.kchunks * P.npad;
    if (sa_dtype == PSK_F64)
      k_sa_fp8<double><<<(unsigned)ceil_div(threads, 256), 256, 0, st>>>(
          (const double *)SA, r, d, P.npad, P.kchunks, P.q, P.sc);
    else
      k_sa_fp8<float><<<(unsigned)ceil_div(threads, 256), 256, 0, st>>>(
          (const float *)SA, r, d, P.npad, P.kchunks, P.q, P.sc);
  }
  return fp8_run(P, m, d, seed, C, st);
}

bool fp8_csr_fusable(const psk_mat &A, int64_t r) {
  return A.format == PSK_CSR && cs_splits(A.n, r) == 1;
}

int gauss_gemm_fp8_csr(int64_t m, int64_t r, const psk_mat &A, const uint32_t *perm,
                       const uint32_t *bptr, uint64_t seed, double *C, Arena &ws,
                       hipStream_t st) {
  if (!fp8_csr_fusable(A, r))
    return fail(PSK_EUNSUPPORTED, "fused CSR quantisation needs one split per bucket");
  Fp8Plan P;
  int rc = fp8_plan(m, r, A.d, ws, P);
  if (rc || ws.dry()) return rc;
  {
    KTimer t("cs_scatter_quant", st);
    const dim3 grid((unsigned)P.kchunks, (unsigned)ceil_div(P.npad / 64, kSlices));
    if (A.dtype == PSK_F64)
      k_scatter_csr_fp8<double><<<grid, 512, 0, st>>>(
          (const double *)A.values, A.indptr, A.indices, P.npad, r, perm, bptr, P.q, P.sc);
    else
      k_scatter_csr_fp8<float><<<grid, 512, 0, st>>>(
          (const float *)A.values, A.indptr, A.indices, P.npad, r, perm, bptr, P.q, P.sc);
  }
  return fp8_run(P, m, A.d, seed, C, st);
}

}  // namespace psk
