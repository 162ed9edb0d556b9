// C = G * (S*A) with BF16 operands on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), G generated in registers.
//
// Paper mapping (arXiv 2203.02798): Algorithm countgauss_multiply's batched
// C += G_i * B, as in the FP64 kernel, with the Gaussian rounded to bfloat16
// and S*A carried as two bfloat16 limbs (hi = bf16(SA), lo = bf16(SA - hi),
// about 16 significant bits together), so C = G_bf16 * (hi + lo) costs two
// matrix instructions per block.  K-split partial products are stored in
// FP32 and summed in FP64 by a second kernel, which applies 1/sqrt(m).
//
// Layout of the limbs (written by k_sa_limbs from a materialised S*A, or for
// CSR A by k_scatter_csr_limbs straight from the binned rows): for 32-bucket
// chunk kc and
// k-quad q (buckets 32kc + 8q .. +7) the 8 values of column n are 16
// contiguous bytes at Lq[kc][q][n][0..7]; a B fragment of the 16x16x32
// instruction (lane l: column l%16, buckets 8(l/16)..+7) is then one 16-byte
// load, and the 16 columns of one quad are 256 contiguous bytes (no LDS bank
// conflicts).  Columns are padded to a multiple of 512 with zeros.
//
// Tiling: 512 threads = 8 wavefronts; workgroup tile 128 rows x 512 columns,
// so every Gaussian value is drawn once per 512 columns.  A chunk is 32
// buckets: the workgroup draws the chunk's 128 x 32 block of G (FP32
// Box-Muller, rounded to bfloat16) into LDS once, and the limb chunk of S*A
// (2 x 32 KiB) is copied into double-buffered LDS by buffer loads one chunk
// ahead.  Each wavefront owns 64 rows x 128 columns (4 x 8 blocks of 16 x
// 16, 128 FP32 accumulators per lane): it reads 4 A fragments and 16 B
// fragments per chunk and issues 64 matrix instructions, so every B
// fragment read from LDS feeds four of them (LDS bandwidth, not the matrix
// cores, bounded the one-row-block layout).
#include "internal.hpp"

namespace psk {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void *lds_ptr_t;

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kBM = 16 * kWaves;  // 128
constexpr int kBN = 512;
constexpr int kBK = 32;
constexpr int kQuadBytes = kBN * 8 * 2;         // 8 KiB: one quad of one chunk-tile
constexpr int kLimbBytes = 4 * kQuadBytes;      // 32 KiB per limb per chunk
constexpr int kChunkBytes = 2 * kLimbBytes;     // 64 KiB (hi + lo)
constexpr int kRB = 4;          // 16-row blocks per wavefront (64 rows)
constexpr int kCB = 8;          // 16-column blocks per wavefront (128 columns)
constexpr int kWR = kBM / 16 / kRB;   // wavefront rows of the tile
constexpr int kWC = kWaves / kWR;     // wavefront columns of the tile
static_assert(kWC * kCB * 16 == kBN, "wavefront tiles cover the block");
constexpr int kGRow = 80;       // LDS row stride of the Gaussian tile (64 B + pad)
constexpr int kGBytes = kBM * kGRow;  // 10 KiB per Gaussian tile

__device__ __forceinline__ uint16_t bf16_bits(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);  // v_cvt_pk_bf16_f32, RNE
}

// bfloat16 (RNE) of a double in one rounding: the double is narrowed to
// FP32 by round-to-odd (truncate toward zero, then set the last bit if the
// value was inexact), which keeps 16 spare bits and therefore cannot make a
// false tie for the second, round-to-nearest-even step.
__device__ __forceinline__ uint16_t bf16_of_f64(double v) {
  if (v != v) return 0x7FC0;
  float f = (float)v;
  if ((double)f != v) {
    uint32_t b = __float_as_uint(f);
    if (fabs((double)f) > fabs(v)) b -= 1;  // step back toward zero
    b |= 1u;
    f = __uint_as_float(b);
  }
  return bf16_bits(f);
}

__device__ __forceinline__ double bf16_to_f64(uint16_t h) {
  return (double)__uint_as_float((uint32_t)h << 16);
}

// SA (r x d, row-major, dtype T) -> two bf16 limb arrays in the chunked
// layout [kc][q][npad][8]; entries outside r x d are zero.
template <typename T>
__global__ __launch_bounds__(256) void k_sa_limbs(const T *__restrict__ SA, int64_t r,
                                                  int64_t d, int64_t npad, int64_t nkc,
                                                  uint16_t *__restrict__ hi,
                                                  uint16_t *__restrict__ lo) {
  // one thread per (kc, q, n): 8 consecutive buckets of one column
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = nkc * 4 * npad;
  if (t >= total) return;
  const int64_t n = t % npad;
  const int64_t q = (t / npad) % 4;
  const int64_t kc = t / (4 * npad);
  uint16_t h8[8], l8[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t k = kc * kBK + q * 8 + e;
    double v = 0.0;
    if (k < r && n < d) v = (double)SA[k * d + n];
    const uint16_t h = bf16_of_f64(v);
    const uint16_t l = bf16_of_f64(v - bf16_to_f64(h));  // exact difference
    h8[e] = h;
    l8[e] = l;
  }
  uint4 ph, pl;
  ph.x = h8[0] | ((uint32_t)h8[1] << 16);
  ph.y = h8[2] | ((uint32_t)h8[3] << 16);
  ph.z = h8[4] | ((uint32_t)h8[5] << 16);
  ph.w = h8[6] | ((uint32_t)h8[7] << 16);
  pl.x = l8[0] | ((uint32_t)l8[1] << 16);
  pl.y = l8[2] | ((uint32_t)l8[3] << 16);
  pl.z = l8[4] | ((uint32_t)l8[5] << 16);
  pl.w = l8[6] | ((uint32_t)l8[7] << 16);
  reinterpret_cast<uint4 *>(hi)[t] = ph;
  reinterpret_cast<uint4 *>(lo)[t] = pl;
}

// S*A of CSR A straight into the limb layout, without the r x d array: a
// workgroup of 8 wavefronts owns the quad of buckets 8 * blockIdx.x + e
// (e = 0..7); wavefront e sums its bucket's rows into an LDS row of npad
// accumulators exactly as the CountSketch scatter does (rows one after
// another in bin order, a row's entries spread over the lanes), then every
// thread turns the 8 sums of one column into its hi and lo limbs (the same
// values k_sa_limbs makes from the materialised S*A).
template <typename T>
__global__ __launch_bounds__(512) void k_scatter_csr_limbs(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, int64_t npad, int64_t r,
    const uint32_t *__restrict__ perm, const uint32_t *__restrict__ bptr,
    uint16_t *__restrict__ hi, uint16_t *__restrict__ lo) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *accs = reinterpret_cast<double *>(smem_raw);  // 8 x npad FP64 sums
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t quad = blockIdx.x;
  const int64_t b = quad * 8 + wave;
  double *acc = accs + (int64_t)wave * npad;
  for (int64_t c = lane; c < npad; c += 64) acc[c] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (b < r) bucket_rows_add(vals, indptr, indices, perm, bptr[b], bptr[b + 1], acc);
  __syncthreads();
  for (int64_t n = threadIdx.x; n < npad; n += 512) {
    uint16_t h8[8], l8[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const double v = accs[(int64_t)e * npad + n];
      const uint16_t h = bf16_of_f64(v);
      h8[e] = h;
      l8[e] = bf16_of_f64(v - bf16_to_f64(h));  // exact difference
    }
    uint4 ph, pl;
    ph.x = h8[0] | ((uint32_t)h8[1] << 16);
    ph.y = h8[2] | ((uint32_t)h8[3] << 16);
    ph.z = h8[4] | ((uint32_t)h8[5] << 16);
    ph.w = h8[6] | ((uint32_t)h8[7] << 16);
    pl.x = l8[0] | ((uint32_t)l8[1] << 16);
    pl.y = l8[2] | ((uint32_t)l8[3] << 16);
    pl.z = l8[4] | ((uint32_t)l8[5] << 16);
    pl.w = l8[6] | ((uint32_t)l8[7] << 16);
    reinterpret_cast<uint4 *>(hi)[quad * npad + n] = ph;
    reinterpret_cast<uint4 *>(lo)[quad * npad + n] = pl;
  }
}

__global__ __launch_bounds__(kThreads) void k_gauss_gemm_bf16(
    int64_t m, int64_t d, int64_t npad, uint64_t seed, const uint16_t *__restrict__ hi,
    const uint16_t *__restrict__ lo, int tiles_m, int tiles_n, int64_t kchunks,
    int64_t cper, float *__restrict__ out /* [splits][m][d] */) {
  __shared__ __align__(16) unsigned char smem[2 * kChunkBytes + 2 * kGBytes];

  const int64_t nblk = (int64_t)gridDim.x;
  int64_t lin = blockIdx.x;
  if ((nblk & 7) == 0) lin = (lin & 7) * (nblk >> 3) + (lin >> 3);
  const int mt = (int)(lin % tiles_m);
  const int64_t rest = lin / tiles_m;
  const int nt = (int)(rest % tiles_n);
  const int ks = (int)(rest / tiles_n);
  const int64_t m0 = (int64_t)mt * kBM;
  const int64_t n0 = (int64_t)nt * kBN;
  const int64_t cb = (int64_t)ks * cper;
  int64_t ce = cb + cper;
  if (ce > kchunks) ce = kchunks;
  const int64_t nch = ce > cb ? ce - cb : 0;

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int q = lane >> 4;
  const int li = lane & 15;
  const int wr = wave / kWC;  // rows 16 kRB wr .. of the tile
  const int wc = wave % kWC;  // columns 16 kCB wc .. of the tile

  v4f acc[kRB][kCB];
#pragma unroll
  for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
    for (int cb2 = 0; cb2 < kCB; ++cb2) acc[rb][cb2] = v4f{0.f, 0.f, 0.f, 0.f};

  // buffer descriptors over this split's chunks of each limb
  const int64_t chunk_stride = 4 * npad * 8;  // bf16 elements per chunk
  const int nbytes = (int)(nch * chunk_stride * 2);
  const __amdgpu_buffer_rsrc_t rh = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(hi + cb * chunk_stride), (short)0, nbytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rl = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(lo + cb * chunk_stride), (short)0, nbytes, 0x00020000);
  // a chunk tile is 4 quads x 8 KiB per limb; wave w copies 1 KiB pieces
  // w, w+8, ... (8 per limb per chunk: 64 KiB / 8 waves / 1 KiB)
  auto copy_chunk = [&](int64_t crel, int buf) {
    unsigned char *base = smem + buf * kChunkBytes;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int piece = wave + kWaves * p;      // 0..31 within one limb
      const int quad = piece >> 3;              // 8 pieces of 1 KiB per quad
      const int off_in_quad = (piece & 7) * 1024;
      const int gsrc = (int)((crel * chunk_stride + (int64_t)quad * npad * 8 + n0 * 8) * 2) +
                       off_in_quad + lane * 16;
      const int ldst = quad * kQuadBytes + off_in_quad;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rh, (lds_ptr_t)(base + ldst), 16, gsrc, 0, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rl, (lds_ptr_t)(base + kLimbBytes + ldst), 16,
                                               gsrc, 0, 0, 0);
    }
  };

  // The Gaussian block of a chunk (128 rows x 32 buckets) is drawn once per
  // workgroup: thread t takes row t / 4 and buckets 8 (t % 4) .. +7 (two
  // Philox blocks), rounds them to bfloat16 and stores 16 bytes in the LDS
  // G tile (row stride kGRow bytes, padded against bank conflicts), from
  // which the wavefronts read their A fragments.
  const int grow = tid >> 2, goct = tid & 3;
  const uint32_t row_g = (uint32_t)(m0 + grow);
  auto gen_g = [&](int64_t c_abs, int gbuf) {
    float z[8];  // bfloat16 values (each the rounding of the FP64 normal)
    const uint64_t qb = (uint64_t)c_abs * 8u + 2u * (uint64_t)goct;
    gauss4_bf16(qb, row_g, seed, z);
    gauss4_bf16(qb + 1, row_g, seed, z + 4);
    v8bf a;
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = (__bf16)z[e];
    *reinterpret_cast<v8bf *>(smem + 2 * kChunkBytes + gbuf * kGBytes + grow * kGRow +
                              goct * 16) = a;
  };

  if (nch > 0) {
    copy_chunk(0, 0);
    gen_g(cb, 0);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  for (int64_t c = 0; c < nch; ++c) {
    const int buf = (int)(c & 1);
    copy_chunk(c + 1, buf ^ 1);  // past the split: range check reads zeros
    gen_g(cb + c + 1, buf ^ 1);  // past the split: an unused tile
    // A fragments: lane (row li of row block rb, quad q) = 8 bf16 of G
    const unsigned char *gt = smem + 2 * kChunkBytes + buf * kGBytes;
    v8bf af[kRB];
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb)
      af[rb] = *reinterpret_cast<const v8bf *>(gt + ((wr * kRB + rb) * 16 + li) * kGRow + q * 16);
    const unsigned char *bh = smem + buf * kChunkBytes + q * kQuadBytes + li * 16 +
                              wc * kCB * 256;
    const unsigned char *bl = bh + kLimbBytes;
#pragma unroll
    for (int cb2 = 0; cb2 < kCB; ++cb2) {
      const v8bf h = *reinterpret_cast<const v8bf *>(bh + cb2 * 256);
      const v8bf l = *reinterpret_cast<const v8bf *>(bl + cb2 * 256);
#pragma unroll
      for (int rb = 0; rb < kRB; ++rb) {
        acc[rb][cb2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[rb], h, acc[rb][cb2], 0, 0, 0);
        acc[rb][cb2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[rb], l, acc[rb][cb2], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  // accumulator element e of block (rb, cb2): row 4 q + e, column li
  float *o = out + (int64_t)ks * m * d;
#pragma unroll
  for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = m0 + (wr * kRB + rb) * 16 + 4 * q + e;
      if (row >= m) continue;
#pragma unroll
      for (int cb2 = 0; cb2 < kCB; ++cb2) {
        const int64_t col = n0 + (wc * kCB + cb2) * 16 + li;
        if (col < d) o[row * d + col] = acc[rb][cb2][e];
      }
    }
}

// C[i] = scale * sum_s part[s][i] (FP32 partials summed in FP64, fixed order)
__global__ __launch_bounds__(256) void k_reduce_splits_f32(const float *__restrict__ part,
                                                           int64_t len, int splits,
                                                           double scale,
                                                           double *__restrict__ C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double acc = (double)part[i];
  for (int s = 1; s < splits; ++s) acc += (double)part[(int64_t)s * len + i];
  C[i] = acc * scale;
}

}  // namespace

namespace {

// Tiling, K split and workspace of one BF16 product (limbs, FP32 partials).
struct Bf16Plan {
  int tiles_m, tiles_n;
  int64_t npad, kchunks, tiles, splits, cper;
  uint16_t *hi, *lo;
  float *part;
};

int bf16_plan(int64_t m, int64_t r, int64_t d, Arena &ws, Bf16Plan &P) {
  P.tiles_m = (int)ceil_div(m, kBM);
  P.tiles_n = (int)ceil_div(d, kBN);
  P.npad = (int64_t)P.tiles_n * kBN;
  P.kchunks = ceil_div(r, kBK);
  P.tiles = (int64_t)P.tiles_m * P.tiles_n;
  int64_t splits = ceil_div(512, P.tiles);
  const int64_t max_splits = P.kchunks / 32 > 0 ? P.kchunks / 32 : 1;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  P.cper = ceil_div(P.kchunks, splits);
  P.splits = ceil_div(P.kchunks, P.cper);
  const int64_t limb_elems = P.kchunks * 4 * P.npad * 8;
  if ((P.cper + 1) * 4 * P.npad * 8 * 2 + 65536 >= ((int64_t)1 << 31))
    return fail(PSK_EUNSUPPORTED, "BF16 Gaussian GEMM: K slice too large for one descriptor");
  P.hi = ws.take<uint16_t>((size_t)limb_elems);
  P.lo = ws.take<uint16_t>((size_t)limb_elems);
  P.part = ws.take<float>((size_t)P.splits * m * d);
  if (!ws.dry() && !ws.ok())
    return fail(PSK_ENOMEM, "workspace too small for the BF16 Gaussian GEMM");
  return 0;
}

// the product of prepared limbs and the FP64 sum of the K-split partials
int bf16_run(const Bf16Plan &P, int64_t m, int64_t d, uint64_t seed, double *C,
             hipStream_t st) {
  {
    KTimer t("gauss_gemm", st);
    k_gauss_gemm_bf16<<<(unsigned)(P.tiles * P.splits), kThreads, 0, st>>>(
        m, d, P.npad, seed, P.hi, P.lo, P.tiles_m, P.tiles_n, P.kchunks, P.cper, P.part);
  }
  {
    KTimer t("gemm_reduce", st);
    const int64_t len = m * d;
    k_reduce_splits_f32<<<(unsigned)ceil_div(len, 256), 256, 0, st>>>(
        P.part, len, (int)P.splits, 1.0 / sqrt((double)m), C);
  }
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

// FP64 bucket sums of 8 buckets over the padded columns
size_t csr_limbs_lds(const psk_mat &A, int64_t d) {
  (void)A;
  return (size_t)8 * ceil_div(d, kBN) * kBN * sizeof(double);
}

}  // namespace

int gauss_gemm_bf16(int64_t m, int64_t r, int64_t d, uint64_t seed, const void *SA,
                    int sa_dtype, double *C, Arena &ws, hipStream_t st) {
  Bf16Plan P;
  int rc = bf16_plan(m, r, d, ws, P);
  if (rc || ws.dry()) return rc;
  {
    KTimer t("sa_limbs", st);
    const int64_t threads = P.kchunks * 4 * P.npad;
    if (sa_dtype == PSK_F64)
      k_sa_limbs<double><<<(unsigned)ceil_div(threads, 256), 256, 0, st>>>(
          (const double *)SA, r, d, P.npad, P.kchunks, P.hi, P.lo);
    else
      k_sa_limbs<float><<<(unsigned)ceil_div(threads, 256), 256, 0, st>>>(
          (const float *)SA, r, d, P.npad, P.kchunks, P.hi, P.lo);
  }
  return bf16_run(P, m, d, seed, C, st);
}

bool bf16_csr_fusable(const psk_mat &A, int64_t r) {
  return A.format == PSK_CSR && cs_splits(A.n, r) == 1 && csr_limbs_lds(A, A.d) <= 65536;
}

int gauss_gemm_bf16_csr(int64_t m, int64_t r, const psk_mat &A, const uint32_t *perm,
                        const uint32_t *bptr, uint64_t seed, double *C, Arena &ws,
                        hipStream_t st) {
  if (!bf16_csr_fusable(A, r))
    return fail(PSK_EUNSUPPORTED, "fused CSR limbs need one split per bucket, d <= 1024");
  Bf16Plan P;
  int rc = bf16_plan(m, r, A.d, ws, P);
  if (rc || ws.dry()) return rc;
  {
    KTimer t("cs_scatter_limbs", st);
    const unsigned quads = (unsigned)(P.kchunks * 4);
    const size_t lds = csr_limbs_lds(A, A.d);
    if (A.dtype == PSK_F64)
      k_scatter_csr_limbs<double><<<quads, 512, lds, st>>>(
          (const double *)A.values, A.indptr, A.indices, P.npad, r, perm, bptr, P.hi, P.lo);
    else
      k_scatter_csr_limbs<float><<<quads, 512, lds, st>>>(
          (const float *)A.values, A.indptr, A.indices, P.npad, r, perm, bptr, P.hi, P.lo);
  }
  return bf16_run(P, m, A.d, seed, C, st);
}

}  // namespace psk
