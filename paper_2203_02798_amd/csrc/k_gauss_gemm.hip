// C = G * (S*A) with the Gaussian G generated inside the GEMM (never stored),
// FP64 on the gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
// Paper mapping (arXiv 2203.02798): Algorithm countgauss_multiply forms, per
// batch of buckets, a fresh Gaussian block and accumulates C += G_i * B with a
// BLAS GEMM; csrcgs/rmcgs scale G by 1/sqrt(m).  Here a batch is a 16-bucket
// K chunk of one workgroup: its Gaussian values are produced in the
// registers that feed the matrix instruction, and the K dimension (r
// buckets) is split over workgroups whose FP64 partial products are summed
// in a fixed order by a second kernel, which also applies 1/sqrt(m).
//
// Tiling: 512 threads = 8 wavefronts; workgroup tile 128 (rows of G / C) x
// 256 (columns of C); each wavefront owns 16 rows x 256 columns = 16 MFMA
// blocks (64 FP64 accumulators per lane).  Generating a Gaussian value costs
// about as much FP64 vector work as a few matrix instructions, so the wide
// column tile matters: each value feeds 256 output columns.  K advances 16
// buckets per chunk: the lane with quad kq = lane/16 draws one Philox block
// for buckets k0+4kq .. k0+4kq+3 of its row, and k-step s (0..3) pairs bucket
// k0+4kq+s of G with the same bucket row of S*A from LDS (any fixed
// permutation of k inside a chunk leaves the contraction unchanged).
// The S*A chunk is staged through double-buffered LDS with a register
// prefetch of the next chunk; the LDS row stride (272 doubles) puts the four
// k rows of one read into two distinct bank halves.
#include "internal.hpp"

namespace psk {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kBM = 16 * kWaves;  // 128
constexpr int kBN = 256;
constexpr int kNB = kBN / 16;      // 16 MFMA blocks per wavefront
constexpr int kBK = 16;
constexpr int kLdsStride = kBN + 16;
constexpr int kPf = kBK * kBN / kThreads;  // 8 prefetched values per thread

typedef __attribute__((address_space(3))) void *lds_ptr_t;

// DIRECT (FP64 S*A, even d, split slice below 2 GiB): each chunk of S*A is
// copied from memory straight into LDS by buffer loads (16 bytes per lane,
// no registers, no LDS stores), issued one chunk ahead.  The buffer
// descriptor covers exactly this workgroup's K slice, so rows past the
// slice read as zero (hardware range check); columns past d of a row read
// the next row's values, which only reach output columns >= d (discarded).
// Otherwise S*A goes through registers (converted to FP64, masked).
template <typename T, bool DIRECT>
__global__ __launch_bounds__(kThreads) void k_gauss_gemm_f64(
    int64_t m, int64_t r, int64_t d, uint64_t seed, const T *__restrict__ SA,
    int tiles_m, int tiles_n, int splits, int64_t kper,
    double *__restrict__ out /* [splits][m][d] */) {
  __shared__ __align__(16) double tile[2][kBK][kLdsStride];

  // XCD-aware order: blocks are dealt round-robin to the 8 XCDs; renumber so
  // that one XCD runs consecutive tiles of the same (column tile, K split),
  // which then share S*A in that XCD's L2.
  const int64_t nblk = (int64_t)gridDim.x;
  int64_t lin = blockIdx.x;
  if ((nblk & 7) == 0) lin = (lin & 7) * (nblk >> 3) + (lin >> 3);
  const int mt = (int)(lin % tiles_m);
  const int64_t rest = lin / tiles_m;
  const int nt = (int)(rest % tiles_n);
  const int ks = (int)(rest / tiles_n);

  const int64_t m0 = (int64_t)mt * kBM;
  const int64_t n0 = (int64_t)nt * kBN;
  const int64_t kb = (int64_t)ks * kper;
  int64_t ke = kb + kper;
  if (ke > r) ke = r;

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int kq = lane >> 4;
  const int li = lane & 15;

  v4d acc[kNB];
#pragma unroll
  for (int b = 0; b < kNB; ++b) acc[b] = v4d{0.0, 0.0, 0.0, 0.0};

  // S*A staging: thread covers column n0 + (tid % 256), rows tid/256 + 2p
  const int lcol = tid & (kBN - 1);
  const int lrow = tid >> 8;
  const bool col_ok = (n0 + lcol) < d;
  double pf[kPf];

  // Branch-free loads (clamped in-bounds address, then a select) keep the
  // whole K iteration one basic block, so the scheduler can interleave the
  // Gaussian generation with the matrix instructions.
  const int64_t ccol = col_ok ? n0 + lcol : d - 1;
  auto load_chunk = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < kPf; ++p) {
      const int64_t k = k0 + lrow + 2 * p;
      const int64_t kc = k < ke ? k : ke - 1;
      const double v = (double)SA[kc * d + ccol];
      pf[p] = (col_ok && k < ke) ? v : 0.0;
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int p = 0; p < kPf; ++p) tile[buf][lrow + 2 * p][lcol] = pf[p];
  };

  // direct path: wave w copies rows 2w, 2w+1 of a chunk, 128 doubles per
  // buffer load (64 lanes x 16 bytes), two loads per row
  __amdgpu_buffer_rsrc_t rsrc;
  if (DIRECT) {
    const int nbytes = (int)((ke > kb ? ke - kb : 0) * d * (int64_t)sizeof(double));
    rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)(SA + kb * d), (short)0, nbytes,
                                             0x00020000);
  }
  auto direct_chunk = [&](int64_t crel, int buf) {
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      const int row = 2 * wave + rr;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int voff =
            (int)(((crel * kBK + row) * d + n0 + hh * 128 + 2 * lane) * (int64_t)sizeof(double));
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_ptr_t)&tile[buf][row][hh * 128],
                                                 16, voff, 0, 0, 0);
      }
    }
  };

  const int64_t nchunks = (ke > kb) ? ceil_div(ke - kb, kBK) : 0;
  const uint32_t row_a = (uint32_t)(m0 + wave * 16 + li);

  // Gaussian values of this lane's row for the four consecutive buckets of a
  // chunk; the values for chunk c+1 are generated while chunk c's matrix
  // instructions run (the vector and matrix pipes work concurrently).
  double g[4];
  if (nchunks > 0) {
    if (DIRECT) {
      direct_chunk(0, 0);
      __builtin_amdgcn_s_waitcnt(0);
    } else {
      load_chunk(kb);
      store_chunk(0);
    }
    gauss4_f64((uint64_t)(kb >> 2) + (uint64_t)kq, row_a, seed, g);
  }
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const int buf = (int)(c & 1);
    const int64_t k0 = kb + c * kBK;
    // the last iteration loads one unused chunk (in bounds or zero-filled)
    // rather than branching
    if (DIRECT)
      direct_chunk(c + 1, buf ^ 1);
    else
      load_chunk(k0 + kBK);
    double gn[4];
    gauss4_f64((uint64_t)((k0 + kBK) >> 2) + (uint64_t)kq, row_a, seed, gn);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double bv[kNB];
#pragma unroll
      for (int nb = 0; nb < kNB; ++nb) bv[nb] = tile[buf][4 * kq + s][nb * 16 + li];
#pragma unroll
      for (int nb = 0; nb < kNB; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[s], bv[nb], acc[nb], 0, 0, 0);
    }
    if (DIRECT)
      __builtin_amdgcn_s_waitcnt(0);  // this wave's copies into buf^1 landed
    else
      store_chunk(buf ^ 1);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) g[s] = gn[s];
  }

  // accumulator element e of block nb: row kq + 4*e, column li
  double *o = out + (int64_t)ks * m * d;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t row = m0 + wave * 16 + kq + 4 * e;
    if (row >= m) continue;
#pragma unroll
    for (int nb = 0; nb < kNB; ++nb) {
      const int64_t col = n0 + nb * 16 + li;
      if (col < d) o[row * d + col] = acc[nb][e];
    }
  }
}

// C[i] = scale * sum_s part[s][i], s in increasing order
__global__ __launch_bounds__(256) void k_reduce_splits(const double *__restrict__ part,
                                                       int64_t len, int splits,
                                                       double scale,
                                                       double *__restrict__ C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double acc = part[i];
  for (int s = 1; s < splits; ++s) acc += part[(int64_t)s * len + i];
  C[i] = acc * scale;
}

}  // namespace

int gauss_gemm(int64_t m, int64_t r, int64_t d, uint64_t seed, int prec,
               const void *SA, int sa_dtype, double *C, Arena &ws,
               hipStream_t st) {
  if (prec == PSK_PREC_BF16) return gauss_gemm_bf16(m, r, d, seed, SA, sa_dtype, C, ws, st);
  if (prec == PSK_PREC_FP8) return gauss_gemm_fp8(m, r, d, seed, SA, sa_dtype, C, ws, st);
  if (prec != PSK_PREC_F64) return fail(PSK_EDTYPE, "unknown Gaussian GEMM precision");
  const int tiles_m = (int)ceil_div(m, kBM);
  const int tiles_n = (int)ceil_div(d, kBN);
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
  // about two rounds of resident workgroups (one 512-thread workgroup per
  // CU), whole 16-bucket batches, at least 64 batches per split
  const int64_t kchunks = ceil_div(r, kBK);
  int64_t splits = ceil_div(512, tiles);
  const int64_t max_splits = kchunks / 64 > 0 ? kchunks / 64 : 1;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  const int64_t kper = ceil_div(kchunks, splits) * kBK;
  splits = ceil_div(r, kper);
  double *part = ws.take<double>((size_t)splits * m * d);
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for the Gaussian GEMM");
  const int64_t nblk = tiles * splits;
  {
    KTimer t("gauss_gemm", st);
    // direct copies need 16-byte aligned rows and a K slice addressable with
    // 32-bit byte offsets (plus one chunk of read-ahead)
    const bool direct = sa_dtype == PSK_F64 && (d % 2) == 0 &&
                        ((uintptr_t)SA % 16) == 0 &&
                        (kper + kBK) * d * (int64_t)sizeof(double) + 65536 < ((int64_t)1 << 31);
    if (direct)
      k_gauss_gemm_f64<double, true><<<(unsigned)nblk, kThreads, 0, st>>>(
          m, r, d, seed, (const double *)SA, tiles_m, tiles_n, (int)splits, kper, part);
    else if (sa_dtype == PSK_F64)
      k_gauss_gemm_f64<double, false><<<(unsigned)nblk, kThreads, 0, st>>>(
          m, r, d, seed, (const double *)SA, tiles_m, tiles_n, (int)splits, kper, part);
    else
      k_gauss_gemm_f64<float, false><<<(unsigned)nblk, kThreads, 0, st>>>(
          m, r, d, seed, (const float *)SA, tiles_m, tiles_n, (int)splits, kper, part);
  }
  const int64_t len = m * d;
  {
    KTimer t("gemm_reduce", st);
    k_reduce_splits<<<(unsigned)ceil_div(len, 256), 256, 0, st>>>(
        part, len, (int)splits, 1.0 / sqrt((double)m), C);
  }
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace psk
