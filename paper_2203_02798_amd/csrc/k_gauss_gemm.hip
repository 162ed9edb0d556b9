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

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gauss_gemm_f64(
    int64_t m, int64_t r, int64_t d, uint64_t seed, const T *__restrict__ SA,
    int tiles_m, int tiles_n, int splits, int64_t kper,
    double *__restrict__ out /* [splits][m][d] */) {
  __shared__ double tile[2][kBK][kLdsStride];

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

  auto load_chunk = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < kPf; ++p) {
      const int64_t k = k0 + lrow + 2 * p;
      pf[p] = (col_ok && k < ke) ? (double)SA[k * d + n0 + lcol] : 0.0;
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int p = 0; p < kPf; ++p) tile[buf][lrow + 2 * p][lcol] = pf[p];
  };

  const int64_t nchunks = (ke > kb) ? ceil_div(ke - kb, kBK) : 0;
  const uint32_t row_a = (uint32_t)(m0 + wave * 16 + li);

  if (nchunks > 0) {
    load_chunk(kb);
    store_chunk(0);
  }
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const int buf = (int)(c & 1);
    const int64_t k0 = kb + c * kBK;
    if (c + 1 < nchunks) load_chunk(k0 + kBK);
    // Gaussian values of this lane's row for four consecutive buckets
    double g[4];
    gauss4_f64((uint64_t)(k0 >> 2) + (uint64_t)kq, row_a, seed, g);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double bv[kNB];
#pragma unroll
      for (int nb = 0; nb < kNB; ++nb) bv[nb] = tile[buf][4 * kq + s][nb * 16 + li];
#pragma unroll
      for (int nb = 0; nb < kNB; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[s], bv[nb], acc[nb], 0, 0, 0);
    }
    if (c + 1 < nchunks) store_chunk(buf ^ 1);
    __syncthreads();
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
  if (prec != PSK_PREC_F64)
    return fail(PSK_EDTYPE, "this build's Gaussian GEMM supports PSK_PREC_F64");
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
    if (sa_dtype == PSK_F64)
      k_gauss_gemm_f64<double><<<(unsigned)nblk, kThreads, 0, st>>>(
          m, r, d, seed, (const double *)SA, tiles_m, tiles_n, (int)splits, kper, part);
    else
      k_gauss_gemm_f64<float><<<(unsigned)nblk, kThreads, 0, st>>>(
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
