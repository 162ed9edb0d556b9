// FP64 dense products on the gfx950 matrix cores (v_mfma_f64_16x16x4f64):
// a general row-major GEMM with optional transposes and K splitting, the
// Gram matrix of a dense A (upper tiles only, mirrored), and the fused
// product-and-row-norm of a dense A times B.
//
// Paper mapping (arXiv 2203.02798): Algorithm gram (row-partitioned Gram:
// private partial Grams of row blocks, then a reduction) becomes the K split
// of A^T*A over row blocks of A followed by a fixed-order reduction kernel;
// rmsqn ("memory efficient" squared row norms of A*B for dense A) becomes a
// GEMM whose epilogue squares and sums each output row, so A*B is never
// stored.
//
// One kernel template covers all three.  A workgroup is 4 wavefronts laid
// out WM x WN; each owns MB x NB blocks of 16 x 16 FP64 accumulators.  K
// advances 16 at a time through LDS tiles kept k-major (As[k][i], Bs[k][j]),
// with the next chunk prefetched into registers while the current one is
// multiplied.  FP32 inputs are widened to FP64 when staged.
#include "internal.hpp"

namespace psk {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kBK = 16;

enum { EPI_PARTIAL = 0, EPI_ROWNORM = 1, EPI_DIRECT = 2 };

template <typename T, bool KMAJOR, int BX>
struct TileLoader {
  // Loads a kBK x BX k-major tile of a logical operand Op[k][x]:
  //   KMAJOR: Op[k][x] = P[k*ld + x] (rows of P are k)
  //   else:   Op[k][x] = P[x*ld + k] (rows of P are x)
  static constexpr int kPer = (kBK * BX) / 256;
  double v[kPer];
  __device__ __forceinline__ void load(const T *__restrict__ P, int64_t ld, int64_t x0,
                                       int64_t xlim, int64_t k0, int64_t klim) {
#pragma unroll
    for (int p = 0; p < kPer; ++p) {
      const int e = threadIdx.x + 256 * p;
      int kk, xx;
      if (KMAJOR) {
        kk = e / BX;
        xx = e % BX;
      } else {
        kk = e % kBK;
        xx = e / kBK;
      }
      const int64_t k = k0 + kk, x = x0 + xx;
      v[p] = (k < klim && x < xlim) ? (double)(KMAJOR ? P[k * ld + x] : P[x * ld + k])
                                    : 0.0;
    }
  }
  __device__ __forceinline__ void store(double (*S)[BX + 4]) const {
#pragma unroll
    for (int p = 0; p < kPer; ++p) {
      const int e = threadIdx.x + 256 * p;
      int kk, xx;
      if (KMAJOR) {
        kk = e / BX;
        xx = e % BX;
      } else {
        kk = e % kBK;
        xx = e / kBK;
      }
      S[kk][xx] = v[p];
    }
  }
};

// Tile scheduling: tile t of the (tiles_m x tiles_n [upper only]) grid,
// split ks.  Blocks are renumbered so one XCD gets consecutive tiles.
struct TileCoord {
  int mt, nt, ks;
};

__device__ __forceinline__ TileCoord tile_of(int tiles_m, int tiles_n, bool upper) {
  const int64_t nblk = (int64_t)gridDim.x;
  int64_t lin = blockIdx.x;
  if ((nblk & 7) == 0) lin = (lin & 7) * (nblk >> 3) + (lin >> 3);
  TileCoord c;
  if (!upper) {
    c.mt = (int)(lin % tiles_m);
    const int64_t rest = lin / tiles_m;
    c.nt = (int)(rest % tiles_n);
    c.ks = (int)(rest / tiles_n);
  } else {
    // upper-triangular tiles (mt <= nt) of a square grid, row-major order
    const int64_t nup = (int64_t)tiles_m * (tiles_m + 1) / 2;
    int64_t t = lin % nup;
    c.ks = (int)(lin / nup);
    int mt = 0;
    int64_t rowlen = tiles_m;
    while (t >= rowlen) {
      t -= rowlen;
      ++mt;
      --rowlen;
    }
    c.mt = mt;
    c.nt = mt + (int)t;
  }
  return c;
}

template <typename TA, typename TB, bool TRA, bool TRB, int WM, int WN, int MB, int NB,
          int EPI, bool UPPER>
__global__ __launch_bounds__(256) void k_dgemm(
    int64_t M, int64_t N, int64_t K, const TA *__restrict__ A, int64_t lda,
    const TB *__restrict__ B, int64_t ldb, int tiles_m, int tiles_n, int64_t kper,
    double *__restrict__ out, int64_t ldo, double alpha, double beta) {
  constexpr int BM = WM * MB * 16;
  constexpr int BN = WN * NB * 16;
  __shared__ double As[kBK][BM + 4];
  __shared__ double Bs[kBK][BN + 4];

  const TileCoord tc = tile_of(tiles_m, tiles_n, UPPER);
  const int64_t m0 = (int64_t)tc.mt * BM;
  const int64_t n0 = (int64_t)tc.nt * BN;
  const int64_t kb = (int64_t)tc.ks * kper;
  int64_t ke = kb + kper;
  if (ke > K) ke = K;

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int kq = lane >> 4;
  const int li = lane & 15;
  const int wm = wave / WN;
  const int wn = wave % WN;

  v4d acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

  // Op_A[i][k]: TRA -> A is K x M (A[k*lda+i]) which is k-major
  TileLoader<TA, TRA, BM> la;
  TileLoader<TB, !TRB, BN> lb;
  const int64_t nchunks = (ke > kb) ? ceil_div(ke - kb, kBK) : 0;
  if (nchunks > 0) {
    la.load(A, lda, m0, M, kb, ke);
    lb.load(B, ldb, n0, N, kb, ke);
  }
  for (int64_t c = 0; c < nchunks; ++c) {
    __syncthreads();
    la.store(As);
    lb.store(Bs);
    __syncthreads();
    if (c + 1 < nchunks) {
      const int64_t k1 = kb + (c + 1) * kBK;
      la.load(A, lda, m0, M, k1, ke);
      lb.load(B, ldb, n0, N, k1, ke);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double av[MB], bv[NB];
#pragma unroll
      for (int a = 0; a < MB; ++a) av[a] = As[4 * s + kq][(wm * MB + a) * 16 + li];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = Bs[4 * s + kq][(wn * NB + b) * 16 + li];
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }

  if (EPI == EPI_DIRECT) {
    // no K split: out = alpha * acc + beta * out (beta == 0 ignores out)
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = m0 + (wm * MB + a) * 16 + kq + 4 * e;
        if (row >= M) continue;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int64_t col = n0 + (wn * NB + b) * 16 + li;
          if (col < N) {
            double *po = out + row * ldo + col;
            *po = beta != 0.0 ? alpha * acc[a][b][e] + beta * *po : alpha * acc[a][b][e];
          }
        }
      }
  } else if (EPI == EPI_PARTIAL) {
    double *o = out + (int64_t)tc.ks * M * ldo;
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = m0 + (wm * MB + a) * 16 + kq + 4 * e;
        if (row >= M) continue;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int64_t col = n0 + (wn * NB + b) * 16 + li;
          if (col < N) o[row * ldo + col] = acc[a][b][e];
        }
      }
  } else {
    // squared row norms over this tile's columns: out[nt][row]
    __shared__ double red[WN][BM];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double s2 = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) s2 += acc[a][b][e] * acc[a][b][e];
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) s2 += __shfl_xor(s2, off, 64);
        if (li == 0) red[wn][(wm * MB + a) * 16 + kq + 4 * e] = s2;
      }
    __syncthreads();
    for (int i = tid; i < BM; i += 256) {
      const int64_t row = m0 + i;
      if (row >= M) continue;
      double s2 = 0.0;
#pragma unroll
      for (int q = 0; q < WN; ++q) s2 += red[q][i];
      out[(int64_t)tc.nt * ldo + row] = s2;
    }
  }
}

// C = alpha * sum_s part[s] + beta * C; part is [splits][M][ldp].  With
// mirror, entries below the diagonal are read from the transposed position
// (only upper tiles were computed).
template <typename TO>
__global__ __launch_bounds__(256) void k_splitk_reduce(
    const double *__restrict__ part, int64_t M, int64_t N, int64_t ldp, int splits,
    double alpha, double beta, TO *__restrict__ C, int64_t ldc, int mirror_tile) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  int64_t i = e / N, j = e % N;
  if (mirror_tile > 0 && (i / mirror_tile) > (j / mirror_tile)) {
    const int64_t t = i;
    i = j;
    j = t;
  }
  double acc = part[i * ldp + j];
  for (int s = 1; s < splits; ++s) acc += part[(int64_t)s * M * ldp + i * ldp + j];
  const int64_t oi = e / N, oj = e % N;
  double v = alpha * acc;
  if (beta != 0.0) v += beta * (double)C[oi * ldc + oj];
  C[oi * ldc + oj] = (TO)v;
}

__global__ __launch_bounds__(256) void k_rownorm_reduce(const double *__restrict__ part,
                                                        int64_t n, int tiles,
                                                        double alpha, double beta,
                                                        double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = part[i];
  for (int t = 1; t < tiles; ++t) s += part[(int64_t)t * n + i];
  double v = alpha * s;
  if (beta != 0.0) v += beta * x[i];
  x[i] = v;
}

int64_t pick_splits(int64_t tiles, int64_t K, int64_t target_blocks) {
  const int64_t kchunks = ceil_div(K, kBK);
  int64_t s = ceil_div(target_blocks, tiles);
  int64_t smax = kchunks / 16;
  if (smax < 1) smax = 1;
  if (s > smax) s = smax;
  return s < 1 ? 1 : s;
}

template <typename TA, typename TB, bool TRA, bool TRB, int WM, int WN, int MB, int NB,
          bool UPPER>
int gemm_partial_launch(int64_t M, int64_t N, int64_t K, const TA *A, int64_t lda,
                        const TB *B, int64_t ldb, double alpha, double beta, void *C,
                        int64_t ldc, bool out_f32, Arena &ws, hipStream_t st) {
  constexpr int BM = WM * MB * 16, BN = WN * NB * 16;
  const int tm = (int)ceil_div(M, BM), tn = (int)ceil_div(N, BN);
  const int64_t tiles = UPPER ? (int64_t)tm * (tm + 1) / 2 : (int64_t)tm * tn;
  int64_t splits = pick_splits(tiles, K, 1024);
  const int64_t kper = ceil_div(ceil_div(K, kBK), splits) * kBK;
  splits = K > 0 ? ceil_div(K, kper) : 1;
  if (splits == 1 && !UPPER && !out_f32) {
    if (ws.dry()) return 0;
    k_dgemm<TA, TB, TRA, TRB, WM, WN, MB, NB, EPI_DIRECT, false>
        <<<(unsigned)tiles, 256, 0, st>>>(M, N, K, A, lda, B, ldb, tm, tn, kper,
                                          (double *)C, ldc, alpha, beta);
    PSK_HIP_TRY(hipGetLastError());
    return 0;
  }
  double *part = ws.take<double>((size_t)splits * M * N);
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for a GEMM");
  k_dgemm<TA, TB, TRA, TRB, WM, WN, MB, NB, EPI_PARTIAL, UPPER>
      <<<(unsigned)(tiles * splits), 256, 0, st>>>(M, N, K, A, lda, B, ldb, tm, tn,
                                                    kper, part, N, 1.0, 0.0);
  const int64_t len = M * N;
  if (out_f32)
    k_splitk_reduce<float><<<(unsigned)ceil_div(len, 256), 256, 0, st>>>(
        part, M, N, N, (int)splits, alpha, beta, (float *)C, ldc, UPPER ? BM : 0);
  else
    k_splitk_reduce<double><<<(unsigned)ceil_div(len, 256), 256, 0, st>>>(
        part, M, N, N, (int)splits, alpha, beta, (double *)C, ldc, UPPER ? BM : 0);
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

// Fused row norms with a column tile of B resident in LDS.  B[:, n0 : n0 +
// BNC] (rows padded to a multiple of the chunk with zeros, row stride BNC + 4) is
// staged once per workgroup; the 8 wavefronts then stream row tiles of A
// (kBresMB blocks of 16 rows) straight from memory into the MFMA operand
// registers (no LDS round trip and no barrier in the main loop) and keep
// kBresMB x BNC/16 accumulator blocks.
// Inside a K chunk of 4 kBresKW columns, lane (li, kq) feeds column
// k0 + kBresKW kq + s of A at step s, and B row k0 + kBresKW kq + s: the same
// permutation of the chunk on both operands, so one lane reads kBresKW
// consecutive elements of its row.
// part[nt * n + row] = the row's squared norm over the tile's BNC columns.
// Workgroups form row groups of tn (one per column tile) that sit on one XCD
// (linear ids equal mod 8) and walk the same rows, so A is fetched into that
// XCD's L2 about once for all tn tiles.
constexpr int kBresThreads = 512;
constexpr int kBresMB = 2;  // 16-row blocks per wavefront tile
constexpr int kBresRows = 16 * kBresMB;
constexpr int kBresKW = 8;

template <typename TA, int BNC, bool VEC>
__global__ __launch_bounds__(kBresThreads) void k_rownorm_bres(
    const TA *__restrict__ A, int64_t ld, int64_t n, int64_t d, const double *__restrict__ B,
    int64_t k, int tn, double *__restrict__ part) {
  static_assert(!VEC || sizeof(TA) == 4, "vector loads are for FP32 A");
  extern __shared__ double Bs[];
  constexpr int LDB = BNC + 4;
  constexpr int NB = BNC / 16;
  constexpr int MB = kBresMB;
  constexpr int KW = kBresKW;  // consecutive elements of a row per lane per chunk
  constexpr int CK = 4 * KW;   // K chunk width
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int64_t lin = blockIdx.x, nblk = gridDim.x;
  const int64_t slot = lin >> 3;
  const int nt = (int)(slot % tn);
  const int64_t ngroups = nblk / tn;
  const int64_t group = (slot / tn) * 8 + (lin & 7);
  const int64_t n0 = (int64_t)nt * BNC;
  const int64_t kch = (d + CK - 1) / CK;
  const int64_t drows = kch * CK;
  for (int64_t e = tid; e < drows * BNC; e += kBresThreads) {
    const int64_t kk = e / BNC;
    const int jj = (int)(e - kk * BNC);
    const int64_t col = n0 + jj;
    Bs[kk * LDB + jj] = (kk < d && col < k) ? B[kk * k + col] : 0.0;
  }
  __syncthreads();
  const int64_t ntiles = (n + kBresRows - 1) / kBresRows;
  for (int64_t t = group * 8 + wave; t < ntiles; t += ngroups * 8) {
    const int64_t r0 = t * kBresRows;
    const TA *arow[MB];
    bool rin[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int64_t row = r0 + mb * 16 + li;
      rin[mb] = row < n;
      arow[mb] = A + (rin[mb] ? row : 0) * ld;
    }
    v4d acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = v4d{0.0, 0.0, 0.0, 0.0};
    auto load = [&](int64_t c, double (&a)[MB][KW]) __attribute__((always_inline)) {
      const int64_t kb = c * CK + KW * kq;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        if constexpr (VEC) {
#pragma unroll
          for (int q = 0; q < KW / 4; ++q) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (rin[mb] && kb + 4 * q < d)
              v = *reinterpret_cast<const float4 *>(arow[mb] + kb + 4 * q);
            a[mb][4 * q + 0] = v.x;
            a[mb][4 * q + 1] = v.y;
            a[mb][4 * q + 2] = v.z;
            a[mb][4 * q + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int s = 0; s < KW; ++s)
            a[mb][s] = (rin[mb] && kb + s < d) ? (double)arow[mb][kb + s] : 0.0;
        }
      }
    };
    auto step = [&](int64_t c, const double (&a)[MB][KW]) __attribute__((always_inline)) {
#pragma unroll
      for (int s = 0; s < KW; ++s) {
        const double *brow = Bs + (c * CK + KW * kq + s) * LDB + li;
        double bv[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bv[nb] = brow[nb * 16];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb][s], bv[nb], acc[mb][nb],
                                                               0, 0, 0);
      }
    };
    double a0[MB][KW], a1[MB][KW];
    load(0, a0);
    for (int64_t c = 0; c < kch; c += 2) {
      if (c + 1 < kch) load(c + 1, a1);
      step(c, a0);
      if (c + 1 >= kch) break;
      if (c + 2 < kch) load(c + 2, a0);
      step(c + 1, a1);
    }
    // lane (li, kq) holds rows kq + 4 e, column li of each 16 x 16 block
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double s2 = 0.0;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) s2 += acc[mb][nb][e] * acc[mb][nb][e];
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) s2 += __shfl_xor(s2, off, 64);
        const int64_t row = r0 + mb * 16 + kq + 4 * e;
        if (li == 0 && row < n) part[(int64_t)nt * n + row] = s2;
      }
  }
}

// Column width of the LDS-resident form for d (0: the tile does not fit).
int bres_width(int64_t d, int64_t k) {
  const int64_t drows = ceil_div(d, (int64_t)(4 * kBresKW)) * (4 * kBresKW);
  if (k > 32 && drows * (64 + 4) * 8 <= 163840) return 64;
  if (drows * (32 + 4) * 8 <= 163840) return 32;
  return 0;
}

template <typename TA, int BNC, bool VEC>
int bres_launch(const psk_mat &Am, const double *B, int64_t k, double *part, int tn,
                hipStream_t st) {
  const int64_t n = Am.n, d = Am.d;
  const size_t lds =
      (size_t)ceil_div(d, (int64_t)(4 * kBresKW)) * (4 * kBresKW) * (BNC + 4) * sizeof(double);
  PSK_HIP_TRY(hipFuncSetAttribute((const void *)k_rownorm_bres<TA, BNC, VEC>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  // one workgroup per CU (the LDS tile), row groups of tn workgroups per XCD
  const int64_t tiles = ceil_div(n, (int64_t)kBresRows);
  int64_t groups = 256 / tn;
  if (groups < 8) groups = 8;
  groups = (groups / 8) * 8;
  const int64_t need = ceil_div(tiles, (int64_t)8);  // 8 wavefronts per workgroup
  while (groups > 8 && groups / 2 >= need) groups /= 2;
  const unsigned nblk = (unsigned)(groups * tn);
  k_rownorm_bres<TA, BNC, VEC><<<nblk, kBresThreads, lds, st>>>(
      (const TA *)Am.values, Am.ld, n, d, B, k, tn, part);
  return 0;
}

template <typename TA>
int rownorm_launch(const psk_mat &Am, const double *B, int64_t k, double alpha,
                   double beta, double *x, Arena &ws, hipStream_t st) {
  const int64_t n = Am.n, d = Am.d;
  const TA *A = (const TA *)Am.values;
  const int bw = bres_width(d, k);
  if (bw > 0) {
    const int tn = (int)ceil_div(k, (int64_t)bw);
    double *part = ws.take<double>((size_t)tn * n);
    if (ws.dry()) return 0;
    if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for row norms");
    // FP32 rows read four elements at a time when every such group is aligned
    const bool vec = Am.ld % 4 == 0 && d % 4 == 0 && ((uintptr_t)Am.values & 15) == 0;
    int rc;
    if constexpr (sizeof(TA) == 4) {
      if (bw == 64)
        rc = vec ? bres_launch<TA, 64, true>(Am, B, k, part, tn, st)
                 : bres_launch<TA, 64, false>(Am, B, k, part, tn, st);
      else
        rc = vec ? bres_launch<TA, 32, true>(Am, B, k, part, tn, st)
                 : bres_launch<TA, 32, false>(Am, B, k, part, tn, st);
    } else {
      (void)vec;
      rc = bw == 64 ? bres_launch<TA, 64, false>(Am, B, k, part, tn, st)
                    : bres_launch<TA, 32, false>(Am, B, k, part, tn, st);
    }
    if (rc) return rc;
    k_rownorm_reduce<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(part, n, tn, alpha, beta, x);
  } else if (k <= 64) {
    constexpr int BM = 32, BN = 64;
    const int tm = (int)ceil_div(n, BM), tn = (int)ceil_div(k, BN);
    double *part = ws.take<double>((size_t)tn * n);
    if (ws.dry()) return 0;
    if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for row norms");
    k_dgemm<TA, double, false, false, 2, 2, 1, 2, EPI_ROWNORM, false>
        <<<(unsigned)((int64_t)tm * tn), 256, 0, st>>>(n, k, d, A, Am.ld, B, k, tm, tn, d,
                                                       part, n, 1.0, 0.0);
    k_rownorm_reduce<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(part, n, tn, alpha,
                                                                  beta, x);
  } else {
    constexpr int BM = 32, BN = 256;
    const int tm = (int)ceil_div(n, BM), tn = (int)ceil_div(k, BN);
    double *part = ws.take<double>((size_t)tn * n);
    if (ws.dry()) return 0;
    if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for row norms");
    k_dgemm<TA, double, false, false, 2, 2, 1, 8, EPI_ROWNORM, false>
        <<<(unsigned)((int64_t)tm * tn), 256, 0, st>>>(n, k, d, A, Am.ld, B, k, tm, tn, d,
                                                       part, n, 1.0, 0.0);
    k_rownorm_reduce<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(part, n, tn, alpha,
                                                                  beta, x);
  }
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace

int dgemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
          const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
          double *C, int64_t ldc, Arena &ws, hipStream_t st) {
  if (M <= 0 || N <= 0) return 0;
  if (K <= 0) return fail(PSK_EINVAL, "internal GEMM with K <= 0");
  // up to 1024 x 1024 outputs (the d x d products of the factorizations),
  // 32 x 32 tiles give the chip four times the workgroups of 64 x 64 ones
#define PSK_DG(TRA, TRB)                                                            \
  return (M * N <= 1024 * 1024)                                                     \
      ? gemm_partial_launch<double, double, TRA, TRB, 2, 2, 1, 1, false>(            \
            M, N, K, A, lda, B, ldb, alpha, beta, C, ldc, false, ws, st)             \
      : gemm_partial_launch<double, double, TRA, TRB, 2, 2, 2, 2, false>(            \
            M, N, K, A, lda, B, ldb, alpha, beta, C, ldc, false, ws, st)
  if (ta && tb) PSK_DG(true, true);
  if (ta) PSK_DG(true, false);
  if (tb) PSK_DG(false, true);
  PSK_DG(false, false);
#undef PSK_DG
}

int gram_dense(double alpha, const psk_mat &A, double beta, void *C, Arena &ws,
               hipStream_t st, bool out_f64) {
  KTimer timer("gram", st, !ws.dry());
  const bool f32 = A.dtype == PSK_F32;
  if (f32)
    return gemm_partial_launch<float, float, true, false, 2, 2, 2, 2, true>(
        A.d, A.d, A.n, (const float *)A.values, A.ld, (const float *)A.values, A.ld,
        alpha, beta, C, A.d, !out_f64, ws, st);
  return gemm_partial_launch<double, double, true, false, 2, 2, 2, 2, true>(
      A.d, A.d, A.n, (const double *)A.values, A.ld, (const double *)A.values, A.ld,
      alpha, beta, C, A.d, false, ws, st);
}

int rownorms_dense(double alpha, const psk_mat &A, const double *B, int64_t k,
                   double beta, double *x, Arena &ws, hipStream_t st) {
  KTimer timer("rownorm", st, !ws.dry());
  if (A.dtype == PSK_F32) return rownorm_launch<float>(A, B, k, alpha, beta, x, ws, st);
  return rownorm_launch<double>(A, B, k, alpha, beta, x, ws, st);
}

}  // namespace psk
