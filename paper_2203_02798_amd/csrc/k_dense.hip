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
#include <type_traits>

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

// Four consecutive elements of one row as loaded (raw, in the dtype of A)
// and whether they are inside the matrix.  The load is branch-free: the
// address is clamped to a valid element and the values are selected and
// widened only when used, so the load stays in flight meanwhile (a load
// inside a branch, or converted right away, is waited for on the spot).
// VEC: one 16-byte FP32 load / two FP64 ones; needs d % 4 == 0 so that a
// column group is wholly inside or outside.
template <typename TA>
struct Raw4 {
  TA x[4];
  bool ok[4];
};

template <typename TA, bool VEC>
__device__ __forceinline__ void raw4_load(const TA *__restrict__ A, int64_t ld, int64_t d,
                                          int64_t row, bool rok, int64_t c, Raw4<TA> &v) {
  if constexpr (VEC) {
    const bool ok = rok && c < d;
    const TA *p = A + (ok ? row * ld + c : 0);
    if constexpr (sizeof(TA) == 4) {
      const float4 x = *reinterpret_cast<const float4 *>(p);
      v.x[0] = x.x; v.x[1] = x.y; v.x[2] = x.z; v.x[3] = x.w;
    } else {
      const double2 x = *reinterpret_cast<const double2 *>(p);
      const double2 y = *reinterpret_cast<const double2 *>(p + 2);
      v.x[0] = x.x; v.x[1] = x.y; v.x[2] = y.x; v.x[3] = y.y;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) v.ok[q] = ok;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = rok && c + q < d;
      v.x[q] = A[ok ? row * ld + c + q : 0];
      v.ok[q] = ok;
    }
  }
}

template <typename TA>
__device__ __forceinline__ double raw4_get(const Raw4<TA> &v, int q) {
  return v.ok[q] ? (double)v.x[q] : 0.0;
}

// Fused row norms with a column tile of B resident in LDS.  A workgroup
// holds 32-column tiles of B: one (PAIR false), or two, tiles p and
// T - 1 - p of the T = ceil(k / 32) tiles (PAIR true; one when they
// coincide).  Its B columns (rows padded to a multiple of the K chunk with
// zeros, row stride BNC + 4) are staged once; the 12 wavefronts then stream
// row tiles of A (kBresMB blocks of 16 rows) straight from memory into the
// MFMA operand registers (no LDS round trip and no barrier in the main loop)
// and keep kBresMB x BNC/16 accumulator blocks.
// While staging, the workgroup finds each tile's row extent: one past the
// last row of B holding a nonzero in the tile's columns.  K chunks at or past
// a tile's extent only add exact zeros to its products, so they are skipped:
// for B = R^{-1} upper triangular, tile t needs its first 32 (t + 1) rows,
// and pairing tile t with tile T - 1 - t gives every workgroup the same
// work.  (Skipped products are a * 0 with a finite: the sums are the same
// bits as the full product's.)
// Inside a K chunk of 4 kBresKW columns, lane (li, kq) feeds column
// k0 + kBresKW kq + s of A at step s, and B row k0 + kBresKW kq + s: the same
// permutation of the chunk on both operands, so one lane reads kBresKW
// consecutive elements of its row.
// The diagonal 32 x 32 block of a triangular B is half zeros.  When the
// staging finds the lower-left 16 x 16 quarter of a tile's diagonal block
// zero (its rows 16 .. 31 in the tile's first 16 columns) and that block is
// the tile's last chunk (and inside the d columns), the chunk is taken in
// another order: one swap of lane halves per pair of elements (lanes
// kq = 0, 1 exchange element s + 4 for element s of kq = 2, 3) gives steps
// 0 .. 3 the chunk's first 16 rows and steps 4 .. 7 its last 16, row
// 16 h + 8 (kq & 1) + 4 (kq >> 1) + s at step 4 h + s, so the products of
// the tile's first column block skip steps 4 .. 7 there.
// part[slot * n + row] = the row's squared norm over the slot's columns.
// Workgroups form row groups of tn (one per slot) that sit on one XCD
// (linear ids equal mod 8) and walk the same rows, so A is fetched into that
// XCD's L2 about once for all tn slots.
constexpr int kBresThreads = 768;  // 12 wavefronts: three per SIMD
constexpr int kBresWaves = kBresThreads / 64;
constexpr int kBresMB = 2;  // 16-row blocks per wavefront tile
constexpr int kBresRows = 16 * kBresMB;
constexpr int kBresKW = 8;
constexpr int kBresTile = 32;  // columns of B per tile

template <typename TA, bool PAIR, bool VEC>
__global__ __launch_bounds__(kBresThreads) void k_rownorm_bres(
    const TA *__restrict__ A, int64_t ld, int64_t n, int64_t d, const double *__restrict__ B,
    int64_t k, int tn, double *__restrict__ part) {
  static_assert(!VEC || sizeof(TA) == 4, "vector loads are for FP32 A");
  extern __shared__ double Bs[];
  __shared__ int ext[2];
  __shared__ int nzq[2];  // a nonzero in the lower-left quarter of the tile's diagonal block
  constexpr int BNC = PAIR ? 2 * kBresTile : kBresTile;
  constexpr int LDB = BNC + 4;
  constexpr int NB = BNC / 16;
  constexpr int NBH = kBresTile / 16;  // blocks per tile
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
  const int64_t ntile = ceil_div(k, (int64_t)kBresTile);
  // first columns of the (one or two) tiles; -1: no second tile
  const int64_t c0a = (int64_t)nt * kBresTile;
  const int64_t tb = PAIR ? ntile - 1 - nt : -1;
  const int64_t c0b = (PAIR && tb != nt) ? tb * kBresTile : -1;
  const int64_t kch = (d + CK - 1) / CK;
  const int64_t drows = kch * CK;
  if (tid < 2) {
    ext[tid] = 0;
    nzq[tid] = 0;
  }
  __syncthreads();
  int exa = 0, exb = 0;
  bool qa = false, qb = false;
  for (int64_t e = tid; e < drows * BNC; e += kBresThreads) {
    const int64_t kk = e / BNC;
    const int jj = (int)(e - kk * BNC);
    const bool hb = jj >= kBresTile;
    const int64_t cb = hb ? c0b : c0a;
    const int jt = hb ? jj - kBresTile : jj;
    const int64_t col = cb + jt;
    const double v = (cb >= 0 && kk < d && col < k) ? B[kk * k + col] : 0.0;
    Bs[kk * LDB + jj] = v;
    if (v != 0.0) {  // NaN counts as nonzero
      const bool quarter = jt < 16 && kk >= cb + 16 && kk < cb + kBresTile;
      if (hb) {
        exb = (int)kk + 1;
        qb = qb || quarter;
      } else {
        exa = (int)kk + 1;
        qa = qa || quarter;
      }
    }
  }
  if (exa) atomicMax(&ext[0], exa);
  if (exb) atomicMax(&ext[1], exb);
  if (qa) atomicOr(&nzq[0], 1);
  if (qb) atomicOr(&nzq[1], 1);
  __syncthreads();
  // K chunks each tile needs (uniform over the workgroup)
  const int64_t kca = __builtin_amdgcn_readfirstlane((ext[0] + CK - 1) / CK);
  const int64_t kcb = __builtin_amdgcn_readfirstlane((ext[1] + CK - 1) / CK);
  // the diagonal chunk of each tile (chunk index = tile index, a chunk
  // spanning one tile's rows) when its quarter is zero and its columns of A
  // are inside d; -1: none
  static_assert(CK == kBresTile, "a K chunk spans one tile's rows");
  const int64_t dga =
      (__builtin_amdgcn_readfirstlane(nzq[0]) || c0a + kBresTile > d) ? -1 : (int64_t)nt;
  const int64_t dgb =
      (c0b < 0 || __builtin_amdgcn_readfirstlane(nzq[1]) || c0b + kBresTile > d) ? -1 : tb;
  const int64_t ntiles = (n + kBresRows - 1) / kBresRows;
  for (int64_t t = group * kBresWaves + wave; t < ntiles; t += ngroups * kBresWaves) {
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
    // the chunk's KW elements of each of the lane's rows, loaded raw and
    // branch-free (Raw4: clamped address, values selected and widened in
    // step), so the next chunk's loads stay in flight during this one's
    // matrix instructions
    typedef Raw4<TA> RawChunk[MB][KW / 4];
    auto load = [&](int64_t c, RawChunk &a) __attribute__((always_inline)) {
      const int64_t kb = c * CK + KW * kq;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int q = 0; q < KW / 4; ++q)
          raw4_load<TA, VEC>(arow[mb], 0, d, 0, rin[mb], kb + 4 * q, a[mb][q]);
    };
    // one K chunk for the blocks of the tiles in HM (bit 0: first tile,
    // bit 1: second tile); DG 1 / 2: a diagonal chunk in the swapped order,
    // the first column block of the first / second tile skipping steps 4 .. 7
    // (every element inside A: no masks; a row past n reads row 0 and
    // feeds only its own outputs, which are not stored)
    auto step = [&](auto hm, auto dg, int64_t c, const RawChunk &raw)
                    __attribute__((always_inline)) {
      constexpr int HM = decltype(hm)::value;
      constexpr int DG = decltype(dg)::value;
      double a[MB][KW];
      if constexpr (DG == 0) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int s = 0; s < KW; ++s) a[mb][s] = raw4_get(raw[mb][s / 4], s % 4);
      } else {
        static_assert(KW == 8, "the swap pairs elements s and s + 4");
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const TA x = raw[mb][0].x[s], y = raw[mb][1].x[s];
            if constexpr (sizeof(TA) == 4) {
              const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x),
                                                              __float_as_uint(y), false, false);
              a[mb][s] = (double)__uint_as_float(r[0]);
              a[mb][4 + s] = (double)__uint_as_float(r[1]);
            } else {
              const uint64_t xb = (uint64_t)__double_as_longlong(x);
              const uint64_t yb = (uint64_t)__double_as_longlong(y);
              const auto rl = __builtin_amdgcn_permlane32_swap((uint32_t)xb, (uint32_t)yb, false,
                                                               false);
              const auto rh = __builtin_amdgcn_permlane32_swap((uint32_t)(xb >> 32),
                                                               (uint32_t)(yb >> 32), false, false);
              a[mb][s] = __longlong_as_double((long long)(((uint64_t)rh[0] << 32) | rl[0]));
              a[mb][4 + s] = __longlong_as_double((long long)(((uint64_t)rh[1] << 32) | rl[1]));
            }
          }
      }
#pragma unroll
      for (int s = 0; s < KW; ++s) {
        const int64_t kr = DG == 0 ? c * CK + KW * kq + s
                                   : c * CK + 16 * (s / 4) + 8 * (kq & 1) + 4 * (kq >> 1) + s % 4;
        const double *brow = Bs + kr * LDB + li;
        auto on = [&](int nb) {
          return ((HM >> (nb / NBH)) & 1) && !(DG && s >= 4 && nb == (DG - 1) * NBH);
        };
        double bv[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          if (on(nb)) bv[nb] = brow[nb * 16];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            if (on(nb))
              acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb][s], bv[nb], acc[mb][nb],
                                                                 0, 0, 0);
      }
    };
    using D0 = std::integral_constant<int, 0>;
    // chunks c0 .. c1 - 1, the next chunk's A loaded while one is multiplied.
    // The loads are unconditional (past the last chunk they reload it, and
    // the copy goes unused): with the same loads in flight on every path,
    // a step waits for its own chunk only, not for the one loading behind it.
    // A phase whose last chunk is the diagonal chunk of its first tile
    // (HM 3, 1) or of its second (HM 2) takes that chunk last, loaded in the
    // same pipeline (its loads are those of any chunk).
    auto run = [&](auto hm, int64_t c0, int64_t c1) __attribute__((always_inline)) {
      constexpr int HM = decltype(hm)::value;
      using DGT = std::integral_constant<int, HM == 2 ? 2 : 1>;
      if (c0 >= c1) return;
      const bool dg = c1 - 1 == (HM == 2 ? dgb : dga);
      const int64_t ce = dg ? c1 - 1 : c1;  // chunks before ce: all products
      const int64_t cl = c1 - 1;
      RawChunk a0, a1;
      load(c0, a0);
      int64_t c = c0;
      for (; c + 1 < ce; c += 2) {
        load(c + 1, a1);
        __builtin_amdgcn_sched_barrier(0);  // keep the next chunk's loads ahead of this step
        step(hm, D0{}, c, a0);
        load(c + 2 < c1 ? c + 2 : cl, a0);
        __builtin_amdgcn_sched_barrier(0);
        step(hm, D0{}, c + 1, a1);
      }
      // c = ce - 1: one more chunk (a0), the next one (the diagonal chunk,
      // or a reload) loading into a1 meanwhile; c = ce: a0 holds the
      // diagonal chunk when there is one
      const bool in1 = c < ce;
      if (in1) {
        load(c + 1 < c1 ? c + 1 : cl, a1);
        __builtin_amdgcn_sched_barrier(0);
        step(hm, D0{}, c, a0);
      }
      if (dg) {
        RawChunk ad;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int q = 0; q < KW / 4; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) ad[mb][q].x[e] = in1 ? a1[mb][q].x[e] : a0[mb][q].x[e];
        step(hm, DGT{}, ce, ad);
      }
    };
    using HBoth = std::integral_constant<int, 3>;
    using HA = std::integral_constant<int, 1>;
    using HB = std::integral_constant<int, 2>;
    if constexpr (PAIR) {
      const int64_t kboth = kca < kcb ? kca : kcb;
      run(HBoth{}, 0, kboth);
      if (kca > kboth) run(HA{}, kboth, kca);
      else if (kcb > kboth) run(HB{}, kboth, kcb);
    } else {
      run(HA{}, 0, kca);
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

// LDS-resident form for d: 2 paired tiles (64 columns) when k > 32 and they
// fit, else 1 tile of 32 columns; 0: the tile does not fit.
int bres_width(int64_t d, int64_t k) {
  const int64_t drows = ceil_div(d, (int64_t)(4 * kBresKW)) * (4 * kBresKW);
  if (k > kBresTile && drows * (2 * kBresTile + 4) * 8 <= 163840) return 2;
  if (drows * (kBresTile + 4) * 8 <= 163840) return 1;
  return 0;
}

template <typename TA, bool PAIR, bool VEC>
int bres_launch(const psk_mat &Am, const double *B, int64_t k, double *part, int tn,
                hipStream_t st) {
  const int64_t n = Am.n, d = Am.d;
  constexpr int BNC = PAIR ? 2 * kBresTile : kBresTile;
  const size_t lds =
      (size_t)ceil_div(d, (int64_t)(4 * kBresKW)) * (4 * kBresKW) * (BNC + 4) * sizeof(double);
  PSK_HIP_TRY(hipFuncSetAttribute((const void *)k_rownorm_bres<TA, PAIR, VEC>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  // one workgroup per CU (the LDS tile), row groups of tn workgroups per XCD
  const int64_t tiles = ceil_div(n, (int64_t)kBresRows);
  int64_t groups = 256 / tn;
  if (groups < 8) groups = 8;
  groups = (groups / 8) * 8;
  const int64_t need = ceil_div(tiles, (int64_t)kBresWaves);  // row tiles per wavefront round
  while (groups > 8 && groups / 2 >= need) groups /= 2;
  const unsigned nblk = (unsigned)(groups * tn);
  KTimer timer("rownorm", st);
  k_rownorm_bres<TA, PAIR, VEC><<<nblk, kBresThreads, lds, st>>>(
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
    // slots: pairs of 32-column tiles (bw 2) or single tiles (bw 1)
    const int64_t ntile = ceil_div(k, (int64_t)kBresTile);
    const int tn = (int)(bw == 2 ? ceil_div(ntile, (int64_t)2) : ntile);
    double *part = ws.take<double>((size_t)tn * n);
    if (ws.dry()) return 0;
    if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for row norms");
    // FP32 rows read four elements at a time when every such group is aligned
    const bool vec = Am.ld % 4 == 0 && d % 4 == 0 && ((uintptr_t)Am.values & 15) == 0;
    int rc;
    if constexpr (sizeof(TA) == 4) {
      if (bw == 2)
        rc = vec ? bres_launch<TA, true, true>(Am, B, k, part, tn, st)
                 : bres_launch<TA, true, false>(Am, B, k, part, tn, st);
      else
        rc = vec ? bres_launch<TA, false, true>(Am, B, k, part, tn, st)
                 : bres_launch<TA, false, false>(Am, B, k, part, tn, st);
    } else {
      (void)vec;
      rc = bw == 2 ? bres_launch<TA, true, false>(Am, B, k, part, tn, st)
                   : bres_launch<TA, false, false>(Am, B, k, part, tn, st);
    }
    if (rc) return rc;
    k_rownorm_reduce<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(part, n, tn, alpha, beta, x);
  } else if (k <= 64) {
    constexpr int BM = 32, BN = 64;
    const int tm = (int)ceil_div(n, BM), tn = (int)ceil_div(k, BN);
    double *part = ws.take<double>((size_t)tn * n);
    if (ws.dry()) return 0;
    if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for row norms");
    {
      KTimer timer("rownorm", st);
      k_dgemm<TA, double, false, false, 2, 2, 1, 2, EPI_ROWNORM, false>
          <<<(unsigned)((int64_t)tm * tn), 256, 0, st>>>(n, k, d, A, Am.ld, B, k, tm, tn, d,
                                                         part, n, 1.0, 0.0);
    }
    k_rownorm_reduce<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(part, n, tn, alpha,
                                                                  beta, x);
  } else {
    constexpr int BM = 32, BN = 256;
    const int tm = (int)ceil_div(n, BM), tn = (int)ceil_div(k, BN);
    double *part = ws.take<double>((size_t)tn * n);
    if (ws.dry()) return 0;
    if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for row norms");
    {
      KTimer timer("rownorm", st);
      k_dgemm<TA, double, false, false, 2, 2, 1, 8, EPI_ROWNORM, false>
          <<<(unsigned)((int64_t)tm * tn), 256, 0, st>>>(n, k, d, A, Am.ld, B, k, tm, tn, d,
                                                         part, n, 1.0, 0.0);
    }
    k_rownorm_reduce<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(part, n, tn, alpha,
                                                                  beta, x);
  }
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}


// ---------------------------------------------------------------------------
// Gram matrix of a dense tall A: C = A^T A as a sum over row slabs
// ---------------------------------------------------------------------------
// Each wavefront owns one 64 x 64 tile (I, J), I <= J, of the upper block
// triangle of C and one slab of consecutive rows of A, and accumulates that
// slab's contribution in registers (4 x 4 blocks of 16 x 16 FP64
// accumulators).  Lane (li, kq) = (lane % 16, lane / 16) reads, for row
// k0 + kq, the four consecutive columns 64 I + 4 li .. + 3 (one vector load)
// and the same four of the tile's J columns: component a of that load is
// row li of the MFMA operand block a, so block a of the tile holds the
// columns 64 I + 4 i + a, i = 0 .. 15 (and likewise for J).  Block (a, b)
// then accumulates C[64 I + 4 i + a][64 J + 4 j + b].  On a diagonal tile
// (I = J) block (b, a) is the transpose of block (a, b), so only a <= b are
// multiplied (10 of 16) and the others are mirrored when the tile is
// written: the executed products are those of the upper triangle at the
// 16 x 16 block level, n d (d + 16) flops for d a multiple of 64.
// Rows past the slab and columns past d read as zero.
// A diagonal tile does 10 of the 16 block products per row step, so its
// slabs are 1.6 times as long (rows_d against rows_o rows): every work item
// then costs about the same, and no SIMD waits on a pair of off-diagonal
// items while others finish early.  The off-diagonal items come first,
// (slab g / Uo, off-diagonal tile g % Uo), then the diagonal ones (slab,
// tile (g' % T, g' % T)); four per workgroup, and workgroups of the same
// XCD (linear ids equal mod 8) take consecutive items, so the tiles of one
// slab read its rows through one L2.  Slab s of tile t writes its 64 x 64
// partial (both triangles of a diagonal tile) to part at gram_part_off(t)
// + s 4096; k_gram_reduce1 sums each tile's slabs in order (no atomics).
// Row steps whose loads are in flight.  Four keep a wavefront at 208
// registers (its 128 accumulators and 80 VGPRs), so beside the kernel's two
// wavefronts per SIMD 96 registers stay free for the smaller kernels of a
// stream beside it (the sketch's binning, the QR's GEMMs at 54).  Eight run
// the Gram alone 4% faster (FP32 4e6 x 256: 4.71 ms at 4, 4.54 at 8) but
// take 240 and leave 32: the sketch-beside-Gram step then takes 11.33 ms
// against 11.17.
constexpr int kGramPF = 4;

// (I, J), I < J, of off-diagonal tile o in row-major order
__device__ __forceinline__ void gram_offdiag_tile(int o, int T, int &I, int &J) {
  I = 0;
  int rest = o;
  while (rest >= T - 1 - I) {
    rest -= T - 1 - I;
    ++I;
  }
  J = I + 1 + rest;
}

// first partial of tile (I, J) (row-major upper triangle): the diagonal
// tiles before it (I of them, one more when J > I) have sd slabs, the others
// so slabs
__host__ __device__ __forceinline__ int64_t gram_part_off(int I, int J, int T, int64_t so,
                                                          int64_t sd) {
  const int t = I * T - I * (I - 1) / 2 + (J - I);
  const int nd = I + (J > I ? 1 : 0);
  return ((int64_t)nd * sd + (int64_t)(t - nd) * so) * 4096;
}

template <typename TA, bool VEC>
__global__ __launch_bounds__(256) void k_gram_syrk(const TA *__restrict__ A, int64_t ld,
                                                   int64_t n, int64_t d, int T,
                                                   int64_t so, int64_t rows_o,
                                                   int64_t sd, int64_t rows_d,
                                                   double *__restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int64_t nblk = gridDim.x;
  int64_t lin = blockIdx.x;
  if ((nblk & 7) == 0) lin = (lin & 7) * (nblk >> 3) + (lin >> 3);
  const int64_t g = lin * 4 + wave;
  const int Uo = T * (T - 1) / 2;
  const int64_t no = so * Uo;
  if (g >= no + sd * T) return;
  int I, J;
  int64_t slab, rows_per;
  if (g < no) {
    slab = g / Uo;
    gram_offdiag_tile((int)(g - slab * Uo), T, I, J);
    rows_per = rows_o;
  } else {
    slab = (g - no) / T;
    I = J = (int)(g - no - slab * T);
    rows_per = rows_d;
  }
  const bool diag = I == J;
  const int64_t k_begin = slab * rows_per;
  int64_t k_end = k_begin + rows_per;
  if (k_end > n) k_end = n;
  const int64_t ci = (int64_t)I * 64 + 4 * li, cj = (int64_t)J * 64 + 4 * li;
  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  auto run = [&](auto dg) __attribute__((always_inline)) {
    constexpr bool DG = decltype(dg)::value;
    Raw4<TA> xa[kGramPF], xb[kGramPF];
    auto fetch = [&](int p, int64_t k0) __attribute__((always_inline)) {
      const int64_t row = k0 + kq;
      const bool rok = row < k_end;
      raw4_load<TA, VEC>(A, ld, d, rok ? row : 0, rok, ci, xa[p]);
      if constexpr (!DG) raw4_load<TA, VEC>(A, ld, d, rok ? row : 0, rok, cj, xb[p]);
    };
#pragma unroll
    for (int p = 0; p < kGramPF; ++p) fetch(p, k_begin + 4 * p);
    for (int64_t k0 = k_begin; k0 < k_end; k0 += 4 * kGramPF) {
#pragma unroll
      for (int p = 0; p < kGramPF; ++p) {
        double av[4], bv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          av[q] = raw4_get(xa[p], q);
          bv[q] = DG ? av[q] : raw4_get(xb[p], q);
        }
        fetch(p, k0 + 4 * (p + kGramPF));
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (!DG || a <= b)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
  };
  if (diag) run(std::true_type{});
  else run(std::false_type{});
  // lane (li, kq) holds rows kq + 4 e, column li of each block: the tile's
  // local element (4 (kq + 4 e) + a, 4 li + b)
  double *o = part + gram_part_off(I, J, T, so, sd) + slab * 4096;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (diag && a > b) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int pr = 4 * (kq + 4 * e) + a, pc = 4 * li + b;
        o[pr * 64 + pc] = acc[a][b][e];
        if (diag && a < b) o[pc * 64 + pr] = acc[a][b][e];
      }
    }
}

// First level of the slab sum: group q of kGramGroups sums its slabs in
// order, gpart[q][p][c] for the d x d output, taken from the upper tile
// (transposed for p > c).
constexpr int kGramGroups = 16;

__global__ __launch_bounds__(256) void k_gram_reduce1(const double *__restrict__ part,
                                                      int64_t d, int T, int64_t so, int64_t sd,
                                                      double *__restrict__ gpart) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t q = blockIdx.y;
  if (e >= d * d) return;
  int64_t p = e / d, c = e % d;
  if (p / 64 > c / 64) {
    const int64_t x = p;
    p = c;
    c = x;
  }
  const int I = (int)(p / 64), J = (int)(c / 64);
  const int64_t slabs = I == J ? sd : so;
  const int64_t off = gram_part_off(I, J, T, so, sd) + (p % 64) * 64 + (c % 64);
  const int64_t s0 = slabs * q / kGramGroups, s1 = slabs * (q + 1) / kGramGroups;
  double acc = 0.0;
  for (int64_t s = s0; s < s1; ++s) acc += part[off + s * 4096];
  gpart[q * d * d + e] = acc;
}

// C = alpha * sum of the groups (in order) + beta * C (beta == 0 ignores C)
template <typename TO>
__global__ __launch_bounds__(256) void k_gram_reduce2(const double *__restrict__ gpart,
                                                      int64_t dd, double alpha, double beta,
                                                      TO *__restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= dd) return;
  double acc = gpart[e];
#pragma unroll
  for (int q = 1; q < kGramGroups; ++q) acc += gpart[q * dd + e];
  double v = alpha * acc;
  if (beta != 0.0) v += beta * (double)C[e];
  C[e] = (TO)v;
}

template <typename TA>
int gram_syrk_launch(double alpha, const psk_mat &Am, double beta, void *C, bool out_f32,
                     Arena &ws, hipStream_t st) {
  const int64_t n = Am.n, d = Am.d;
  const int T = (int)ceil_div(d, (int64_t)64);
  const int Uo = T * (T - 1) / 2;
  const uintptr_t addr = (uintptr_t)Am.values;
  const bool vec = (Am.ld % 4 == 0) && (d % 4 == 0) && (addr % 16 == 0);
  // about two wavefronts per SIMD in one round: 2048 work items of equal
  // cost, a diagonal item 10/16 of an off-diagonal one per row; slabs of
  // whole loop iterations
  constexpr int64_t kStep = 4 * kGramPF;
  int64_t so = (int64_t)(2048.0 / (Uo + 0.625 * T));
  if (so < 8) so = 8;
  const int64_t rows_o = ceil_div(ceil_div(n, so), kStep) * kStep;
  so = ceil_div(n, rows_o);
  const int64_t rows_d = ceil_div((rows_o * 16) / 10, kStep) * kStep;
  const int64_t sd = ceil_div(n, rows_d);
  double *part = ws.take<double>((size_t)(so * Uo + sd * T) * 4096);
  double *gpart = ws.take<double>((size_t)kGramGroups * d * d);
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for the Gram matrix");
  const int64_t items = so * Uo + sd * T;
  int64_t nblk = ceil_div(items, (int64_t)4);
  nblk = ceil_div(nblk, (int64_t)8) * 8;  // whole XCD rounds for the remap
  {
    KTimer timer("gram", st);
    if (vec)
      k_gram_syrk<TA, true><<<(unsigned)nblk, 256, 0, st>>>((const TA *)Am.values, Am.ld, n, d,
                                                            T, so, rows_o, sd, rows_d, part);
    else
      k_gram_syrk<TA, false><<<(unsigned)nblk, 256, 0, st>>>((const TA *)Am.values, Am.ld, n, d,
                                                             T, so, rows_o, sd, rows_d, part);
  }
  KTimer rtimer("gram_reduce", st);
  const int64_t dd = d * d;
  dim3 g1((unsigned)ceil_div(dd, (int64_t)256), kGramGroups);
  k_gram_reduce1<<<g1, 256, 0, st>>>(part, d, T, so, sd, gpart);
  if (out_f32)
    k_gram_reduce2<float><<<(unsigned)ceil_div(dd, (int64_t)256), 256, 0, st>>>(
        gpart, dd, alpha, beta, (float *)C);
  else
    k_gram_reduce2<double><<<(unsigned)ceil_div(dd, (int64_t)256), 256, 0, st>>>(
        gpart, dd, alpha, beta, (double *)C);
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
  if (A.dtype == PSK_F32) return gram_syrk_launch<float>(alpha, A, beta, C, !out_f64, ws, st);
  return gram_syrk_launch<double>(alpha, A, beta, C, false, ws, st);
}

int rownorms_dense(double alpha, const psk_mat &A, const double *B, int64_t k,
                   double beta, double *x, Arena &ws, hipStream_t st) {
  if (A.dtype == PSK_F32) return rownorm_launch<float>(A, B, k, alpha, beta, x, ws, st);
  return rownorm_launch<double>(A, B, k, alpha, beta, x, ws, st);
}

}  // namespace psk
