// C = G * (S*A) for CSR A over the nonzeros of S*A only.
//
// Paper mapping (arXiv 2203.02798): Algorithm countgauss_multiply's product
// C = G (S A), evaluated as C = sum_b G[:, b] (S A)[b, :], the sum running
// over the nonzero entries of S*A (the (G S) A form of the sparse sketches).
// A CountSketch of a sparse matrix has few nonzeros per bucket row (about
// nnz(A) / r), so this costs 2 m nnz(S A) flops instead of the dense
// product's 2 m r d, besides drawing the m x r Gaussian once.  The result is
// the same product in the same precision as the dense kernels:
//   FP64  G and S*A in FP64;
//   BF16  G rounded to bfloat16, S*A as its two bfloat16 limbs hi + lo;
//   FP8   both in OCP e4m3: S*A with one E8M0 scale per 128-bucket block
//         of each column, G with the fixed scale 2^-6.
// Only the 4-bucket quads of G that meet an entry of S*A are drawn: with
// counter-based normals and G's rounding decided per value, the others are
// never needed.  The product walks G in blocks of QB such quads (QB = 128,
// 64 with G in FP64) taken from the list of occupied quads in bucket order,
// so the number of blocks follows the nonzeros of S*A, not r.
// FP64 accumulates in FP64.  BF16 and FP8 accumulate in FP32 within a K
// split, as the dense reduced-precision kernels do (each product is exact
// inside the FMA; BF16's value hi + lo is rounded to FP32 where its limbs
// span more than 24 bits), and the split partials are summed in FP64.
//
// Steps (all on the binned rows of cs_bin):
//   k_row_nnz + scan   offsets: bucket b's entries occupy slots
//                      eoff[bptr[b]] .. eoff[bptr[b+1]] (its rows' lengths);
//   k_sa_entries       a lane per bucket sums the bucket's rows in
//                      registers (the CountSketch scatter's order, so the
//                      same bits as S*A; longer buckets through a dense LDS
//                      row per wavefront) and writes its nonzeros (bucket,
//                      column, value) in column order into its slots, the
//                      unused slots as holes (column -1);
//   k_entries_fp8      (FP8) the per-column, per-128-bucket scale and the
//                      e4m3 rounding of the values;
//   k_quad_flags + scan  the rank of every occupied 4-bucket quad;
//   k_quad_list        the occupied quads in order, the G blocks of QB of
//                      them, each block's first entry slot, the count;
//   k_block_csc        each G block's entries sorted by (column, slot of
//                      their bucket in the block: 4 rank + bucket mod 4),
//                      packed with their column's run length;
//   k_gauss_sparse     workgroup (32- or 16-row tile of C, a range of G
//                      blocks): per block it draws G for its rows into LDS
//                      and stages the block's entries; each thread adds the
//                      entries of its column into its rows of C, held in
//                      registers; the tile goes out as one K-split partial;
//   k_sparse_reduce    C = (1/sqrt m) sum of the partials in split order.
#include <type_traits>

#include "internal.hpp"

namespace psk {
namespace {

constexpr int kBlk = 128;  // buckets per FP8 scale block

// rn[j] = number of entries of the row at bin position j; 0 at and past
// the binned count bptr[r] (at most n; rows without entries are not binned)
__global__ __launch_bounds__(256) void k_row_nnz(const int64_t *__restrict__ indptr,
                                                 const uint32_t *__restrict__ perm,
                                                 const uint32_t *__restrict__ bptr, int64_t r,
                                                 int64_t n, uint32_t *__restrict__ rn) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j > n) return;
  uint32_t v = 0;
  if (j < (int64_t)bptr[r]) {
    const int64_t row = (int64_t)(perm[j] & 0x7fffffffu);
    v = (uint32_t)(indptr[row + 1] - indptr[row]);
  }
  rn[j] = v;
}

// qf[q] = 1 when quad q (buckets 4q .. 4q + 3) holds an entry, else 0;
// qf[nquads] = 0 (an exclusive scan then gives ranks and the count)
__global__ __launch_bounds__(256) void k_quad_flags(const uint32_t *__restrict__ bptr,
                                                    const uint32_t *__restrict__ eoff, int64_t r,
                                                    int64_t nquads, uint32_t *__restrict__ qf) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q > nquads) return;
  uint32_t f = 0u;
  if (q < nquads) {
    const int64_t b0 = 4 * q, b1 = b0 + 4 < r ? b0 + 4 : r;
    f = eoff[bptr[b1]] > eoff[bptr[b0]] ? 1u : 0u;
  }
  qf[q] = f;
}

// From the scanned flags (qrank[q] = occupied quads before q, qrank[nquads]
// = their count): qlist[rank] = q for every occupied quad; G block s holds
// ranks QB s .. QB s + QB - 1 and its entries start at slot be[s] (the
// quads between two occupied ones own no slots); be[blocks] = all slots.
__global__ __launch_bounds__(256) void k_quad_list(const uint32_t *__restrict__ bptr,
                                                   const uint32_t *__restrict__ eoff,
                                                   const uint32_t *__restrict__ qrank, int64_t r,
                                                   int64_t nquads, int qb,
                                                   uint32_t *__restrict__ qlist,
                                                   uint32_t *__restrict__ be) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q > nquads) return;
  if (q == nquads) {
    const uint32_t nb = (qrank[nquads] + (uint32_t)qb - 1u) / (uint32_t)qb;
    be[nb] = eoff[bptr[r]];
    return;
  }
  const uint32_t rk = qrank[q];
  if (qrank[q + 1] == rk) return;  // empty quad
  qlist[rk] = (uint32_t)q;
  if (rk % (uint32_t)qb == 0u) be[rk / (uint32_t)qb] = eoff[bptr[4 * q]];
}

// bfloat16 (RNE) of a double in one rounding (round-to-odd to FP32 first)
__device__ __forceinline__ double bf16_round(double v) {
  if (v != v) return v;
  float f = (float)v;
  if ((double)f != v) {
    uint32_t b = __float_as_uint(f);
    if (fabs((double)f) > fabs(v)) b -= 1;
    b |= 1u;
    f = __uint_as_float(b);
  }
  return (double)(float)(__bf16)f;
}

// exponent e of the E8M0 block scale: smallest integer with 448 * 2^e >= amax
// (amax = f 2^x, f in [1/2, 1); 448 = 0.875 2^9), 0 for amax == 0 or not
// finite, clamped
__device__ __forceinline__ int e8m0_exp(double amax) {
  int x;
  const double f = frexp(amax, &x);
  int e = (f <= 0.875) ? x - 9 : x - 8;
  if (!(amax > 0.0 && amax <= 1.7976931348623157e308)) e = 0;
  return e < -127 ? -127 : (e > 127 ? 127 : e);
}

// e4m3 (OCP, RNE) of v 2^-e, returned as its value times 2^e; v 2^-e goes
// to FP32 by round-to-odd first, so the e4m3 rounding is a single one
__device__ __forceinline__ double e4m3_round(double v, int e) {
  const double x = ldexp(v, -e);
  float f = (float)x;
  if ((double)f != x && x == x) {
    uint32_t b = __float_as_uint(f);
    if (fabs((double)f) > fabs(x)) b -= 1;
    b |= 1u;
    f = __uint_as_float(b);
  }
  f = fabsf(f) <= 3.4028234663852886e38f ? f : __builtin_nanf("");  // non-finite: NaN
  const int byte = __builtin_amdgcn_cvt_pk_fp8_f32(f, 0.0f, 0, false) & 0xff;
  return ldexp((double)__builtin_amdgcn_cvt_f32_fp8(byte, 0), e);
}

// The value written for an S*A entry: BF16 keeps hi + lo, its two limbs
template <bool LIMBS>
__device__ __forceinline__ double entry_value(double v) {
  if (!LIMBS) return v;
  const double hi = bf16_round(v);
  return hi + bf16_round(v - hi);
}

// Bucket b's S*A entries through a dense LDS row of d (one wavefront): its
// rows summed in the CountSketch scatter's order, the nonzeros written in
// column order into the slots e0 .. e0 + cap, the rest as holes.
template <typename T, bool LIMBS>
__device__ void bucket_entries_wave(const T *__restrict__ vals, const int64_t *__restrict__ indptr,
                                    const int32_t *__restrict__ indices,
                                    const uint32_t *__restrict__ perm, uint32_t j0, uint32_t j1,
                                    uint32_t e0, uint32_t cap, int64_t b, int64_t d,
                                    int64_t dpad, double scale, double *acc,
                                    uint32_t *__restrict__ eb, int32_t *__restrict__ ec,
                                    double *__restrict__ ev) {
  const int lane = (int)(threadIdx.x & 63u);
  for (int64_t c = lane; c < dpad; c += 64) acc[c] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  bucket_rows_add(vals, indptr, indices, perm, j0, j1, acc);
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  uint32_t cnt = 0;
  for (int64_t c0 = 0; c0 < d; c0 += 64) {
    const int64_t c = c0 + lane;
    const double v = c < d ? acc[c] : 0.0;
    const bool nz = v != 0.0;
    const uint64_t mask = __ballot(nz);
    if (nz) {
      const uint32_t pos = e0 + cnt + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
      eb[pos] = (uint32_t)b;
      ec[pos] = (int32_t)c;
      ev[pos] = entry_value<LIMBS>(v * scale);
    }
    cnt += (uint32_t)__popcll(mask);
  }
  for (uint32_t p = cnt + lane; p < cap; p += 64) {
    eb[e0 + p] = (uint32_t)b;
    ec[e0 + p] = -1;
    ev[e0 + p] = 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();  // acc is reused by the wavefront's next bucket
}

constexpr int kLaneEnt = 8;  // entries a bucket may have for the lane path

// S*A entries of buckets 256 blockIdx.x .. +255, a lane per bucket: the
// bucket's rows (at most kLaneEnt entries in all) are added into a list of
// (column, value) in registers, row after row in list order, so each value
// is summed in the CountSketch scatter's order and has the same bits as
// S*A; the list is sorted by column and its nonzeros written in that order,
// then the holes.  Buckets with more entries are taken afterwards, one at a
// time, by their wavefront through a dense LDS row (bucket_entries_wave).
// BF16: the value written is hi + lo (the two limbs); otherwise S*A itself.
// Each bucket's sum is multiplied by scale once (1 for CountSketch, 1/sqrt(s)
// for an OSNAP's bins of (row, non-zero) pairs), as S*A itself is formed.
template <typename T, bool LIMBS>
__global__ __launch_bounds__(256) void k_sa_entries(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, int64_t d, int64_t dpad, int64_t r,
    const uint32_t *__restrict__ perm, const uint32_t *__restrict__ bptr,
    const uint32_t *__restrict__ eoff, double scale, uint32_t *__restrict__ eb,
    int32_t *__restrict__ ec, double *__restrict__ ev) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = (int)(threadIdx.x & 63u);
  double *acc = reinterpret_cast<double *>(smem_raw) + (int64_t)(threadIdx.x >> 6) * dpad;
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  uint32_t j0 = 0, j1 = 0, e0 = 0, cap = 0;
  if (b < r) {
    j0 = bptr[b];
    j1 = bptr[b + 1];
    e0 = eoff[j0];
    cap = eoff[j1] - e0;
  }
  const bool lng = cap > (uint32_t)kLaneEnt;
  if (cap > 0 && !lng) {
    int col[kLaneEnt];
    double val[kLaneEnt];  // FP64 sums, FP32 entries widened exactly
#pragma unroll
    for (int k = 0; k < kLaneEnt; ++k) {
      col[k] = INT32_MAX;
      val[k] = 0.0;
    }
    int n = 0;
    for (uint32_t j = j0; j < j1; ++j) {
      const uint32_t pv = perm[j];
      const int64_t row = (int64_t)(pv & 0x7fffffffu);
      const bool ng = (pv >> 31) != 0u;
      const int64_t p1 = indptr[row + 1];
      for (int64_t p = indptr[row]; p < p1; ++p) {
        const int32_t c = indices[p];
        const double v0 = (double)vals[p];
        const double v = ng ? -v0 : v0;
        bool hit = false;
#pragma unroll
        for (int k = 0; k < kLaneEnt; ++k)
          if (col[k] == c) {
            val[k] += v;
            hit = true;
          }
        if (!hit) {
#pragma unroll
          for (int k = 0; k < kLaneEnt; ++k)
            if (k == n) {
              col[k] = c;
              val[k] = v;
            }
          ++n;
        }
      }
    }
    // sort by column (odd-even transposition; unused slots hold INT32_MAX)
#pragma unroll
    for (int ph = 0; ph < kLaneEnt; ++ph)
#pragma unroll
      for (int k = ph & 1; k + 1 < kLaneEnt; k += 2)
        if (col[k] > col[k + 1]) {
          const int tc = col[k];
          col[k] = col[k + 1];
          col[k + 1] = tc;
          const double tv = val[k];
          val[k] = val[k + 1];
          val[k + 1] = tv;
        }
    uint32_t pos = 0;
#pragma unroll
    for (int k = 0; k < kLaneEnt; ++k) {
      const double v = (double)val[k];
      if (k < n && v != 0.0) {
        eb[e0 + pos] = (uint32_t)b;
        ec[e0 + pos] = col[k];
        ev[e0 + pos] = entry_value<LIMBS>(v * scale);
        ++pos;
      }
    }
    for (; pos < cap; ++pos) {
      eb[e0 + pos] = (uint32_t)b;
      ec[e0 + pos] = -1;
      ev[e0 + pos] = 0.0;
    }
  }
  uint64_t lm = __ballot(lng);
  while (lm) {
    const int i = __ffsll((unsigned long long)lm) - 1;
    lm &= lm - 1;
    const uint32_t bj0 = __shfl(j0, i, 64), bj1 = __shfl(j1, i, 64);
    const uint32_t be0 = __shfl(e0, i, 64), bcap = __shfl(cap, i, 64);
    const int64_t bb = b - lane + i;
    bucket_entries_wave<T, LIMBS>(vals, indptr, indices, perm, bj0, bj1, be0, bcap, bb, d, dpad,
                                  scale, acc, eb, ec, ev);
  }
}

// FP8: entry values of 128-bucket block blockIdx.x rounded to e4m3 with the
// scale of their column in that block (amax over the block's entries of the
// column, taken exactly with integer max on the bit patterns).
__global__ __launch_bounds__(256) void k_entries_fp8(const uint32_t *__restrict__ bptr,
                                                     const uint32_t *__restrict__ eoff,
                                                     int64_t r, int64_t d,
                                                     const int32_t *__restrict__ ec,
                                                     double *__restrict__ ev) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned long long *amax = reinterpret_cast<unsigned long long *>(smem_raw);  // d
  const int64_t b0 = (int64_t)blockIdx.x * kBlk;
  const int64_t b1 = b0 + kBlk < r ? b0 + kBlk : r;
  const uint32_t e0 = eoff[bptr[b0]], e1 = eoff[bptr[b1]];
  for (int64_t c = threadIdx.x; c < d; c += 256) amax[c] = 0ull;
  __syncthreads();
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int32_t c = ec[e];
    if (c >= 0)
      atomicMax(&amax[c], (unsigned long long)__double_as_longlong(fabs(ev[e])));
  }
  __syncthreads();
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int32_t c = ec[e];
    if (c >= 0) {
      const int ex = e8m0_exp(__longlong_as_double((long long)amax[c]));
      ev[e] = e4m3_round(ev[e], ex);
    }
  }
}

// Packed sorted entry: column (bits 0-9), bucket offset in its G block
// (10-18), entries of the column left in the block counting this one
// (19-28), first entry of the column in the block (29); kHole for none.
constexpr uint32_t kHole = 0xffffffffu;
constexpr int kCscCols = 1024;  // columns of S*A the block sort takes at most

// Entries of G block blockIdx.x (8 W occupied quads, slots be[k] ..
// be[k+1]) in (column, bucket) order: the valid ones first, packed, then
// the holes.  A bucket's place in the block is 4 (rank of its quad in the
// block) + bucket mod 4, below 32 W.  Each bucket holds a column at most
// once, so an entry's place among its column's entries is the number of the
// column's buckets before its own: a bitmap of buckets per column, its
// popcounts and a scan over the columns give every entry its slot, with no
// dependence on timing.  Blocks past the count (qrank[nquads] quads) exit.
template <int W, typename VT>
__global__ __launch_bounds__(512) void k_block_csc(const uint32_t *__restrict__ be,
                                                   const uint32_t *__restrict__ eb,
                                                   const int32_t *__restrict__ ec,
                                                   const double *__restrict__ ev, int64_t d,
                                                   const uint32_t *__restrict__ qrank,
                                                   int64_t nquads,
                                                   uint32_t *__restrict__ sp,
                                                   VT *__restrict__ sv) {
  __shared__ uint32_t bits[kCscCols * W];   // [column][word]: buckets present
  __shared__ uint16_t wpre[kCscCols * W];   // buckets present in the words before
  __shared__ uint32_t ccnt[kCscCols];       // entries per column
  __shared__ uint32_t cst[kCscCols];        // exclusive scan of ccnt
  const int tid = threadIdx.x;
  const int64_t k = blockIdx.x;
  const uint32_t nblk = (qrank[nquads] + (uint32_t)(8 * W) - 1u) / (uint32_t)(8 * W);
  if ((uint32_t)k >= nblk) return;
  const uint32_t lo = be[k], hi = be[k + 1];
  const uint32_t r0 = (uint32_t)(k * (8 * W));  // rank of the block's first quad
  // slot of bucket b in the block
  auto slot_of = [&](uint32_t b) { return 4u * (qrank[b >> 2] - r0) + (b & 3u); };
  for (int64_t i = tid; i < d * W; i += 512) bits[i] = 0u;
  __syncthreads();
  for (uint32_t e = lo + tid; e < hi; e += 512) {
    const int32_t c = ec[e];
    if (c >= 0) {
      const uint32_t bo = slot_of(eb[e]);
      atomicOr(&bits[c * W + (bo >> 5)], 1u << (bo & 31));
    }
  }
  __syncthreads();
  for (int64_t c = tid; c < d; c += 512) {
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      wpre[c * W + w] = (uint16_t)run;
      run += (uint32_t)__popc(bits[c * W + w]);
    }
    ccnt[c] = run;
  }
  __syncthreads();
  if (tid < 64) {  // one wavefront scans the column counts
    const int64_t per = ceil_div(d, (int64_t)64);
    const int64_t c0 = tid * per, c1 = c0 + per < d ? c0 + per : d;
    uint32_t s = 0;
    for (int64_t c = c0; c < c1; ++c) s += ccnt[c];
    uint32_t x = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (tid >= off) x += y;
    }
    uint32_t ex = x - s;
    for (int64_t c = c0; c < c1; ++c) {
      cst[c] = ex;
      ex += ccnt[c];
    }
  }
  __syncthreads();
  for (uint32_t e = lo + tid; e < hi; e += 512) {
    const int32_t c = ec[e];
    if (c >= 0) {
      const uint32_t bo = slot_of(eb[e]), w = bo >> 5;
      const uint32_t rank =
          wpre[c * W + w] + (uint32_t)__popc(bits[c * W + w] & ((1u << (bo & 31)) - 1u));
      const uint32_t pos = lo + cst[c] + rank;
      sp[pos] = (uint32_t)c | (bo << 10) | ((ccnt[c] - rank) << 19) | ((rank == 0u) << 29);
      sv[pos] = (VT)ev[e];
    }
  }
  const uint32_t nv = cst[d - 1] + ccnt[d - 1];
  for (uint32_t p = lo + nv + tid; p < hi; p += 512) {
    sp[p] = kHole;
    sv[p] = VT(0);
  }
}

// G precision of the sparse product
enum { kG64 = 0, kGbf16 = 1, kGfp8 = 2 };

constexpr int kSThreads = 1024;
// entries of a block staged in LDS at once: 2048 with FP64 values, 4096
// with FP32 ones (the same registers per thread)
constexpr int kStageMax = 4 * kSThreads;
// A column with more than kHeavy entries in a staged turn (a dense column
// of A, or b appended to A) is summed by all threads together; a turn holds
// at most kStageMax / (kHeavy + 1) < kHeavyMax such columns, so the list never
// overflows and which columns take that path depends on the data alone.
constexpr int kHeavy = 32;
constexpr int kHeavyMax = 128;
static_assert(kStageMax / (kHeavy + 1) < kHeavyMax, "heavy list capacity");

// Workgroup (row tile mt, K split ks), 1024 threads: rows a0 .. a0 + MT of
// C (MT = 16 1024 / DP) and the G blocks ks bper .. ks bper + bper - 1, a
// block being QB = BLK / 4 occupied quads of buckets (BLK = 512 with G in
// FP32, 256 with G in FP64; bper from the number of blocks, read here).
// Thread (h, j) = (tid / DP, tid % DP) holds C[a0 + 16 h + i, j], i < 16, in
// FP64 registers.  Per block: every thread draws its share of
// the block of G into LDS (bucket-major, so one bucket's MT values are
// contiguous); the block's entries, sorted by (column, bucket), are staged
// in LDS with, per column, the range of its entries; thread (h, j) then
// adds G[a, b] s for the entries (b, j, s) of its column in bucket order
// (FP64, or FP32 when G is drawn in FP32).
// So each element of C is summed by one thread, over buckets in ascending
// order, with no atomics.  Entries are fetched two blocks ahead, the block
// bounds three; a block of more than KS entries is staged in turns.
template <int GP, int DP, int BLK>
__global__ __launch_bounds__(kSThreads) void k_gauss_sparse(
    int64_t m, int64_t d, int64_t r, uint64_t seed, const uint32_t *__restrict__ be,
    const uint32_t *__restrict__ sp, const void *__restrict__ sv_raw,
    const uint32_t *__restrict__ qlist, const uint32_t *__restrict__ nqp, int tiles_m,
    double *__restrict__ part /* [splits][m][d] */) {
  typedef typename std::conditional<GP == kG64, double, float>::type GT;
  typedef GT AT;  // accumulator and staged value: FP64, or FP32 with G in FP32
  constexpr int KS = sizeof(AT) == 4 ? kStageMax : kStageMax / 2;
  const AT *__restrict__ sv = reinterpret_cast<const AT *>(sv_raw);  // the sorted values
  constexpr int RG = kSThreads / DP;                // row groups
  constexpr int MT = 16 * RG;                       // tile rows
  constexpr int GS = MT + 16 / (int)sizeof(GT);     // LDS stride of a bucket of G
  constexpr int kQ = BLK / 4;                       // quads (Philox blocks) per G block
  constexpr int NIT = MT * kQ / kSThreads;          // G items per thread
  static_assert(NIT >= 1 && MT * kQ % kSThreads == 0, "whole G items per thread");
  static_assert(kQ <= kSThreads, "one thread per quad of the block's list");
  __shared__ __align__(16) GT Gb[BLK * GS];
  __shared__ uint32_t stp[KS];
  __shared__ AT stv[KS];
  __shared__ uint2 crng[DP];  // per column: tag, first staged slot | count << 16
  // heavy columns of the turn: column, first slot | count << 16; the count
  // alternates with the turn's parity so that it is cleared a turn ahead
  __shared__ uint2 hlist[kHeavyMax];
  __shared__ uint32_t hcnt[2];
  constexpr int NSTR = kSThreads / MT;  // entry streams of a heavy column
  __shared__ AT hred[NSTR * MT];
  const int tid = threadIdx.x;
  const int mt = (int)(blockIdx.x % tiles_m);
  const int64_t ks = blockIdx.x / tiles_m;
  const int64_t splits = gridDim.x / tiles_m;
  const int64_t a0 = (int64_t)mt * MT;
  const int64_t nq = (int64_t)nqp[0];  // occupied quads
  const int64_t nblk = ceil_div(nq, (int64_t)kQ);
  const int64_t bper = ceil_div(nblk, splits);
  const int64_t k0 = ks * bper < nblk ? ks * bper : nblk;
  const int64_t k1 = k0 + bper < nblk ? k0 + bper : nblk;
  const int j = tid % DP, h = tid / DP;
  for (int i = tid; i < DP; i += kSThreads) crng[i] = make_uint2(kHole, 0u);
  if (tid < 2) hcnt[tid] = 0u;
  AT acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = AT(0);
  uint32_t tag = 0;  // one per staged turn, never kHole
  // block bounds, loaded per lane (through vz, a zero the compiler cannot
  // see) so that they join the entries in the in-order vector load counter
  struct Bnd {
    uint32_t lo, hi;
  };
  struct ESet {
    uint32_t p[KS / kSThreads];
    AT v[KS / kSThreads];
    uint32_t lo, hi;
  };
  int vz;
  asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
  auto bounds = [&](int64_t k, Bnd &B) {
    B.lo = be[(k < k1 ? k : k1) + vz];
    B.hi = be[(k + 1 < k1 ? k + 1 : k1) + vz];
  };
  // the quads of the next blocks in an LDS ring of four: quad i of block k
  // (0 past the split) is loaded by thread i three steps ahead and stored at
  // the end of the step's draw, before its barrier
  __shared__ uint32_t qring[4][kQ];
  auto quad_of = [&](int64_t k) -> uint32_t {
    const int64_t e = k * kQ + tid;
    const int64_t ec2 = e < nq ? e : (nq > 0 ? nq - 1 : 0);
    const uint32_t q = qlist[ec2];
    return (k < k1 && e < nq) ? q : 0u;
  };
  auto load = [&](uint32_t base, uint32_t hi, uint32_t *pp, AT *vv) {
#pragma unroll
    for (int s2 = 0; s2 < KS / kSThreads; ++s2) {
      const uint32_t e = base + (uint32_t)(tid + kSThreads * s2);
      const uint32_t ei = e < hi ? e : (hi ? hi - 1 : 0u);  // clamped; masked when staged
      pp[s2] = sp[ei];
      vv[s2] = sv[ei];
    }
  };
  auto fetch = [&](const Bnd &B, ESet &R) {
    load(B.lo, B.hi, R.p, R.v);
    R.lo = B.lo;
    R.hi = B.hi;
  };
  // stage one turn (nch entries) and its column ranges; barrier before and after
  auto stage = [&](const uint32_t *pp, const AT *vv, uint32_t nch)
                   __attribute__((always_inline)) {
#pragma unroll
    for (int s2 = 0; s2 < KS / kSThreads; ++s2) {
      const int idx = tid + kSThreads * s2;
      const uint32_t pv = (uint32_t)idx < nch ? pp[s2] : kHole;
      stp[idx] = pv;
      stv[idx] = vv[s2];
      if (pv != kHole && (((pv >> 29) & 1u) || idx == 0)) {
        const uint32_t left = (pv >> 19) & 1023u;
        const uint32_t room = nch - (uint32_t)idx;
        const uint32_t cnt = left < room ? left : room;
        const uint32_t rng = (uint32_t)idx | (cnt << 16);
        if (cnt > (uint32_t)kHeavy) {
          // all threads sum it in consume; its owner skips it (no tag is
          // kHole, this turn's or a later one's)
          const uint32_t k = atomicAdd(&hcnt[tag & 1u], 1u);
          hlist[k] = make_uint2(pv & 1023u, rng);
          crng[pv & 1023u] = make_uint2(kHole, 0u);
        } else {
          crng[pv & 1023u] = make_uint2(tag, rng);
        }
      }
    }
  };
  auto consume = [&]() __attribute__((always_inline)) {
    const uint2 cr = crng[j];
    if (cr.x == tag) {
      const int s0 = (int)(cr.y & 0xffffu), s1 = s0 + (int)(cr.y >> 16);
      for (int i = s0; i < s1; ++i) {
        const uint32_t pv = stp[i];
        const AT v = stv[i];
        const GT *gp = Gb + ((pv >> 10) & 511u) * GS + 16 * h;
        GT gv[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) gv[t] = gp[t];
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] = fma(gv[t], v, acc[t]);
      }
    }
    // heavy columns: thread (stream st, row a) takes the column's entries
    // st, st + NSTR, ... for row a; the streams' sums are added to the
    // owners' accumulators in stream order
    const uint32_t nh = hcnt[tag & 1u];
    if (tid == 0) hcnt[(tag & 1u) ^ 1u] = 0u;  // the next turn's count
    const int ha = tid % MT, hs = tid / MT;
#pragma unroll 1
    for (uint32_t q = 0; __builtin_expect(q < nh, 0); ++q) {
      const uint2 hv = hlist[q];
      const int s0 = (int)(hv.y & 0xffffu), s1 = s0 + (int)(hv.y >> 16);
      AT part = AT(0);
#pragma unroll 1
      for (int i = s0 + hs; i < s1; i += NSTR) {
        const uint32_t pv = stp[i];
        part = fma((AT)Gb[((pv >> 10) & 511u) * GS + ha], stv[i], part);
      }
      hred[hs * MT + ha] = part;
      __syncthreads();
      if ((uint32_t)j == hv.x) {
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          AT sum = AT(0);
#pragma unroll 4
          for (int q2 = 0; q2 < NSTR; ++q2) sum += hred[q2 * MT + 16 * h + t];
          acc[t] += sum;
        }
      }
      __syncthreads();
    }
    ++tag;
  };
  auto step = [&](int64_t kb, ESet &X, Bnd &BX, Bnd &BY) __attribute__((always_inline)) {
    // Block kb: the occupied quads kQ kb .. kQ kb + kQ - 1 of the list
    // (fewer in the last block); item it of the block is row it % MT of its
    // (it / MT)-th quad, drawn into the G slots 4 (it / MT) .. + 3; thread
    // tid takes items tid, tid + 1024, ...
    const int64_t qleft = nq - kb * kQ;
    const int nqb = kb < k1 ? (int)(qleft < kQ ? qleft : kQ) : 0;
    // the quads of block kb + 3, stored into the ring after the draw
    uint32_t qnext = 0;
    if (tid < kQ) qnext = quad_of(kb + 3);
    const int nitems = nqb * MT;
    const uint32_t *qr = qring[kb & 3];
    // row, slot quad and first bucket of item u (r < 2^31: 32-bit)
    auto item_of = [&](int u, int &a, int &q, uint32_t &bq) __attribute__((always_inline)) {
      const int it = tid + kSThreads * u;
      a = it % MT;
      q = it / MT;
      bq = 4u * qr[q];
    };
    const uint32_t ru = (uint32_t)r;
    const int mi = (int)m, a0i = (int)a0;
    // the drawn values: FP64, or (BF16, FP8: exact in bfloat16) two
    // bfloat16 per register
    constexpr int GW = GP == kG64 ? 4 : 2;
    typedef typename std::conditional<GP == kG64, double, uint32_t>::type GR;
    GR g[NIT][GW];
    // values within the window of a rounding midpoint (4 bits per item):
    // redrawn in FP64 after the store, when g is no longer live
    uint32_t nearm = 0;
#pragma unroll
    for (int u = 0; u < NIT; ++u) {
      if (tid + kSThreads * u < nitems) {
        int a, q;
        uint32_t bq;
        item_of(u, a, q, bq);
        const int ga = a0i + a;
        if constexpr (GP == kG64) {
          double z[4] = {0.0, 0.0, 0.0, 0.0};
          if (ga < mi && bq < ru) gauss4_f64((uint64_t)(bq >> 2), (uint32_t)ga, seed, z);
#pragma unroll
          for (int t = 0; t < 4; ++t) g[u][t] = z[t];
        } else {
          float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
          if (ga < mi && bq < ru) {
            const u32x4 x = philox_g((uint64_t)(bq >> 2), (uint32_t)ga, seed);
            if (GP == kGbf16) {
              nearm |= gauss4_bf16_fast(x, z) << (4 * u);
            } else {
              // FP8: G's fixed scale, so a quad's rounding needs no other values
              uint32_t nr;
              const uint32_t by = gauss4_e4m3_fast(x, &nr);
              nearm |= nr << (4 * u);
#pragma unroll
              for (int t = 0; t < 4; ++t) z[t] = e4m3_g_value(by, t);
            }
          }
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (bq + t >= ru) z[t] = 0.0f;  // G ends at bucket r
          // bfloat16 patterns (exact: the values are bfloat16 or e4m3)
          g[u][0] = (__float_as_uint(z[0]) >> 16) | (__float_as_uint(z[1]) & 0xFFFF0000u);
          g[u][1] = (__float_as_uint(z[2]) >> 16) | (__float_as_uint(z[3]) & 0xFFFF0000u);
        }
      }
    }
    if (tid < kQ) qring[(kb + 3) & 3][tid] = qnext;  // ring slot of block kb - 1, read
    __syncthreads();  // the previous block is done with Gb, the stage and crng
#pragma unroll
    for (int u = 0; u < NIT; ++u)
      if (tid + kSThreads * u < nitems) {
        int a, q;
        uint32_t bq;
        item_of(u, a, q, bq);
        GT gv[4];
        if constexpr (GP == kG64) {
#pragma unroll
          for (int t = 0; t < 4; ++t) gv[t] = (GT)g[u][t];
        } else {
          gv[0] = (GT)__uint_as_float(g[u][0] << 16);
          gv[1] = (GT)__uint_as_float(g[u][0] & 0xFFFF0000u);
          gv[2] = (GT)__uint_as_float(g[u][1] << 16);
          gv[3] = (GT)__uint_as_float(g[u][1] & 0xFFFF0000u);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) Gb[(4 * q + t) * GS + a] = gv[t];
      }
    if constexpr (GP != kG64) {
      // the FP64 decisions, written over this thread's own slots (made
      // visible by the barrier after the stage)
      if (__builtin_expect(nearm != 0u, 0)) {
#pragma unroll 1
        for (int u = 0; u < NIT; ++u) {
          const uint32_t nb = (nearm >> (4 * u)) & 15u;
          if (nb == 0u) continue;
          int a, q;
          uint32_t bq;
          item_of(u, a, q, bq);
          const int ga = a0i + a;
          const u32x4 x = philox_g((uint64_t)(bq >> 2), (uint32_t)ga, seed);
          float z[4];
          if (GP == kGbf16) {
            gauss4_bf16_fix(x, nb, z);
          } else {
            const uint32_t by = gauss4_e4m3_fix(x, nb, 0u);
#pragma unroll
            for (int t = 0; t < 4; ++t) z[t] = e4m3_g_value(by, t);
          }
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (((nb >> t) & 1u) && bq + t < ru) Gb[(4 * q + t) * GS + a] = (GT)z[t];
        }
      }
    }
    const uint32_t lo = X.lo, hi = X.hi;
    stage(X.p, X.v, hi - lo < (uint32_t)KS ? hi - lo : (uint32_t)KS);
    __syncthreads();
    bounds(kb + 3, BY);  // block kb + 3 is fetched in the next step
    fetch(BX, X);        // block kb + 2, bounds loaded in the previous step
    consume();
    // more than KS entries: the further turns, loaded here
    for (uint32_t base = lo + KS; base < hi; base += KS) {
      uint32_t pp[KS / kSThreads];
      AT vv[KS / kSThreads];
      load(base, hi, pp, vv);
      __syncthreads();
      stage(pp, vv, hi - base < (uint32_t)KS ? hi - base : (uint32_t)KS);
      __syncthreads();
      consume();
    }
  };
  if (tid < kQ) {  // ring slots are block index mod 4
    qring[k0 & 3][tid] = quad_of(k0);
    qring[(k0 + 1) & 3][tid] = quad_of(k0 + 1);
    qring[(k0 + 2) & 3][tid] = quad_of(k0 + 2);
  }
  __syncthreads();
  Bnd BA, BB;
  ESet RA, RB;
  bounds(k0, BA);
  fetch(BA, RA);
  bounds(k0 + 1, BB);
  fetch(BB, RB);
  bounds(k0 + 2, BA);
  // both steps unconditional (a conditional one would copy set B at the
  // loop's end): a step at k1 has empty bounds and adds nothing
  for (int64_t kb = k0; kb < k1; kb += 2) {
    step(kb, RA, BA, BB);
    step(kb + 1, RB, BB, BA);
  }
  if (j < d) {
    double *o = part + (ks * m + a0 + 16 * h) * d + j;
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (a0 + 16 * h + i < m) o[(int64_t)i * d] = (double)acc[i];
  }
}

// perm[j] = j (sign +1), bptr[b] = b: bucket b holds row b alone
__global__ __launch_bounds__(256) void k_identity_bins(int64_t n, uint32_t *__restrict__ perm,
                                                       uint32_t *__restrict__ bptr) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < n) perm[j] = (uint32_t)j;
  if (j <= n) bptr[j] = (uint32_t)j;
}

// C[i] = scale * sum_s part[s][i], splits in order
__global__ __launch_bounds__(256) void k_sparse_reduce(const double *__restrict__ part,
                                                       int64_t len, int splits, double scale,
                                                       double *__restrict__ C) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  double s = part[i];
  for (int q = 1; q < splits; ++q) s += part[(int64_t)q * len + i];
  C[i] = s * scale;
}

}  // namespace

bool gauss_sparse_fits(const psk_mat &A, int64_t per_row) {
  if (A.format != PSK_CSR) return false;
  // the dense bucket rows of the entry kernel: 4 x d accumulators in 64 KiB of LDS
  if ((size_t)4 * ((A.d + 3) & ~(int64_t)3) * sizeof(double) > 65536) return false;
  if (A.d > 1023) return false;
  // bin entries (n per_row) and entry slots (nnz per_row) in 32 bits
  return A.nnz * per_row < ((int64_t)1 << 31) && A.n * per_row < ((int64_t)1 << 31);
}

bool gauss_sparse_ok(const psk_mat &A, int64_t r, int64_t m, int64_t per_row) {
  if (m <= 0 || !gauss_sparse_fits(A, per_row)) return false;
  // S*A from the binned rows has the bits of S*A from cs_apply when no
  // bucket's rows are split
  if (cs_splits(A.n * per_row, r) != 1) return false;
  // S*A (at most nnz per_row nonzeros) no denser than 1 in 32 of its r x d
  // entries (measured: in FP64 at 1/16 the product over the nonzeros is
  // already slower than the dense GEMM, at 1/8 forty times slower; its
  // contraction reads G from LDS once per nonzero and waits on the longest
  // column run of each wavefront)
  return A.nnz * per_row * 32 <= r * A.d;
}

int identity_bins(int64_t n, Arena &ws, uint32_t **perm, uint32_t **bptr, hipStream_t st) {
  *perm = ws.take<uint32_t>((size_t)n + 1);
  *bptr = ws.take<uint32_t>((size_t)n + 1);
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for the bins of G*A");
  k_identity_bins<<<(unsigned)ceil_div(n + 1, 256), 256, 0, st>>>(n, *perm, *bptr);
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

bool gauss_sparse_pick(const psk_mat &A, int64_t r, int64_t m, int prec, int64_t per_row) {
  if (!gauss_sparse_ok(A, r, m, per_row)) return false;
  const int64_t nz = A.nnz * per_row;  // bound on the nonzeros of S*A
  if (prec != PSK_PREC_FP8) return true;
  // FP8: both forms draw the same m r normals; the dense form adds the FP8
  // MFMA contraction over all r d entries and the scatter of S*A, the sparse
  // form m FP32 updates per nonzero.  Measured crossover near 1/500 of r d
  // (CSR 1e7 x 1000 at 1e-3 of r d: sparse 8.1 ms, dense 11.2 ms; CSR
  // 1e6 x 500 at 4e-3: sparse 1.09 ms, dense 1.00 ms).
  // FP8 (its dense form fused from the bins, or from S*A for an OSNAP)
  return nz * 512 <= r * A.d;
}

int gauss_gemm_sparse(int64_t m, int64_t r, const psk_mat &A, const uint32_t *perm,
                      const uint32_t *bptr, uint64_t seed, int prec, double *C, Arena &ws,
                      hipStream_t st, int64_t per_row, double sa_scale) {
  if (m <= 0 || !gauss_sparse_fits(A, per_row))
    return fail(PSK_EUNSUPPORTED, "sparse Gaussian product: CSR, d <= 1023, nnz < 2^31");
  // bin entries: n (CountSketch) or n per_row (OSNAP pairs); entry slots
  // likewise nnz per_row
  const int64_t n = A.n * per_row, d = A.d;
  const int64_t nslots = A.nnz * per_row;
  const int mtr = d <= 512 ? 32 : 16;
  const int tiles_m = (int)ceil_div(m, mtr);
  const int64_t blk = prec == PSK_PREC_F64 ? 256 : 512;  // G slots (4 per quad) per block
  const int64_t nquads = ceil_div(r, 4);
  const int64_t nblk = ceil_div(nquads, blk / 4);  // blocks when every quad is occupied
  // one 1024-thread workgroup per CU: about 256 of them in all
  int64_t splits = 256 / tiles_m;
  if (splits > nblk / 4) splits = nblk / 4;
  if (splits < 1) splits = 1;
  const int64_t bper = ceil_div(nblk, splits);
  splits = ceil_div(nblk, bper);
  uint32_t *eoff = ws.take<uint32_t>((size_t)n + 1);
  uint32_t *be = ws.take<uint32_t>((size_t)nblk + 1);
  uint32_t *sums = nullptr;
  scan_plan(n + 1, ws, &sums);
  uint32_t *eb = ws.take<uint32_t>((size_t)nslots + 1);
  int32_t *ec = ws.take<int32_t>((size_t)nslots + 1);
  double *ev = ws.take<double>((size_t)nslots + 1);
  uint32_t *sp = ws.take<uint32_t>((size_t)nslots + 1);
  // the sorted values in the precision the product stages them in
  void *sv = prec == PSK_PREC_F64 ? (void *)ws.take<double>((size_t)nslots + 1)
                                  : (void *)ws.take<float>((size_t)nslots + 1);
  uint32_t *qrank = ws.take<uint32_t>((size_t)nquads + 1);
  uint32_t *qlist = ws.take<uint32_t>((size_t)nquads);
  uint32_t *qsums = nullptr;
  scan_plan(nquads + 1, ws, &qsums);
  double *part = ws.take<double>((size_t)splits * m * d);
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for the sparse Gaussian product");
  {
    KTimer t("sa_entries", st);
    k_row_nnz<<<(unsigned)ceil_div(n + 1, 256), 256, 0, st>>>(A.indptr, perm, bptr, r, n, eoff);
    scan_run(eoff, n + 1, sums, st);
    const int64_t dpad = (d + 3) & ~(int64_t)3;
    const size_t lds = (size_t)4 * dpad * sizeof(double);
    const unsigned nb = (unsigned)ceil_div(r, 256);
    const bool limbs = prec == PSK_PREC_BF16;
#define PSK_SAE(TT, LB)                                                                   \
  k_sa_entries<TT, LB><<<nb, 256, lds, st>>>((const TT *)A.values, A.indptr, A.indices, d, \
                                              dpad, r, perm, bptr, eoff, sa_scale, eb, ec, ev)
    if (A.dtype == PSK_F64) {
      if (limbs) PSK_SAE(double, true); else PSK_SAE(double, false);
    } else {
      if (limbs) PSK_SAE(float, true); else PSK_SAE(float, false);
    }
#undef PSK_SAE
    if (prec == PSK_PREC_FP8)
      k_entries_fp8<<<(unsigned)ceil_div(r, kBlk), 256, (size_t)d * 8, st>>>(bptr, eoff, r, d,
                                                                          ec, ev);
    const unsigned qg = (unsigned)ceil_div(nquads + 1, 256);
    k_quad_flags<<<qg, 256, 0, st>>>(bptr, eoff, r, nquads, qrank);
    scan_run(qrank, nquads + 1, qsums, st);
    k_quad_list<<<qg, 256, 0, st>>>(bptr, eoff, qrank, r, nquads, (int)(blk / 4), qlist, be);
    if (blk == 256)
      k_block_csc<8, double><<<(unsigned)nblk, 512, 0, st>>>(be, eb, ec, ev, d, qrank, nquads,
                                                             sp, (double *)sv);
    else
      k_block_csc<16, float><<<(unsigned)nblk, 512, 0, st>>>(be, eb, ec, ev, d, qrank, nquads,
                                                             sp, (float *)sv);
  }
  {
    KTimer t("gauss_gemm", st);
    const unsigned grid = (unsigned)(tiles_m * splits);
#define PSK_GSP(GP, DP, BLK)                                                                 \
  k_gauss_sparse<GP, DP, BLK><<<grid, kSThreads, 0, st>>>(m, d, r, seed, be, sp, sv, qlist, \
                                                         qrank + nquads, tiles_m, part)
#define PSK_GSP_MT(GP, BLK)                   \
  do {                                        \
    if (d <= 512) PSK_GSP(GP, 512, BLK);      \
    else PSK_GSP(GP, 1024, BLK);              \
  } while (0)
    if (prec == PSK_PREC_F64) PSK_GSP_MT(kG64, 256);
    else if (prec == PSK_PREC_BF16) PSK_GSP_MT(kGbf16, 512);
    else PSK_GSP_MT(kGfp8, 512);
#undef PSK_GSP_MT
#undef PSK_GSP
  }
  {
    KTimer t("gemm_reduce", st);
    const int64_t len = m * d;
    k_sparse_reduce<<<(unsigned)ceil_div(len, 256), 256, 0, st>>>(part, len, (int)splits,
                                                                  1.0 / sqrt((double)m), C);
  }
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace psk
