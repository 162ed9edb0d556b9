// CountSketch on gfx950: hash, stable binning of rows by bucket, and the
// bucket-owned row reduction that forms S*A.
//
// Paper mapping (arXiv 2203.02798): the hash is Definition 3; the binned row
// list is the Block-Column CountSketch of section 2.3 (b_r = r: per bucket a
// list of signed row indices, n indices in total); the reduction is Algorithm
// bcs_multiply with one bucket's rows summed by one wavefront, so no two
// workers ever write the same output row (no atomics, deterministic order).
//
// Binning is a stable LSD radix sort of (bucket, row|sign) pairs with 8-bit
// digits: per 2048-key tile a digit histogram, one exclusive scan over
// (digit, tile), then a stable scatter whose in-tile ranks come from
// wavefront ballots.  Stability keeps each bucket's rows in increasing row
// order, which fixes the summation order.
#include "internal.hpp"

namespace psk {
namespace {

constexpr int kRadix = 256;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;  // 2048 keys per block
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096 per block
// the sort's kernels give each thread one digit (histogram, offsets, runs),
// keep per-wavefront digit counts for four wavefronts, and call the block
// scan, which is sized for kScanThreads
static_assert(kRadix == kSortThreads && kSortThreads == kScanThreads,
              "one thread per digit in the sort and scan kernels");
static_assert(kSortThreads == 4 * 64, "the scatter's per-wavefront counts assume four wavefronts");

// ---------------------------------------------------------------------------
// hash
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_hash_export(int64_t row0, int64_t count,
                                                     uint32_t r, uint64_t seed,
                                                     int32_t *__restrict__ h,
                                                     int8_t *__restrict__ sign) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  uint32_t b, neg;
  cs_hash_row((uint64_t)(row0 + j), r, seed, b, neg);
  if (h) h[j] = (int32_t)b;
  if (sign) sign[j] = neg ? (int8_t)-1 : (int8_t)1;
}

__global__ __launch_bounds__(256) void k_hash_keys(int64_t n, uint32_t r,
                                                   uint64_t seed,
                                                   uint32_t *__restrict__ keys,
                                                   uint32_t *__restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t b, neg;
  cs_hash_row((uint64_t)i, r, seed, b, neg);
  keys[i] = b;
  vals[i] = (uint32_t)i | (neg << 31);
}

// OSNAP with s non-zeros per row of A (block construction): pair j = i s + k
// is non-zero k of row i, so each row's s entries are adjacent and, after the
// stable sort, every bucket lists its rows in increasing order
__global__ __launch_bounds__(256) void k_hash_keys_osnap(int64_t pairs, uint32_t s,
                                                         uint32_t rb, uint64_t seed,
                                                         uint32_t *__restrict__ keys,
                                                         uint32_t *__restrict__ vals) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= pairs) return;
  const int64_t i = j / s;
  const uint32_t k = (uint32_t)(j - i * s);
  uint32_t b, neg;
  osnap_hash_nz((uint64_t)i, k, rb, seed, b, neg);
  keys[j] = b;
  vals[j] = (uint32_t)i | (neg << 31);
}

__global__ __launch_bounds__(256) void k_hash_export_osnap(int64_t row0, int64_t pairs,
                                                           uint32_t s, uint32_t rb,
                                                           uint64_t seed,
                                                           int32_t *__restrict__ h,
                                                           int8_t *__restrict__ sign) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= pairs) return;
  const int64_t i = j / s;
  const uint32_t k = (uint32_t)(j - i * s);
  uint32_t b, neg;
  osnap_hash_nz((uint64_t)(row0 + i), k, rb, seed, b, neg);
  if (h) h[j] = (int32_t)b;
  if (sign) sign[j] = neg ? (int8_t)-1 : (int8_t)1;
}

// CSR A: only rows that hold an entry are binned (an empty row adds nothing
// to any sum, so the bins and the sums of the others are unchanged).
// f[i] = 1 when row i holds an entry (f[n] = 0); after an exclusive scan
// k_row_compact lists them in order and writes their count.
__global__ __launch_bounds__(256) void k_row_flags(const int64_t *__restrict__ indptr, int64_t n,
                                                   uint32_t *__restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  f[i] = (i < n && indptr[i + 1] > indptr[i]) ? 1u : 0u;
}

// cnt[0] = rows listed, cnt[1] = s times that (the pairs to bin)
__global__ __launch_bounds__(256) void k_row_compact(const int64_t *__restrict__ indptr,
                                                     const uint32_t *__restrict__ rank,
                                                     int64_t n, uint32_t s,
                                                     uint32_t *__restrict__ rows,
                                                     uint32_t *__restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == n) {
    cnt[0] = rank[n];
    cnt[1] = rank[n] * s;
    return;
  }
  if (indptr[i + 1] > indptr[i]) rows[rank[i]] = (uint32_t)i;
}

// (bucket, row | sign) pairs of the listed rows, s non-zeros each (s = 1:
// the CountSketch hash, non-zero 0 with rb = r); cnt[0] rows listed
__global__ __launch_bounds__(256) void k_hash_keys_rows(const uint32_t *__restrict__ rows,
                                                        const uint32_t *__restrict__ cnt,
                                                        uint32_t s, uint32_t rb, uint64_t seed,
                                                        uint32_t *__restrict__ keys,
                                                        uint32_t *__restrict__ vals) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= (int64_t)cnt[0] * s) return;
  const int64_t q = j / s;
  const uint32_t k = (uint32_t)(j - q * s);
  const uint32_t i = rows[q];
  uint32_t b, neg;
  osnap_hash_nz((uint64_t)i, k, rb, seed, b, neg);
  keys[j] = b;
  vals[j] = i | (neg << 31);
}

// ---------------------------------------------------------------------------
// radix sort pass: per-tile digit histogram (digit-major layout)
// ---------------------------------------------------------------------------
// The keys in use: n, or the count at dn (at most n) when given.
__device__ __forceinline__ int64_t keys_in_use(int64_t n, const uint32_t *dn) {
  return dn ? (int64_t)dn[0] : n;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(
    const uint32_t *__restrict__ keys, int64_t n, const uint32_t *__restrict__ dn, int shift,
    uint32_t mask, uint32_t *__restrict__ hist, int64_t ntiles) {
  __shared__ uint32_t h[kRadix];
  n = keys_in_use(n, dn);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= n) {  // a tile past the keys in use: an empty histogram
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = 0u;
    return;
  }
  h[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t idx = base + it * kSortThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// ---------------------------------------------------------------------------
// exclusive scan of uint32 (three kernels: tile scan, scan of tile sums, add)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t t, uint32_t &total) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  uint32_t inc = t;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t pre = 0;
  total = 0;
#pragma unroll
  for (int q = 0; q < kScanThreads / 64; ++q) {
    if (q < w) pre += wsum[q];
    total += wsum[q];
  }
  __syncthreads();
  return pre + inc - t;
}

// Stable scatter of one tile.  Ranks come from wavefront ballots as the
// keys are read (tile order within each digit); each key is first placed in
// LDS at its digit's tile-local run, then the tile is written out run by
// run, consecutive threads to consecutive addresses of a digit's run in
// kout / vout (instead of every key straight to its own run).  The tile's
// count of a digit is the difference of two neighbouring scanned offsets.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    int64_t n, const uint32_t *__restrict__ dn, int shift, int nbits,
    const uint32_t *__restrict__ offs, int64_t ntiles, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout) {
  __shared__ uint32_t lrun[kRadix];    // next tile-local position of each digit
  __shared__ uint32_t lstart[kRadix];  // tile-local start of each digit's run
  __shared__ uint32_t goff[kRadix];    // where this tile's run of each digit goes
  __shared__ uint32_t wc[4][kRadix];
  __shared__ uint32_t sk[kSortTile], sv[kSortTile];
  n = keys_in_use(n, dn);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= n) return;  // nothing of this tile in use
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int64_t L = (int64_t)kRadix * ntiles;
  const int64_t o = (int64_t)tid * ntiles + blockIdx.x;
  const uint32_t g0 = offs[o];
  const uint32_t g1 = o + 1 < L ? offs[o + 1] : (uint32_t)n;
  uint32_t total;
  const uint32_t ls = block_excl_scan(g1 - g0, total);
  goff[tid] = g0;
  lstart[tid] = ls;
  lrun[tid] = ls;
#pragma unroll
  for (int q = 0; q < 4; ++q) wc[q][tid] = 0;
  __syncthreads();
  const uint32_t mask = (1u << nbits) - 1u;
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t idx = base + it * kSortThreads + tid;
    const bool valid = idx < n;
    const uint32_t k = valid ? kin[idx] : 0u;
    const uint32_t v = valid ? vin[idx] : 0u;
    const uint32_t dg = (k >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (dg >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wc[w][dg] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = lrun[dg] + rank;
      for (int q = 0; q < w; ++q) pos += wc[q][dg];
      sk[pos] = k;
      sv[pos] = v;
    }
    __syncthreads();
    lrun[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
#pragma unroll
    for (int q = 0; q < 4; ++q) wc[q][tid] = 0;
    __syncthreads();
  }
  const int cnt = (int)(n - base < kSortTile ? n - base : kSortTile);
  for (int e = tid; e < cnt; e += kSortThreads) {
    const uint32_t k = sk[e];
    const uint32_t dg = (k >> shift) & mask;
    const uint32_t pos = goff[dg] + ((uint32_t)e - lstart[dg]);
    kout[pos] = k;
    vout[pos] = sv[e];
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(uint32_t *__restrict__ data,
                                                             int64_t L,
                                                             uint32_t *__restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t t = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < L) ? data[base + i] : 0u;
    t += v[i];
  }
  uint32_t total;
  uint32_t run = block_excl_scan(t, total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < L) data[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(uint32_t *__restrict__ sums,
                                                            int64_t nb) {
  uint32_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kScanTile) {
    const int64_t base = c0 + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = (base + i < nb) ? sums[base + i] : 0u;
      t += v[i];
    }
    uint32_t total;
    uint32_t run = carry + block_excl_scan(t, total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (base + i < nb) sums[base + i] = run;
      run += v[i];
    }
    carry += total;
  }
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t *__restrict__ data, int64_t L,
                                                  const uint32_t *__restrict__ sums) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < L) data[i] += sums[i / kScanTile];
}

int scan_plan_impl(int64_t L, Arena &ws, uint32_t **sums) {
  *sums = ws.take<uint32_t>((size_t)ceil_div(L, kScanTile) + 1);
  return 0;
}

void scan_run_impl(uint32_t *data, int64_t L, uint32_t *sums, hipStream_t st) {
  const int64_t nb = ceil_div(L, kScanTile);
  k_scan_tiles<<<(unsigned)nb, kScanThreads, 0, st>>>(data, L, sums);
  k_scan_sums<<<1, kScanThreads, 0, st>>>(sums, nb);
  k_scan_add<<<(unsigned)ceil_div(L, 256), 256, 0, st>>>(data, L, sums);
}

// bucket b's range starts at the first sorted position whose key is >= b
__global__ __launch_bounds__(256) void k_bucket_ptr(const uint32_t *__restrict__ skeys,
                                                    int64_t n, const uint32_t *__restrict__ dn,
                                                    uint32_t r, uint32_t *__restrict__ bptr) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  n = keys_in_use(n, dn);
  if (j > n) return;
  const int64_t prev = j > 0 ? (int64_t)skeys[j - 1] : -1;
  const int64_t cur = j < n ? (int64_t)skeys[j] : (int64_t)r;
  for (int64_t b = prev + 1; b <= cur; ++b) bptr[b] = (uint32_t)j;
}

// The same pointers with the key count on the device: one thread per
// bucket b in [0, r], bptr[b] = the first position whose key is >= b
// (a binary search, so the work stays bounded when the keys in use are few
// and the buckets many).
__global__ __launch_bounds__(256) void k_bucket_ptr_search(const uint32_t *__restrict__ skeys,
                                                           const uint32_t *__restrict__ dn,
                                                           uint32_t r,
                                                           uint32_t *__restrict__ bptr) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > (int64_t)r) return;
  uint32_t lo = 0, hi = dn[0];
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if ((int64_t)skeys[mid] < b) lo = mid + 1;
    else hi = mid;
  }
  bptr[b] = lo;
}

__global__ void k_fill_identity_ptr(uint32_t *bptr, int64_t n, const uint32_t *dn) {
  bptr[0] = 0;
  bptr[1] = (uint32_t)keys_in_use(n, dn);
}

// ---------------------------------------------------------------------------
// S*A, dense A: one wavefront per (bucket, split); each lane owns VW adjacent
// columns in each of CH column groups, accumulating in registers.
// ---------------------------------------------------------------------------
template <typename T, int VW>
struct Vec;
template <>
struct Vec<double, 1> { typedef double type; };
template <>
struct Vec<double, 2> { typedef double2 type; };
template <>
struct Vec<float, 1> { typedef float type; };
template <>
struct Vec<float, 2> { typedef float2 type; };
template <>
struct Vec<float, 4> { typedef float4 type; };
template <>
struct Vec<double, 4> { typedef double4 type; };

template <typename T, int VW>
__device__ __forceinline__ void vload(const T *p, T (&x)[VW]) {
  typedef typename Vec<T, VW>::type V;
  const V v = *reinterpret_cast<const V *>(p);
  const T *e = reinterpret_cast<const T *>(&v);
#pragma unroll
  for (int q = 0; q < VW; ++q) x[q] = e[q];
}

template <typename T, int VW>
__device__ __forceinline__ void vstore(T *p, const T (&x)[VW]) {
  typedef typename Vec<T, VW>::type V;
  V v;
  T *e = reinterpret_cast<T *>(&v);
#pragma unroll
  for (int q = 0; q < VW; ++q) e[q] = x[q];
  *reinterpret_cast<V *>(p) = v;
}

// VW adjacent outputs: one vector store where the vector type exists (the
// row of out is aligned whenever the loads of A are), else element stores
template <typename TO, int VW>
__device__ __forceinline__ void store_out(TO *p, const TO (&x)[VW]) {
  if constexpr (sizeof(TO) * VW <= 16) {
    vstore<TO, VW>(p, x);
  } else {
#pragma unroll
    for (int q = 0; q < VW; q += 2) {
      const TO y[2] = {x[q], x[q + 1]};
      vstore<TO, 2>(p + q, y);
    }
  }
}

// The U rows of a batch are loaded together and branch-free (a row past the
// bucket, or columns past d, load an element of row 0 at column 0 and are
// masked), so all of them are in flight at once, and the bin entries of the
// next batch are loaded while this one is summed.  Rows are added in bin
// order, in FP64.
template <typename T, typename TO, int VW, int CH, int U>
__global__ __launch_bounds__(256) void k_scatter_dense(
    const T *__restrict__ A, int64_t ld, int64_t d, int64_t r,
    const uint32_t *__restrict__ perm, const uint32_t *__restrict__ bptr,
    int splits, double scale, TO *__restrict__ out) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wave >= r * splits) return;
  const int64_t b = wave / splits;
  const int s = (int)(wave - b * splits);
  const uint32_t lo = bptr[b];
  const uint32_t len = bptr[b + 1] - lo;
  const uint32_t j0 = lo + (uint32_t)(((uint64_t)len * s) / splits);
  const uint32_t j1 = lo + (uint32_t)(((uint64_t)len * (s + 1)) / splits);
  TO *orow = out + ((int64_t)s * r + b) * d;
  const int lane = threadIdx.x & 63;
  constexpr int64_t kSpan = 64 * VW * CH;
  for (int64_t c0 = 0; c0 < d; c0 += kSpan) {
    double acc[CH][VW];
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int q = 0; q < VW; ++q) acc[c][q] = 0.0;
    // column offsets of this lane's groups, clamped to 0 past d
    int64_t coff[CH];
    bool cok[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int64_t col = c0 + (int64_t)(c * 64 + lane) * VW;
      cok[c] = col < d;
      coff[c] = cok[c] ? col : 0;
    }
    uint32_t pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) pv[u] = perm[(j0 + u < j1) ? j0 + u : lo];
    for (uint32_t j = j0; j < j1; j += U) {
      T x[U][CH][VW];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool rok = j + u < j1;
        const int64_t row = rok ? (int64_t)(pv[u] & 0x7fffffffu) : 0;
#pragma unroll
        for (int c = 0; c < CH; ++c) vload<T, VW>(A + row * ld + coff[c], x[u][c]);
      }
      double sg[U];
#pragma unroll
      for (int u = 0; u < U; ++u) sg[u] = (j + u < j1) ? ((pv[u] >> 31) ? -1.0 : 1.0) : 0.0;
      // the next batch's bin entries
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t jn = j + U + u;
        pv[u] = perm[jn < j1 ? jn : lo];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < CH; ++c)
#pragma unroll
          for (int q = 0; q < VW; ++q) {
            const double xv = cok[c] ? (double)x[u][c][q] : 0.0;
            acc[c][q] = fma(sg[u], xv, acc[c][q]);
          }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (cok[c]) {
        TO ov[VW];
#pragma unroll
        for (int q = 0; q < VW; ++q) ov[q] = (TO)(acc[c][q] * scale);
        store_out<TO, VW>(orow + coff[c], ov);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// S*A, CSR A: one wavefront per (bucket, split) with a private LDS row of d
// FP64 accumulators; rows of the bucket are applied one after another
// (bucket_rows_add).
// ---------------------------------------------------------------------------
template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_scatter_csr(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, int64_t d, int64_t dpad, int64_t r,
    const uint32_t *__restrict__ perm, const uint32_t *__restrict__ bptr,
    int splits, double scale, TO *__restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw) + (threadIdx.x >> 6) * dpad;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wave >= r * splits) return;
  const int lane = threadIdx.x & 63;
  const int64_t b = wave / splits;
  const int s = (int)(wave - b * splits);
  const uint32_t lo = bptr[b];
  const uint32_t len = bptr[b + 1] - lo;
  const uint32_t j0 = lo + (uint32_t)(((uint64_t)len * s) / splits);
  const uint32_t j1 = lo + (uint32_t)(((uint64_t)len * (s + 1)) / splits);
  for (int64_t c = lane; c < d; c += 64) acc[c] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  bucket_rows_add(vals, indptr, indices, perm, j0, j1, acc);
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  TO *orow = out + ((int64_t)s * r + b) * d;
  for (int64_t c = lane; c < d; c += 64) orow[c] = (TO)(acc[c] * scale);
}

// SA[b, c] = sum over splits of partial[s, b, c] (FP64), splits in
// increasing order, rounded once to the output type
template <typename TO>
__global__ __launch_bounds__(256) void k_combine_splits(const double *__restrict__ part,
                                                        int64_t rd, int splits,
                                                        double scale,
                                                        TO *__restrict__ SA) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rd) return;
  double acc = part[e];
  for (int s = 1; s < splits; ++s) acc += part[(int64_t)s * rd + e];
  SA[e] = (TO)(acc * scale);
}

int choose_splits(int64_t n, int64_t r) {
  // Enough wavefronts to cover the chip when buckets are few and long;
  // at least ~32 rows per split on average.
  const int64_t target_waves = 8192;
  if (r >= target_waves) return 1;
  int64_t s = ceil_div(target_waves, r);
  const int64_t by_rows = n / (r * 32);
  if (s > by_rows) s = by_rows;
  if (s > 64) s = 64;
  return s < 1 ? 1 : (int)s;
}

template <typename T, typename TO, int VW>
void launch_dense(const psk_mat &A, int64_t r, const uint32_t *perm,
                  const uint32_t *bptr, int splits, double scale, TO *out, hipStream_t st) {
  const int64_t waves = r * splits;
  const unsigned blocks = (unsigned)ceil_div(waves, 4);
  const int64_t span1 = 64 * VW;  // columns per lane group
  // one column group: six rows a batch (84 VGPRs with FP32 rows, against
  // 104 at eight) run as fast alone and leave a wavefront of room beside the
  // Gram on another stream (C3's sketch-beside-Gram step 11.22 -> 11.06 ms)
  if (A.d <= span1)
    k_scatter_dense<T, TO, VW, 1, 6><<<blocks, 256, 0, st>>>(
        (const T *)A.values, A.ld, A.d, r, perm, bptr, splits, scale, out);
  else if (A.d <= 2 * span1)
    k_scatter_dense<T, TO, VW, 2, 4><<<blocks, 256, 0, st>>>(
        (const T *)A.values, A.ld, A.d, r, perm, bptr, splits, scale, out);
  else
    k_scatter_dense<T, TO, VW, 4, 4><<<blocks, 256, 0, st>>>(
        (const T *)A.values, A.ld, A.d, r, perm, bptr, splits, scale, out);
}

// VW adjacent columns per lane where the rows of A and of the output allow
// aligned vector accesses
template <typename T, typename TO>
void launch_dense_vw(const psk_mat &A, int64_t r, const uint32_t *perm,
                     const uint32_t *bptr, int splits, double scale, TO *out,
                     hipStream_t st) {
  const uintptr_t addr = (uintptr_t)A.values, oaddr = (uintptr_t)out;
  constexpr int es = (int)sizeof(T), os = (int)sizeof(TO);
  const bool v4 = es == 4 && (A.d % 4 == 0) && (A.ld % 4 == 0) && (addr % 16 == 0) &&
                  oaddr % (os == 4 ? 16 : 16) == 0;
  const bool v2 = (A.d % 2 == 0) && (A.ld % 2 == 0) && (addr % (2 * es) == 0) &&
                  oaddr % (2 * os) == 0;
  if constexpr (sizeof(T) == 4) {
    if (v4) return launch_dense<T, TO, 4>(A, r, perm, bptr, splits, scale, out, st);
  }
  if (v2) return launch_dense<T, TO, 2>(A, r, perm, bptr, splits, scale, out, st);
  launch_dense<T, TO, 1>(A, r, perm, bptr, splits, scale, out, st);
}

// LDS of the CSR scatter: FP64 accumulators of wpb wavefronts
constexpr size_t kCsrLdsMax = 163840;

}  // namespace

// ---------------------------------------------------------------------------
// host entry points
// ---------------------------------------------------------------------------
int cs_splits(int64_t n, int64_t r) { return choose_splits(n, r); }
int scan_plan(int64_t L, Arena &ws, uint32_t **sums) { return scan_plan_impl(L, ws, sums); }
void scan_run(uint32_t *data, int64_t L, uint32_t *sums, hipStream_t st) {
  scan_run_impl(data, L, sums, st);
}

int cs_hash_export(int64_t row0, int64_t count, uint32_t r, uint64_t seed,
                   int32_t *h, int8_t *sign, hipStream_t st) {
  if (count == 0) return 0;
  k_hash_export<<<(unsigned)ceil_div(count, 256), 256, 0, st>>>(row0, count, r,
                                                                 seed, h, sign);
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

int sort_pairs(uint32_t *keys, uint32_t *vals, int64_t n, uint32_t r, Arena &ws,
               hipStream_t st, uint32_t **skeys, uint32_t **svals, uint32_t *ptr,
               const uint32_t *dn) {
  int bits = 0;
  while (bits < 32 && ((uint64_t)1 << bits) < (uint64_t)r) ++bits;
  const int passes = (bits + 7) / 8;
  const int64_t ntiles = ceil_div(n, kSortTile);
  const int64_t L = (int64_t)kRadix * ntiles;
  uint32_t *k1 = passes ? ws.take<uint32_t>(n) : nullptr;
  uint32_t *v1 = passes ? ws.take<uint32_t>(n) : nullptr;
  uint32_t *hist = passes ? ws.take<uint32_t>(L) : nullptr;
  uint32_t *sums = nullptr;
  if (passes) scan_plan_impl(L, ws, &sums);
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for a radix sort");
  uint32_t *kin = keys, *vin = vals, *kout = k1, *vout = v1;
  for (int p = 0; p < passes && n > 0; ++p) {
    const int shift = 8 * p;
    const int nb = (bits - shift) < 8 ? (bits - shift) : 8;
    const uint32_t mask = (1u << nb) - 1u;
    k_radix_hist<<<(unsigned)ntiles, kSortThreads, 0, st>>>(kin, n, dn, shift, mask, hist,
                                                            ntiles);
    scan_run_impl(hist, L, sums, st);
    k_radix_scatter<<<(unsigned)ntiles, kSortThreads, 0, st>>>(kin, vin, n, dn, shift, nb,
                                                               hist, ntiles, kout, vout);
    uint32_t *t;
    t = kin; kin = kout; kout = t;
    t = vin; vin = vout; vout = t;
  }
  if (ptr) {
    if (passes && dn)
      k_bucket_ptr_search<<<(unsigned)ceil_div((int64_t)r + 1, 256), 256, 0, st>>>(kin, dn, r,
                                                                                  ptr);
    else if (passes)
      k_bucket_ptr<<<(unsigned)ceil_div(n + 1, 256), 256, 0, st>>>(kin, n, nullptr, r, ptr);
    else
      k_fill_identity_ptr<<<1, 1, 0, st>>>(ptr, n, dn);
  }
  PSK_HIP_TRY(hipGetLastError());
  *skeys = kin;
  *svals = vin;
  return 0;
}

int osnap_hash_export(int64_t row0, int64_t count, uint32_t s, uint32_t r, uint64_t seed,
                      int32_t *h, int8_t *sign, hipStream_t st) {
  const int64_t pairs = count * (int64_t)s;
  if (pairs == 0) return 0;
  k_hash_export_osnap<<<(unsigned)ceil_div(pairs, 256), 256, 0, st>>>(row0, pairs, s, r / s,
                                                                       seed, h, sign);
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

// Bins of the (row, non-zero) pairs: s per row (s = 1 for CountSketch,
// rb = r / s rows of S per block).  For CSR A only the rows holding an
// entry are listed first (their count stays on the device and bounds the
// sort), so a matrix with many empty rows sorts only the others.
static int bin_pairs(const psk_mat &A, uint32_t s, uint32_t r, uint64_t seed, Arena &ws,
                     hipStream_t st, uint32_t **perm, uint32_t **bptr) {
  const int64_t n = A.n;
  const int64_t pairs = n * (int64_t)s;
  const bool compact = A.format == PSK_CSR;
  uint32_t *k0 = ws.take<uint32_t>(pairs);
  uint32_t *v0 = ws.take<uint32_t>(pairs);
  uint32_t *bp = ws.take<uint32_t>((size_t)r + 1);
  uint32_t *rank = nullptr, *rows = nullptr, *cnt = nullptr, *sums = nullptr;
  if (compact) {
    rank = ws.take<uint32_t>((size_t)n + 1);
    rows = ws.take<uint32_t>((size_t)n);
    cnt = ws.take<uint32_t>(2);
    scan_plan_impl(n + 1, ws, &sums);
  }
  if (!ws.dry() && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for the binning");
  KTimer timer("cs_bin", st, !ws.dry());
  if (!ws.dry()) {
    if (compact) {
      const unsigned g = (unsigned)ceil_div(n + 1, 256);
      k_row_flags<<<g, 256, 0, st>>>(A.indptr, n, rank);
      scan_run_impl(rank, n + 1, sums, st);
      k_row_compact<<<g, 256, 0, st>>>(A.indptr, rank, n, s, rows, cnt);
      k_hash_keys_rows<<<(unsigned)ceil_div(pairs, 256), 256, 0, st>>>(rows, cnt, s, r / s,
                                                                        seed, k0, v0);
    } else if (s == 1) {
      k_hash_keys<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(n, r, seed, k0, v0);
    } else {
      k_hash_keys_osnap<<<(unsigned)ceil_div(pairs, 256), 256, 0, st>>>(pairs, s, r / s, seed,
                                                                         k0, v0);
    }
  }
  uint32_t *sk = nullptr;
  // for CSR A the pairs of the listed rows (cnt[1]) bound the sort
  const int rc =
      sort_pairs(k0, v0, pairs, r, ws, st, &sk, perm, bp, compact ? cnt + 1 : nullptr);
  if (rc) return rc;
  *bptr = bp;
  return 0;
}

int cs_bin(const psk_mat &A, uint32_t r, uint64_t seed, Arena &ws, hipStream_t st,
           uint32_t **perm, uint32_t **bptr) {
  return bin_pairs(A, 1u, r, seed, ws, st, perm, bptr);
}

int osnap_bin(const psk_mat &A, uint32_t s, uint32_t r, uint64_t seed, Arena &ws,
              hipStream_t st, uint32_t **perm, uint32_t **bptr) {
  return bin_pairs(A, s, r, seed, ws, st, perm, bptr);
}

int cs_apply(const psk_mat &A, uint32_t r, const uint32_t *perm,
             const uint32_t *bptr, void *SA, Arena &ws, hipStream_t st, bool out_f64,
             double scale, int64_t entries) {
  const int splits = choose_splits(entries > 0 ? entries : A.n, r);
  const bool o64 = out_f64 || A.dtype == PSK_F64;
  void *part = nullptr;
  if (splits > 1) part = ws.take<double>((size_t)splits * r * A.d);
  const int64_t dpad = (A.d + 3) & ~(int64_t)3;
  if (A.format == PSK_CSR && (size_t)dpad * 8 > kCsrLdsMax)
    return fail(PSK_EUNSUPPORTED, "CSR S*A supports d <= 20480");
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for S*A");
  KTimer timer("cs_scatter", st);
  if (A.format == PSK_DENSE) {
    // K-split partials are written unscaled; the combine applies the scale
    if (splits > 1) {
      if (A.dtype == PSK_F64)
        launch_dense_vw<double, double>(A, r, perm, bptr, splits, 1.0, (double *)part, st);
      else
        launch_dense_vw<float, double>(A, r, perm, bptr, splits, 1.0, (double *)part, st);
    } else if (A.dtype == PSK_F64) {
      launch_dense_vw<double, double>(A, r, perm, bptr, 1, scale, (double *)SA, st);
    } else if (o64) {
      launch_dense_vw<float, double>(A, r, perm, bptr, 1, scale, (double *)SA, st);
    } else {
      launch_dense_vw<float, float>(A, r, perm, bptr, 1, scale, (float *)SA, st);
    }
  } else {
    int wpb = 4;
    while (wpb > 1 && (size_t)wpb * dpad * 8 > 65536) --wpb;
    const size_t lds = (size_t)wpb * dpad * 8;
    const int64_t waves = (int64_t)r * splits;
    const unsigned blocks = (unsigned)ceil_div(waves, wpb);
#define PSK_SCSR(T, TO, OUT, SC)                                                           \
  do {                                                                                     \
    if (lds > 65536)                                                                       \
      PSK_HIP_TRY(hipFuncSetAttribute((const void *)k_scatter_csr<T, TO>,                  \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
    k_scatter_csr<T, TO><<<blocks, 64 * wpb, lds, st>>>((const T *)A.values, A.indptr,     \
                                                        A.indices, A.d, dpad, r, perm, bptr, \
                                                        splits, (SC), (TO *)(OUT));        \
  } while (0)
    if (splits > 1) {
      if (A.dtype == PSK_F64) PSK_SCSR(double, double, part, 1.0);
      else PSK_SCSR(float, double, part, 1.0);
    } else if (A.dtype == PSK_F64) {
      PSK_SCSR(double, double, SA, scale);
    } else if (o64) {
      PSK_SCSR(float, double, SA, scale);
    } else {
      PSK_SCSR(float, float, SA, scale);
    }
#undef PSK_SCSR
  }
  if (splits > 1) {
    const int64_t rd = (int64_t)r * A.d;
    if (o64)
      k_combine_splits<double><<<(unsigned)ceil_div(rd, 256), 256, 0, st>>>(
          (const double *)part, rd, splits, scale, (double *)SA);
    else
      k_combine_splits<float><<<(unsigned)ceil_div(rd, 256), 256, 0, st>>>(
          (const double *)part, rd, splits, scale, (float *)SA);
  }
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace psk
