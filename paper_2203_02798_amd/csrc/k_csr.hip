// Gram matrix and squared row norms of a CSR matrix on gfx950, FP64.
//
// Paper mapping (arXiv 2203.02798):
// * Gram: Algorithm gram_serial's outer-product loop (B[J_k, J_j] +=
//   V_k V_j over pairs of a row's entries), parallelised by output rows as
//   Algorithm gram_parallel_memory_effcient does (each worker owns output
//   rows, so no partial Grams and no reduction), but where that algorithm
//   scans every row of A and filters its entries, here the entries are first
//   sorted by column (a stable radix sort: the column index of A), so the
//   wavefront owning output row j visits exactly the rows with an entry in
//   column j: nnz_2(A) work in total.  Only k >= j is accumulated and the
//   other triangle is mirrored, so C is exactly symmetric.
// * Row norms: Algorithm squared_row_norms: Bt = B B^T once, then per row
//   sum_{k,j} V_k V_j Bt[J_j, J_k].  Short rows take one lane each; rows
//   longer than 32 entries are taken by the whole wavefront (lanes over k).
//   That costs a row nnz^2 scattered reads of Bt; a row with more than
//   max(32, k/8) entries costs less as the product itself, ||V B[J, :]||^2
//   (nnz contiguous rows of B, k values each): such rows are listed and
//   taken by k_rownorm_csr_long, a workgroup per row.
#include "internal.hpp"

namespace psk {
namespace {

// rowidx[p] = row of stored entry p
__global__ __launch_bounds__(256) void k_row_of_entry(const int64_t *__restrict__ indptr,
                                                      int64_t n, uint32_t *__restrict__ rowidx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t p = indptr[i]; p < indptr[i + 1]; ++p) rowidx[p] = (uint32_t)i;
}

// (column, position) pairs of the stored entries, to be sorted by column
__global__ __launch_bounds__(256) void k_col_keys(const int32_t *__restrict__ indices,
                                                  int64_t nnz, uint32_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  keys[p] = (uint32_t)indices[p];
  vals[p] = (uint32_t)p;
}

// One wavefront per output row j: for every entry A[i, j] of column j (rows
// in increasing order), add A[i, j] * A[i, k] over the entries of row i with
// k >= j into a private LDS row; then write C[j, k] and its mirror C[k, j].
template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_gram_csc(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, const uint32_t *__restrict__ rowidx,
    const uint32_t *__restrict__ cperm, const uint32_t *__restrict__ cptr, int64_t d,
    int64_t dpad, double alpha, double beta, TO *__restrict__ C) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw) + (threadIdx.x >> 6) * dpad;
  const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (j >= d) return;
  const int lane = threadIdx.x & 63;
  for (int64_t c = j + lane; c < d; c += 64) acc[c] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const uint32_t e1 = cptr[j + 1];
  for (uint32_t e0 = cptr[j]; e0 < e1; e0 += 64) {
    const uint32_t e = e0 + lane;
    if (e < e1) {
      const uint32_t p = cperm[e];
      const double v = (double)vals[p];
      const uint32_t i = rowidx[p];
      for (int64_t h = indptr[i]; h < indptr[i + 1]; ++h) {
        const int32_t c = indices[h];
        if (c >= j) atomicAdd(&acc[c], v * (double)vals[h]);
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int64_t k = j + lane; k < d; k += 64) {
    const double g = alpha * acc[k];
    const int64_t up = j * d + k, lo = k * d + j;
    C[up] = (TO)(beta != 0.0 ? g + beta * (double)C[up] : g);
    if (k > j) C[lo] = (TO)(beta != 0.0 ? g + beta * (double)C[lo] : g);
  }
}

// nlong[0] = 0 (the list of rows for the product form)
__global__ void k_clear_count(uint32_t *__restrict__ nlong) {
  if (threadIdx.x == 0) nlong[0] = 0u;
}

// Rows of more than tl entries are only listed here (longlist, nlong); the
// order of the list does not matter, each row's value is computed alone.
template <typename T>
__global__ __launch_bounds__(256) void k_rownorm_csr(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, int64_t n, int64_t d,
    const double *__restrict__ Bt, double alpha, double beta, double *__restrict__ x,
    int64_t tl, uint32_t *__restrict__ longlist, uint32_t *__restrict__ nlong) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  bool have = i < n;
  int64_t p0 = 0, p1 = 0;
  if (have) {
    p0 = indptr[i];
    p1 = indptr[i + 1];
  }
  if (have && p1 - p0 > tl) {
    longlist[atomicAdd(nlong, 1u)] = (uint32_t)i;
    have = false;
  }
  const bool longrow = have && (p1 - p0) > 32;
  if (have && !longrow) {
    double acc = 0.0;
    for (int64_t k = p0; k < p1; ++k) {
      const double vk = (double)vals[k];
      const int64_t ck = indices[k];
      double s = 0.0;
      for (int64_t j = p0; j < p1; ++j) s += (double)vals[j] * Bt[(int64_t)indices[j] * d + ck];
      acc += vk * s;
    }
    x[i] = beta != 0.0 ? alpha * acc + beta * x[i] : alpha * acc;
  }
  uint64_t pending = __ballot(longrow);
  while (pending) {
    const int src = __ffsll((unsigned long long)pending) - 1;
    pending &= pending - 1;
    const int64_t q0 = __shfl(p0, src, 64);
    const int64_t q1 = __shfl(p1, src, 64);
    const int64_t row = __shfl(i, src, 64);
    double part = 0.0;
    for (int64_t k = q0 + lane; k < q1; k += 64) {
      const double vk = (double)vals[k];
      const int64_t ck = indices[k];
      double s = 0.0;
      for (int64_t j = q0; j < q1; ++j) s += (double)vals[j] * Bt[(int64_t)indices[j] * d + ck];
      part += vk * s;
    }
    part = wave_sum(part);
    if (lane == 0) x[row] = beta != 0.0 ? alpha * part + beta * x[row] : alpha * part;
  }
}

// The listed rows as the product itself: workgroup per row (grid-stride
// over the list), thread t holds y_j = sum_p V_p B[J_p, j] for its columns
// j = t + 256 q, q < Q (k <= 256 Q), the entries taken in row order, kU at a
// time with their rows of B loaded together; then ||y||^2 summed in a
// fixed order (thread, wavefront, workgroup).
constexpr int kRnU = 8;  // entries whose B rows are in flight together
template <typename T, int Q>
__global__ __launch_bounds__(256) void k_rownorm_csr_long(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, const uint32_t *__restrict__ longlist,
    const uint32_t *__restrict__ nlong, const double *__restrict__ B, int64_t k, double alpha,
    double beta, double *__restrict__ x) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const uint32_t cnt = nlong[0];
  for (uint32_t l = blockIdx.x; l < cnt; l += gridDim.x) {
    const int64_t i = (int64_t)longlist[l];
    const int64_t p0 = indptr[i], p1 = indptr[i + 1];
    double y[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) y[q] = 0.0;
    for (int64_t p = p0; p < p1; p += kRnU) {
      double v[kRnU];
      int64_t c[kRnU];
#pragma unroll
      for (int u = 0; u < kRnU; ++u) {
        const bool ok = p + u < p1;
        const int64_t pu = ok ? p + u : p0;  // clamped, value zeroed
        v[u] = ok ? (double)vals[pu] : 0.0;
        c[u] = indices[pu];
      }
      double b[kRnU][Q];
#pragma unroll
      for (int u = 0; u < kRnU; ++u)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int64_t j = tid + 256 * q;
          b[u][q] = B[c[u] * k + (j < k ? j : 0)];
        }
#pragma unroll
      for (int u = 0; u < kRnU; ++u)
#pragma unroll
        for (int q = 0; q < Q; ++q) y[q] = fma(v[u], b[u][q], y[q]);
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q)
      if (tid + 256 * q < k) s = fma(y[q], y[q], s);
    s = wave_sum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
      const double t = ((red[0] + red[1]) + red[2]) + red[3];
      x[i] = beta != 0.0 ? alpha * t + beta * x[i] : alpha * t;
    }
    __syncthreads();  // red is reused by the next row
  }
}

}  // namespace

int gram_csr(double alpha, const psk_mat &A, double beta, void *C, Arena &ws,
             hipStream_t st, bool out_f64) {
  const int64_t d = A.d, n = A.n, nnz = A.nnz;
  if (d > 8192) return fail(PSK_EUNSUPPORTED, "CSR gram supports d <= 8192");
  if (nnz >= ((int64_t)1 << 32)) return fail(PSK_EUNSUPPORTED, "CSR gram needs nnz < 2^32");
  const int64_t cnt = nnz > 0 ? nnz : 1;
  uint32_t *keys = ws.take<uint32_t>(cnt);
  uint32_t *vals = ws.take<uint32_t>(cnt);
  uint32_t *rowidx = ws.take<uint32_t>(cnt);
  uint32_t *cptr = ws.take<uint32_t>((size_t)d + 1);
  if (!ws.dry()) {
    k_col_keys<<<(unsigned)ceil_div(cnt, 256), 256, 0, st>>>(A.indices, nnz, keys, vals);
    k_row_of_entry<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(A.indptr, n, rowidx);
  }
  uint32_t *skeys = nullptr, *cperm = nullptr;
  int rc = sort_pairs(keys, vals, nnz, (uint32_t)d, ws, st, &skeys, &cperm, cptr);
  if (rc) return rc;
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for CSR gram");
  const int64_t dpad = (d + 1) & ~(int64_t)1;
  int wpb = 4;
  while (wpb > 1 && (size_t)wpb * dpad * sizeof(double) > 65536) --wpb;
  const size_t lds = (size_t)wpb * dpad * sizeof(double);
  const unsigned blocks = (unsigned)ceil_div(d, wpb);
  KTimer timer("gram", st);
  if (A.dtype == PSK_F64)
    k_gram_csc<double, double><<<blocks, 64 * wpb, lds, st>>>(
        (const double *)A.values, A.indptr, A.indices, rowidx, cperm, cptr, d, dpad, alpha,
        beta, (double *)C);
  else if (out_f64)
    k_gram_csc<float, double><<<blocks, 64 * wpb, lds, st>>>(
        (const float *)A.values, A.indptr, A.indices, rowidx, cperm, cptr, d, dpad, alpha,
        beta, (double *)C);
  else
    k_gram_csc<float, float><<<blocks, 64 * wpb, lds, st>>>(
        (const float *)A.values, A.indptr, A.indices, rowidx, cperm, cptr, d, dpad, alpha,
        beta, (float *)C);
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

int rownorms_csr(double alpha, const psk_mat &A, const double *B, int64_t k,
                 double beta, double *x, Arena &ws, hipStream_t st) {
  const int64_t d = A.d;
  if (d > 8192) return fail(PSK_EUNSUPPORTED, "CSR row norms support d <= 8192");
  double *Bt = ws.take<double>((size_t)d * d);
  // rows for the product form: more than max(32, k/8) entries (k <= 2048)
  const int64_t tl = k <= 2048 ? (k / 8 > 32 ? k / 8 : 32) : INT64_MAX;
  uint32_t *longlist = ws.take<uint32_t>((size_t)A.n);
  uint32_t *nlong = ws.take<uint32_t>(1);
  // B * B^T (d x d) with the FP64 GEMM
  int rc = dgemm(false, true, d, d, k, 1.0, B, k, B, k, 0.0, Bt, d, ws, st);
  if (rc) return rc;
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for CSR row norms");
  const unsigned blocks = (unsigned)ceil_div(A.n, 256);
  KTimer timer("rownorm", st);
  k_clear_count<<<1, 64, 0, st>>>(nlong);
#define PSK_RNC(T)                                                                         \
  k_rownorm_csr<T><<<blocks, 256, 0, st>>>((const T *)A.values, A.indptr, A.indices, A.n, d, \
                                           Bt, alpha, beta, x, tl, longlist, nlong)
  if (A.dtype == PSK_F64) PSK_RNC(double); else PSK_RNC(float);
#undef PSK_RNC
  if (tl != INT64_MAX) {
    // a fixed grid walks the listed rows (their count stays on the device)
    const unsigned lb = 2048;
#define PSK_RNL(T, Q)                                                                   \
  k_rownorm_csr_long<T, Q><<<lb, 256, 0, st>>>((const T *)A.values, A.indptr, A.indices, \
                                              longlist, nlong, B, k, alpha, beta, x)
    if (A.dtype == PSK_F64) {
      if (k <= 1024) PSK_RNL(double, 4); else PSK_RNL(double, 8);
    } else {
      if (k <= 1024) PSK_RNL(float, 4); else PSK_RNL(float, 8);
    }
#undef PSK_RNL
  }
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace psk
