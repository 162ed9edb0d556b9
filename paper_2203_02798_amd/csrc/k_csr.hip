// Gram matrix and squared row norms of a CSR matrix on gfx950, FP64.
//
// Paper mapping (arXiv 2203.02798):
// * Gram: Algorithm gram_serial's outer-product loop (B[J_k, J_j] +=
//   V_k V_j over pairs of a row's entries), parallelised by combining the two
//   parallel algorithms of section 3: like Algorithm
//   gram_parallel_memory_effcient a workgroup owns a range of output rows
//   (kept in LDS) and filters each row's entries against that range; like
//   Algorithm gram the rows of A are split into chunks whose partial results
//   are summed afterwards (in a fixed order).  Inside a workgroup each
//   output row belongs to one wavefront, so every LDS element is updated by
//   one wavefront in row order.
// * Row norms: Algorithm squared_row_norms: Bt = B B^T once, then per row
//   sum_{k,j} V_k V_j Bt[J_j, J_k].  Short rows take one lane each; rows
//   longer than 32 entries are taken by the whole wavefront (lanes over k).
#include "internal.hpp"

namespace psk {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_gram_csr(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, int64_t n, int64_t d, int rb,
    int64_t rows_per_chunk, int nranges, double *__restrict__ part) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw);  // [rb][d]
  const int range = (int)(blockIdx.x % nranges);
  const int chunk = (int)(blockIdx.x / nranges);
  const int64_t r0 = (int64_t)range * rb;
  const int rows_here = (int)((r0 + rb <= d) ? rb : (d - r0));
  for (int64_t e = threadIdx.x; e < (int64_t)rb * d; e += blockDim.x) acc[e] = 0.0;
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t i0 = (int64_t)chunk * rows_per_chunk;
  int64_t i1 = i0 + rows_per_chunk;
  if (i1 > n) i1 = n;
  for (int64_t g = i0; g < i1; g += 64) {
    const int64_t i = g + lane;
    if (i < i1) {
      const int64_t p0 = indptr[i], p1 = indptr[i + 1];
      for (int64_t kk = p0; kk < p1; ++kk) {
        const int64_t c = (int64_t)indices[kk] - r0;
        if (c < 0 || c >= rows_here || (int)(c & 3) != wave) continue;
        const double vk = (double)vals[kk];
        double *arow = acc + c * d;
        for (int64_t h = p0; h < p1; ++h)
          atomicAdd(&arow[indices[h]], vk * (double)vals[h]);
      }
    }
  }
  __syncthreads();
  double *o = part + (int64_t)chunk * d * d + r0 * d;
  for (int64_t e = threadIdx.x; e < (int64_t)rows_here * d; e += blockDim.x) o[e] = acc[e];
}

// C = alpha * sum_chunks part + beta * C; both (i, j) and (j, i) take the
// upper-triangle entry (min, max), so C is exactly symmetric.
template <typename TO>
__global__ __launch_bounds__(256) void k_gram_reduce(const double *__restrict__ part,
                                                     int64_t d, int chunks, double alpha,
                                                     double beta, TO *__restrict__ C) {
  const int64_t dd = d * d;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= dd) return;
  const int64_t i = e / d, j = e % d;
  const int64_t src = i <= j ? e : j * d + i;
  double s = part[src];
  for (int c = 1; c < chunks; ++c) s += part[(int64_t)c * dd + src];
  double v = alpha * s;
  if (beta != 0.0) v += beta * (double)C[e];
  C[e] = (TO)v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_rownorm_csr(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, int64_t n, int64_t d,
    const double *__restrict__ Bt, double alpha, double beta, double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool have = i < n;
  int64_t p0 = 0, p1 = 0;
  if (have) {
    p0 = indptr[i];
    p1 = indptr[i + 1];
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

}  // namespace

int gram_csr(double alpha, const psk_mat &A, double beta, void *C, Arena &ws,
             hipStream_t st) {
  const int64_t d = A.d;
  if (d > 8192) return fail(PSK_EUNSUPPORTED, "CSR gram supports d <= 8192");
  int rb = (int)(8192 / d);  // rb x d FP64 rows in 64 KiB of LDS
  if (rb > 64) rb = 64;
  if (rb < 1) rb = 1;
  const int nranges = (int)ceil_div(d, rb);
  int64_t chunks = ceil_div(1024, nranges);
  if (chunks > 16) chunks = 16;
  if (chunks > A.n) chunks = A.n;
  if (chunks < 1) chunks = 1;
  const int64_t rows_per_chunk = ceil_div(A.n, chunks);
  chunks = ceil_div(A.n, rows_per_chunk);
  double *part = ws.take<double>((size_t)chunks * d * d);
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for CSR gram");
  const size_t lds = (size_t)rb * d * sizeof(double);
  const unsigned blocks = (unsigned)(nranges * chunks);
  KTimer timer("gram", st);
  if (A.dtype == PSK_F64)
    k_gram_csr<double><<<blocks, 256, lds, st>>>((const double *)A.values, A.indptr,
                                                 A.indices, A.n, d, rb, rows_per_chunk,
                                                 nranges, part);
  else
    k_gram_csr<float><<<blocks, 256, lds, st>>>((const float *)A.values, A.indptr,
                                                A.indices, A.n, d, rb, rows_per_chunk,
                                                nranges, part);
  const int64_t dd = d * d;
  if (A.dtype == PSK_F64)
    k_gram_reduce<double><<<(unsigned)ceil_div(dd, 256), 256, 0, st>>>(
        part, d, (int)chunks, alpha, beta, (double *)C);
  else
    k_gram_reduce<float><<<(unsigned)ceil_div(dd, 256), 256, 0, st>>>(
        part, d, (int)chunks, alpha, beta, (float *)C);
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

int rownorms_csr(double alpha, const psk_mat &A, const double *B, int64_t k,
                 double beta, double *x, Arena &ws, hipStream_t st) {
  const int64_t d = A.d;
  if (d > 8192) return fail(PSK_EUNSUPPORTED, "CSR row norms support d <= 8192");
  double *Bt = ws.take<double>((size_t)d * d);
  // B * B^T (d x d) with the FP64 GEMM
  int rc = dgemm(false, true, d, d, k, 1.0, B, k, B, k, 0.0, Bt, d, ws, st);
  if (rc) return rc;
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for CSR row norms");
  const unsigned blocks = (unsigned)ceil_div(A.n, 256);
  KTimer timer("rownorm", st);
  if (A.dtype == PSK_F64)
    k_rownorm_csr<double><<<blocks, 256, 0, st>>>((const double *)A.values, A.indptr,
                                                  A.indices, A.n, d, Bt, alpha, beta, x);
  else
    k_rownorm_csr<float><<<blocks, 256, 0, st>>>((const float *)A.values, A.indptr,
                                                 A.indices, A.n, d, Bt, alpha, beta, x);
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace psk
