// Direct least squares and exact leverage scores from the Gram matrix, and
// the sketch-and-solve least-squares solver.
//
// Paper mapping (arXiv 2203.02798), section 4 (applications):
//   leverage_gram     Algorithm ls_direct: B = A^T A, theta_i =
//                     ||e_i^T A V Sigma^{-1}||^2 from the SVD of B;
//   lsq_gram          Algorithm least_squares_gram: B = A^T A, c = A^T b,
//                     x = V Sigma^+ V^T c;
//   lsq_sketch_solve  Algorithm least_squares_approx: [A~ b~] = G S [A b],
//                     x = argmin ||A~ x - b~|| from the SVD of A~.
// As in the factorization of the sketch, a triangular factor stands in for
// the SVD: with B = R^T R (Cholesky) or A~ = Q R (sketch_qr), A R^{-1} has
// the column space of A V Sigma^{-1} and orthonormal columns, so the
// leverage scores and the least-squares solutions are the same.  Full
// column rank is assumed (the paper's truncation is not applied): a
// Cholesky pivot that is not positive returns PSK_ERANK.  The Gram route
// squares the condition number (B is as ill-conditioned as A^2); the
// sketch-and-solve route works on A~ through its QR.
//
// Kernels (all sums in a fixed order):
//   k_atb_csr / k_atb_dense  partial A^T b per block of rows (a wavefront's
//                            private LDS row for CSR, one column per thread
//                            for dense), written per block;
//   k_sum_parts              the block partials summed in block order;
//   k_trmv_t                 y = X^T c for upper triangular X (a thread per
//                            output, the terms in row order);
//   k_trmv_n                 x (+)= X y (a wavefront per row, a fixed
//                            reduction tree);
//   k_resid_dense            r = b - C x for a dense FP64 C (a wavefront per
//                            row);
//   k_augment_csr / _dense   [A b] with FP64 values (sketch-and-solve
//                            sketches it once, so G is drawn once), and
//                            k_split_aug splits its sketch into A~ and b~.
// sketch-and-solve applies the semi-normal equations x = X X^T C^T b~ with
// C = A~ and X = R^{-1}, then one correction with the residual b~ - C x
// (corrected semi-normal equations: the accuracy of the QR solution).
#include "internal.hpp"

namespace psk {
namespace {

constexpr int kAtbBlocks = 512;  // row blocks of A^T b
constexpr int kDenseCols = 16;   // columns a thread of k_atb_dense holds (d <= 4096)

__device__ __forceinline__ void row_block(int64_t n, int64_t &r0, int64_t &r1) {
  const int64_t per = ceil_div(n, (int64_t)gridDim.x);
  r0 = (int64_t)blockIdx.x * per;
  r1 = r0 + per < n ? r0 + per : n;
}

// part[blk][j] = sum over the block's rows i of A[i, j] b[i] (CSR): lane per
// row, the row's entries in order, into the wavefront's LDS row (lanes of one
// instruction that share a column are applied in lane order); the
// wavefronts' rows are then summed in wavefront order.
template <typename T>
__global__ __launch_bounds__(256) void k_atb_csr(const T *__restrict__ vals,
                                                 const int64_t *__restrict__ indptr,
                                                 const int32_t *__restrict__ indices, int64_t n,
                                                 int64_t d, int wpb, const double *__restrict__ b,
                                                 double *__restrict__ part) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *acc = reinterpret_cast<double *>(smem_raw);  // wpb x d
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t c = threadIdx.x; c < (int64_t)wpb * d; c += 256) acc[c] = 0.0;
  __syncthreads();
  int64_t r0, r1;
  row_block(n, r0, r1);
  if (wave < wpb) {
    double *aw = acc + (int64_t)wave * d;
    for (int64_t base = r0 + (int64_t)wave * 64; base < r1; base += 64 * wpb) {
      const int64_t i = base + lane;
      if (i < r1) {
        const double bi = b[i];
        const int64_t p1 = indptr[i + 1];
        for (int64_t p = indptr[i]; p < p1; ++p) atomicAdd(&aw[indices[p]], (double)vals[p] * bi);
      }
    }
  }
  __syncthreads();
  for (int64_t j = threadIdx.x; j < d; j += 256) {
    double s = 0.0;
    for (int w = 0; w < wpb; ++w) s += acc[(int64_t)w * d + j];
    part[(int64_t)blockIdx.x * d + j] = s;
  }
}

// the same for dense A (row stride ld): thread t holds columns t + 256 q
template <typename T>
__global__ __launch_bounds__(256) void k_atb_dense(const T *__restrict__ A, int64_t ld,
                                                   int64_t n, int64_t d,
                                                   const double *__restrict__ b,
                                                   double *__restrict__ part) {
  int64_t r0, r1;
  row_block(n, r0, r1);
  double acc[kDenseCols];
#pragma unroll
  for (int q = 0; q < kDenseCols; ++q) acc[q] = 0.0;
  for (int64_t i = r0; i < r1; ++i) {
    const double bi = b[i];
    const T *row = A + i * ld;
#pragma unroll
    for (int q = 0; q < kDenseCols; ++q) {
      const int64_t j = threadIdx.x + 256 * q;
      if (j < d) acc[q] = fma((double)row[j], bi, acc[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < kDenseCols; ++q) {
    const int64_t j = threadIdx.x + 256 * q;
    if (j < d) part[(int64_t)blockIdx.x * d + j] = acc[q];
  }
}

// out[j] = sum_p part[p][j], p in order
__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ part, int nparts,
                                                   int64_t d, double *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= d) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * d + j];
  out[j] = s;
}

// y[j] = sum_{i <= j} X[i][j] c[i] (X upper triangular, row-major)
__global__ __launch_bounds__(256) void k_trmv_t(const double *__restrict__ X, int64_t d,
                                                const double *__restrict__ c,
                                                double *__restrict__ y) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= d) return;
  double s = 0.0;
  for (int64_t i = 0; i <= j; ++i) s = fma(X[i * d + j], c[i], s);
  y[j] = s;
}

// x[i] (+)= sum_{j >= i} X[i][j] y[j]: a wavefront per row
__global__ __launch_bounds__(256) void k_trmv_n(const double *__restrict__ X, int64_t d,
                                                const double *__restrict__ y,
                                                double *__restrict__ x, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= d) return;
  double s = 0.0;
  for (int64_t j = i + lane; j < d; j += 64) s = fma(X[i * d + j], y[j], s);
  s = wave_sum(s);
  if (lane == 0) x[i] = accumulate ? x[i] + s : s;
}

// r[i] = b[i] - sum_j C[i][j] x[j] (C dense FP64, m x d): a wavefront per row
__global__ __launch_bounds__(256) void k_resid_dense(const double *__restrict__ C, int64_t m,
                                                     int64_t d, const double *__restrict__ x,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= m) return;
  double s = 0.0;
  for (int64_t j = lane; j < d; j += 64) s = fma(C[i * d + j], x[j], s);
  s = wave_sum(s);
  if (lane == 0) r[i] = b[i] - s;
}

// [A b] as CSR with FP64 values: row i's entries, then (d, b_i)
template <typename T>
__global__ __launch_bounds__(256) void k_augment_csr(const T *__restrict__ vals,
                                                     const int64_t *__restrict__ indptr,
                                                     const int32_t *__restrict__ indices,
                                                     int64_t n, int64_t d,
                                                     const double *__restrict__ b,
                                                     int64_t *__restrict__ oip,
                                                     int32_t *__restrict__ oidx,
                                                     double *__restrict__ oval) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i > n) return;
  oip[i] = (i < n ? indptr[i] : indptr[n]) + i;
  if (i == n) return;
  const int64_t p0 = indptr[i], p1 = indptr[i + 1], o = p0 + i;
  for (int64_t p = p0; p < p1; ++p) {
    oidx[o + p - p0] = indices[p];
    oval[o + p - p0] = (double)vals[p];
  }
  oidx[o + p1 - p0] = (int32_t)d;
  oval[o + p1 - p0] = b[i];
}

// [A b] dense, FP64, row stride d + 1
template <typename T>
__global__ __launch_bounds__(256) void k_augment_dense(const T *__restrict__ A, int64_t ld,
                                                       int64_t n, int64_t d,
                                                       const double *__restrict__ b,
                                                       double *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t w = d + 1;
  if (e >= n * w) return;
  const int64_t i = e / w, j = e - i * w;
  out[e] = j < d ? (double)A[i * ld + j] : b[i];
}

// C (m x d) and cb (m) from the sketch of [A b] (m x (d + 1))
__global__ __launch_bounds__(256) void k_split_aug(const double *__restrict__ Ca, int64_t m,
                                                   int64_t d, double *__restrict__ C,
                                                   double *__restrict__ cb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t w = d + 1;
  if (e >= m * w) return;
  const int64_t i = e / w, j = e - i * w;
  if (j < d) C[i * d + j] = Ca[e];
  else cb[i] = Ca[e];
}

// c = A^T b (d FP64) through kAtbBlocks row-block partials
int atb(const psk_mat &A, const double *b, double *c, Arena &ws, hipStream_t st) {
  const int64_t d = A.d;
  if (A.format == PSK_DENSE && d > 256 * kDenseCols)
    return fail(PSK_EUNSUPPORTED, "A^T b of dense A supports d <= 4096");
  int wpb = 4;
  while (wpb > 1 && (size_t)wpb * d * sizeof(double) > 65536) --wpb;
  if (A.format == PSK_CSR && (size_t)d * sizeof(double) > 65536)
    return fail(PSK_EUNSUPPORTED, "A^T b of CSR A supports d <= 8192");
  double *part = ws.take<double>((size_t)kAtbBlocks * d);
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for A^T b");
  if (A.format == PSK_CSR) {
    const size_t lds = (size_t)wpb * d * sizeof(double);
    if (A.dtype == PSK_F64)
      k_atb_csr<double><<<kAtbBlocks, 256, lds, st>>>((const double *)A.values, A.indptr,
                                                      A.indices, A.n, d, wpb, b, part);
    else
      k_atb_csr<float><<<kAtbBlocks, 256, lds, st>>>((const float *)A.values, A.indptr,
                                                     A.indices, A.n, d, wpb, b, part);
  } else if (A.dtype == PSK_F64) {
    k_atb_dense<double><<<kAtbBlocks, 256, 0, st>>>((const double *)A.values, A.ld, A.n, d, b,
                                                    part);
  } else {
    k_atb_dense<float><<<kAtbBlocks, 256, 0, st>>>((const float *)A.values, A.ld, A.n, d, b,
                                                   part);
  }
  k_sum_parts<<<(unsigned)ceil_div(d, 256), 256, 0, st>>>(part, kAtbBlocks, d, c);
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

// x (+)= X X^T c (X = R^{-1}, upper triangular d x d); y: d scratch
void apply_xxt(const double *X, int64_t d, const double *c, double *y, double *x,
               int accumulate, hipStream_t st) {
  k_trmv_t<<<(unsigned)ceil_div(d, 256), 256, 0, st>>>(X, d, c, y);
  k_trmv_n<<<(unsigned)ceil_div(d, 4), 256, 0, st>>>(X, d, y, x, accumulate);
}

// B = A^T A in FP64 (both triangles) whatever the dtype of A
int gram_f64(const psk_mat &A, double *B, Arena &ws, hipStream_t st) {
  return A.format == PSK_DENSE ? gram_dense(1.0, A, 0.0, B, ws, st, true)
                               : gram_csr(1.0, A, 0.0, B, ws, st, true);
}

// the status word of the factorization (and of the finiteness check of the
// result, count values at out), read back once the stream reaches it
int rank_check(int *flag, const double *out, int64_t count, hipStream_t st) {
  flag_nonfinite(out, count, flag, st);
  int h = 0;
  PSK_HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  PSK_HIP_TRY(hipStreamSynchronize(st));
  return factor_status(h, "a Cholesky pivot was not positive: A is numerically rank deficient");
}

}  // namespace

int leverage_gram_impl(const psk_mat &A, double *theta, Arena &ws, hipStream_t st) {
  const int64_t d = A.d;
  if (d > 4096) return fail(PSK_EUNSUPPORTED, "leverage_gram supports d <= 4096");
  double *B = ws.take<double>((size_t)d * d);
  double *R = ws.take<double>((size_t)d * d);
  double *X = ws.take<double>((size_t)d * d);
  int *flag = ws.take<int>(4);
  if (!ws.dry() && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for leverage_gram");
  const size_t mk = ws.mark();
  int rc;
  if ((rc = gram_f64(A, B, ws, st))) return rc;
  ws.release(mk);
  if ((rc = chol_factor(B, d, R, X, flag, ws, st))) return rc;
  ws.release(mk);
  rc = A.format == PSK_DENSE ? rownorms_dense(1.0, A, X, d, 0.0, theta, ws, st)
                             : rownorms_csr(1.0, A, X, d, 0.0, theta, ws, st);
  if (rc || ws.dry()) return rc;
  return rank_check(flag, theta, A.n, st);
}

int lsq_gram_impl(const psk_mat &A, const double *b, double *x, Arena &ws, hipStream_t st) {
  const int64_t d = A.d;
  if (d > 4096) return fail(PSK_EUNSUPPORTED, "lsq_gram supports d <= 4096");
  double *B = ws.take<double>((size_t)d * d);
  double *R = ws.take<double>((size_t)d * d);
  double *X = ws.take<double>((size_t)d * d);
  double *c = ws.take<double>((size_t)d);
  double *y = ws.take<double>((size_t)d);
  int *flag = ws.take<int>(4);
  if (!ws.dry() && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for lsq_gram");
  const size_t mk = ws.mark();
  int rc;
  if ((rc = gram_f64(A, B, ws, st))) return rc;
  ws.release(mk);
  if ((rc = chol_factor(B, d, R, X, flag, ws, st))) return rc;
  ws.release(mk);
  if ((rc = atb(A, b, c, ws, st))) return rc;
  ws.release(mk);
  if (ws.dry()) return 0;
  apply_xxt(X, d, c, y, x, 0, st);
  PSK_HIP_TRY(hipGetLastError());
  return rank_check(flag, x, d, st);
}

int lsq_sketch_solve_impl(const psk_mat &A, const double *b, double *x, int64_t m, int64_t r,
                          uint64_t seed, int prec, Arena &ws, hipStream_t st) {
  const int64_t d = A.d;
  if (d > 4096) return fail(PSK_EUNSUPPORTED, "lsq_sketch_solve supports d <= 4096");
  double *Ca = ws.take<double>((size_t)m * (d + 1));
  double *C = ws.take<double>((size_t)m * d);
  double *cb = ws.take<double>((size_t)m);
  double *rr = ws.take<double>((size_t)m);
  double *R = ws.take<double>((size_t)d * d);
  double *X = ws.take<double>((size_t)d * d);
  double *z = ws.take<double>((size_t)d);
  double *y = ws.take<double>((size_t)d);
  if (!ws.dry() && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for lsq_sketch_solve");
  const size_t mk = ws.mark();
  int rc;
  // [A~ b~] = G S [A b], one sketch of the matrix with b as its last
  // column (FP64 values), so that G is drawn once
  psk_mat ab{};
  ab.dtype = PSK_F64;
  ab.n = A.n;
  ab.d = d + 1;
  const bool run = !ws.dry();
  if (A.format == PSK_CSR) {
    int64_t *oip = ws.take<int64_t>((size_t)A.n + 1);
    int32_t *oidx = ws.take<int32_t>((size_t)(A.nnz + A.n));
    double *oval = ws.take<double>((size_t)(A.nnz + A.n));
    if (run && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for lsq_sketch_solve");
    ab.format = PSK_CSR;
    ab.ld = d + 1;
    ab.nnz = A.nnz + A.n;
    ab.values = oval;
    ab.indptr = oip;
    ab.indices = oidx;
    if (run) {
      const unsigned g = (unsigned)ceil_div(A.n + 1, 256);
      if (A.dtype == PSK_F64)
        k_augment_csr<double><<<g, 256, 0, st>>>((const double *)A.values, A.indptr, A.indices,
                                                 A.n, d, b, oip, oidx, oval);
      else
        k_augment_csr<float><<<g, 256, 0, st>>>((const float *)A.values, A.indptr, A.indices,
                                                A.n, d, b, oip, oidx, oval);
    }
  } else {
    double *ad = ws.take<double>((size_t)A.n * (d + 1));
    if (run && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for lsq_sketch_solve");
    ab.format = PSK_DENSE;
    ab.ld = d + 1;
    ab.values = ad;
    if (run) {
      const unsigned g = (unsigned)ceil_div(A.n * (d + 1), 256);
      if (A.dtype == PSK_F64)
        k_augment_dense<double><<<g, 256, 0, st>>>((const double *)A.values, A.ld, A.n, d, b,
                                                   ad);
      else
        k_augment_dense<float><<<g, 256, 0, st>>>((const float *)A.values, A.ld, A.n, d, b, ad);
    }
  }
  if ((rc = do_sketch_gcs(ab, m, r, seed, prec, Ca, ws, st))) return rc;
  ws.release(mk);
  if (run)
    k_split_aug<<<(unsigned)ceil_div(m * (d + 1), 256), 256, 0, st>>>(Ca, m, d, C, cb);
  // the QR's workspace stays held: its pivot flag is read at the end
  int *flag = nullptr;
  if ((rc = sketch_qr_impl(C, m, d, R, X, ws, st, &flag))) return rc;
  const size_t mk2 = ws.mark();
  psk_mat cm{};
  cm.format = PSK_DENSE;
  cm.dtype = PSK_F64;
  cm.n = m;
  cm.d = d;
  cm.ld = d;
  cm.values = C;
  // x = X X^T C^T b~, then once more with the residual b~ - C x
  if ((rc = atb(cm, cb, z, ws, st))) return rc;
  ws.release(mk2);
  if (!ws.dry()) {
    apply_xxt(X, d, z, y, x, 0, st);
    k_resid_dense<<<(unsigned)ceil_div(m, 4), 256, 0, st>>>(C, m, d, x, cb, rr);
  }
  if ((rc = atb(cm, rr, z, ws, st))) return rc;
  ws.release(mk2);
  if (ws.dry()) return 0;
  apply_xxt(X, d, z, y, x, 1, st);
  PSK_HIP_TRY(hipGetLastError());
  return rank_check(flag, x, d, st);
}

}  // namespace psk
