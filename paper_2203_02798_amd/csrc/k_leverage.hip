// Leverage scores from a sketch, end to end (Algorithm
// ls_approximate_drineas of arXiv 2203.02798, section 4):
//   1. the sketch: S A (the algorithm as stated, m = 0) or G S A (m > 0);
//   2. its triangular factor R and R^{-1} (sketch_qr; the QR stands in for
//      the paper's SVD: A R^{-1} and A V Sigma^{-1} differ by an orthogonal
//      d x d factor, so their row norms agree);
//   3. optionally the Johnson-Lindenstrauss step X = R^{-1} Pi with Pi a d x t
//      Gaussian of variance 1/t (t = O(log n / eps^2) keeps every row norm to
//      within 1 +- eps), which cuts the dense row-norm product from n d^2 to
//      n d t multiply-adds;
//   4. theta_i = ||e_i^T A X||^2 (Algorithm squared_row_norms).
// Pi is drawn by the generator of G on counter stream 2: Pi[b, j] =
// z(row j, column b) / sqrt(t), so Pi^T is a t x d Gaussian of that stream.
//
// Kernels: k_jl_normals writes the unscaled normals of Pi (a thread per four
// consecutive columns b of one row j of Pi^T, stored as Pi[b, j] so that
// neighbouring threads write neighbouring j); k_widen_f32 turns an FP32 S A
// into the FP64 operand of the factorization.
#include "internal.hpp"

namespace psk {
namespace {

// Z[b * t + j] = z_{b mod 4}(q = b div 4, row j, stream 2), b < d, j < t.
__global__ __launch_bounds__(256) void k_jl_normals(int64_t d, int64_t t, uint64_t seed,
                                                    double *__restrict__ Z) {
  const int64_t nq = (d + 3) / 4;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nq * t) return;
  const int64_t q = idx / t, j = idx - q * t;
  double z[4];
  gauss4_f64((uint64_t)q, (uint32_t)j, seed, z, 2u);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t b = 4 * q + k;
    if (b < d) Z[b * t + j] = z[k];
  }
}

}  // namespace

int sketch_f64(const psk_mat &A, int64_t m, int64_t r, uint64_t seed, int prec, double *C,
               Arena &ws, hipStream_t st) {
  if (m > 0) return do_sketch_gcs(A, m, r, seed, prec, C, ws, st);
  // S A as its FP64 sums (FP32 A is widened exactly and summed in FP64)
  return do_sketch_cs(A, r, seed, C, ws, st, true);
}

int leverage_sketch_impl(const psk_mat &A, int64_t m, int64_t r, int64_t t, uint64_t seed,
                         int prec, double *theta, bool check_rank, Arena &ws, hipStream_t st) {
  const int64_t d = A.d;
  if (d > 4096) return fail(PSK_EUNSUPPORTED, "leverage_sketch supports d <= 4096");
  // rows of the sketch: G S A has m, S A alone has r
  const int64_t rows = m > 0 ? m : r;
  double *C = ws.take<double>((size_t)rows * d);
  double *R = ws.take<double>((size_t)d * d);
  double *Ri = ws.take<double>((size_t)d * d);
  double *X = t > 0 ? ws.take<double>((size_t)d * t) : Ri;
  const bool run = !ws.dry();
  if (run && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for leverage_sketch");
  const size_t mk = ws.mark();
  int rc;
  if ((rc = sketch_f64(A, m, r, seed, prec, C, ws, st))) return rc;
  ws.release(mk);
  int *flag = nullptr;
  if ((rc = sketch_qr_impl(C, rows, d, R, Ri, ws, st, &flag))) return rc;
  // the factorization's workspace stays taken: its pivot flag is read last
  const size_t mk2 = ws.mark();
  if (t > 0) {
    double *Z = ws.take<double>((size_t)d * t);
    if (run && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for leverage_sketch");
    if (run) {
      const int64_t thr = ((d + 3) / 4) * t;
      KTimer timer("jl_normals", st);
      k_jl_normals<<<(unsigned)ceil_div(thr, 256), 256, 0, st>>>(d, t, seed, Z);
    }
    if ((rc = dgemm(false, false, d, t, d, 1.0 / sqrt((double)t), Ri, d, Z, t, 0.0, X, t, ws,
                    st)))
      return rc;
  }
  ws.release(mk2);
  const int64_t k = t > 0 ? t : d;
  rc = A.format == PSK_DENSE ? rownorms_dense(1.0, A, X, k, 0.0, theta, ws, st)
                             : rownorms_csr(1.0, A, X, k, 0.0, theta, ws, st);
  if (rc) return rc;
  if (!run) return 0;
  PSK_HIP_TRY(hipGetLastError());
  if (!check_rank) return 0;
  // a NaN or infinity of A that a reduced-precision sketch did not carry
  // still reaches its row's score
  flag_nonfinite(theta, A.n, flag, st);
  int h = 0;
  PSK_HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  PSK_HIP_TRY(hipStreamSynchronize(st));
  return factor_status(h, "a Cholesky pivot was not positive: the sketch is numerically rank deficient");
}

}  // namespace psk
