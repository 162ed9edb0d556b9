// R and R^{-1} of an FP64 sketch C (m x d) on gfx950 by shifted
// Cholesky-QR with two extra Cholesky-QR passes (sCQR3: Fukaya, Kannan,
// Nakatsukasa, Yamamoto, Yanagisawa, "Shifted Cholesky QR for computing the
// QR factorization of ill-conditioned matrices", SIAM J. Sci. Comput. 2020).
//
// Paper mapping (arXiv 2203.02798): the sketch-based algorithms
// (ls_approximate_drineas, least_squares_precondition) factor the sketch
// G*S*A and use the inverse factor as an orthogonaliser / right
// preconditioner; the paper uses an SVD, here the triangular factor of a QR
// (the same column space, so the same leverage scores and an equally good
// preconditioner).  Cholesky-QR keeps the work in GEMMs on the matrix cores
// (W = C^T C, Q = C R^{-1}); the shift s = 11 (m d + d (d+1)) u ||C||_F^2 on
// the first pass keeps the Cholesky factorization defined for condition
// numbers up to about 1/u, and two unshifted passes restore orthogonality.
//
// The d x d Cholesky is blocked (64 columns): a one-workgroup kernel factors
// the diagonal block in LDS and inverts it, then two GEMMs form the block
// row of R and update the trailing matrix.  R^{-1} is assembled by block
// columns: X[0:j, j] = -X[0:j, 0:j] R[0:j, j] X[j, j].
#include "internal.hpp"

namespace psk {
namespace {

constexpr int kNB = 64;

__global__ void k_fill(double *__restrict__ p, int64_t count, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// W[i][i] += coef * trace(W)
__global__ __launch_bounds__(256) void k_shift_diag(double *__restrict__ W, int64_t d,
                                                    double coef) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 256) s += W[i * d + i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double tr = red[0] + red[1] + red[2] + red[3];
  for (int64_t i = threadIdx.x; i < d; i += 256) W[i * d + i] += coef * tr;
}

// Upper Cholesky U^T U = W[j0:j0+nb, j0:j0+nb] and its inverse by one
// wavefront: lane j keeps column j of the block in registers; each step
// publishes one row through a 64-entry LDS buffer that every lane reads with
// broadcast loads (no barriers beyond the wavefront).  Rows stay unscaled
// during elimination (step k subtracts U[k][i] U[k][j] / U[k][k]) and are
// scaled by 1/sqrt(U[k][k]) at the end.  A block narrower than 64 is padded
// with the identity.  The inverse is back substitution on each column:
// x_i = (e_j[i] - sum_{k>i} U[i][k] x_k) / U[i][i].
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(64) void k_potrf_block(const double *__restrict__ W,
                                                    int64_t d, int64_t j0, int nb,
                                                    double *__restrict__ R,
                                                    double *__restrict__ X,
                                                    int *__restrict__ flag) {
  __shared__ double rowbuf[kNB];
  const int j = threadIdx.x;
  double c[kNB];
#pragma unroll
  for (int i = 0; i < kNB; ++i)
    c[i] = (i < nb && j < nb) ? W[(j0 + i) * d + j0 + j] : (i == j ? 1.0 : 0.0);
  bool bad = false;
  double mypiv = 1.0;  // this lane's pivot U[j][j] once step j is reached
#pragma clang loop unroll(full)
  for (int k = 0; k < kNB; ++k) {
    rowbuf[j] = c[k];  // row k of the (unscaled) factor
    wave_sync_lds();
    double piv = rowbuf[k];
    mypiv = (k == j) ? piv : mypiv;
    bad |= !(piv > 0.0);
    piv = piv > 0.0 ? piv : 1.0;
    const double f = c[k] / piv;  // U[k][j] / U[k][k]
#pragma clang loop unroll(full)
    for (int i = k + 1; i < kNB; ++i) c[i] -= rowbuf[i] * f;
    wave_sync_lds();
  }
  // scale row k by 1/sqrt(U[k][k]) (the diagonal entries sit in lane k)
  rowbuf[j] = sqrt(mypiv > 0.0 ? mypiv : 1.0);
  wave_sync_lds();
#pragma unroll
  for (int k = 0; k < kNB; ++k) {
    const double v = (k <= j) ? c[k] / rowbuf[k] : 0.0;
    if (k < nb && j < nb) R[(j0 + k) * d + j0 + j] = v;
  }
  if (bad && j == 0) atomicOr(flag, 1);
}

// Inverse of the upper-triangular diagonal block R[j0:j0+nb, j0:j0+nb] into
// the same block of X: lane j solves U x = e_j by back substitution,
// x_i = (e_j[i] - sum_{k>i} U[i][k] x_k) / U[i][i], reading U from LDS
// (broadcast loads).  Padding beyond nb is the identity.
__global__ __launch_bounds__(64) void k_trinv_block(const double *__restrict__ R, int64_t d,
                                                    int64_t j0, int nb,
                                                    double *__restrict__ X) {
  __shared__ double Ul[kNB][kNB + 1];
  const int j = threadIdx.x;
#pragma unroll
  for (int i = 0; i < kNB; ++i)
    Ul[i][j] = (i < nb && j < nb) ? R[(j0 + i) * d + j0 + j] : (i == j ? 1.0 : 0.0);
  wave_sync_lds();
  double x[kNB];
#pragma clang loop unroll(full)
  for (int i = kNB - 1; i >= 0; --i) {
    double s = (i == j) ? 1.0 : 0.0;
#pragma clang loop unroll(full)
    for (int k = i + 1; k < kNB; ++k) s -= Ul[i][k] * x[k];
    x[i] = s / Ul[i][i];
  }
  if (j < nb) {
#pragma unroll
    for (int i = 0; i < kNB; ++i)
      if (i < nb) X[(j0 + i) * d + j0 + j] = (i <= j) ? x[i] : 0.0;
  }
}

void fill(double *p, int64_t count, double v, hipStream_t st) {
  k_fill<<<(unsigned)ceil_div(count, 256), 256, 0, st>>>(p, count, v);
}

// Upper Cholesky of W (destroyed) into R, and X = R^{-1}.  T is d x d scratch.
int chol_inv(double *W, int64_t d, double *R, double *X, double *T, int *flag,
             Arena &ws, hipStream_t st) {
  const bool run = !ws.dry();
  if (run) {
    fill(R, d * d, 0.0, st);
    fill(X, d * d, 0.0, st);
  }
  const size_t mk = ws.mark();
  for (int64_t j0 = 0; j0 < d; j0 += kNB) {
    const int nb = (int)((d - j0) < kNB ? (d - j0) : kNB);
    if (run) {
      k_potrf_block<<<1, 64, 0, st>>>(W, d, j0, nb, R, X, flag);
      k_trinv_block<<<1, 64, 0, st>>>(R, d, j0, nb, X);
    }
    const int64_t rest = d - j0 - nb;
    if (rest > 0) {
      int rc = dgemm(true, false, nb, rest, nb, 1.0, X + j0 * d + j0, d,
                     W + j0 * d + j0 + nb, d, 0.0, R + j0 * d + j0 + nb, d, ws, st);
      ws.release(mk);
      if (rc) return rc;
      rc = dgemm(true, false, rest, rest, nb, -1.0, R + j0 * d + j0 + nb, d,
                 R + j0 * d + j0 + nb, d, 1.0, W + (j0 + nb) * d + j0 + nb, d, ws, st);
      ws.release(mk);
      if (rc) return rc;
    }
  }
  for (int64_t j0 = kNB; j0 < d; j0 += kNB) {
    const int nb = (int)((d - j0) < kNB ? (d - j0) : kNB);
    int rc = dgemm(false, false, j0, nb, j0, 1.0, X, d, R + j0, d, 0.0, T, d, ws, st);
    ws.release(mk);
    if (rc) return rc;
    rc = dgemm(false, false, j0, nb, nb, -1.0, T, d, X + j0 * d + j0, d, 0.0, X + j0, d,
               ws, st);
    ws.release(mk);
    if (rc) return rc;
  }
  return 0;
}

}  // namespace

int sketch_qr_impl(const double *C, int64_t m, int64_t d, double *R, double *Rinv,
                   Arena &ws, hipStream_t st, int **flag_out) {
  if (d > 4096) return fail(PSK_EUNSUPPORTED, "sketch_qr supports d <= 4096");
  double *Qa = ws.take<double>((size_t)m * d);
  double *Qb = ws.take<double>((size_t)m * d);
  double *W = ws.take<double>((size_t)d * d);
  double *R1 = ws.take<double>((size_t)d * d);
  double *R2 = ws.take<double>((size_t)d * d);
  double *R3 = ws.take<double>((size_t)d * d);
  double *X1 = ws.take<double>((size_t)d * d);
  double *X2 = ws.take<double>((size_t)d * d);
  double *X3 = ws.take<double>((size_t)d * d);
  double *T = ws.take<double>((size_t)d * d);
  int *flag = ws.take<int>(4);
  const bool run = !ws.dry();
  if (run && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for sketch_qr");
  const size_t mk = ws.mark();
  int rc;
  KTimer timer("sketch_qr", st);
  if (run) k_fill<<<1, 64, 0, st>>>(reinterpret_cast<double *>(flag), 2, 0.0);
  if (flag_out) *flag_out = flag;
  // pass 1 (shifted): W = C^T C + s I
  if ((rc = dgemm(true, false, d, d, m, 1.0, C, d, C, d, 0.0, W, d, ws, st))) return rc;
  ws.release(mk);
  const double u = 1.1102230246251565e-16;
  const double coef = 11.0 * ((double)m * d + (double)d * (d + 1)) * u;
  if (run) k_shift_diag<<<1, 256, 0, st>>>(W, d, coef);
  if ((rc = chol_inv(W, d, R1, X1, T, flag, ws, st))) return rc;
  ws.release(mk);
  if ((rc = dgemm(false, false, m, d, d, 1.0, C, d, X1, d, 0.0, Qa, d, ws, st))) return rc;
  ws.release(mk);
  // pass 2
  if ((rc = dgemm(true, false, d, d, m, 1.0, Qa, d, Qa, d, 0.0, W, d, ws, st))) return rc;
  ws.release(mk);
  if ((rc = chol_inv(W, d, R2, X2, T, flag, ws, st))) return rc;
  ws.release(mk);
  if ((rc = dgemm(false, false, m, d, d, 1.0, Qa, d, X2, d, 0.0, Qb, d, ws, st))) return rc;
  ws.release(mk);
  // pass 3
  if ((rc = dgemm(true, false, d, d, m, 1.0, Qb, d, Qb, d, 0.0, W, d, ws, st))) return rc;
  ws.release(mk);
  if ((rc = chol_inv(W, d, R3, X3, T, flag, ws, st))) return rc;
  ws.release(mk);
  // R = R3 R2 R1, R^{-1} = X1 X2 X3
  if ((rc = dgemm(false, false, d, d, d, 1.0, R2, d, R1, d, 0.0, T, d, ws, st))) return rc;
  ws.release(mk);
  if ((rc = dgemm(false, false, d, d, d, 1.0, R3, d, T, d, 0.0, R, d, ws, st))) return rc;
  ws.release(mk);
  if ((rc = dgemm(false, false, d, d, d, 1.0, X1, d, X2, d, 0.0, T, d, ws, st))) return rc;
  ws.release(mk);
  if ((rc = dgemm(false, false, d, d, d, 1.0, T, d, X3, d, 0.0, Rinv, d, ws, st))) return rc;
  ws.release(mk);
  if (run) PSK_HIP_TRY(hipGetLastError());
  return 0;
}

}  // namespace psk
