// Column subset selection and the leverage scores of the selected columns
// (arXiv 2203.02798, section 4.1 Algorithm cgrrqr and section 4.3 Algorithm
// ls_hrn_exact).
//
// css_select: the sketch B = G S A (or S A for m == 0), then the first k
// steps of the column-pivoted Householder QR of B (Businger and Golub): at
// step j the remaining column with the largest norm of its rows j .. rows-1
// is chosen (lowest index on ties) and a Householder reflector that zeroes
// its rows below j is applied to every remaining column.  The chosen columns
// are the selection.  Only the permutation is kept (R is not returned).
//
// leverage_css: the exact leverage scores of A[:, K] for the selected K
// (Algorithm ls_direct on the column subset).  A[:, K] is never formed: its
// Gram matrix is the K x K block of A^T A, whose Cholesky factor R_K gives
// theta_i = ||e_i^T A[:, K] R_K^{-1}||^2 = ||e_i^T A B||^2 with B the d x k
// matrix that holds the rows of R_K^{-1} at the rows K and zeros elsewhere.
//
// Layout and kernels.  The sketch (rows x d, row-major) is transposed once so
// that every column is contiguous (k_transpose, 32 x 32 tiles through LDS).
// k_col_norms gives the squared column norms.  One k_qrcp_step launch per
// pivot: every workgroup finds the pivot p from the norms of the previous
// step (a redundant argmax over d values), and each wavefront owns one
// column: it forms w = v^T c with the reflector v read from column p, updates
// its column and recomputes the squared norm of its rows j+1 .. rows-1
// exactly (no downdating).  The norms are double-buffered across launches, so
// no launch reads what it writes; column p is only read during its step.
// Sums run over lanes in a fixed order and then a fixed butterfly, so the
// selection is deterministic.
#include "internal.hpp"

namespace psk {
namespace {

constexpr int kTile = 32;

// Bt[c * rows + i] = C[i * d + c]; blockIdx.x over row tiles, blockIdx.y
// over column tiles; 256 threads = 32 x 8.
__global__ __launch_bounds__(256) void k_transpose(const double *__restrict__ C, int64_t rows,
                                                   int64_t d, double *__restrict__ Bt) {
  __shared__ double tile[kTile][kTile + 1];
  const int64_t i0 = (int64_t)blockIdx.x * kTile, c0 = (int64_t)blockIdx.y * kTile;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < kTile; y += 8) {
    const int64_t i = i0 + y, c = c0 + tx;
    if (i < rows && c < d) tile[y][tx] = C[i * d + c];
  }
  __syncthreads();
  for (int y = ty; y < kTile; y += 8) {
    const int64_t c = c0 + y, i = i0 + tx;
    if (i < rows && c < d) Bt[c * rows + i] = tile[tx][y];
  }
}

// norms[c] = sum_i Bt[c, i]^2, a wavefront per column.
__global__ __launch_bounds__(256) void k_col_norms(const double *__restrict__ Bt, int64_t rows,
                                                   int64_t d, double *__restrict__ norms) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= d) return;
  const double *col = Bt + c * rows;
  double s = 0.0;
  for (int64_t i = lane; i < rows; i += 64) s = fma(col[i], col[i], s);
  s = wave_sum(s);
  if (lane == 0) norms[c] = s;
}

// Rows per lane that k_qrcp_step keeps in registers (the rows below the
// pivot row of up to 64 * kQrReg rows); longer columns stream through memory
// twice.  Both forms add the same terms in the same order.
constexpr int kQrReg = 16;

// (v, i) pair reduction: the larger value, the lower index on equal values.
__device__ __forceinline__ void argmax_merge(double &v, int &i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// One pivot step j.  nin: squared norms of rows j.. of the live columns, -1
// for chosen ones; nout receives the same for step j + 1.
__global__ __launch_bounds__(256) void k_qrcp_step(double *__restrict__ Bt, int64_t rows,
                                                   int64_t d, int64_t j,
                                                   const double *__restrict__ nin,
                                                   double *__restrict__ nout,
                                                   int32_t *__restrict__ cols) {
  __shared__ double sv[4];
  __shared__ int si[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // argmax over the live columns, lowest index on equal norms; a NaN norm
  // (non-finite input) counts as -0.5, below every other live column but
  // above the chosen ones (-1), so p is always a live column (j < d)
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int c = tid; c < d; c += 256) {
    const double v0 = nin[c];
    const double v = v0 != v0 ? -0.5 : v0;
    if (v > best) {
      best = v;
      bi = c;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
    argmax_merge(best, bi, __shfl_xor(best, off, 64), __shfl_xor(bi, off, 64));
  if (lane == 0) {
    sv[wave] = best;
    si[wave] = bi;
  }
  __syncthreads();
  best = sv[0];
  bi = si[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) argmax_merge(best, bi, sv[w], si[w]);
  const int p = bi;
  const double n2 = best;
  // no barrier below this point
  const int64_t c = (int64_t)blockIdx.x * 4 + wave;
  if (c >= d) return;
  const double nc = nin[c];
  if (nc < 0.0) {
    if (lane == 0) nout[c] = -1.0;
    return;
  }
  if (c == p) {
    if (lane == 0) {
      nout[c] = -1.0;
      cols[j] = (int32_t)c;
    }
    return;
  }
  double *col = Bt + c * rows;
  const double *x = Bt + (int64_t)p * rows;
  // reflector H = I - 2 v v^T / (v^T v), v = x - beta e_j on rows j..
  double v0 = 0.0, vtv = 1.0;
  const bool reflect = n2 > 0.0;
  if (reflect) {
    const double alpha = x[j];
    const double nx = sqrt(n2);
    const double beta = alpha >= 0.0 ? -nx : nx;
    v0 = alpha - beta;
    vtv = 2.0 * beta * (beta - alpha);
  }
  const double cj = col[j];
  const int64_t i0 = j + 1 + lane;
  double nn;
  if (rows - (j + 1) <= 64 * kQrReg) {
    double xr[kQrReg], cr[kQrReg];
#pragma unroll
    for (int t = 0; t < kQrReg; ++t) {
      const int64_t i = i0 + 64 * t;
      xr[t] = i < rows ? x[i] : 0.0;
      cr[t] = i < rows ? col[i] : 0.0;
    }
    double s = 0.0;
    if (reflect) {
      double part = 0.0;
#pragma unroll
      for (int t = 0; t < kQrReg; ++t) part = fma(xr[t], cr[t], part);
      s = 2.0 * fma(v0, cj, wave_sum(part)) / vtv;
    }
    double part2 = 0.0;
#pragma unroll
    for (int t = 0; t < kQrReg; ++t) {
      const int64_t i = i0 + 64 * t;
      const double y = fma(-s, xr[t], cr[t]);
      if (i < rows) col[i] = y;
      part2 = fma(y, y, part2);
    }
    nn = wave_sum(part2);
    if (lane == 0) col[j] = fma(-s, v0, cj);
  } else {
    double s = 0.0;
    if (reflect) {
      double part = 0.0;
#pragma unroll 4
      for (int64_t i = i0; i < rows; i += 64) part = fma(x[i], col[i], part);
      s = 2.0 * fma(v0, cj, wave_sum(part)) / vtv;
    }
    double part2 = 0.0;
#pragma unroll 4
    for (int64_t i = i0; i < rows; i += 64) {
      const double y = fma(-s, x[i], col[i]);
      col[i] = y;
      part2 = fma(y, y, part2);
    }
    nn = wave_sum(part2);
    if (lane == 0) col[j] = fma(-s, v0, cj);
  }
  if (lane == 0) nout[c] = nn;
}

// W[a, b] = G[cols[a], cols[b]] (k x k block of the d x d Gram matrix).
__global__ __launch_bounds__(256) void k_gather_block(const double *__restrict__ G, int64_t d,
                                                      const int32_t *__restrict__ cols, int64_t k,
                                                      double *__restrict__ W) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= k * k) return;
  const int64_t a = idx / k, b = idx - a * k;
  W[idx] = G[(int64_t)cols[a] * d + cols[b]];
}

// B (d x k, zero on entry) gets row a of X (k x k) at row cols[a].
__global__ __launch_bounds__(256) void k_scatter_rows(const double *__restrict__ X, int64_t k,
                                                      const int32_t *__restrict__ cols,
                                                      double *__restrict__ B) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= k * k) return;
  const int64_t a = idx / k, b = idx - a * k;
  B[(int64_t)cols[a] * k + b] = X[idx];
}

__global__ __launch_bounds__(256) void k_zero(double *__restrict__ p, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = 0.0;
}

unsigned grid_for(int64_t count) {
  const int64_t b = ceil_div(count, 256);
  return (unsigned)(b < 8192 ? b : 8192);
}

}  // namespace

int css_select_impl(const psk_mat &A, int64_t m, int64_t r, int64_t k, uint64_t seed, int prec,
                    int32_t *cols, Arena &ws, hipStream_t st) {
  const int64_t d = A.d;
  if (d > 4096) return fail(PSK_EUNSUPPORTED, "column subset selection supports d <= 4096");
  const int64_t rows = m > 0 ? m : r;
  double *C = ws.take<double>((size_t)rows * d);
  double *Bt = ws.take<double>((size_t)rows * d);
  double *na = ws.take<double>((size_t)d);
  double *nb = ws.take<double>((size_t)d);
  int *flag = ws.take<int>(2);
  const bool run = !ws.dry();
  if (run && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for css_select");
  const size_t mk = ws.mark();
  int rc;
  if ((rc = sketch_f64(A, m, r, seed, prec, C, ws, st))) return rc;
  ws.release(mk);
  if (!run) return 0;
  // pivots chosen by norms with a NaN in them are meaningless: the sketch is
  // checked first and read back before the selection runs
  k_zero<<<1, 64, 0, st>>>(reinterpret_cast<double *>(flag), 1);
  flag_nonfinite(C, rows * d, flag, st);
  int h = 0;
  PSK_HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  PSK_HIP_TRY(hipStreamSynchronize(st));
  if ((rc = factor_status(h, ""))) return rc;
  KTimer timer("qrcp", st);
  const dim3 tg((unsigned)ceil_div(rows, (int64_t)kTile), (unsigned)ceil_div(d, (int64_t)kTile));
  k_transpose<<<tg, 256, 0, st>>>(C, rows, d, Bt);
  const unsigned cb = (unsigned)ceil_div(d, (int64_t)4);
  k_col_norms<<<cb, 256, 0, st>>>(Bt, rows, d, na);
  for (int64_t j = 0; j < k; ++j) {
    k_qrcp_step<<<cb, 256, 0, st>>>(Bt, rows, d, j, na, nb, cols);
    double *t = na;
    na = nb;
    nb = t;
  }
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

int leverage_css_impl(const psk_mat &A, int64_t m, int64_t r, int64_t k, uint64_t seed, int prec,
                      double *theta, int32_t *cols, Arena &ws, hipStream_t st) {
  const int64_t d = A.d;
  if (d > 4096) return fail(PSK_EUNSUPPORTED, "leverage_css supports d <= 4096");
  int32_t *kc = cols ? cols : ws.take<int32_t>((size_t)k);
  double *G = ws.take<double>((size_t)d * d);
  double *W = ws.take<double>((size_t)k * k);
  double *R = ws.take<double>((size_t)k * k);
  double *X = ws.take<double>((size_t)k * k);
  double *B = ws.take<double>((size_t)d * k);
  int *flag = ws.take<int>(4);
  const bool run = !ws.dry();
  if (run && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for leverage_css");
  const size_t mk = ws.mark();
  int rc;
  if ((rc = css_select_impl(A, m, r, k, seed, prec, kc, ws, st))) return rc;
  ws.release(mk);
  rc = A.format == PSK_DENSE ? gram_dense(1.0, A, 0.0, G, ws, st, true)
                             : gram_csr(1.0, A, 0.0, G, ws, st, true);
  if (rc) return rc;
  ws.release(mk);
  if (run) k_gather_block<<<(unsigned)ceil_div(k * k, (int64_t)256), 256, 0, st>>>(G, d, kc, k, W);
  if ((rc = chol_factor(W, k, R, X, flag, ws, st))) return rc;
  ws.release(mk);
  if (run) {
    k_zero<<<grid_for(d * k), 256, 0, st>>>(B, d * k);
    k_scatter_rows<<<(unsigned)ceil_div(k * k, (int64_t)256), 256, 0, st>>>(X, k, kc, B);
  }
  rc = A.format == PSK_DENSE ? rownorms_dense(1.0, A, B, k, 0.0, theta, ws, st)
                             : rownorms_csr(1.0, A, B, k, 0.0, theta, ws, st);
  if (rc) return rc;
  if (!run) return 0;
  PSK_HIP_TRY(hipGetLastError());
  flag_nonfinite(theta, A.n, flag, st);
  int h = 0;
  PSK_HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  PSK_HIP_TRY(hipStreamSynchronize(st));
  return factor_status(h, "a Cholesky pivot was not positive: the selected columns are numerically rank deficient");
}

}  // namespace psk
