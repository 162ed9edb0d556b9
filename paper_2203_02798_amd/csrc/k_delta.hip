// The perturbation of a sketch against a reference sketch,
// delta = ||(C^ - C) R^{-1}||_2 with R from the QR of C.
//
// Paper mapping (arXiv 2203.02798): the sketches of Algorithms
// ls_approximate_drineas and least_squares_precondition are used through
// R^{-1} only; C^ R^{-1} = Q + F with ||F||_2 = delta keeps the singular
// values of R^ R^{-1} in [1 - delta, 1 + delta], so the leverage scores from
// C^ and C differ by a factor in [(1 + delta)^-2, (1 - delta)^-2] and the
// preconditioned condition numbers by (1 + delta) / (1 - delta).  delta
// states how much a reduced-precision (BF16, FP8) sketch moves those results
// against the FP64 one.
//
// Steps: R^{-1} of C (sketch_qr), D = C^ - C, F = D R^{-1}, W = F^T F (all
// FP64 on the matrix cores); then ||F||_2^2 = lambda_max(W) by repeated
// squaring, M_0 = W / ||W||_F, M_{i+1} = M_i^2 / ||M_i^2||_F (each squaring
// doubles the power, so after kSquarings the top eigenvector dominates
// every column by (lambda_2 / lambda_1)^(2^kSquarings)), and the Rayleigh
// quotient v^T W v of the largest column v of the last M.  The estimate is
// a Rayleigh quotient, so it never exceeds lambda_max.
#include "internal.hpp"

namespace psk {
namespace {

constexpr int kSquarings = 12;

__global__ __launch_bounds__(256) void k_sub(const double *__restrict__ a,
                                             const double *__restrict__ b, int64_t len,
                                             double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < len) out[i] = a[i] - b[i];
}

__device__ double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
  return t;
}

// M <- M / ||M||_F (M = 0 stays 0) in two launches: k_frob_parts sums the
// squares of kNrmParts equal slices of M, one workgroup each; k_frob_scale
// adds the slice sums (one wavefront's fixed butterfly, the same in every
// workgroup) and scales M.
constexpr int kNrmParts = 64;

__global__ __launch_bounds__(256) void k_frob_parts(const double *__restrict__ M, int64_t len,
                                                    double *__restrict__ part) {
  __shared__ double red[4];
  const int64_t per = ceil_div(len, (int64_t)kNrmParts);
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < len ? lo + per : len;
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += M[i] * M[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_frob_scale(double *__restrict__ M, int64_t len,
                                                    const double *__restrict__ part) {
  static_assert(kNrmParts == 64, "one partial per lane");
  const double t = wave_sum(part[threadIdx.x & 63]);
  const double nrm = sqrt(t);
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * 256)
    M[i] *= inv;
}

// Squared column norms of M in kColSlices row slices: workgroup (x, y) takes
// columns 64 x .. 64 x + 63 (lanes) over the rows of slice y, its four
// wavefronts every fourth row, and writes the slice's sums (wavefronts in
// order) to cnp[y][j].
constexpr int kColSlices = 16;

__global__ __launch_bounds__(256) void k_col_norms(const double *__restrict__ M, int64_t d,
                                                   double *__restrict__ cnp) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + lane;
  const int64_t per = ceil_div(d, (int64_t)kColSlices);
  const int64_t lo = (int64_t)blockIdx.y * per;
  const int64_t hi = lo + per < d ? lo + per : d;
  double s = 0.0;
  if (j < d)
    for (int64_t i = lo + w; i < hi; i += 4) {
      const double v = M[i * d + j];
      s += v * v;
    }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < d) cnp[blockIdx.y * d + j] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// The Rayleigh quotient's terms for v = the column of M of largest norm (the
// first such column on ties; the slices' sums added in slice order): every
// workgroup finds that column the same way, then each wavefront takes one
// row i of W, lanes along the row, and writes qv[i] = v_i (W v)_i and
// qv[d + i] = v_i^2.
__global__ __launch_bounds__(256) void k_rayleigh_rows(const double *__restrict__ M,
                                                       const double *__restrict__ W, int64_t d,
                                                       const double *__restrict__ cnp,
                                                       double *__restrict__ qv) {
  __shared__ double best_s[256];
  __shared__ int best_j[256];
  double bs = -1.0;
  int bj = 0;
  for (int64_t j = threadIdx.x; j < d; j += 256) {
    double s = 0.0;
    for (int q = 0; q < kColSlices; ++q) s += cnp[q * d + j];
    if (s > bs) {
      bs = s;
      bj = (int)j;
    }
  }
  best_s[threadIdx.x] = bs;
  best_j[threadIdx.x] = bj;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 1; t < 256; ++t)
      if (best_s[t] > best_s[0] || (best_s[t] == best_s[0] && best_j[t] < best_j[0])) {
        best_s[0] = best_s[t];
        best_j[0] = best_j[t];
      }
  }
  __syncthreads();
  const int64_t j = best_j[0];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + w;
  if (i >= d) return;
  double acc = 0.0;
  for (int64_t k = lane; k < d; k += 64) acc += W[i * d + k] * M[k * d + j];
  acc = wave_sum(acc);
  if (lane == 0) {
    const double vi = M[i * d + j];
    qv[i] = vi * acc;
    qv[d + i] = vi * vi;
  }
}

// delta = sqrt(v^T W v / v^T v) from the row terms (0 when v is 0); one
// workgroup, fixed order
__global__ __launch_bounds__(256) void k_rayleigh_final(const double *__restrict__ qv,
                                                        int64_t d, double *__restrict__ delta) {
  __shared__ double red[4];
  double q = 0.0, nv = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 256) {
    q += qv[i];
    nv += qv[d + i];
  }
  q = block_sum(q, red);
  nv = block_sum(nv, red);
  if (threadIdx.x == 0) *delta = nv > 0.0 ? sqrt(fmax(q / nv, 0.0)) : 0.0;
}

void frob_normalise(double *M, int64_t len, double *part, hipStream_t st) {
  k_frob_parts<<<kNrmParts, 256, 0, st>>>(M, len, part);
  const int64_t nb = ceil_div(len, (int64_t)256);
  k_frob_scale<<<(unsigned)(nb < 2048 ? nb : 2048), 256, 0, st>>>(M, len, part);
}

}  // namespace

int delta_from_factor(const double *Chat, const double *C, const double *Ri, int64_t m,
                      int64_t d, double *delta, Arena &ws, hipStream_t st) {
  double *D = ws.take<double>((size_t)m * d);
  double *F = ws.take<double>((size_t)m * d);
  double *W = ws.take<double>((size_t)d * d);
  double *M0 = ws.take<double>((size_t)d * d);
  double *M1 = ws.take<double>((size_t)d * d);
  double *part = ws.take<double>(kNrmParts);
  double *cnp = ws.take<double>((size_t)kColSlices * d);
  double *qv = ws.take<double>((size_t)2 * d);
  const bool run = !ws.dry();
  if (run && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for sketch_delta");
  const size_t mk = ws.mark();
  int rc;
  KTimer timer("sketch_delta", st, run);
  if (run) {
    const int64_t len = m * d;
    k_sub<<<(unsigned)ceil_div(len, 256), 256, 0, st>>>(Chat, C, len, D);
  }
  if ((rc = dgemm(false, false, m, d, d, 1.0, D, d, Ri, d, 0.0, F, d, ws, st))) return rc;
  ws.release(mk);
  if ((rc = dgemm(true, false, d, d, m, 1.0, F, d, F, d, 0.0, W, d, ws, st))) return rc;
  ws.release(mk);
  if (run) {
    PSK_HIP_TRY(hipMemcpyAsync(M0, W, (size_t)d * d * sizeof(double), hipMemcpyDeviceToDevice,
                               st));
    frob_normalise(M0, d * d, part, st);
  }
  double *a = M0, *b = M1;
  for (int i = 0; i < kSquarings; ++i) {
    if ((rc = dgemm(false, false, d, d, d, 1.0, a, d, a, d, 0.0, b, d, ws, st))) return rc;
    ws.release(mk);
    if (run) frob_normalise(b, d * d, part, st);
    double *t = a;
    a = b;
    b = t;
  }
  if (run) {
    k_col_norms<<<dim3((unsigned)ceil_div(d, (int64_t)64), kColSlices), 256, 0, st>>>(a, d, cnp);
    k_rayleigh_rows<<<(unsigned)ceil_div(d, (int64_t)4), 256, 0, st>>>(a, W, d, cnp, qv);
    k_rayleigh_final<<<1, 256, 0, st>>>(qv, d, delta);
    PSK_HIP_TRY(hipGetLastError());
  }
  return 0;
}

int sketch_delta_impl(const double *Chat, const double *C, int64_t m, int64_t d, double *delta,
                      Arena &ws, hipStream_t st) {
  if (d > 4096) return fail(PSK_EUNSUPPORTED, "sketch_delta supports d <= 4096");
  double *R = ws.take<double>((size_t)d * d);
  double *Ri = ws.take<double>((size_t)d * d);
  if (!ws.dry() && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for sketch_delta");
  const size_t mk = ws.mark();
  int rc;
  if ((rc = sketch_qr_impl(C, m, d, R, Ri, ws, st))) return rc;
  ws.release(mk);
  return delta_from_factor(Chat, C, Ri, m, d, delta, ws, st);
}

}  // namespace psk
