// Sketch-and-precondition least squares on gfx950 (FP64):
// C = G*S*A, R from sketch_qr(C), LSQR on the right-preconditioned operator
// A*R^{-1}, x = R^{-1} y, then refinement passes on the residual.
//
// Paper mapping (arXiv 2203.02798): Algorithm least_squares_precondition
// (B = GSA, factor B, N = inverse factor, solve min ||A N y - b|| with a
// preconditioned iterative method, x = N y).  The iterative method is LSQR
// (Paige & Saunders, ACM TOMS 8(1), 1982), which the paper leaves open.
//
// One LSQR iteration reads A once: for every row, u_i <- A_i vhat - alpha u_i
// and A_i^T u_i is accumulated immediately (the normalisation by beta is a
// scalar applied afterwards), so the two products A v and A^T u of the
// bidiagonalisation share one pass over A.  The scalar recurrences run in a
// one-workgroup kernel; all state stays on the device, and a `done` flag set
// by the convergence test turns the remaining enqueued iterations into
// no-ops, so the host only synchronises every `check_every` iterations.
#include <math.h>

#include "internal.hpp"

namespace psk {
namespace {

struct LsqrState {
  double alpha, beta_new, rhobar, phibar, anorm2, bnorm, ufac, ynorm2;
  double rnorm, arnorm, test2;
  int done, iters, pad0, pad1;
};

constexpr int kPassBlocks = 512;

template <typename T, bool CSR, bool INIT>
__global__ __launch_bounds__(256) void k_pass(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, int64_t n, int64_t d, int64_t ld,
    const double *__restrict__ vhat, const double *__restrict__ rhs,
    double *__restrict__ u, const LsqrState *__restrict__ st,
    double *__restrict__ part_t, double *__restrict__ part_b2) {
  if (!INIT && st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double *tl = reinterpret_cast<double *>(smem_raw) + (int64_t)wave * d;
  __shared__ double b2s[4];
  for (int64_t c = lane; c < d; c += 64) tl[c] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const double au = INIT ? 0.0 : st->alpha * st->ufac;
  const int64_t rows_per_blk = ceil_div(n, (int64_t)gridDim.x);
  const int64_t rb0 = (int64_t)blockIdx.x * rows_per_blk;
  int64_t rb1 = rb0 + rows_per_blk;
  if (rb1 > n) rb1 = n;
  const int64_t rows_per_wave = ceil_div(rb1 - rb0 > 0 ? rb1 - rb0 : 0, 4);
  const int64_t i0 = rb0 + wave * rows_per_wave;
  int64_t i1 = i0 + rows_per_wave;
  if (i1 > rb1) i1 = rb1;
  double b2 = 0.0;
  for (int64_t i = i0; i < i1; ++i) {
    double ui;
    if (CSR) {
      const int64_t p0 = indptr[i], p1 = indptr[i + 1];
      if (INIT) {
        ui = rhs[i];
      } else {
        double dot = 0.0;
        for (int64_t p = p0 + lane; p < p1; p += 64) dot += (double)vals[p] * vhat[indices[p]];
        ui = wave_sum(dot) - au * u[i];
      }
      for (int64_t p = p0 + lane; p < p1; p += 64)
        atomicAdd(&tl[indices[p]], (double)vals[p] * ui);
    } else {
      const T *row = vals + i * ld;
      if (INIT) {
        ui = rhs[i];
      } else {
        double dot = 0.0;
        for (int64_t c = lane; c < d; c += 64) dot += (double)row[c] * vhat[c];
        ui = wave_sum(dot) - au * u[i];
      }
      for (int64_t c = lane; c < d; c += 64) tl[c] += (double)row[c] * ui;
    }
    if (lane == 0) u[i] = ui;
    b2 += ui * ui;
  }
  if (lane == 0) b2s[wave] = b2;
  __syncthreads();
  const double *t0 = reinterpret_cast<const double *>(smem_raw);
  for (int64_t c = threadIdx.x; c < d; c += 256)
    part_t[(int64_t)blockIdx.x * d + c] = ((t0[c] + t0[d + c]) + t0[2 * d + c]) + t0[3 * d + c];
  if (threadIdx.x == 0) part_b2[blockIdx.x] = ((b2s[0] + b2s[1]) + b2s[2]) + b2s[3];
}

// beta = sqrt(sum part_b2); tv = (sum_blocks part_t) / beta
__global__ __launch_bounds__(256) void k_reduce_t(const double *__restrict__ part_t,
                                                  const double *__restrict__ part_b2,
                                                  int nb, int64_t d, LsqrState *__restrict__ st,
                                                  double *__restrict__ tv, int init) {
  if (!init && st->done) return;
  __shared__ double bsh;
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 64) s += part_b2[b];
    s = wave_sum(s);
    if (threadIdx.x == 0) bsh = sqrt(s);
  }
  __syncthreads();
  const double beta = bsh;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < d) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part_t[(int64_t)b * d + j];
    tv[j] = beta > 0.0 ? t / beta : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->beta_new = beta;
}

// vnew_j = sum_{i<=j} Rinv[i][j] tv_i - beta v_j ; part_a2[block] = sum vnew^2
__global__ __launch_bounds__(256) void k_vnew(const double *__restrict__ Rinv, int64_t d,
                                              const double *__restrict__ tv,
                                              const double *__restrict__ v,
                                              const LsqrState *__restrict__ st,
                                              double *__restrict__ vnew,
                                              double *__restrict__ part_a2, int init) {
  if (!init && st->done) return;
  __shared__ double red[4];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double val = 0.0;
  if (j < d) {
    double s = 0.0;
    for (int64_t i = 0; i <= j; ++i) s += Rinv[i * d + j] * tv[i];
    val = init ? s : s - st->beta_new * v[j];
    vnew[j] = val;
  }
  double a2 = wave_sum(val * val);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a2;
  __syncthreads();
  if (threadIdx.x == 0) part_a2[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// scalar recurrences, v/w/y updates and the stopping test (one workgroup)
__global__ __launch_bounds__(256) void k_update(LsqrState *__restrict__ st, int64_t d,
                                                double *__restrict__ v,
                                                const double *__restrict__ vnew,
                                                double *__restrict__ w,
                                                double *__restrict__ y,
                                                const double *__restrict__ part_a2, int nb,
                                                double atol, double btol, int init) {
  if (!init && st->done) return;
  __shared__ double sh[8];
  __shared__ double red[4];
  if (threadIdx.x == 0) {
    double a2 = 0.0;
    for (int b = 0; b < nb; ++b) a2 += part_a2[b];
    const double alpha = sqrt(a2);
    const double beta = st->beta_new;
    double phi = 0.0, rho = 1.0, theta = 0.0;
    int done = 0;
    if (init) {
      st->bnorm = beta;
      st->phibar = beta;
      st->rhobar = alpha;
      st->anorm2 = 0.0;
      st->iters = 0;
      if (beta == 0.0 || alpha == 0.0) done = 1;
    } else {
      st->anorm2 += st->alpha * st->alpha + beta * beta;
      const double rhobar = st->rhobar;
      rho = sqrt(rhobar * rhobar + beta * beta);
      const double c = rhobar / rho;
      const double s = beta / rho;
      theta = s * alpha;
      st->rhobar = -c * alpha;
      phi = c * st->phibar;
      st->phibar = s * st->phibar;
      st->iters += 1;
      const double anorm = sqrt(st->anorm2);
      const double rnorm = st->phibar;
      const double arnorm = rnorm * alpha * fabs(c);
      st->rnorm = rnorm;
      st->arnorm = arnorm;
      st->test2 = (anorm > 0.0 && rnorm > 0.0) ? arnorm / (anorm * rnorm) : 0.0;
      if (arnorm <= atol * anorm * rnorm) done = 1;
      if (rnorm <= btol * st->bnorm + atol * anorm * sqrt(st->ynorm2)) done = 1;
      if (alpha == 0.0 || beta == 0.0) done = 1;
    }
    st->alpha = alpha;
    st->ufac = beta > 0.0 ? 1.0 / beta : 0.0;
    sh[0] = alpha > 0.0 ? 1.0 / alpha : 0.0;
    sh[1] = init ? 0.0 : phi / rho;
    sh[2] = init ? 0.0 : theta / rho;
    sh[3] = done;
  }
  __syncthreads();
  const double ainv = sh[0], fx = sh[1], fw = sh[2];
  double y2 = 0.0;
  for (int64_t j = threadIdx.x; j < d; j += 256) {
    const double vj = vnew[j] * ainv;
    if (init) {
      w[j] = vj;
      y[j] = 0.0;
    } else {
      const double wj = w[j];
      const double yj = y[j] + fx * wj;
      y[j] = yj;
      y2 += yj * yj;
      w[j] = vj - fw * wj;
    }
    v[j] = vj;
  }
  y2 = wave_sum(y2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = y2;
  __syncthreads();
  if (threadIdx.x == 0) {
    st->ynorm2 = ((red[0] + red[1]) + red[2]) + red[3];
    if (sh[3] != 0.0) st->done = 1;
  }
}

// out_i = (accumulate ? out_i : 0) + sum_{j>=i} Rinv[i][j] vec_j  (RinvT = Rinv^T)
__global__ __launch_bounds__(256) void k_trmv(const double *__restrict__ RinvT, int64_t d,
                                              const double *__restrict__ vec,
                                              double *__restrict__ out,
                                              const LsqrState *__restrict__ st,
                                              int check_done, int accumulate) {
  if (check_done && st->done) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d) return;
  double s = 0.0;
  for (int64_t j = i; j < d; ++j) s += RinvT[j * d + i] * vec[j];
  out[i] = accumulate ? out[i] + s : s;
}

__global__ void k_transpose(const double *__restrict__ A, int64_t d, double *__restrict__ T) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  const int64_t i = e / d, j = e % d;
  T[j * d + i] = A[i * d + j];
}

__global__ void k_state_reset(LsqrState *st) {
  if (threadIdx.x == 0) {
    st->alpha = st->beta_new = st->rhobar = st->phibar = 0.0;
    st->anorm2 = st->bnorm = st->ufac = st->ynorm2 = 0.0;
    st->rnorm = st->arnorm = st->test2 = 0.0;
    st->done = 0;
    st->iters = 0;
  }
}

__global__ void k_zero(double *p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// res_i = b_i - A_i x (one wavefront per row)
template <typename T, bool CSR>
__global__ __launch_bounds__(256) void k_resid(const T *__restrict__ vals,
                                               const int64_t *__restrict__ indptr,
                                               const int32_t *__restrict__ indices,
                                               int64_t n, int64_t d, int64_t ld,
                                               const double *__restrict__ x,
                                               const double *__restrict__ b,
                                               double *__restrict__ res) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double dot = 0.0;
  if (CSR) {
    for (int64_t p = indptr[i] + lane; p < indptr[i + 1]; p += 64)
      dot += (double)vals[p] * x[indices[p]];
  } else {
    for (int64_t c = lane; c < d; c += 64) dot += (double)vals[i * ld + c] * x[c];
  }
  dot = wave_sum(dot);
  if (lane == 0) res[i] = b[i] - dot;
}

struct LsqBufs {
  double *u, *part_t, *part_b2, *tv, *vnew, *part_a2, *v, *w, *y, *vhat;
  double *RinvT;
  LsqrState *st;
};

template <typename T>
void launch_pass(const psk_mat &A, bool init, const LsqBufs &B, const double *rhs,
                 hipStream_t stream) {
  const size_t lds = (size_t)4 * A.d * sizeof(double);
  const T *vals = (const T *)A.values;
  if (A.format == PSK_CSR) {
    if (init)
      k_pass<T, true, true><<<kPassBlocks, 256, lds, stream>>>(
          vals, A.indptr, A.indices, A.n, A.d, A.ld, B.vhat, rhs, B.u, B.st, B.part_t,
          B.part_b2);
    else
      k_pass<T, true, false><<<kPassBlocks, 256, lds, stream>>>(
          vals, A.indptr, A.indices, A.n, A.d, A.ld, B.vhat, rhs, B.u, B.st, B.part_t,
          B.part_b2);
  } else {
    if (init)
      k_pass<T, false, true><<<kPassBlocks, 256, lds, stream>>>(
          vals, A.indptr, A.indices, A.n, A.d, A.ld, B.vhat, rhs, B.u, B.st, B.part_t,
          B.part_b2);
    else
      k_pass<T, false, false><<<kPassBlocks, 256, lds, stream>>>(
          vals, A.indptr, A.indices, A.n, A.d, A.ld, B.vhat, rhs, B.u, B.st, B.part_t,
          B.part_b2);
  }
}

void one_step(const psk_mat &A, bool init, const LsqBufs &B, const double *Rinv,
              const double *rhs, const psk_lsq_opts &o, hipStream_t stream) {
  const int64_t d = A.d;
  const unsigned db = (unsigned)ceil_div(d, 256);
  {
    KTimer t("lsqr_pass", stream);
    if (A.dtype == PSK_F64)
      launch_pass<double>(A, init, B, rhs, stream);
    else
      launch_pass<float>(A, init, B, rhs, stream);
  }
  k_reduce_t<<<db, 256, 0, stream>>>(B.part_t, B.part_b2, kPassBlocks, d, B.st, B.tv,
                                     init ? 1 : 0);
  k_vnew<<<db, 256, 0, stream>>>(Rinv, d, B.tv, B.v, B.st, B.vnew, B.part_a2, init ? 1 : 0);
  k_update<<<1, 256, 0, stream>>>(B.st, d, B.v, B.vnew, B.w, B.y, B.part_a2, (int)db,
                                  o.atol, o.btol, init ? 1 : 0);
  k_trmv<<<db, 256, 0, stream>>>(B.RinvT, d, B.v, B.vhat, B.st, init ? 0 : 1, 0);
}

}  // namespace

int lsq_impl(const psk_mat &A, const double *b, double *x, const psk_lsq_opts &o,
             psk_lsq_info *info, Arena &ws, hipStream_t st) {
  const int64_t n = A.n, d = A.d, m = o.m;
  if (d > 1024) return fail(PSK_EUNSUPPORTED, "lsq_solve supports d <= 1024");
  const bool own = o.Rinv == nullptr;  // sketch and factor here
  double *C = own ? ws.take<double>((size_t)m * d) : nullptr;
  double *R = own ? ws.take<double>((size_t)d * d) : nullptr;
  double *Rinv = own ? ws.take<double>((size_t)d * d) : const_cast<double *>(o.Rinv);
  LsqBufs B;
  B.RinvT = ws.take<double>((size_t)d * d);
  B.u = ws.take<double>((size_t)n);
  B.part_t = ws.take<double>((size_t)kPassBlocks * d);
  B.part_b2 = ws.take<double>(kPassBlocks);
  B.tv = ws.take<double>((size_t)d);
  B.vnew = ws.take<double>((size_t)d);
  B.part_a2 = ws.take<double>((size_t)ceil_div(d, 256));
  B.v = ws.take<double>((size_t)d);
  B.w = ws.take<double>((size_t)d);
  B.y = ws.take<double>((size_t)d);
  B.vhat = ws.take<double>((size_t)d);
  double *res = ws.take<double>((size_t)n);
  B.st = ws.take<LsqrState>(1);
  const size_t mk = ws.mark();
  int rc = 0;
  int *flag = nullptr;
  if (own) {
    // sketch and factor (their scratch is released afterwards)
    void *SA = ws.take<unsigned char>((size_t)o.r * d * elem_size(A.dtype));
    uint32_t *perm = nullptr, *bptr = nullptr;
    if ((rc = cs_bin(n, (uint32_t)o.r, o.seed, ws, st, &perm, &bptr))) return rc;
    if ((rc = cs_apply(A, (uint32_t)o.r, perm, bptr, SA, ws, st))) return rc;
    if ((rc = gauss_gemm(m, o.r, d, o.seed, o.prec, SA, A.dtype, C, ws, st))) return rc;
    if ((rc = sketch_qr_impl(C, m, d, R, Rinv, ws, st, &flag))) return rc;
  }
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for lsq_solve");
  ws.release(mk);
  k_transpose<<<(unsigned)ceil_div(d * d, 256), 256, 0, st>>>(Rinv, d, B.RinvT);
  if (own) {
    int hflag = 0;
    PSK_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    PSK_HIP_TRY(hipStreamSynchronize(st));
    if (hflag) return fail(PSK_ERANK, "sketch is numerically rank deficient");
  }

  const unsigned db = (unsigned)ceil_div(d, 256);
  k_zero<<<(unsigned)ceil_div(d, 256), 256, 0, st>>>(x, d);
  int total_iters = 0;
  bool converged = true;
  LsqrState hs{};
  for (int pass = 0; pass <= o.refine; ++pass) {
    const double *rhs = b;
    if (pass > 0) {
      const unsigned rb = (unsigned)ceil_div(n * 64, 256);
      if (A.format == PSK_CSR) {
        if (A.dtype == PSK_F64)
          k_resid<double, true><<<rb, 256, 0, st>>>((const double *)A.values, A.indptr,
                                                     A.indices, n, d, A.ld, x, b, res);
        else
          k_resid<float, true><<<rb, 256, 0, st>>>((const float *)A.values, A.indptr,
                                                   A.indices, n, d, A.ld, x, b, res);
      } else {
        if (A.dtype == PSK_F64)
          k_resid<double, false><<<rb, 256, 0, st>>>((const double *)A.values, nullptr,
                                                      nullptr, n, d, A.ld, x, b, res);
        else
          k_resid<float, false><<<rb, 256, 0, st>>>((const float *)A.values, nullptr,
                                                    nullptr, n, d, A.ld, x, b, res);
      }
      rhs = res;
    }
    k_state_reset<<<1, 64, 0, st>>>(B.st);
    k_zero<<<db, 256, 0, st>>>(B.v, d);
    one_step(A, true, B, Rinv, rhs, o, st);
    int it = 0;
    bool done = false;
    while (it < o.max_iter) {
      int batch = o.check_every;
      if (batch > o.max_iter - it) batch = o.max_iter - it;
      for (int q = 0; q < batch; ++q) one_step(A, false, B, Rinv, rhs, o, st);
      it += batch;
      PSK_HIP_TRY(hipMemcpyAsync(&hs, B.st, sizeof(hs), hipMemcpyDeviceToHost, st));
      PSK_HIP_TRY(hipStreamSynchronize(st));
      if (hs.done) {
        done = true;
        break;
      }
    }
    if (!done) converged = false;
    total_iters += hs.iters;
    // x += R^{-1} y
    k_trmv<<<db, 256, 0, st>>>(B.RinvT, d, B.y, x, B.st, 0, 1);
  }
  PSK_HIP_TRY(hipGetLastError());
  PSK_HIP_TRY(hipStreamSynchronize(st));
  if (info) {
    info->iters = total_iters;
    info->status = converged ? PSK_OK : PSK_ENOCONV;
    info->resid = hs.rnorm;
    info->ne_resid = hs.test2;
  }
  if (!converged) return fail(PSK_ENOCONV, "LSQR reached max_iter before its tolerance");
  return 0;
}

}  // namespace psk
