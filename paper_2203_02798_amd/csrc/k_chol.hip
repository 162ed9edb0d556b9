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
// numbers up to about 1/u, and up to two unshifted passes restore
// orthogonality.  The second pass stops the factorisation when its Gram
// matrix is within 1e-4 of the identity: then the first pass's Q was
// already orthonormal to that level, the second pass leaves it orthonormal
// to rounding level (Cholesky-QR loses orthogonality like cond(Q)^2 u), and
// a third pass would change R only by rounding.  Otherwise (ill-conditioned
// C) the third pass runs as in sCQR3.
//
// The d x d Cholesky and the inverse of its factor are blocked by 64 columns
// with one launch per block step (k_chol_step, below): the panel, the
// trailing update, the partial products of R^{-1} and the factorization of
// the next diagonal block all happen in the same launch, so a pass costs
// ceil(d/64) + 2 launches besides its two GEMMs with C.
#include "internal.hpp"

namespace psk {
namespace {

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

// ---------------------------------------------------------------------------
// Blocked Cholesky W = R^T R with X = R^{-1}, 64-column blocks, one kernel
// launch per block step.  Step j (k_chol_step) runs one 256-thread workgroup
// per 64 x 64 tile of work:
//   panel    R[j, J]  = X_jj^T W[j, J]                       (J > j)
//   trailing W[I, J] -= P_I^T P_J,  P_K = X_jj^T W[j, K]     (j < I <= J)
//   partial  P_j[I][K] = X[I, K] R[K, j]                     (I <= K <= j-2)
//   finish   X[I, c]  = -(sum_K P_c[I][K] + X[I, c-1] R[c-1, c]) X_cc
//                                                   (c = j - 1, I < c)
// and the workgroup that owns the next diagonal tile (j+1, j+1), whose update
// is the last one it receives, factors it in the same launch (Cholesky and
// triangular inverse of the 64 x 64 block), so the next step finds R_{j+1,j+1}
// and X_{j+1,j+1} ready.  The off-diagonal blocks of X = R^{-1}, whose sums
// run over up to d - 64 terms, are split into 64-term partial products so
// that no workgroup carries a long sum; a block column is summed (in K
// order) and finished one launch after its partials, and one extra launch
// finishes the last column.  Block 0 is factored by k_chol_first.  W is read
// in its upper block triangle and destroyed.
// ---------------------------------------------------------------------------
constexpr int kLd = 68;      // LDS row stride of 64-wide tiles (doubles)
constexpr int kUt = 66;      // LDS row stride of the transposed factor
constexpr int kTh = 256;

struct CholSmem {
  double As[16 * kLd];
  double Bs[16 * kLd];
  double PI[64 * kLd];       // also the diagonal tile to factor
  double PJ[64 * kLd];
  double Ut[64 * kUt];       // block inverses of the diagonal factor
  double rowbuf[2][64];
  double rinv[64];
};

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, l);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// 1/sqrt(x) to about one ulp: the hardware estimate, then one third-order
// and one Newton correction, each from the residual e = 1 - x y^2 taken with
// an FMA.
__device__ __forceinline__ double rsqrt_acc(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-(x * y), y, 1.0);
  y = fma(y * e, fma(e, 0.375, 0.5), y);
  e = fma(-(x * y), y, 1.0);
  return fma(y * e, 0.5, y);
}

constexpr int kVb = 16 * 17;  // one 16 x 16 block inverse in LDS (row stride 17)

// Wavefront 0: Cholesky of the 16 x 16 block at (o, o) of the LDS tile T
// (its upper triangle is read), right-looking with lane l % 16 holding
// column l % 16: step k takes the pivot from lane k, scales row k, publishes
// it through LDS and applies the rank-1 update to its column.  The same row
// operations (scale row k by 1/U_kk, subtract U_ki times row k from row i)
// applied to the identity leave L^{-1} = U^{-T} in z, lane l holding its
// column l, i.e. row l of V = U^{-1}.  U overwrites the block's upper
// triangle and V goes to Vb (row-major, stride 17).  Lanes 16..63 repeat
// lanes 0..15 and store nothing.  Returns bit 1 when a pivot was not
// positive (it is then replaced by 1), bit 2 when one was NaN or infinite.
__device__ __forceinline__ int factor16(double *__restrict__ T, int o,
                                         double *__restrict__ rowbuf,
                                         double *__restrict__ Vb) {
  const int l = threadIdx.x & 15;
  const bool st = threadIdx.x < 16;
  double c[16], z[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    c[i] = T[(o + i) * kLd + o + l];
    z[i] = (i == l) ? 1.0 : 0.0;
  }
  int bad = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    double piv = readlane_f64(c[k], k);
    bad |= !(piv > 0.0) ? 1 : 0;
    bad |= !(fabs(piv) <= 1.7976931348623157e308) ? 2 : 0;  // NaN or infinite
    piv = piv > 0.0 ? piv : 1.0;
    const double rs = rsqrt_acc(piv);
    const double u = (l >= k) ? c[k] * rs : 0.0;
    z[k] *= rs;
    double *rb = rowbuf + (k & 1) * 16;
    if (st) {
      rb[l] = u;
      if (l >= k) T[(o + k) * kLd + o + l] = u;
    }
    wave_sync_lds();
    double rbv[16];
#pragma unroll
    for (int i = k + 1; i < 16; ++i) rbv[i] = rb[i];
#pragma unroll
    for (int i = k + 1; i < 16; ++i) {
      c[i] -= rbv[i] * u;
      z[i] -= rbv[i] * z[k];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if (st) {
#pragma unroll
    for (int i = 0; i < 16; ++i) Vb[l * 17 + i] = z[i];
  }
  return bad;
}

// All 256 threads.  T = S.PI: the 64 x 64 tile (row-major, stride kLd), of
// which the leading nb x nb block is used (the rest is taken as identity).
// Blocked right-looking Cholesky over four 16-column blocks: block kb is
// factored by wavefront 0 (factor16, which also gives the block's inverse),
// then the panel right of it is solved (U[kb, J] = V_kb^T T[kb, J]) and the
// trailing block updated (T[I, J] -= U[kb, I]^T U[kb, J]) by the whole
// workgroup, each thread owning a small register tile of outputs with its
// operands loaded ahead.  The inverse X = U^{-1} is built block column by
// block column: X[I, J] = -(sum_{K = I..J-1} X[I, K] U[K, J]) V_J.  Writes
// the nb x nb blocks of R (= U, zero below the diagonal) and X at (j0, j0).
template <int TR>
__device__ __forceinline__ void trailing_update(double *__restrict__ T, int o) {
  // rows / columns o + 16 + t + 16 a (a < TR) of thread (ti, tj)
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
  const int b0 = o + 16;
  double acc[TR][TR];
#pragma unroll
  for (int a = 0; a < TR; ++a)
#pragma unroll
    for (int b = 0; b < TR; ++b) acc[a][b] = 0.0;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const double *row = T + (o + m) * kLd;
    double ri[TR], cj[TR];
#pragma unroll
    for (int a = 0; a < TR; ++a) {
      ri[a] = row[b0 + ti + 16 * a];
      cj[a] = row[b0 + tj + 16 * a];
    }
#pragma unroll
    for (int a = 0; a < TR; ++a)
#pragma unroll
      for (int b = 0; b < TR; ++b) acc[a][b] = fma(ri[a], cj[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < TR; ++a)
#pragma unroll
    for (int b = 0; b < TR; ++b) T[(b0 + ti + 16 * a) * kLd + b0 + tj + 16 * b] -= acc[a][b];
}

__device__ __forceinline__ void factor_diag(CholSmem &S, int nb, int64_t d, int64_t j0,
                                            double *__restrict__ R, double *__restrict__ X,
                                            int *__restrict__ flag) {
  double *T = S.PI;
  double *XT = S.PJ;
  double *V = S.Ut;   // four block inverses, kVb doubles each
  double *P = S.As;   // up to three 16 x 16 partial products (stride 17)
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += kTh) {
    const int i = e >> 6, j = e & 63;
    if (i >= nb || j >= nb) T[i * kLd + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  int bad = 0;
#pragma unroll 1
  for (int kb = 0; kb < 4; ++kb) {
    const int o = 16 * kb;
    if (tid < 64) bad |= factor16(T, o, S.rowbuf[0], V + kb * kVb);
    __syncthreads();
    const int rest = 48 - o;  // columns right of the block
    if (rest == 0) break;
    {
      // panel rows o..o+15, columns o+16..63: U[o+r][j] = sum_{m<=r} V[m][r] T[o+m][j]
      const double *Vk = V + kb * kVb;
      const int r = tid & 15, jg = tid >> 4;
      double vc[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) vc[m] = (m <= r) ? Vk[m * 17 + r] : 0.0;
      double pv[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int j = o + 16 + jg + 16 * q;
        const int jc = j < 64 ? j : 63;
        double tc[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) tc[m] = T[(o + m) * kLd + jc];
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int m = 0; m < 16; m += 2) {
          a0 = fma(vc[m], tc[m], a0);
          a1 = fma(vc[m + 1], tc[m + 1], a1);
        }
        pv[q] = a0 + a1;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int j = o + 16 + jg + 16 * q;
        if (j < 64) T[(o + r) * kLd + j] = pv[q];
      }
      __syncthreads();
    }
    // trailing block rows / columns o+16..63
    if (rest == 48) trailing_update<3>(T, o);
    else if (rest == 32) trailing_update<2>(T, o);
    else trailing_update<1>(T, o);
    __syncthreads();
  }
  // X: diagonal blocks from the block inverses, zero below them
  for (int e = tid; e < 64 * 64; e += kTh) {
    const int i = e >> 6, j = e & 63;
    const int bi = i >> 4, bj = j >> 4;
    XT[i * kLd + j] = (bi == bj) ? V[bi * kVb + (i & 15) * 17 + (j & 15)]
                                 : 0.0;
  }
  __syncthreads();
  {
    const int r = tid >> 4, c = tid & 15;
#pragma unroll 1
    for (int J = 1; J < 4; ++J) {
      // P[I] = sum_{K=I}^{J-1} X[I, K] U[K, J] for every I < J at once:
      // thread (r, c) keeps one accumulator per I
      double acc[3] = {0.0, 0.0, 0.0};
      for (int K = 0; K < J; ++K) {
        double tcol[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) tcol[m] = T[(16 * K + m) * kLd + 16 * J + c];
#pragma unroll
        for (int I = 0; I < 3; ++I) {
          if (I <= K) {
            double xr[16];
#pragma unroll
            for (int m = 0; m < 16; ++m) xr[m] = XT[(16 * I + r) * kLd + 16 * K + m];
#pragma unroll
            for (int m = 0; m < 16; ++m) acc[I] = fma(xr[m], tcol[m], acc[I]);
          }
        }
      }
#pragma unroll
      for (int I = 0; I < 3; ++I)
        if (I < J) P[I * kVb + r * 17 + c] = acc[I];
      __syncthreads();
      // X[I, J] = -P[I] V_J (V_J upper triangular)
      const double *VJ = V + J * kVb;
      double vcol[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) vcol[m] = (m <= c) ? VJ[m * 17 + c] : 0.0;
#pragma unroll
      for (int I = 0; I < 3; ++I) {
        if (I < J) {
          double pr[16];
#pragma unroll
          for (int m = 0; m < 16; ++m) pr[m] = P[I * kVb + r * 17 + m];
          double a0 = 0.0, a1 = 0.0;
#pragma unroll
          for (int m = 0; m < 16; m += 2) {
            a0 = fma(pr[m], vcol[m], a0);
            a1 = fma(pr[m + 1], vcol[m + 1], a1);
          }
          XT[(16 * I + r) * kLd + 16 * J + c] = -(a0 + a1);
        }
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < 64 * 64; e += kTh) {
    const int i = e >> 6, j = e & 63;
    if (i < nb && j < nb) {
      R[(j0 + i) * d + j0 + j] = (i <= j) ? T[i * kLd + j] : 0.0;
      X[(j0 + i) * d + j0 + j] = XT[i * kLd + j];
    }
  }
  if (bad) atomicOr(flag, bad);
}

// acc (this thread's 4 x 4 of a 64 x 64 tile: rows 4*ty.., columns 4*tx..)
// += op(A) op(B) over K, staged through LDS 16 k at a time with the next
// chunk prefetched into registers.  fa(i, k) = op(A)[i][k], fb(k, j) =
// op(B)[k][j]; both return 0 outside the operand.  KCONTIG_A tells which
// index of A is contiguous in memory (coalesced staging).
template <bool KCONTIG_A, class FA, class FB>
__device__ __forceinline__ void tile_mm(double acc[4][4], FA fa, FB fb, int K, CholSmem &S) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double pa[4], pb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + kTh * e;  // 0..1023
      int i, kk;
      if (KCONTIG_A) { kk = idx & 15; i = idx >> 4; } else { i = idx & 63; kk = idx >> 6; }
      pa[e] = (k0 + kk < K) ? fa(i, k0 + kk) : 0.0;
      const int jj = idx & 63, kb = idx >> 6;
      pb[e] = (k0 + kb < K) ? fb(k0 + kb, jj) : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + kTh * e;
      int i, kk;
      if (KCONTIG_A) { kk = idx & 15; i = idx >> 4; } else { i = idx & 63; kk = idx >> 6; }
      S.As[kk * kLd + i] = pa[e];
      S.Bs[(idx >> 6) * kLd + (idx & 63)] = pb[e];
    }
    __syncthreads();
    if (k0 + 16 < K) fetch(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const double4 a = *reinterpret_cast<const double4 *>(S.As + kk * kLd + 4 * ty);
      const double4 bq = *reinterpret_cast<const double4 *>(S.Bs + kk * kLd + 4 * tx);
      const double av[4] = {a.x, a.y, a.z, a.w};
      const double bv[4] = {bq.x, bq.y, bq.z, bq.w};
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = fma(av[r], bv[q], acc[r][q]);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void zero_acc(double acc[4][4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;
}

// acc -> LDS tile (row-major, stride kLd)
__device__ __forceinline__ void acc_to_lds(const double acc[4][4], double *T) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    *reinterpret_cast<double4 *>(T + (4 * ty + r) * kLd + 4 * tx) =
        double4{acc[r][0], acc[r][1], acc[r][2], acc[r][3]};
}

// P = X_jj^T W[j, K] (64 x 64) into the LDS tile P.
__device__ __forceinline__ void panel_tile(const double *__restrict__ W, const double *__restrict__ X,
                           int64_t d, int64_t j0, int nbj, int64_t c0, double *P,
                           CholSmem &S) {
  double acc[4][4];
  zero_acc(acc);
  // op(A)[i][k] = X[j0+k][j0+i] (i, k < nbj): contiguous in i
  auto fa = [&](int i, int k) {
    return (i < nbj && k < nbj) ? X[(j0 + k) * d + j0 + i] : 0.0;
  };
  auto fb = [&](int k, int jj) {
    return (k < nbj && c0 + jj < d) ? W[(j0 + k) * d + c0 + jj] : 0.0;
  };
  tile_mm<false>(acc, fa, fb, nbj, S);
  acc_to_lds(acc, P);
  __syncthreads();
}

__global__ __launch_bounds__(kTh) void k_chol_first(const double *__restrict__ W, int64_t d,
                                                    double *__restrict__ R,
                                                    double *__restrict__ X,
                                                    int *__restrict__ flag) {
  __shared__ CholSmem S;
  const int nb = (int)(d < 64 ? d : 64);
  for (int e = threadIdx.x; e < 64 * 64; e += kTh) {
    const int i = e >> 6, jj = e & 63;
    S.PI[i * kLd + jj] = (i < nb && jj < nb) ? W[(int64_t)i * d + jj] : 0.0;
  }
  __syncthreads();
  factor_diag(S, nb, d, 0, R, X, flag);
}

__global__ __launch_bounds__(kTh) void k_chol_step(double *__restrict__ W, int64_t d,
                                                   int nblk, int j,
                                                   double *__restrict__ R,
                                                   double *__restrict__ X,
                                                   int *__restrict__ flag,
                                                   double *__restrict__ xpart) {
  __shared__ CholSmem S;
  const int p = j < nblk ? nblk - j - 1 : 0;
  const int ntrail = p * (p + 1) / 2;
  const int npart = (j >= 2 && j < nblk) ? (j - 1) * j / 2 : 0;
  const int cfin = j - 1;  // the X block column finished in this launch
  const int nfin = cfin >= 1 ? cfin : 0;
  int t = blockIdx.x;
  const int64_t j0 = (int64_t)j * 64;
  const int nbj = (int)((d - j0) < 64 ? (d - j0) : 64);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  if (t < ntrail) {
    // trailing tile (I, J), enumerated row by row of the upper block triangle
    int I = j + 1, rem = t;
    while (rem >= nblk - I) { rem -= nblk - I; ++I; }
    const int J = I + rem;
    const int64_t r0 = (int64_t)I * 64, c0 = (int64_t)J * 64;
    panel_tile(W, X, d, j0, nbj, r0, S.PI, S);
    if (J != I) panel_tile(W, X, d, j0, nbj, c0, S.PJ, S);
    const double *PJ = (J != I) ? S.PJ : S.PI;
    double acc[4][4];
    zero_acc(acc);
#pragma unroll 4
    for (int k = 0; k < 64; ++k) {
      const double4 a = *reinterpret_cast<const double4 *>(S.PI + k * kLd + 4 * ty);
      const double4 bq = *reinterpret_cast<const double4 *>(PJ + k * kLd + 4 * tx);
      const double av[4] = {a.x, a.y, a.z, a.w};
      const double bv[4] = {bq.x, bq.y, bq.z, bq.w};
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = fma(av[r], bv[q], acc[r][q]);
    }
    if (I == j + 1 && J == j + 1) {
      // the next diagonal tile: update in LDS and factor it here
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t gi = r0 + 4 * ty + r, gj = c0 + 4 * tx + q;
          const double w = (gi < d && gj < d) ? W[gi * d + gj] : 0.0;
          S.PI[(4 * ty + r) * kLd + 4 * tx + q] = w - acc[r][q];
        }
      __syncthreads();
      const int nb1 = (int)((d - r0) < 64 ? (d - r0) : 64);
      factor_diag(S, nb1, d, r0, R, X, flag);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t gi = r0 + 4 * ty + r, gj = c0 + 4 * tx + q;
          if (gi < d && gj < d) W[gi * d + gj] -= acc[r][q];
        }
    }
    return;
  }
  t -= ntrail;
  const int64_t half = (int64_t)(nblk - 2) * (nblk - 1) / 2 * 4096;  // tiles per parity
  if (t < npart) {
    // partial product P_j[I][K] = X[I, K] R[K, j] for I <= K <= j - 2
    int K = 0;
    while ((K + 1) * (K + 2) / 2 <= t) ++K;
    const int I = t - K * (K + 1) / 2;
    const int64_t r0 = (int64_t)I * 64, k0 = (int64_t)K * 64;
    double acc[4][4];
    zero_acc(acc);
    auto fa = [&](int i, int k) { return X[(r0 + i) * d + k0 + k]; };  // in range
    auto fb = [&](int k, int jj) { return jj < nbj ? R[(k0 + k) * d + j0 + jj] : 0.0; };
    tile_mm<true>(acc, fa, fb, 64, S);
    double *P = xpart + (j & 1) * half + (int64_t)t * 4096;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) P[(4 * ty + r) * 64 + 4 * tx + q] = acc[r][q];
    return;
  }
  t -= npart;
  if (t < nfin) {
    // X[I, c] = -(sum_{K=I}^{c-2} P_c[I][K] + X[I, c-1] R[c-1, c]) X_cc, c = cfin
    const int I = t, c = cfin;
    const int64_t r0 = (int64_t)I * 64, cm0 = (int64_t)(c - 1) * 64, c0 = (int64_t)c * 64;
    const int nbc = (int)((d - c0) < 64 ? (d - c0) : 64);
    double acc[4][4];
    zero_acc(acc);
    auto fa = [&](int i, int k) { return X[(r0 + i) * d + cm0 + k]; };  // in range
    auto fb = [&](int k, int jj) { return jj < nbc ? R[(cm0 + k) * d + c0 + jj] : 0.0; };
    tile_mm<true>(acc, fa, fb, 64, S);
    const double *Pc = xpart + (c & 1) * half;
    double sum[4][4];
    zero_acc(sum);
#pragma unroll 4
    for (int K = I; K <= c - 2; ++K) {
      const double *pk = Pc + (int64_t)(K * (K + 1) / 2 + I) * 4096 + 4 * tx;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double4 v = *reinterpret_cast<const double4 *>(pk + (4 * ty + r) * 64);
        sum[r][0] += v.x;
        sum[r][1] += v.y;
        sum[r][2] += v.z;
        sum[r][3] += v.w;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[r][q] = sum[r][q] + acc[r][q];
    acc_to_lds(acc, S.PI);
    __syncthreads();
    zero_acc(acc);
    auto ga = [&](int i, int k) { return S.PI[i * kLd + k]; };
    auto gb = [&](int k, int jj) {
      return (k < nbc && jj < nbc) ? X[(c0 + k) * d + c0 + jj] : 0.0;
    };
    tile_mm<true>(acc, ga, gb, nbc, S);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = r0 + 4 * ty + r, gj = c0 + 4 * tx + q;
        if (gj < d) X[gi * d + gj] = -acc[r][q];
      }
    return;
  }
  t -= nfin;
  if (t < p) {
    // panel tile R[j, J] = X_jj^T W[j, J]
    const int64_t c0 = (int64_t)(j + 1 + t) * 64;
    panel_tile(W, X, d, j0, nbj, c0, S.PI, S);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = j0 + 4 * ty + r, gj = c0 + 4 * tx + q;
        if (4 * ty + r < nbj && gj < d) R[gi * d + gj] = S.PI[(4 * ty + r) * kLd + 4 * tx + q];
      }
  }
}

// ---------------------------------------------------------------------------
// Cholesky factor and inverse of a near-identity W = I + E by matrix products
// only (used for the second and third Cholesky-QR passes, whose Gram matrix
// is the identity up to a small E when the previous pass was accurate).
// With R = I + U (U upper triangular), R^T R = W reads U + U^T = E - U^T U,
// so U = Phi(E - U^T U) where Phi keeps the strict upper triangle and half
// the diagonal.  The fixed point iteration U_0 = Phi(E), U_{t+1} =
// Phi(E - U_t^T U_t) gains a factor ~||E|| per step; X = R^{-1} is the
// Neumann series I - U + U^2 - ..., evaluated as X_{t+1} = I - U X_t.  For
// ||E||_F <= kSeriesTol = 1e-4 two steps of each leave errors below 1e-16;
// smaller ||E|| needs fewer (series_depth).  ||E||_F is read back to the
// host (one stream synchronisation per pass), which picks the series or
// the blocked Cholesky and, after a second pass that took the series, ends
// the factorisation there.
// ---------------------------------------------------------------------------
constexpr double kSeriesTol = 1e-4;
constexpr int kParts = 64;

// part[b] = sum over a fixed slice of (W - I)^2, fixed reduction order
__global__ __launch_bounds__(256) void k_fro_partials(const double *__restrict__ W, int64_t d,
                                                      double *__restrict__ part) {
  __shared__ double red[4];
  const int64_t n = d * d;
  const int64_t chunk = ceil_div(n, kParts);
  const int64_t b0 = (int64_t)blockIdx.x * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  double s = 0.0;
  for (int64_t e = b0 + threadIdx.x; e < b1; e += 256) {
    const int64_t i = e / d, jj = e - i * d;
    const double v = W[e] - (i == jj ? 1.0 : 0.0);
    s = fma(v, v, s);
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// U = Phi(W - I) (the whole matrix: zero below the diagonal)
__global__ __launch_bounds__(256) void k_series_u0(const double *__restrict__ W, int64_t d,
                                                   double *__restrict__ U) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= d * d) return;
  const int64_t i = e / d, jj = e - i * d;
  U[e] = jj > i ? W[e] : (jj == i ? 0.5 * (W[e] - 1.0) : 0.0);
}

// U = Phi(W - I - T), T = U_prev^T U_prev
__global__ __launch_bounds__(256) void k_series_phi(const double *__restrict__ W,
                                                    const double *__restrict__ T, int64_t d,
                                                    double *__restrict__ U) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= d * d) return;
  const int64_t i = e / d, jj = e - i * d;
  const double m = W[e] - (i == jj ? 1.0 : 0.0) - T[e];
  U[e] = jj > i ? m : (jj == i ? 0.5 * m : 0.0);
}

// R = I + U, X = I - U (whole matrices)
__global__ __launch_bounds__(256) void k_series_rx(const double *__restrict__ U, int64_t d,
                                                   double *__restrict__ R,
                                                   double *__restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= d * d) return;
  const int64_t i = e / d, jj = e - i * d;
  const double id = (i == jj) ? 1.0 : 0.0;
  R[e] = id + U[e];
  X[e] = id - U[e];
}

// X = I - T on and above the diagonal, 0 below (T = U X_prev, upper)
__global__ __launch_bounds__(256) void k_series_x(const double *__restrict__ T, int64_t d,
                                                  double *__restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= d * d) return;
  const int64_t i = e / d, jj = e - i * d;
  X[e] = jj >= i ? (i == jj ? 1.0 : 0.0) - T[e] : 0.0;
}

void fill(double *p, int64_t count, double v, hipStream_t st) {
  k_fill<<<(unsigned)ceil_div(count, 256), 256, 0, st>>>(p, count, v);
}

// Upper Cholesky of W (destroyed) into R, and X = R^{-1}; R and X must be
// zero on entry.
// xpart: scratch of at least d * d doubles for the partial products of the
// off-diagonal blocks of X (two block columns' worth, by parity).
void chol_inv(double *W, int64_t d, double *R, double *X, int *flag, double *xpart,
              hipStream_t st) {
  const int nblk = (int)ceil_div(d, 64);
  k_chol_first<<<1, kTh, 0, st>>>(W, d, R, X, flag);
  // launch j = nblk only finishes the last block column of X
  for (int j = 0; j <= nblk; ++j) {
    const int p = j < nblk ? nblk - j - 1 : 0;
    const int npart = (j >= 2 && j < nblk) ? (j - 1) * j / 2 : 0;
    const int nfin = j - 1 >= 1 ? j - 1 : 0;
    const int tiles = p * (p + 1) / 2 + npart + nfin + p;
    if (tiles > 0)
      k_chol_step<<<tiles, kTh, 0, st>>>(W, d, nblk, j, R, X, flag, xpart);
  }
}

// ||W - I||_F^2, summed on the host in a fixed order from kParts device
// partials (synchronises the stream).
int fro_dist_identity_sq(const double *W, int64_t d, double *part, hipStream_t st,
                         double *out) {
  k_fro_partials<<<kParts, 256, 0, st>>>(W, d, part);
  double h[kParts];
  PSK_HIP_TRY(hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, st));
  PSK_HIP_TRY(hipStreamSynchronize(st));
  double sum = 0.0;
  for (int b = 0; b < kParts; ++b) sum += h[b];
  *out = sum;
  return 0;
}

// Products of the series for ||E||_F = eps: after t fixed-point steps U is
// off by about 2^t eps^(t+2), and I - U + ... + (-U)^(t+1) by eps^(t+2).
int series_depth(double eps) {
  if (eps <= 1e-8) return 0;
  if (eps <= 3e-6) return 1;
  return 2;
}

// R = I + U, X = R^{-1} of W = I + E with ||E||_F <= kSeriesTol: U_0 =
// Phi(E), U_{t+1} = Phi(E - U_t^T U_t), X_1 = I - U, X_{t+1} = I - U X_t,
// `depth` steps of each.  B0, B1, B2: d x d scratch.
int series_chol(const double *W, int64_t d, int depth, double *R, double *X, double *B0,
                double *B1, double *B2, Arena &ws, hipStream_t st) {
  const bool run = !ws.dry();
  const unsigned ew = (unsigned)ceil_div(d * d, 256);
  const size_t mk = ws.mark();
  int rc;
  if (run) k_series_u0<<<ew, 256, 0, st>>>(W, d, B0);
  double *u = B0, *v = B1;
  for (int t = 0; t < depth; ++t) {
    if ((rc = dgemm(true, false, d, d, d, 1.0, u, d, u, d, 0.0, B2, d, ws, st))) return rc;
    ws.release(mk);
    if (run) k_series_phi<<<ew, 256, 0, st>>>(W, B2, d, v);
    double *tmp = u; u = v; v = tmp;
  }
  if (run) k_series_rx<<<ew, 256, 0, st>>>(u, d, R, X);
  for (int t = 0; t < depth; ++t) {
    if ((rc = dgemm(false, false, d, d, d, 1.0, u, d, X, d, 0.0, B2, d, ws, st))) return rc;
    ws.release(mk);
    if (run) k_series_x<<<ew, 256, 0, st>>>(B2, d, X);
  }
  return 0;
}

// R, X of the Gram matrix W = Q^T Q of a pass after the first: the series
// when ||W - I||_F <= kSeriesTol, else the blocked Cholesky.  In a planning
// run (no data) both are planned.  *series tells which ran.
int later_pass_chol(double *W, int64_t d, double *R, double *X, double *B0, double *B1,
                    double *B2, double *part, int *flag, bool *series, Arena &ws,
                    hipStream_t st) {
  int rc;
  if (ws.dry()) {
    *series = false;
    return series_chol(W, d, 2, R, X, B0, B1, B2, ws, st);
  }
  double e2;
  if ((rc = fro_dist_identity_sq(W, d, part, st, &e2))) return rc;
  *series = e2 <= kSeriesTol * kSeriesTol;
  if (*series) return series_chol(W, d, series_depth(sqrt(e2)), R, X, B0, B1, B2, ws, st);
  fill(R, d * d, 0.0, st);
  fill(X, d * d, 0.0, st);
  chol_inv(W, d, R, X, flag, B2, st);
  return 0;
}

}  // namespace

int chol_factor(double *W, int64_t d, double *R, double *X, int *flag, Arena &ws,
                hipStream_t st) {
  if (d > 4096) return fail(PSK_EUNSUPPORTED, "the Cholesky factorization supports d <= 4096");
  double *xpart = ws.take<double>((size_t)d * d);
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for the Cholesky factorization");
  k_fill<<<1, 64, 0, st>>>(reinterpret_cast<double *>(flag), 2, 0.0);
  fill(R, d * d, 0.0, st);
  fill(X, d * d, 0.0, st);
  chol_inv(W, d, R, X, flag, xpart, st);
  PSK_HIP_TRY(hipGetLastError());
  return 0;
}

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
  double *B0 = ws.take<double>((size_t)d * d);
  double *B1 = ws.take<double>((size_t)d * d);
  double *B2 = ws.take<double>((size_t)d * d);
  double *part = ws.take<double>(kParts);
  int *flag = ws.take<int>(4);
  const bool run = !ws.dry();
  if (run && !ws.ok()) return fail(PSK_ENOMEM, "workspace too small for sketch_qr");
  const size_t mk = ws.mark();
  int rc;
  KTimer timer("sketch_qr", st, run);
  // flag[0]: a Cholesky pivot failed
  if (run) k_fill<<<1, 64, 0, st>>>(reinterpret_cast<double *>(flag), 2, 0.0);
  if (flag_out) *flag_out = flag;
  // pass 1 (shifted): W = C^T C + s I, blocked Cholesky
  if ((rc = dgemm(true, false, d, d, m, 1.0, C, d, C, d, 0.0, W, d, ws, st))) return rc;
  ws.release(mk);
  const double u = 1.1102230246251565e-16;
  const double coef = 11.0 * ((double)m * d + (double)d * (d + 1)) * u;
  if (run) {
    k_shift_diag<<<1, 256, 0, st>>>(W, d, coef);
    fill(R1, d * d, 0.0, st);
    fill(X1, d * d, 0.0, st);
    chol_inv(W, d, R1, X1, flag, B0, st);  // B0 is not in use yet
  }
  if ((rc = dgemm(false, false, m, d, d, 1.0, C, d, X1, d, 0.0, Qa, d, ws, st))) return rc;
  ws.release(mk);
  // pass 2: W = Qa^T Qa
  if ((rc = dgemm(true, false, d, d, m, 1.0, Qa, d, Qa, d, 0.0, W, d, ws, st))) return rc;
  ws.release(mk);
  bool series2 = false, series3 = false;
  if ((rc = later_pass_chol(W, d, R2, X2, B0, B1, B2, part, flag, &series2, ws, st)))
    return rc;
  ws.release(mk);
  // When pass 2 took the series (Qa was orthonormal to within 1e-4), its
  // result is orthonormal to rounding level and a third pass would change R
  // only at that level: R = R2 R1, R^{-1} = X1 X2.
  if (series2) {
    if ((rc = dgemm(false, false, d, d, d, 1.0, R2, d, R1, d, 0.0, R, d, ws, st))) return rc;
    ws.release(mk);
    if ((rc = dgemm(false, false, d, d, d, 1.0, X1, d, X2, d, 0.0, Rinv, d, ws, st))) return rc;
    ws.release(mk);
    if (run) PSK_HIP_TRY(hipGetLastError());
    return 0;
  }
  if ((rc = dgemm(false, false, m, d, d, 1.0, Qa, d, X2, d, 0.0, Qb, d, ws, st))) return rc;
  ws.release(mk);
  // pass 3: W = Qb^T Qb
  if ((rc = dgemm(true, false, d, d, m, 1.0, Qb, d, Qb, d, 0.0, W, d, ws, st))) return rc;
  ws.release(mk);
  if ((rc = later_pass_chol(W, d, R3, X3, B0, B1, B2, part, flag, &series3, ws, st)))
    return rc;
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
