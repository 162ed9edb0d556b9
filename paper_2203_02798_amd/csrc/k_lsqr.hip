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
// bidiagonalisation share one pass over A.  An iteration is three kernels:
//   pass    (512 workgroups)  per-workgroup partial A^T u and ||u||^2;
//   vnew    (d/16)            beta, t = A^T u / beta for 16 rows each, and
//                             those rows' share of R^{-T} t;
//   update  (d/8 + 1)         vnew = R^{-T} t - beta v and alpha = ||vnew||
//                             (every workgroup sums the shares in the same
//                             order), vhat = R^{-1} vnew / alpha for the next
//                             pass, and (the extra workgroup) the scalar
//                             recurrences, v, w, y and the stopping test.
// All state stays on the device; a `done` flag set by the stopping test turns
// the remaining enqueued iterations into no-ops, so the host reads the state
// only after groups of up to `check_every` iterations, each group's copy
// while the next group runs, and cuts the last group short where the
// stopping margin's observed rate predicts the stop.  Every sum has a fixed order (CSR rows
// scatter A_i^T u_i into per-wavefront LDS rows in a fixed instruction
// order).
#include <math.h>

#include <cmath>

#include <mutex>
#include <vector>

#include "internal.hpp"

namespace psk {
namespace {

struct LsqrState {
  double alpha, beta_new, rhobar, phibar, anorm2, bnorm, ufac, ynorm2;
  double rnorm, arnorm, test2;
  int done, iters, pad0, pad1;
};

// Pinned host copies of the LSQR state with their events: the host reads a
// group's convergence flag while the next group runs.  Kept for the life of
// the process and reused (one pair per running solve, per device).
struct StateSlot {
  int dev = -1;
  LsqrState *h = nullptr;  // two snapshots
  hipEvent_t ev[2] = {nullptr, nullptr};
};
std::mutex g_slot_mu;
std::vector<StateSlot> g_free_slots;

int take_slot(StateSlot *out) {
  int dev = 0;
  PSK_HIP_TRY(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_slot_mu);
    for (size_t i = 0; i < g_free_slots.size(); ++i)
      if (g_free_slots[i].dev == dev) {
        *out = g_free_slots[i];
        g_free_slots.erase(g_free_slots.begin() + (long)i);
        return 0;
      }
  }
  StateSlot sl;
  sl.dev = dev;
  PSK_HIP_TRY(hipHostMalloc((void **)&sl.h, 2 * sizeof(LsqrState), hipHostMallocDefault));
  for (int k = 0; k < 2; ++k)
    PSK_HIP_TRY(hipEventCreateWithFlags(&sl.ev[k], hipEventDisableTiming));
  *out = sl;
  return 0;
}

// returns the slot to the pool once no copy into it is pending
struct SlotGuard {
  StateSlot sl;
  bool held = false;
  ~SlotGuard() {
    if (!held) return;
    for (int k = 0; k < 2; ++k) (void)hipEventSynchronize(sl.ev[k]);
    std::lock_guard<std::mutex> lk(g_slot_mu);
    g_free_slots.push_back(sl);
  }
};

constexpr int kPassBlocks = 512;  // partial A^T u vectors per pass
constexpr int kCsrWaves = 8;      // wavefronts of a CSR pass workgroup
constexpr int kShortRow = 16;   // CSR rows up to this length take one lane each
constexpr int kRowsPerLane = 4; // CSR rows a lane works on at once in a pass
constexpr int kRegEntries = 4;  // entries per short CSR row held in registers

__device__ __forceinline__ void block_rows(int64_t n, int64_t &r0, int64_t &r1) {
  const int64_t per = ceil_div(n, (int64_t)gridDim.x);
  r0 = (int64_t)blockIdx.x * per;
  r1 = r0 + per;
  if (r1 > n) r1 = n;
}

// partial A^T u and ||u||^2 of this workgroup's rows, u_i updated in place.
// vhat is staged in LDS, so the gathers vhat[col] are LDS reads; the first
// kRegEntries entries of every short row are loaded at once and kept in
// registers for both products (A vhat and A^T u), so a row costs two
// dependent global loads (row pointers, then entries) whatever its length up
// to kRegEntries.  Additions keep the order: entries in sequence within a
// row; rows r, then lanes, into a wavefront's LDS accumulator row.
template <typename T, bool INIT>
__global__ __launch_bounds__(64 * kCsrWaves, 4) void k_pass_csr(
    const T *__restrict__ vals, const int64_t *__restrict__ indptr,
    const int32_t *__restrict__ indices, int64_t n, int64_t d,
    const double *__restrict__ vhat, const double *__restrict__ rhs,
    double *__restrict__ u, const LsqrState *__restrict__ st,
    double *__restrict__ part_t, double *__restrict__ part_b2) {
  const int stop = INIT ? 0 : st->done;  // tested after the first barrier
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *tl = reinterpret_cast<double *>(smem_raw);  // kCsrWaves x d accumulators
  double *vh = tl + kCsrWaves * d;                     // vhat, d
  __shared__ double b2s[kCsrWaves];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  int64_t rb0, rb1;
  block_rows(n, rb0, rb1);
  // row pointers and u (rhs on the first pass) of a batch of rows, fetched
  // ahead: the first batch's loads are in flight while the LDS is prepared,
  // the next batch's are issued at the end of the one before
  int64_t fq0[kRowsPerLane], fq1[kRowsPerLane];
  double fu[kRowsPerLane];
  auto fetch = [&](int64_t b) {
#pragma unroll
    for (int r = 0; r < kRowsPerLane; ++r) {
      const int64_t i = b + 64 * r + lane;
      fq0[r] = 0;
      fq1[r] = 0;
      fu[r] = 0.0;
      if (i < rb1) {
        fq0[r] = indptr[i];
        fq1[r] = indptr[i + 1];
        fu[r] = INIT ? rhs[i] : u[i];
      }
    }
  };
  int64_t base = rb0 + wave * 64 * kRowsPerLane;
  fetch(base);
  for (int64_t c = threadIdx.x; c < kCsrWaves * d; c += 64 * kCsrWaves) tl[c] = 0.0;
  if (!INIT)
    for (int64_t c = threadIdx.x; c < d; c += 64 * kCsrWaves) vh[c] = vhat[c];
  __syncthreads();
  if (stop) return;  // uniform per workgroup; nothing global written yet
  double *tw = tl + (int64_t)wave * d;
  const double au = INIT ? 0.0 : st->alpha * st->ufac;
  double b2 = 0.0;
  for (; base < rb1; base += 64 * kCsrWaves * kRowsPerLane) {
    int64_t p0[kRowsPerLane];
    int len[kRowsPerLane];  // entries of a short row, 0 for long or absent rows
    uint64_t longmask[kRowsPerLane];
    double ux[kRowsPerLane];  // u_i (rhs_i on the first pass) of short rows, else 0
#pragma unroll
    for (int r = 0; r < kRowsPerLane; ++r) {
      const bool lr = (fq1[r] - fq0[r]) > kShortRow;
      p0[r] = fq0[r];
      len[r] = lr ? 0 : (int)(fq1[r] - fq0[r]);
      longmask[r] = __ballot(lr);
      ux[r] = lr ? 0.0 : fu[r];
    }
    int maxlen = 0;
#pragma unroll
    for (int r = 0; r < kRowsPerLane; ++r) maxlen = max(maxlen, len[r]);
    // the first kRegEntries entries of every short row, all loads issued together
    int ci[kRowsPerLane][kRegEntries];
    double xv[kRowsPerLane][kRegEntries];
#pragma unroll
    for (int r = 0; r < kRowsPerLane; ++r)
#pragma unroll
      for (int e = 0; e < kRegEntries; ++e) {
        ci[r][e] = 0;
        xv[r][e] = 0.0;
        if (e < len[r]) {
          ci[r][e] = indices[p0[r] + e];
          xv[r][e] = (double)vals[p0[r] + e];
        }
      }
    double ui[kRowsPerLane];
    if (INIT) {
#pragma unroll
      for (int r = 0; r < kRowsPerLane; ++r) ui[r] = ux[r];
    } else {
      double dot[kRowsPerLane];
#pragma unroll
      for (int r = 0; r < kRowsPerLane; ++r) dot[r] = 0.0;
#pragma unroll
      for (int e = 0; e < kRegEntries; ++e)
#pragma unroll
        for (int r = 0; r < kRowsPerLane; ++r)
          if (e < len[r]) dot[r] += xv[r][e] * vh[ci[r][e]];
      for (int e = kRegEntries; e < maxlen; ++e) {
#pragma unroll
        for (int r = 0; r < kRowsPerLane; ++r) {
          const int64_t p = p0[r] + e;
          if (e < len[r]) dot[r] += (double)vals[p] * vh[indices[p]];
        }
      }
#pragma unroll
      for (int r = 0; r < kRowsPerLane; ++r) ui[r] = dot[r] - au * ux[r];
    }
#pragma unroll
    for (int r = 0; r < kRowsPerLane; ++r) {
      const int64_t i = base + 64 * r + lane;
      if (i < rb1 && !((longmask[r] >> lane) & 1)) {
        u[i] = ui[r];
        b2 += ui[r] * ui[r];
      }
    }
    // A^T u into this wavefront's LDS row, entries e, then rows r, then lanes
#pragma unroll
    for (int e = 0; e < kRegEntries; ++e)
#pragma unroll
      for (int r = 0; r < kRowsPerLane; ++r)
        if (e < len[r]) atomicAdd(&tw[ci[r][e]], xv[r][e] * ui[r]);
    for (int e = kRegEntries; e < maxlen; ++e) {
#pragma unroll
      for (int r = 0; r < kRowsPerLane; ++r) {
        const int64_t p = p0[r] + e;
        if (e < len[r]) atomicAdd(&tw[indices[p]], (double)vals[p] * ui[r]);
      }
    }
    // rows longer than kShortRow: the whole wavefront, one row at a time
#pragma unroll
    for (int r = 0; r < kRowsPerLane; ++r) {
      uint64_t pending = longmask[r];
      while (pending) {
        const int src = __ffsll((unsigned long long)pending) - 1;
        pending &= pending - 1;
        const int64_t row = base + 64 * r + src;
        const int64_t q0 = indptr[row];
        const int64_t q1 = indptr[row + 1];
        double uv;
        if (INIT) {
          uv = rhs[row];
        } else {
          double dt = 0.0;
          for (int64_t p = q0 + lane; p < q1; p += 64) dt += (double)vals[p] * vh[indices[p]];
          uv = wave_sum(dt) - au * u[row];
        }
        if (lane == 0) {
          u[row] = uv;
          b2 += uv * uv;
        }
        for (int64_t p = q0 + lane; p < q1; p += 64)
          atomicAdd(&tw[indices[p]], (double)vals[p] * uv);
      }
    }
    if (base + 64 * kCsrWaves * kRowsPerLane < rb1)
      fetch(base + 64 * kCsrWaves * kRowsPerLane);
  }
  b2 = wave_sum(b2);
  if (lane == 0) b2s[wave] = b2;
  __syncthreads();
  for (int64_t c = threadIdx.x; c < d; c += 64 * kCsrWaves) {
    double t = tl[c];
#pragma unroll
    for (int w = 1; w < kCsrWaves; ++w) t += tl[(int64_t)w * d + c];
    part_t[(int64_t)blockIdx.x * d + c] = t;
  }
  if (threadIdx.x == 0) {
    double t = b2s[0];
#pragma unroll
    for (int w = 1; w < kCsrWaves; ++w) t += b2s[w];
    part_b2[blockIdx.x] = t;
  }
}

// dense rows: wavefront per row, lane owns columns lane + 64k (k < KC);
// a wavefront takes RB of its rows (every fourth of the workgroup's) at a
// time, with their entries of u, so that short rows still keep a few KiB
// per wavefront in flight (launch_dense_pass picks RB).  A row past the
// workgroup's reads the batch's first row and counts as zero.
template <typename T, bool INIT, int KC, int RB>
__global__ __launch_bounds__(256) void k_pass_dense(
    const T *__restrict__ A, int64_t ld, int64_t n, int64_t d,
    const double *__restrict__ vhat, const double *__restrict__ rhs,
    double *__restrict__ u, const LsqrState *__restrict__ st,
    double *__restrict__ part_t, double *__restrict__ part_b2) {
  // the stop flag is read now and tested once vhat and the first batch of
  // rows are in flight (nothing is written before the test)
  const int stop = INIT ? 0 : st->done;
  __shared__ double tl[4][64 * KC];
  __shared__ double b2s[4];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const double au = INIT ? 0.0 : st->alpha * st->ufac;
  int64_t rb0, rb1;
  block_rows(n, rb0, rb1);
  double vh[KC], tacc[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int64_t c = lane + 64 * k;
    vh[k] = (!INIT && c < d) ? vhat[c] : 0.0;
    tacc[k] = 0.0;
  }
  double x[RB][KC], uo[RB];
  bool ok[RB];
  auto fetch = [&](int64_t i) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      ok[r] = i + 4 * r < rb1;
      const int64_t row = ok[r] ? i + 4 * r : i;
      const T *ra = A + row * ld;
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const int64_t c = lane + 64 * k;
        x[r][k] = (ok[r] && c < d) ? (double)ra[c] : 0.0;
      }
      uo[r] = INIT ? rhs[row] : u[row];
    }
  };
  int64_t i = rb0 + wave;
  if (i < rb1) fetch(i);
  if (stop) return;
  double b2 = 0.0;
  for (; i < rb1; i += 4 * RB) {
    double uu[RB];
    if (INIT) {
#pragma unroll
      for (int r = 0; r < RB; ++r) uu[r] = ok[r] ? uo[r] : 0.0;
    } else {
      double dt[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        dt[r] = 0.0;
#pragma unroll
        for (int k = 0; k < KC; ++k) dt[r] += x[r][k] * vh[k];
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < RB; ++r) dt[r] += __shfl_xor(dt[r], off, 64);
#pragma unroll
      for (int r = 0; r < RB; ++r) uu[r] = ok[r] ? dt[r] - au * uo[r] : 0.0;
    }
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (ok[r]) u[i + 4 * r] = uu[r];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) b2 += uu[r] * uu[r];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < RB; ++r) t += x[r][k] * uu[r];
      tacc[k] += t;
    }
    if (i + 4 * RB < rb1) fetch(i + 4 * RB);
  }
#pragma unroll
  for (int k = 0; k < KC; ++k) tl[wave][lane + 64 * k] = tacc[k];
  if (lane == 0) b2s[wave] = b2;  // every lane holds the same b2
  __syncthreads();
  for (int64_t c = threadIdx.x; c < d; c += 256)
    part_t[(int64_t)blockIdx.x * d + c] =
        ((tl[0][c] + tl[1][c]) + tl[2][c]) + tl[3][c];
  if (threadIdx.x == 0) part_b2[blockIdx.x] = ((b2s[0] + b2s[1]) + b2s[2]) + b2s[3];
}

// Triangular products with R^{-1}: a workgroup owns 8 rows (or columns);
// its 256 threads split the other index into 32 phases.
constexpr int kColsPerBlk = 8;
constexpr int kPhases = 32;
constexpr int kMaxK = 1024 / kPhases;  // terms per thread in a phase (d <= 1024)

// sum_{k<K} rv[k] * tv[first + kPhases k] with four accumulators: the full
// quads of k go round-robin to a0..a3, the remaining k to a0, and the result
// is (a0 + a1) + (a2 + a3).  rv holds the matrix entries, loaded ahead.
__device__ __forceinline__ double phased_dot(const double (&rv)[kMaxK],
                                             const double *__restrict__ tv, int64_t first,
                                             int K) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const int full = K & ~3;
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) {
    if (k < K) {
      const double t = tv[first + (int64_t)kPhases * k];
      if (k < full) {
        if ((k & 3) == 0) a0 += rv[k] * t;
        else if ((k & 3) == 1) a1 += rv[k] * t;
        else if ((k & 3) == 2) a2 += rv[k] * t;
        else a3 += rv[k] * t;
      } else {
        a0 += rv[k] * t;
      }
    }
  }
  return (a0 + a1) + (a2 + a3);
}

// beta = ||u||, t = (A^T u) / beta and the contributions of rows
// i0 .. i0 + kVRows - 1 of R^{-1} to vnew_j = sum_{i<=j} Rinv[i][j] t_i
// (the -beta v term is added where the partials are summed, k_update).
// Workgroup b owns those rows: it sums their t_i from the kPassBlocks pass
// partials (thread (g, c): column i0 + c, partials g, g + kVGroups, ...;
// the groups then in order) and writes vpart[b][j] for j >= i0.
constexpr int kVRows = 16;
constexpr int kVThreads = 512;
constexpr int kVGroups = kVThreads / kVRows;  // 32
constexpr int kVSlots = 1024 / kVThreads;     // columns j per thread (d <= 1024)

__global__ __launch_bounds__(kVThreads) void k_vnew_rows(
    const double *__restrict__ part_t, const double *__restrict__ part_b2,
    const double *__restrict__ Rinv, int64_t d, LsqrState *__restrict__ st,
    double *__restrict__ vpart, int init) {
  const int stop = init ? 0 : st->done;  // tested after the first barrier
  __shared__ double red[kVGroups][kVRows + 1];
  __shared__ double tv[kVRows];
  __shared__ double bred[kVThreads / 64];
  const int tid = threadIdx.x;
  const int c = tid % kVRows, g = tid / kVRows;
  const int64_t i0 = (int64_t)blockIdx.x * kVRows;
  const int64_t i = i0 + c;
  // loads first, all unconditional (indices clamped into range, values
  // masked afterwards): the pass partials, one partial square and the
  // R^{-1} entries of this thread's columns j in the workgroup's rows
  const int64_t ic = i < d ? i : d - 1;
  double pt[kPassBlocks / kVGroups];
#pragma unroll
  for (int q = 0; q < kPassBlocks / kVGroups; ++q)
    pt[q] = part_t[(int64_t)(g + kVGroups * q) * d + ic];
  double s = part_b2[tid < kPassBlocks ? tid : 0];
  double rr[kVSlots][kVRows];
#pragma unroll
  for (int sl = 0; sl < kVSlots; ++sl) {
    const int64_t j = i0 + tid + kVThreads * sl;
    const int64_t jc = j < d ? j : d - 1;
#pragma unroll
    for (int r = 0; r < kVRows; ++r) {
      const int64_t row = (i0 + r) <= jc ? i0 + r : jc;
      rr[sl][r] = Rinv[row * d + jc];
    }
  }
  if (tid >= kPassBlocks) s = 0.0;
  // beta from the kPassBlocks partial squares (same order in every workgroup)
  s = wave_sum(s);
  if ((tid & 63) == 0) bred[tid >> 6] = s;
  double ts = 0.0;
#pragma unroll
  for (int q = 0; q < kPassBlocks / kVGroups; ++q) ts += pt[q];
  red[g][c] = i < d ? ts : 0.0;
  __syncthreads();
  if (stop) return;  // uniform per workgroup; nothing written yet
  double b2 = bred[0];
#pragma unroll
  for (int w = 1; w < kVThreads / 64; ++w) b2 += bred[w];
  const double beta = sqrt(b2);
  const double binv = beta > 0.0 ? 1.0 / beta : 0.0;
  if (tid < kVRows) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kVGroups; ++q) t += red[q][tid];
    tv[tid] = t * binv;
  }
  __syncthreads();
#pragma unroll
  for (int sl = 0; sl < kVSlots; ++sl) {
    const int64_t j = i0 + tid + kVThreads * sl;
    if (j < d) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < kVRows; ++r)
        if (i0 + r <= j) acc += rr[sl][r] * tv[r];
      vpart[(int64_t)blockIdx.x * d + j] = acc;
    }
  }
  if (blockIdx.x == 0 && tid == 0) st->beta_new = beta;
}

// scalar recurrences, v/w/y updates and the stopping test (run by one
// whole workgroup of 256 threads).  ss is the workgroup's LDS copy of the
// state, loaded at the kernel's start; wp, yp the thread's first kUpdPre
// entries of w and y (j = tid + 256 q), likewise loaded early, so that
// nothing here waits on memory but the few entries of d > 256 kUpdPre.
constexpr int kUpdPre = 4;

__device__ void lsqr_update(LsqrState *__restrict__ st, const LsqrState &ss, int64_t d,
                            double *__restrict__ v, const double *__restrict__ vnew,
                            double *__restrict__ w, double *__restrict__ y,
                            const double (&wp)[kUpdPre], const double (&yp)[kUpdPre],
                            double alpha, double atol, double btol, int init) {
  __shared__ double sh[8];
  __shared__ double red[4];
  if (threadIdx.x == 0) {
    const double beta = ss.beta_new;
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
      const double anorm2 = ss.anorm2 + ss.alpha * ss.alpha + beta * beta;
      st->anorm2 = anorm2;
      const double rhobar = ss.rhobar;
      rho = sqrt(rhobar * rhobar + beta * beta);
      const double c = rhobar / rho;
      const double s = beta / rho;
      theta = s * alpha;
      st->rhobar = -c * alpha;
      phi = c * ss.phibar;
      const double phibar = s * ss.phibar;
      st->phibar = phibar;
      st->iters = ss.iters + 1;
      const double anorm = sqrt(anorm2);
      const double rnorm = phibar;
      const double arnorm = rnorm * alpha * fabs(c);
      st->rnorm = rnorm;
      st->arnorm = arnorm;
      st->test2 = (anorm > 0.0 && rnorm > 0.0) ? arnorm / (anorm * rnorm) : 0.0;
      if (arnorm <= atol * anorm * rnorm) done = 1;
      if (rnorm <= btol * ss.bnorm + atol * anorm * sqrt(ss.ynorm2)) done = 1;
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
  auto step = [&](int64_t j, double wj, double yj0) {
    const double vj = vnew[j] * ainv;
    if (init) {
      w[j] = vj;
      y[j] = 0.0;
    } else {
      const double yj = yj0 + fx * wj;
      y[j] = yj;
      y2 += yj * yj;
      w[j] = vj - fw * wj;
    }
    v[j] = vj;
  };
#pragma unroll
  for (int q = 0; q < kUpdPre; ++q) {
    const int64_t j = threadIdx.x + 256 * q;
    if (j < d) step(j, wp[q], yp[q]);
  }
  for (int64_t j = threadIdx.x + 256 * kUpdPre; j < d; j += 256) step(j, w[j], y[j]);
  y2 = wave_sum(y2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = y2;
  __syncthreads();
  if (threadIdx.x == 0) {
    st->ynorm2 = ((red[0] + red[1]) + red[2]) + red[3];
    if (sh[3] != 0.0) st->done = 1;
  }
}

// out_i = (accumulate ? out_i : 0) + sum_{j>=i} Rinv[i][j] vec_j; a workgroup
// owns 8 rows, 32 column phases per row (four accumulators each)
__global__ __launch_bounds__(256) void k_trmv(const double *__restrict__ Rinv, int64_t d,
                                              const double *__restrict__ vec,
                                              double *__restrict__ out,
                                              const LsqrState *__restrict__ st,
                                              int check_done, int accumulate) {
  if (check_done && st->done) return;
  __shared__ double red[kColsPerBlk][kPhases + 1];
  const int tid = threadIdx.x;
  const int c = tid >> 5;  // row within the block
  const int g = tid & 31;  // column phase
  const int64_t i = (int64_t)blockIdx.x * kColsPerBlk + c;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (i < d) {
    int64_t jj = i + ((g - (i & 31)) & 31);  // first j >= i with j = g mod 32
    const double *row = Rinv + i * d;
    for (; jj + 3 * kPhases < d; jj += 4 * kPhases) {
      a0 += row[jj] * vec[jj];
      a1 += row[jj + kPhases] * vec[jj + kPhases];
      a2 += row[jj + 2 * kPhases] * vec[jj + 2 * kPhases];
      a3 += row[jj + 3 * kPhases] * vec[jj + 3 * kPhases];
    }
    for (; jj < d; jj += kPhases) a0 += row[jj] * vec[jj];
  }
  red[c][g] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (tid < kColsPerBlk) {
    const int64_t ii = (int64_t)blockIdx.x * kColsPerBlk + tid;
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kPhases; ++q) t += red[tid][q];
    if (ii < d) out[ii] = accumulate ? out[ii] + t : t;
  }
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

// out[0] = max_i |R_ii|, out[1] = min_i |R_ii| (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_diag_ratio(const double *__restrict__ R, int64_t d,
                                                    double *__restrict__ out) {
  __shared__ double mx[256], mn[256];
  double a = 0.0, b = INFINITY;
  for (int64_t i = threadIdx.x; i < d; i += 256) {
    const double v = fabs(R[i * d + i]);
    a = fmax(a, v);
    b = fmin(b, v);
  }
  mx[threadIdx.x] = a;
  mn[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + s]);
      mn[threadIdx.x] = fmin(mn[threadIdx.x], mn[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = mx[0];
    out[1] = mn[0];
  }
}

// res_i = b_i - A_i x.  Dense: one wavefront per row.  CSR: one lane per
// row, and rows longer than kShortRow are taken by the whole wavefront.
template <typename T, bool CSR>
__global__ __launch_bounds__(256) void k_resid(const T *__restrict__ vals,
                                               const int64_t *__restrict__ indptr,
                                               const int32_t *__restrict__ indices,
                                               int64_t n, int64_t d, int64_t ld,
                                               const double *__restrict__ x,
                                               const double *__restrict__ b,
                                               double *__restrict__ res) {
  const int lane = threadIdx.x & 63;
  if (CSR) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool have = i < n;
    int64_t p0 = 0, p1 = 0;
    if (have) {
      p0 = indptr[i];
      p1 = indptr[i + 1];
    }
    const bool longrow = have && (p1 - p0) > kShortRow;
    if (have && !longrow) {
      double dot = 0.0;
      for (int64_t p = p0; p < p1; ++p) dot += (double)vals[p] * x[indices[p]];
      res[i] = b[i] - dot;
    }
    uint64_t pending = __ballot(longrow);
    while (pending) {
      const int src = __ffsll((unsigned long long)pending) - 1;
      pending &= pending - 1;
      const int64_t q0 = __shfl(p0, src, 64);
      const int64_t q1 = __shfl(p1, src, 64);
      const int64_t row = __shfl(i, src, 64);
      double dot = 0.0;
      for (int64_t p = q0 + lane; p < q1; p += 64) dot += (double)vals[p] * x[indices[p]];
      dot = wave_sum(dot);
      if (lane == 0) res[row] = b[row] - dot;
    }
    return;
  }
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (i >= n) return;
  double dot = 0.0;
  for (int64_t c = lane; c < d; c += 64) dot += (double)vals[i * ld + c] * x[c];
  dot = wave_sum(dot);
  if (lane == 0) res[i] = b[i] - dot;
}

// The second half of an iteration in one launch: every workgroup computes
// v of the previous iteration is read from v_in and the new one written to
// v_out (the two alternate), since every workgroup reads v while the extra
// one writes it.
// vnew_j = sum_{b <= j / kVRows} vpart[b][j] - beta v_j (partials in order),
// alpha = ||vnew|| (one fixed order, so every workgroup has the same bits)
// and rows of vhat = R^{-1} (vnew / alpha), 8 rows per workgroup.  The one
// extra workgroup (index nb) runs the scalar recurrences, the v, w, y
// updates and the stopping test, which no other workgroup of this launch
// reads; a stop it signals turns the following launches into no-ops.
template <int NBV>  // bound on the number of vnew partials (ceil(d / kVRows))
__global__ __launch_bounds__(256) void k_update(const double *__restrict__ Rinv, int64_t d,
                                                const double *__restrict__ vpart, int nb,
                                                LsqrState *__restrict__ st,
                                                const double *__restrict__ v_in,
                                                double *__restrict__ v_out,
                                                double *__restrict__ w, double *__restrict__ y,
                                                double *__restrict__ vhat, double atol,
                                                double btol, int init) {
  // the stop flag is read now and tested after the first barrier, so that
  // this launch's loads are already in flight (nothing is written before)
  const int stop = init ? 0 : st->done;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *vn = reinterpret_cast<double *>(smem_raw);  // vnew, d doubles
  __shared__ double red[kColsPerBlk][kPhases + 1];
  __shared__ double a2red[4];
  __shared__ LsqrState ss;  // the update workgroup's copy of the state
  const int tid = threadIdx.x;
  const bool upd = (int)blockIdx.x == nb;
  // the update workgroup loads the state and its w, y entries up front
  static_assert(sizeof(LsqrState) % 8 == 0 && sizeof(LsqrState) / 8 <= 256, "state words");
  double wp[kUpdPre], yp[kUpdPre];
#pragma unroll
  for (int q = 0; q < kUpdPre; ++q) {
    wp[q] = 0.0;
    yp[q] = 0.0;
  }
  if (upd) {
    if (tid < (int)(sizeof(LsqrState) / 8))
      reinterpret_cast<double *>(&ss)[tid] = reinterpret_cast<const double *>(st)[tid];
    if (!init) {
#pragma unroll
      for (int q = 0; q < kUpdPre; ++q) {
        const int64_t j = tid + 256 * q;
        const int64_t jc = j < d ? j : d - 1;
        wp[q] = w[jc];
        yp[q] = y[jc];
      }
    }
  }
  const int c = tid >> 5;  // row within the block
  const int g = tid & 31;  // column phase
  const int64_t i = (int64_t)blockIdx.x * kColsPerBlk + c;
  const int64_t jj0 = i + ((g - (i & 31)) & 31);  // first j >= i with j = g mod 32
  const int K = (!upd && i < d && jj0 < d) ? (int)ceil_div(d - jj0, kPhases) : 0;
  // loads first: this thread's R^{-1} entries
  double rv[kMaxK];
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) rv[k] = k < K ? Rinv[i * d + jj0 + kPhases * k] : 0.0;
  const double beta = st->beta_new;
  // entries j = tid + 256 q; for d <= 512 both of a thread's entries load
  // their partials at once (one round of memory latency instead of two)
  constexpr int kSl = NBV <= 512 / kVRows ? 2 : 1;
  double a2 = 0.0;
  for (int64_t j0 = tid; j0 < d; j0 += 256 * kSl) {
    // the shares of workgroups b <= j / kVRows, loaded unconditionally for
    // j < d (row index clamped) and summed in order; an entry j >= d loads
    // nothing and is not used
    double pv[kSl][NBV], vj[kSl];
#pragma unroll
    for (int q = 0; q < kSl; ++q) {
      const int64_t j = j0 + 256 * q;
      if (j < d) {
        const int nbj = (int)(j / kVRows) + 1;
#pragma unroll
        for (int b = 0; b < NBV; ++b)
          pv[q][b] = vpart[(int64_t)(b < nbj ? b : nbj - 1) * d + j];
        vj[q] = init ? 0.0 : v_in[j];
      }
    }
#pragma unroll
    for (int q = 0; q < kSl; ++q) {
      const int64_t j = j0 + 256 * q;
      if (j < d) {
        const int nbj = (int)(j / kVRows) + 1;
        double sv = 0.0;
#pragma unroll
        for (int b = 0; b < NBV; ++b)
          if (b < nbj) sv += pv[q][b];
        const double val = init ? sv : sv - beta * vj[q];
        vn[j] = val;
        a2 += val * val;
      }
    }
  }
  a2 = wave_sum(a2);
  if ((tid & 63) == 0) a2red[tid >> 6] = a2;
  __syncthreads();
  if (stop) return;  // uniform: every workgroup read the same flag
  const double alpha = sqrt(((a2red[0] + a2red[1]) + a2red[2]) + a2red[3]);
  if (upd) {
    lsqr_update(st, ss, d, v_out, vn, w, y, wp, yp, alpha, atol, btol, init);
    return;
  }
  const double ainv = alpha > 0.0 ? 1.0 / alpha : 0.0;
  red[c][g] = phased_dot(rv, vn, jj0, K);
  __syncthreads();
  if (tid < kColsPerBlk) {
    const int64_t ii = (int64_t)blockIdx.x * kColsPerBlk + tid;
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kPhases; ++q) t += red[tid][q];
    if (ii < d) vhat[ii] = t * ainv;
  }
}

struct LsqBufs {
  double *u, *part_t, *part_b2, *vpart, *v[2], *w, *y, *vhat;
  LsqrState *st;
};

template <typename T, bool INIT>
void launch_dense_pass(const psk_mat &A, const LsqBufs &B, const double *rhs,
                       hipStream_t s) {
  const T *a = (const T *)A.values;
  const int64_t d = A.d;
  // rows per wavefront batch (FP64, n = 1e6: d = 32 135 us a pass with 8
  // against 166 with 2; n = 2e4, d = 50: 10.1 us with 2 against 11.4 with
  // 8, a wavefront then holding about ten rows; d = 128: 4 better than 2)
#define PSK_DP(KC, RB)                                                                  \
  k_pass_dense<T, INIT, KC, RB><<<kPassBlocks, 256, 0, s>>>(a, A.ld, A.n, d, B.vhat, rhs, \
                                                            B.u, B.st, B.part_t, B.part_b2)
  if (d <= 64) {
    if (A.n >= 65536) PSK_DP(1, 8);
    else PSK_DP(1, 2);
  } else if (d <= 128) {
    PSK_DP(2, 4);
  } else if (d <= 256) {
    PSK_DP(4, 2);
  } else if (d <= 512) {
    PSK_DP(8, 2);
  } else {
    PSK_DP(16, 2);
  }
#undef PSK_DP
}

template <typename T>
void launch_pass(const psk_mat &A, bool init, const LsqBufs &B, const double *rhs,
                 hipStream_t s) {
  if (A.format == PSK_CSR) {
    const size_t lds = (size_t)(kCsrWaves + 1) * A.d * sizeof(double);
    const T *vals = (const T *)A.values;
    if (init)
      k_pass_csr<T, true><<<kPassBlocks, 64 * kCsrWaves, lds, s>>>(vals, A.indptr, A.indices, A.n, A.d,
                                                        B.vhat, rhs, B.u, B.st, B.part_t,
                                                        B.part_b2);
    else
      k_pass_csr<T, false><<<kPassBlocks, 64 * kCsrWaves, lds, s>>>(vals, A.indptr, A.indices, A.n, A.d,
                                                         B.vhat, rhs, B.u, B.st, B.part_t,
                                                         B.part_b2);
  } else {
    if (init)
      launch_dense_pass<T, true>(A, B, rhs, s);
    else
      launch_dense_pass<T, false>(A, B, rhs, s);
  }
}

// step k of a solve reads v[k & 1] and writes v[(k + 1) & 1]
void one_step(const psk_mat &A, bool init, int k, const LsqBufs &B, const double *Rinv,
              const double *rhs, const psk_lsq_opts &o, hipStream_t s) {
  const int64_t d = A.d;
  const unsigned nb16 = (unsigned)ceil_div(d, kColsPerBlk);
  {
    KTimer t("lsqr_pass", s);
    if (A.dtype == PSK_F64)
      launch_pass<double>(A, init, B, rhs, s);
    else
      launch_pass<float>(A, init, B, rhs, s);
  }
  const unsigned nbv = (unsigned)ceil_div(d, kVRows);
  k_vnew_rows<<<nbv, kVThreads, 0, s>>>(B.part_t, B.part_b2, Rinv, d, B.st, B.vpart,
                                        init ? 1 : 0);
  const size_t lds = (size_t)d * sizeof(double);
  if (nbv <= 512 / kVRows)
    k_update<512 / kVRows><<<nb16 + 1, 256, lds, s>>>(
        Rinv, d, B.vpart, (int)nb16, B.st, B.v[k & 1], B.v[(k + 1) & 1], B.w, B.y, B.vhat,
        o.atol, o.btol, init ? 1 : 0);
  else
    k_update<1024 / kVRows><<<nb16 + 1, 256, lds, s>>>(
        Rinv, d, B.vpart, (int)nb16, B.st, B.v[k & 1], B.v[(k + 1) & 1], B.w, B.y, B.vhat,
        o.atol, o.btol, init ? 1 : 0);
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
  B.u = ws.take<double>((size_t)n);
  B.part_t = ws.take<double>((size_t)kPassBlocks * d);
  B.part_b2 = ws.take<double>(kPassBlocks);
  B.vpart = ws.take<double>((size_t)ceil_div(d, kVRows) * d);
  B.v[0] = ws.take<double>((size_t)d);
  B.v[1] = ws.take<double>((size_t)d);
  B.w = ws.take<double>((size_t)d);
  B.y = ws.take<double>((size_t)d);
  B.vhat = ws.take<double>((size_t)d);
  double *res = ws.take<double>((size_t)n);  // residual of the refinement passes
  B.st = ws.take<LsqrState>(1);
  double *ratio = ws.take<double>(2);       // max |R_ii|, min |R_ii|
  // the reduced-precision sketch's perturbation against the FP64 one, on
  // request: that sketch kept (Chat), the FP64 sketch and its factor
  const bool want_delta = own && o.want_delta != 0 && o.prec != PSK_PREC_F64;
  double *Chat = want_delta ? ws.take<double>((size_t)m * d) : nullptr;
  double *C64 = want_delta ? ws.take<double>((size_t)m * d) : nullptr;
  double *R64 = want_delta ? ws.take<double>((size_t)d * d) : nullptr;
  double *Ri64 = want_delta ? ws.take<double>((size_t)d * d) : nullptr;
  double *dl = want_delta ? ws.take<double>(1) : nullptr;
  const size_t mk = ws.mark();
  int rc = 0;
  int *flag = nullptr;
  int prec_used = o.prec;
  // default limits: the BF16 sketch carries ~1e-5 relative error, the FP8
  // one ~5e-2
  const double cond_limit =
      o.escalate_cond != 0.0 ? o.escalate_cond : (o.prec == PSK_PREC_FP8 ? 10.0 : 1e4);
  const bool may_escalate =
      own && (o.prec == PSK_PREC_BF16 || o.prec == PSK_PREC_FP8) && cond_limit > 0.0;
  // CSR A whose S*A is sparse: the product over the nonzeros of S*A from
  // the binned rows (the FP64 rebuild too, whatever the first precision).
  // Otherwise, CSR A with the BF16 or FP8 GEMM: its operand comes straight
  // from the binned rows and S*A is only formed if the solve escalates to
  // FP64.
  const bool sparse_ok = own && gauss_sparse_ok(A, o.r, m);
  const bool sparse = sparse_ok && gauss_sparse_pick(A, o.r, m, o.prec);
  const bool fused = own && !sparse &&
                     ((o.prec == PSK_PREC_BF16 && bf16_csr_fusable(A, o.r)) ||
                      (o.prec == PSK_PREC_FP8 && fp8_csr_fusable(A, o.r)));
  void *SA = nullptr;
  uint32_t *perm = nullptr, *bptr = nullptr;
  // the FP64 sketch (after a reduced-precision one), S*A formed here if needed
  auto rebuild_f64 = [&](double *Cout) -> int {
    int e;
    if (sparse_ok)
      return gauss_gemm_sparse(m, o.r, A, perm, bptr, o.seed, PSK_PREC_F64, Cout, ws, st);
    if (fused && !SA) {
      SA = ws.take<double>((size_t)o.r * d);
      if ((e = cs_apply(A, (uint32_t)o.r, perm, bptr, SA, ws, st, true))) return e;
    }
    return gauss_gemm(m, o.r, d, o.seed, PSK_PREC_F64, SA, PSK_F64, Cout, ws, st);
  };
  size_t mk_sketch = 0;  // scratch above S*A and the bins: the sketch's
  if (own) {
    // sketch and factor (their scratch is released afterwards); S*A (or the
    // binned rows it is formed from) stays until the precision decision so
    // that an FP64 rebuild can reuse it
    if (!fused && !sparse) SA = ws.take<double>((size_t)o.r * d);
    if ((rc = cs_bin(A, (uint32_t)o.r, o.seed, ws, st, &perm, &bptr))) return rc;
    if (!fused && !sparse && (rc = cs_apply(A, (uint32_t)o.r, perm, bptr, SA, ws, st, true)))
      return rc;
    const size_t mk2 = ws.mark();
    mk_sketch = mk2;
    if (sparse)
      rc = gauss_gemm_sparse(m, o.r, A, perm, bptr, o.seed, o.prec, C, ws, st);
    else if (fused && o.prec == PSK_PREC_BF16)
      rc = gauss_gemm_bf16_csr(m, o.r, A, perm, bptr, o.seed, C, ws, st);
    else if (fused)
      rc = gauss_gemm_fp8_csr(m, o.r, A, perm, bptr, o.seed, C, ws, st);
    else
      rc = gauss_gemm(m, o.r, d, o.seed, o.prec, SA, PSK_F64, C, ws, st);
    if (rc) return rc;
    ws.release(mk2);
    if ((rc = sketch_qr_impl(C, m, d, R, Rinv, ws, st, &flag))) return rc;
    if (want_delta) {
      // delta = ||(Chat - C64) R64^{-1}||_2 for the FP64 sketch C64 of the
      // same S*A, its scratch above the factorization's (whose pivot flag is
      // read below); S*A formed here (fused forms) stays for an escalation
      if (!ws.dry())
        PSK_HIP_TRY(hipMemcpyAsync(Chat, C, (size_t)m * d * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
      if ((rc = rebuild_f64(C64))) return rc;
      const size_t mk3 = ws.mark();
      if ((rc = sketch_qr_impl(C64, m, d, R64, Ri64, ws, st))) return rc;
      ws.release(mk3);
      if ((rc = delta_from_factor(Chat, C64, Ri64, m, d, dl, ws, st))) return rc;
      ws.release(mk3);
    } else {
      ws.release(mk2);
    }
    if (may_escalate && ws.dry()) {
      // plan the FP64 rebuild as well
      if ((rc = rebuild_f64(C))) return rc;
      ws.release(mk2);
    }
  }
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for lsq_solve");
  // delta of the sketch LSQR is preconditioned with: 0 for the FP64 sketch,
  // NaN when not measured (not requested, or the caller's R^{-1})
  double delta_est = (own && o.prec == PSK_PREC_F64) ? 0.0 : NAN;
  if (own) {
    int hflag = 0;
    double hr[2] = {1.0, 1.0};
    k_diag_ratio<<<1, 256, 0, st>>>(R, d, ratio);
    PSK_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    PSK_HIP_TRY(hipMemcpyAsync(hr, ratio, sizeof(hr), hipMemcpyDeviceToHost, st));
    if (want_delta)
      PSK_HIP_TRY(hipMemcpyAsync(&delta_est, dl, sizeof(double), hipMemcpyDeviceToHost, st));
    PSK_HIP_TRY(hipStreamSynchronize(st));
    // A reduced-precision sketch only preconditions well while its relative
    // error (about 1e-5 for the BF16 GEMM) times cond(A) stays small; the
    // diagonal ratio of R is a cheap lower estimate of cond(A).
    // a NaN or an infinity in the sketch is not cured by an FP64 one
    if (hflag & 2) return factor_status(hflag, "");
    if (may_escalate && (hflag || !(hr[0] <= cond_limit * hr[1]))) {
      // the first factorization's flag has been read: its scratch is free
      ws.release(mk_sketch);
      const size_t mk2 = ws.mark();
      if (want_delta) {
        PSK_HIP_TRY(hipMemcpyAsync(C, C64, (size_t)m * d * sizeof(double),
                                   hipMemcpyDeviceToDevice, st));
      } else if ((rc = rebuild_f64(C))) {
        return rc;
      }
      ws.release(mk2);
      if ((rc = sketch_qr_impl(C, m, d, R, Rinv, ws, st, &flag))) return rc;
      ws.release(mk2);
      PSK_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
      PSK_HIP_TRY(hipStreamSynchronize(st));
      prec_used = PSK_PREC_F64;
      delta_est = 0.0;  // LSQR runs on the FP64 sketch now
    }
    if ((rc = factor_status(hflag, "sketch is numerically rank deficient"))) return rc;
  }
  ws.release(mk);

  const unsigned db = (unsigned)ceil_div(d, 256);
  const unsigned nb16 = (unsigned)ceil_div(d, kColsPerBlk);
  SlotGuard slot;
  if ((rc = take_slot(&slot.sl))) return rc;
  slot.held = true;
  k_zero<<<db, 256, 0, st>>>(x, d);
  int total_iters = 0;
  bool converged = true, nonfinite = false;
  LsqrState hs{};
  double rate = 0.0;  // d log(stopping margin) / d iteration, from the last pass
  for (int pass = 0; pass <= o.refine; ++pass) {
    const double *rhs = b;
    if (pass > 0) {
      // CSR: a lane per row; dense: a wavefront per row
      const unsigned rb = (unsigned)ceil_div(A.format == PSK_CSR ? n : n * 64, 256);
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
    k_zero<<<db, 256, 0, st>>>(B.v[0], d);
    one_step(A, true, 0, B, Rinv, rhs, o, st);
    int kstep = 1;
    // Groups of at most check_every iterations; after each, the state is
    // copied to pinned memory and the host reads the previous group's copy
    // while this one runs.  A group enqueued after convergence costs only
    // no-op launches (the device-side done flag), so the host sizes the
    // groups near the end: the stopping margin q (1 at the stopping test)
    // falls about geometrically, and from its rate over the known states the
    // last group is cut to end one iteration past the predicted stop and is
    // read at once.  A refinement pass starts from the first pass's rate,
    // with a short first group read at once (it usually needs few
    // iterations).  The prediction only sizes groups: the stop itself is the
    // device's test, and a wrong prediction costs a wait or no-op launches.
    int it = 0, ngroup = 0;
    int queue[2], queued = 0;  // slots of the groups enqueued and not yet read
    int known_it = -1, prev_it = -1;
    double known_q = 0.0, prev_q = 0.0;
    bool done = false;
    auto margin = [&](const LsqrState &s2) {
      double q = INFINITY;
      const double anorm = sqrt(s2.anorm2);
      if (o.atol > 0.0) q = s2.test2 / o.atol;
      const double den = o.btol * s2.bnorm + o.atol * anorm * sqrt(s2.ynorm2);
      if (den > 0.0) q = fmin(q, s2.rnorm / den);
      return q;
    };
    while (it < o.max_iter || queued > 0) {
      if (prev_it >= 0 && known_it > prev_it && prev_q > 0.0 && known_q > 0.0) {
        const double r = log(known_q / prev_q) / (known_it - prev_it);
        if (std::isfinite(r) && r < -1e-3) rate = r;
      }
      int batch = o.check_every;
      bool read_now = false;
      if (pass > 0 && ngroup == 0) {
        batch = batch < 4 ? batch : 4;
        read_now = true;
      } else if (known_it >= 0 && rate < 0.0 && known_q > 0.0 && std::isfinite(known_q)) {
        const int need =
            known_q <= 1.0 ? 0 : (int)fmin(ceil(log(known_q) / -rate), (double)o.max_iter);
        const int left = need - (it - known_it);  // predicted, beyond what is enqueued
        if (left <= 0 && queued > 0) {
          batch = 0;
        } else if (left < batch) {
          batch = left > 0 ? left + 1 : 1;
          read_now = true;
        }
      }
      if (batch > o.max_iter - it) batch = o.max_iter - it;
      if (batch > 0) {
        for (int q = 0; q < batch; ++q) one_step(A, false, kstep++, B, Rinv, rhs, o, st);
        it += batch;
        const int cur = ngroup++ & 1;
        PSK_HIP_TRY(hipMemcpyAsync(&slot.sl.h[cur], B.st, sizeof(LsqrState),
                                   hipMemcpyDeviceToHost, st));
        PSK_HIP_TRY(hipEventRecord(slot.sl.ev[cur], st));
        queue[queued++] = cur;
      }
      // read the older group while the newer one runs; everything when a
      // group was cut short, nothing was enqueued or max_iter is reached
      const int keep = (read_now || batch == 0 || it >= o.max_iter) ? 0 : 1;
      while (queued > keep) {
        const int sl = queue[0];
        queue[0] = queue[1];
        --queued;
        PSK_HIP_TRY(hipEventSynchronize(slot.sl.ev[sl]));
        hs = slot.sl.h[sl];
        prev_it = known_it;
        prev_q = known_q;
        known_it = hs.iters;
        known_q = margin(hs);
        if (hs.done) {
          done = true;
          break;
        }
        // a NaN or an infinity in A or b makes the norms non-finite and the
        // stopping test never true: stop at the first read that shows it
        if (!std::isfinite(hs.bnorm) || !std::isfinite(hs.rnorm) ||
            !std::isfinite(hs.anorm2)) {
          nonfinite = true;
          break;
        }
      }
      if (done || nonfinite) break;
    }
    if (nonfinite) break;
    // the groups still enqueued after the stop are no-ops; the stream
    // synchronisation below waits for them
    if (!done) converged = false;
    total_iters += hs.iters;
    // x += R^{-1} y
    k_trmv<<<nb16, 256, 0, st>>>(Rinv, d, B.y, x, B.st, 0, 1);
  }
  PSK_HIP_TRY(hipGetLastError());
  PSK_HIP_TRY(hipStreamSynchronize(st));
  if (nonfinite)
    return fail(PSK_ENONFINITE, "LSQR's norms are not finite: A or b holds a NaN or an infinity");
  if (info) {
    info->iters = total_iters;
    info->status = converged ? PSK_OK : PSK_ENOCONV;
    info->resid = hs.rnorm;
    info->ne_resid = hs.test2;
    info->prec_used = own ? prec_used : -1;
    info->reserved = 0;
    info->delta_est = delta_est;
  }
  if (!converged) return fail(PSK_ENOCONV, "LSQR reached max_iter before its tolerance");
  return 0;
}

}  // namespace psk
