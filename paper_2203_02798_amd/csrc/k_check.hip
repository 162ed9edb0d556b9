// Validation of a matrix operand before any kernel that walks it: the CSR
// structure (offsets from 0 to nnz, never decreasing; column indices in
// [0, d), Section 1 notation) and, on request, the finiteness of the stored
// values.  One pass reads the offsets and indices (and values) once, ORs the
// predicates of csr_check.hpp into a device word, and the host reads that
// word once after the pass.
#include "csr_check.hpp"
#include "internal.hpp"

namespace psk {
namespace {

constexpr int kChkThreads = 256;
constexpr int kChkUnroll = 4;

__global__ void k_check_clear(uint32_t *__restrict__ flag) {
  if (threadIdx.x == 0) flag[0] = 0u;
}

template <typename T>
__global__ void __launch_bounds__(kChkThreads)
    k_check_csr(const int64_t *__restrict__ indptr, const int32_t *__restrict__ indices,
                const T *__restrict__ values, int64_t n, int64_t d, int64_t nnz,
                int check_values, uint32_t *__restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * kChkThreads;
  const int64_t t0 = (int64_t)blockIdx.x * kChkThreads + threadIdx.x;
  uint32_t code = 0;
  // row offsets: row i reads indptr[i] and indptr[i + 1] (i + 1 <= n)
  for (int64_t i = t0; i < n; i += stride)
    code |= csr_row_code(indptr[i], indptr[i + 1], i, n, nnz);
  // entries, kChkUnroll loads in flight per thread: addresses are clamped to
  // the last entry, the codes of the clamped copies are masked out
  const int64_t last = nnz - 1;
  for (int64_t k = t0; k < nnz; k += stride * kChkUnroll) {
    int32_t c[kChkUnroll];
#pragma unroll
    for (int u = 0; u < kChkUnroll; ++u) {
      const int64_t e = k + u * stride;
      c[u] = indices[e < nnz ? e : last];
    }
#pragma unroll
    for (int u = 0; u < kChkUnroll; ++u)
      if (k + u * stride < nnz) code |= csr_index_code(c[u], d);
    if (check_values) {
      T v[kChkUnroll];
#pragma unroll
      for (int u = 0; u < kChkUnroll; ++u) {
        const int64_t e = k + u * stride;
        v[u] = values[e < nnz ? e : last];
      }
#pragma unroll
      for (int u = 0; u < kChkUnroll; ++u)
        if (k + u * stride < nnz) code |= value_code(v[u]);
    }
  }
  if (code) atomicOr(flag, code);
}

// Dense values: one wavefront per row (grid-stride over rows), lanes across
// the row's d entries at stride ld.
template <typename T>
__global__ void __launch_bounds__(kChkThreads)
    k_check_dense(const T *__restrict__ values, int64_t n, int64_t d, int64_t ld,
                  uint32_t *__restrict__ flag) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (kChkThreads / 64);
  uint32_t code = 0;
  for (int64_t i = (int64_t)blockIdx.x * (kChkThreads / 64) + (threadIdx.x >> 6); i < n;
       i += waves) {
    const T *row = values + i * ld;
    for (int64_t j = lane; j < d; j += 64) code |= value_code(row[j]);
  }
  if (code) atomicOr(flag, code);
}

// count FP64 values: kCheckNonFinite into *flag when one is NaN or infinite
__global__ void __launch_bounds__(kChkThreads)
    k_flag_nonfinite(const double *__restrict__ p, int64_t count, int *__restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * kChkThreads;
  const int64_t last = count - 1;
  uint32_t code = 0;
  for (int64_t k = (int64_t)blockIdx.x * kChkThreads + threadIdx.x; k < count;
       k += stride * kChkUnroll) {
    double v[kChkUnroll];
#pragma unroll
    for (int u = 0; u < kChkUnroll; ++u) {
      const int64_t e = k + u * stride;
      v[u] = p[e < count ? e : last];
    }
#pragma unroll
    for (int u = 0; u < kChkUnroll; ++u)
      if (k + u * stride < count) code |= value_code(v[u]);
  }
  if (code) atomicOr(flag, (int)code);
}

int read_code(const uint32_t *flag, hipStream_t st, uint32_t *code) {
  uint32_t h = 0;
  PSK_HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, st));
  PSK_HIP_TRY(hipStreamSynchronize(st));
  *code = h;
  return 0;
}

}  // namespace

int check_operand(const psk_mat &A, bool values, Arena &ws, hipStream_t st) {
  uint32_t *flag = ws.take<uint32_t>(1);
  if (ws.dry()) return 0;
  if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for the operand check");
  if (A.format == PSK_DENSE && !values) return 0;
  KTimer timer("check", st);
  k_check_clear<<<1, 64, 0, st>>>(flag);
  if (A.format == PSK_CSR) {
    const int64_t work = A.n > A.nnz ? A.n : A.nnz;
    const int64_t blocks = ceil_div(work, (int64_t)kChkThreads * kChkUnroll);
    const unsigned grid = (unsigned)(blocks < 1 ? 1 : blocks > 8192 ? 8192 : blocks);
    const int cv = values ? 1 : 0;
    if (A.dtype == PSK_F64)
      k_check_csr<double><<<grid, kChkThreads, 0, st>>>(A.indptr, A.indices,
                                                         (const double *)A.values, A.n, A.d,
                                                         A.nnz, cv, flag);
    else
      k_check_csr<float><<<grid, kChkThreads, 0, st>>>(A.indptr, A.indices,
                                                        (const float *)A.values, A.n, A.d,
                                                        A.nnz, cv, flag);
  } else {
    const int64_t blocks = ceil_div(A.n, (int64_t)(kChkThreads / 64));
    const unsigned grid = (unsigned)(blocks > 8192 ? 8192 : blocks);
    if (A.dtype == PSK_F64)
      k_check_dense<double><<<grid, kChkThreads, 0, st>>>((const double *)A.values, A.n, A.d,
                                                           A.ld, flag);
    else
      k_check_dense<float><<<grid, kChkThreads, 0, st>>>((const float *)A.values, A.n, A.d,
                                                          A.ld, flag);
  }
  PSK_HIP_TRY(hipGetLastError());
  uint32_t code = 0;
  int rc = read_code(flag, st, &code);
  if (rc) return rc;
  if (code & kCheckStructure)
    return fail(PSK_EINVAL,
                "CSR A is malformed: indptr must start at 0, never decrease and end at nnz, "
                "and every column index must lie in [0, d)");
  if (code & kCheckNonFinite) return fail(PSK_ENONFINITE, "A holds a NaN or an infinity");
  return 0;
}

void flag_nonfinite(const double *p, int64_t count, int *flag, hipStream_t st) {
  if (count <= 0) return;
  const int64_t blocks = ceil_div(count, (int64_t)kChkThreads * kChkUnroll);
  k_flag_nonfinite<<<(unsigned)(blocks > 2048 ? 2048 : blocks), kChkThreads, 0, st>>>(p, count,
                                                                                      flag);
}

int factor_status(int h, const char *rank_msg) {
  if (h & (int)kCheckNonFinite)
    return fail(PSK_ENONFINITE,
                "a NaN or an infinity reached the factorization or its result: the input "
                "holds one, or a sum overflowed");
  if (h) return fail(PSK_ERANK, rank_msg);
  return 0;
}

int validate_csr(const psk_mat &A, Arena &ws, hipStream_t st) {
  // dense A has no structure to check; a CSR matrix flagged as checked was
  // accepted by psk_check before, on the caller's word
  if (A.format != PSK_CSR || (A.flags & PSK_MAT_CHECKED)) return 0;
  const size_t mk = ws.mark();
  const int rc = check_operand(A, false, ws, st);
  ws.release(mk);
  return rc;
}

}  // namespace psk
