// C-ABI layer of libpsk: argument validation, workspace planning and
// dispatch to the kernel files.  Every entry point checks its arguments on
// the host before anything is enqueued and reports failures as psk_status
// codes with a thread-local message; no C++ exception crosses the boundary.
#include <math.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace psk {

static thread_local std::string g_last_error;

// ---- kernel timing -----------------------------------------------------------
namespace {
struct Pending {
  std::string name;
  hipEvent_t a, b;
};
struct Agg {
  double ms = 0.0;
  int64_t n = 0;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<Pending> g_pending;
std::map<std::string, Agg> g_agg;
std::string g_only;  // ",name,name," to record only those brackets; empty: all
std::string g_names;

void drain_locked() {
  for (auto &p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      Agg &g = g_agg[p.name];
      g.ms += ms;
      g.n += 1;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
}
}  // namespace

bool timing_enabled() { return g_timing; }

int timing_begin(const char *name, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!g_only.empty() && g_only.find("," + std::string(name) + ",") == std::string::npos)
    return -1;
  Pending p;
  p.name = name;
  if (hipEventCreate(&p.a) != hipSuccess) return -1;
  if (hipEventCreate(&p.b) != hipSuccess) {
    (void)hipEventDestroy(p.a);
    return -1;
  }
  (void)hipEventRecord(p.a, st);
  g_pending.push_back(p);
  return (int)g_pending.size() - 1;
}

void timing_end(int slot, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (slot >= 0 && slot < (int)g_pending.size()) (void)hipEventRecord(g_pending[slot].b, st);
}

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int status, const std::string &msg) {
  g_last_error = msg;
  return status;
}

int check_mat(const psk_mat *A) {
  if (!A) return fail(PSK_EINVAL, "A is NULL");
  if (A->format != PSK_DENSE && A->format != PSK_CSR)
    return fail(PSK_EINVAL, "A->format must be PSK_DENSE or PSK_CSR");
  if (A->dtype != PSK_F64 && A->dtype != PSK_F32)
    return fail(PSK_EDTYPE, "A->dtype must be PSK_F64 or PSK_F32");
  if (A->n < 1 || A->d < 1) return fail(PSK_EINVAL, "A must have n >= 1 and d >= 1");
  if (A->n >= ((int64_t)1 << 31)) return fail(PSK_EUNSUPPORTED, "n must be < 2^31");
  if ((A->flags & ~(uint32_t)PSK_MAT_CHECKED) != 0u || A->reserved != 0u)
    return fail(PSK_EINVAL, "A->flags may hold PSK_MAT_CHECKED only; A->reserved must be 0");
  if (A->format == PSK_DENSE) {
    if (A->ld < A->d) return fail(PSK_EINVAL, "dense A needs ld >= d");
    if (!A->values) return fail(PSK_EINVAL, "A->values is NULL");
  } else {
    if (A->nnz < 0) return fail(PSK_EINVAL, "CSR A needs nnz >= 0");
    if (!A->indptr) return fail(PSK_EINVAL, "CSR A->indptr is NULL");
    if (A->nnz > 0 && (!A->values || !A->indices))
      return fail(PSK_EINVAL, "CSR A->values/indices is NULL");
    if (A->d > INT32_MAX) return fail(PSK_EUNSUPPORTED, "CSR d must fit int32");
  }
  return 0;
}

int check_r(int64_t r) {
  if (r < 1 || r >= ((int64_t)1 << 31)) return fail(PSK_EINVAL, "r must be in [1, 2^31)");
  return 0;
}

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// plan + run helpers shared by the entry points, psk_workspace_size and the
// request server
int do_sketch_cs(const psk_mat &A, int64_t r, uint64_t seed, void *SA, Arena &ws,
                 hipStream_t st, bool out_f64) {
  uint32_t *perm = nullptr, *bptr = nullptr;
  int rc = cs_bin(A, (uint32_t)r, seed, ws, st, &perm, &bptr);
  if (rc) return rc;
  return cs_apply(A, (uint32_t)r, perm, bptr, SA, ws, st, out_f64);
}

int do_sketch_gcs(const psk_mat &A, int64_t m, int64_t r, uint64_t seed, int prec,
                  void *C, Arena &ws, hipStream_t st) {
  if (m == 0) return do_sketch_cs(A, r, seed, C, ws, st);
  if (gauss_sparse_pick(A, r, m, prec)) {
    // S*A is sparse: the product over its nonzeros
    uint32_t *perm = nullptr, *bptr = nullptr;
    int rc = cs_bin(A, (uint32_t)r, seed, ws, st, &perm, &bptr);
    if (rc) return rc;
    return gauss_gemm_sparse(m, r, A, perm, bptr, seed, prec, (double *)C, ws, st);
  }
  const bool fb = prec == PSK_PREC_BF16 && bf16_csr_fusable(A, r);
  const bool f8 = prec == PSK_PREC_FP8 && fp8_csr_fusable(A, r);
  if (fb || f8) {
    // the BF16 limbs / FP8 bytes of S*A straight from the binned rows
    uint32_t *perm = nullptr, *bptr = nullptr;
    int rc = cs_bin(A, (uint32_t)r, seed, ws, st, &perm, &bptr);
    if (rc) return rc;
    if (fb) return gauss_gemm_bf16_csr(m, r, A, perm, bptr, seed, (double *)C, ws, st);
    return gauss_gemm_fp8_csr(m, r, A, perm, bptr, seed, (double *)C, ws, st);
  }
  // S*A as its FP64 sums (FP32 A too), the operand of every Gaussian GEMM
  void *SA = ws.take<double>((size_t)r * A.d);
  int rc = do_sketch_cs(A, r, seed, SA, ws, st, true);
  if (rc) return rc;
  return gauss_gemm(m, r, A.d, seed, prec, SA, PSK_F64, (double *)C, ws, st);
}

int do_sketch_osnap(const psk_mat &A, int64_t s, int64_t m, int64_t r, uint64_t seed,
                    int prec, void *C, Arena &ws, hipStream_t st) {
  if (s == 1) return do_sketch_gcs(A, m, r, seed, prec, C, ws, st);
  uint32_t *perm = nullptr, *bptr = nullptr;
  int rc = osnap_bin(A, (uint32_t)s, (uint32_t)r, seed, ws, st, &perm, &bptr);
  if (rc) return rc;
  // each bucket's signed rows summed in FP64, times 1/sqrt(s) once
  const double scale = 1.0 / sqrt((double)s);
  const int64_t entries = A.n * s;
  if (m == 0)
    return cs_apply(A, (uint32_t)r, perm, bptr, C, ws, st, false, scale, entries);
  // CSR A whose S*A is sparse: the product over its nonzeros, formed from
  // the same bins with the same sums
  if (gauss_sparse_pick(A, r, m, prec, s))
    return gauss_gemm_sparse(m, r, A, perm, bptr, seed, prec, (double *)C, ws, st, s, scale);
  void *SA = ws.take<double>((size_t)r * A.d);
  if ((rc = cs_apply(A, (uint32_t)r, perm, bptr, SA, ws, st, true, scale, entries))) return rc;
  return gauss_gemm(m, r, A.d, seed, prec, SA, PSK_F64, (double *)C, ws, st);
}

int do_sketch_g(const psk_mat &A, int64_t m, uint64_t seed, int prec, double *C, Arena &ws,
                hipStream_t st) {
  if (A.format == PSK_CSR) {
    if (!gauss_sparse_fits(A))
      return fail(PSK_EUNSUPPORTED, "sketch_g of CSR A needs d <= 1023 and nnz < 2^31");
    uint32_t *perm = nullptr, *bptr = nullptr;
    int rc = identity_bins(A.n, ws, &perm, &bptr, st);
    if (rc) return rc;
    return gauss_gemm_sparse(m, A.n, A, perm, bptr, seed, prec, C, ws, st);
  }
  const void *op = A.values;
  if (A.ld != A.d) {
    // the GEMM reads its operand with row stride d
    const size_t es = elem_size(A.dtype);
    void *cp = ws.take<unsigned char>((size_t)A.n * A.d * es);
    if (!ws.dry()) {
      if (!ws.ok()) return fail(PSK_ENOMEM, "workspace too small for sketch_g");
      PSK_HIP_TRY(hipMemcpy2DAsync(cp, (size_t)A.d * es, A.values, (size_t)A.ld * es,
                                   (size_t)A.d * es, (size_t)A.n, hipMemcpyDeviceToDevice, st));
    }
    op = cp;
  }
  return gauss_gemm(m, A.n, A.d, seed, prec, op, A.dtype, C, ws, st);
}

}  // namespace psk

using namespace psk;

extern "C" {

const char *psk_version(void) { return "psk 0.1.0 (gfx950)"; }

int psk_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing = on != 0;
  return PSK_OK;
}

int psk_timing_only(const char *names) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_only = (names && *names) ? "," + std::string(names) + "," : std::string();
  return PSK_OK;
}

int psk_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_tmu);
  drain_locked();
  g_agg.clear();
  return PSK_OK;
}

int psk_timing_collect(const char *name, double *total_ms, int64_t *launches) {
  if (!name || !total_ms || !launches) return fail(PSK_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(g_tmu);
  drain_locked();
  auto it = g_agg.find(name);
  *total_ms = it == g_agg.end() ? 0.0 : it->second.ms;
  *launches = it == g_agg.end() ? 0 : it->second.n;
  return PSK_OK;
}

const char *psk_timing_names(void) {
  std::lock_guard<std::mutex> lk(g_tmu);
  drain_locked();
  g_names.clear();
  for (auto &kv : g_agg) {
    if (!g_names.empty()) g_names += ",";
    g_names += kv.first;
  }
  return g_names.c_str();
}

const char *psk_last_error(void) { return g_last_error.c_str(); }

// Shapes of an OSNAP: 1 <= s <= r with s | r, and n s < 2^32 (bin positions
// are 32-bit).
static int check_osnap(const psk_mat &A, int64_t s, int64_t r) {
  if (s < 1 || s > r || r % s != 0)
    return fail(PSK_EINVAL, "OSNAP needs 1 <= s <= r with s dividing r");
  if (A.n * s >= ((int64_t)1 << 32)) return fail(PSK_EUNSUPPORTED, "OSNAP needs n * s < 2^32");
  return 0;
}

// Shapes of leverage_sketch: the sketch has m >= d rows (G S A) or, with
// m == 0, r >= d rows (S A); t >= 0 columns of Pi, d * t < 2^31.
static int check_leverage_sketch(const psk_mat &A, int64_t m, int64_t r, int64_t t,
                                 int prec) {
  int rc = check_r(r);
  if (rc) return rc;
  if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PSK_EINVAL, "m must be in [0, 2^31)");
  if (m == 0 && r < A.d) return fail(PSK_EINVAL, "leverage_sketch with m == 0 needs r >= d");
  if (m > 0 && m < A.d) return fail(PSK_EINVAL, "leverage_sketch needs m >= d (or m == 0)");
  if (t < 0 || A.d * t >= ((int64_t)1 << 31))
    return fail(PSK_EINVAL, "t must be >= 0 with d * t < 2^31");
  if (m > 0 && prec != PSK_PREC_F64 && prec != PSK_PREC_BF16 && prec != PSK_PREC_FP8)
    return fail(PSK_EDTYPE, "prec must be PSK_PREC_F64, PSK_PREC_BF16 or PSK_PREC_FP8");
  return 0;
}

// Shapes of the column subset selection: the sketch as for leverage_sketch,
// 1 <= k <= d <= 4096.
static int check_css(const psk_mat &A, int64_t m, int64_t r, int64_t k, int prec) {
  int rc = check_leverage_sketch(A, m, r, 0, prec);
  if (rc) return rc;
  if (k < 1 || k > A.d) return fail(PSK_EINVAL, "k must be in [1, d]");
  return 0;
}

int psk_workspace_size(int op, const psk_mat *A, int64_t m, int64_t r, int64_t k,
                       int prec, size_t *bytes) {
  if (!bytes) return fail(PSK_EINVAL, "bytes is NULL");
  if (!A) return fail(PSK_EINVAL, "A is NULL");
  if ((A->flags & ~(uint32_t)PSK_MAT_CHECKED) != 0u || A->reserved != 0u)
    return fail(PSK_EINVAL, "A->flags may hold PSK_MAT_CHECKED only; A->reserved must be 0");
  Arena ws;  // dry run
  int rc = 0;
  // every call that walks a CSR A checks its structure first (its result
  // word is released before the call's own scratch is taken)
  if (op != PSK_OP_QR && op != PSK_OP_DELTA && op != PSK_OP_CHECK &&
      (rc = validate_csr(*A, ws, nullptr)))
    return rc;
  switch (op) {
    case PSK_OP_CHECK:
      rc = check_operand(*A, true, ws, nullptr);
      break;
    case PSK_OP_SKETCH_OSNAP:
      if ((rc = check_r(r))) return rc;
      if ((rc = check_osnap(*A, k, r))) return rc;
      if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PSK_EINVAL, "m must be in [0, 2^31)");
      rc = do_sketch_osnap(*A, k, m, r, 0, prec, nullptr, ws, nullptr);
      break;
    case PSK_OP_SKETCH_CS:
      if ((rc = check_r(r))) return rc;
      rc = do_sketch_cs(*A, r, 0, nullptr, ws, nullptr);
      break;
    case PSK_OP_SKETCH_GCS:
      if ((rc = check_r(r))) return rc;
      if (m < 0) return fail(PSK_EINVAL, "m must be >= 0");
      rc = do_sketch_gcs(*A, m, r, 0, prec, nullptr, ws, nullptr);
      break;
    case PSK_OP_GRAM:
      rc = A->format == PSK_DENSE ? gram_dense(1.0, *A, 0.0, nullptr, ws, nullptr)
                                  : gram_csr(1.0, *A, 0.0, nullptr, ws, nullptr);
      break;
    case PSK_OP_ROWNORMS:
      if (k < 1) return fail(PSK_EINVAL, "k must be >= 1");
      rc = A->format == PSK_DENSE
               ? rownorms_dense(1.0, *A, nullptr, k, 0.0, nullptr, ws, nullptr)
               : rownorms_csr(1.0, *A, nullptr, k, 0.0, nullptr, ws, nullptr);
      break;
    case PSK_OP_QR:
      rc = sketch_qr_impl(nullptr, A->n, A->d, nullptr, nullptr, ws, nullptr);
      break;
    case PSK_OP_DELTA:
      if (A->d < 1 || A->n < A->d) return fail(PSK_EINVAL, "PSK_OP_DELTA needs n = m >= d >= 1");
      rc = sketch_delta_impl(nullptr, nullptr, A->n, A->d, nullptr, ws, nullptr);
      break;
    case PSK_OP_LSQ: {
      psk_lsq_opts o{};
      if (m == 0) {
        // the caller passes its own R^{-1}: no sketch, no factorization
        static const double dummy = 0.0;
        o.Rinv = &dummy;
      } else {
        if ((rc = check_r(r))) return rc;
        if (m < A->d || r < m) return fail(PSK_EINVAL, "LSQ workspace needs d <= m <= r");
      }
      o.m = m;
      o.r = r;
      o.prec = prec;
      o.max_iter = 1;
      o.check_every = 1;
      o.want_delta = k != 0 ? 1 : 0;
      rc = lsq_impl(*A, nullptr, nullptr, o, nullptr, ws, nullptr);
      break;
    }
    case PSK_OP_SKETCH_G:
      if (m < 1 || m >= ((int64_t)1 << 31)) return fail(PSK_EINVAL, "m must be in [1, 2^31)");
      rc = do_sketch_g(*A, m, 0, prec, nullptr, ws, nullptr);
      break;
    case PSK_OP_LEVERAGE_GRAM:
      rc = leverage_gram_impl(*A, nullptr, ws, nullptr);
      break;
    case PSK_OP_LSQ_GRAM:
      rc = lsq_gram_impl(*A, nullptr, nullptr, ws, nullptr);
      break;
    case PSK_OP_LSQ_SKETCH:
      if ((rc = check_r(r))) return rc;
      if (m < A->d || m >= ((int64_t)1 << 31))
        return fail(PSK_EINVAL, "lsq_sketch_solve needs d <= m < 2^31");
      rc = lsq_sketch_solve_impl(*A, nullptr, nullptr, m, r, 0, prec, ws, nullptr);
      break;
    case PSK_OP_LEVERAGE_SKETCH:
      if ((rc = check_leverage_sketch(*A, m, r, k, prec))) return rc;
      rc = leverage_sketch_impl(*A, m, r, k, 0, prec, nullptr, true, ws, nullptr);
      break;
    case PSK_OP_CSS:
      if ((rc = check_css(*A, m, r, k, prec))) return rc;
      rc = css_select_impl(*A, m, r, k, 0, prec, nullptr, ws, nullptr);
      break;
    case PSK_OP_LEVERAGE_CSS:
      if ((rc = check_css(*A, m, r, k, prec))) return rc;
      rc = leverage_css_impl(*A, m, r, k, 0, prec, nullptr, nullptr, ws, nullptr);
      break;
    default:
      return fail(PSK_EINVAL, "unknown op");
  }
  if (rc) return rc;
  *bytes = ws.peak + 256;
  return PSK_OK;
}

int cs_hash(int64_t row0, int64_t count, int64_t r, uint64_t seed, int32_t *h,
            int8_t *sign, void *stream) {
  if (count < 0 || row0 < 0) return fail(PSK_EINVAL, "count and row0 must be >= 0");
  int rc = check_r(r);
  if (rc) return rc;
  return cs_hash_export(row0, count, (uint32_t)r, seed, h, sign, as_stream(stream));
}

int sketch_cs(const psk_mat *A, int64_t r, uint64_t seed, void *SA, void *wsp,
              size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if ((rc = check_r(r))) return rc;
  if (!SA) return fail(PSK_EINVAL, "SA is NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  if ((rc = do_sketch_cs(*A, r, seed, nullptr, plan, nullptr))) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_SKETCH_CS)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return do_sketch_cs(*A, r, seed, SA, ws, as_stream(stream));
}

int sketch_gcs(const psk_mat *A, int64_t m, int64_t r, uint64_t seed, int prec,
               void *C, void *wsp, size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if ((rc = check_r(r))) return rc;
  if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PSK_EINVAL, "m must be in [0, 2^31)");
  if (m > 0 && prec != PSK_PREC_F64 && prec != PSK_PREC_BF16 && prec != PSK_PREC_FP8)
    return fail(PSK_EDTYPE, "prec must be PSK_PREC_F64, PSK_PREC_BF16 or PSK_PREC_FP8");
  if (!C) return fail(PSK_EINVAL, "C is NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  if ((rc = do_sketch_gcs(*A, m, r, seed, prec, nullptr, plan, nullptr))) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_SKETCH_GCS)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return do_sketch_gcs(*A, m, r, seed, prec, C, ws, as_stream(stream));
}

int osnap_hash(int64_t row0, int64_t count, int64_t s, int64_t r, uint64_t seed, int32_t *h,
               int8_t *sign, void *stream) {
  if (count < 0 || row0 < 0) return fail(PSK_EINVAL, "count and row0 must be >= 0");
  int rc = check_r(r);
  if (rc) return rc;
  if (s < 1 || s > r || r % s != 0)
    return fail(PSK_EINVAL, "OSNAP needs 1 <= s <= r with s dividing r");
  if (count > (((int64_t)1 << 40) - 1) / s) return fail(PSK_EINVAL, "count * s must be < 2^40");
  return osnap_hash_export(row0, count, (uint32_t)s, (uint32_t)r, seed, h, sign,
                           as_stream(stream));
}

int sketch_osnap(const psk_mat *A, int64_t s, int64_t m, int64_t r, uint64_t seed, int prec,
                 void *C, void *wsp, size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if ((rc = check_r(r))) return rc;
  if ((rc = check_osnap(*A, s, r))) return rc;
  if (m < 0 || m >= ((int64_t)1 << 31)) return fail(PSK_EINVAL, "m must be in [0, 2^31)");
  if (m > 0 && prec != PSK_PREC_F64 && prec != PSK_PREC_BF16 && prec != PSK_PREC_FP8)
    return fail(PSK_EDTYPE, "prec must be PSK_PREC_F64, PSK_PREC_BF16 or PSK_PREC_FP8");
  if (!C) return fail(PSK_EINVAL, "C is NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  if ((rc = do_sketch_osnap(*A, s, m, r, seed, prec, nullptr, plan, nullptr))) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_SKETCH_OSNAP)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return do_sketch_osnap(*A, s, m, r, seed, prec, C, ws, as_stream(stream));
}

int sketch_g(const psk_mat *A, int64_t m, uint64_t seed, int prec, double *C, void *wsp,
             size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if (m < 1 || m >= ((int64_t)1 << 31)) return fail(PSK_EINVAL, "m must be in [1, 2^31)");
  if (prec != PSK_PREC_F64 && prec != PSK_PREC_BF16 && prec != PSK_PREC_FP8)
    return fail(PSK_EDTYPE, "prec must be PSK_PREC_F64, PSK_PREC_BF16 or PSK_PREC_FP8");
  if (!C) return fail(PSK_EINVAL, "C is NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  if ((rc = do_sketch_g(*A, m, seed, prec, nullptr, plan, nullptr))) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_SKETCH_G)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return do_sketch_g(*A, m, seed, prec, C, ws, as_stream(stream));
}

int leverage_gram(const psk_mat *A, double *theta, void *wsp, size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if (!theta) return fail(PSK_EINVAL, "theta is NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  if ((rc = leverage_gram_impl(*A, nullptr, plan, nullptr))) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_LEVERAGE_GRAM)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return leverage_gram_impl(*A, theta, ws, as_stream(stream));
}

int lsq_gram(const psk_mat *A, const double *b, double *x, void *wsp, size_t ws_bytes,
             void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if (!b || !x) return fail(PSK_EINVAL, "b and x must be non-NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  if ((rc = lsq_gram_impl(*A, nullptr, nullptr, plan, nullptr))) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_LSQ_GRAM)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return lsq_gram_impl(*A, b, x, ws, as_stream(stream));
}

int lsq_sketch_solve(const psk_mat *A, const double *b, double *x, int64_t m, int64_t r,
                     uint64_t seed, int prec, void *wsp, size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if ((rc = check_r(r))) return rc;
  if (m < A->d || m >= ((int64_t)1 << 31))
    return fail(PSK_EINVAL, "lsq_sketch_solve needs d <= m < 2^31");
  if (prec != PSK_PREC_F64 && prec != PSK_PREC_BF16 && prec != PSK_PREC_FP8)
    return fail(PSK_EDTYPE, "prec must be PSK_PREC_F64, PSK_PREC_BF16 or PSK_PREC_FP8");
  if (!b || !x) return fail(PSK_EINVAL, "b and x must be non-NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  if ((rc = lsq_sketch_solve_impl(*A, nullptr, nullptr, m, r, seed, prec, plan, nullptr)))
    return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_LSQ_SKETCH)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return lsq_sketch_solve_impl(*A, b, x, m, r, seed, prec, ws, as_stream(stream));
}

int leverage_sketch(const psk_mat *A, int64_t m, int64_t r, int64_t t, uint64_t seed, int prec,
                    double *theta, void *wsp, size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if ((rc = check_leverage_sketch(*A, m, r, t, prec))) return rc;
  if (!theta) return fail(PSK_EINVAL, "theta is NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  if ((rc = leverage_sketch_impl(*A, m, r, t, seed, prec, nullptr, true, plan, nullptr)))
    return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_LEVERAGE_SKETCH)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return leverage_sketch_impl(*A, m, r, t, seed, prec, theta, true, ws, as_stream(stream));
}

int css_select(const psk_mat *A, int64_t m, int64_t r, int64_t k, uint64_t seed, int prec,
               int32_t *cols, void *wsp, size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if ((rc = check_css(*A, m, r, k, prec))) return rc;
  if (!cols) return fail(PSK_EINVAL, "cols is NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  if ((rc = css_select_impl(*A, m, r, k, seed, prec, nullptr, plan, nullptr))) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_CSS)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return css_select_impl(*A, m, r, k, seed, prec, cols, ws, as_stream(stream));
}

int leverage_css(const psk_mat *A, int64_t m, int64_t r, int64_t k, uint64_t seed, int prec,
                 double *theta, int32_t *cols, void *wsp, size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if ((rc = check_css(*A, m, r, k, prec))) return rc;
  if (!theta) return fail(PSK_EINVAL, "theta is NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  // planned without the caller's cols, so the bound covers both forms
  if ((rc = leverage_css_impl(*A, m, r, k, seed, prec, nullptr, nullptr, plan, nullptr)))
    return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_LEVERAGE_CSS)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return leverage_css_impl(*A, m, r, k, seed, prec, theta, cols, ws, as_stream(stream));
}

int gram(double alpha, const psk_mat *A, double beta, void *C, void *wsp,
         size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if (!C) return fail(PSK_EINVAL, "C is NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  rc = A->format == PSK_DENSE ? gram_dense(alpha, *A, beta, nullptr, plan, nullptr)
                              : gram_csr(alpha, *A, beta, nullptr, plan, nullptr);
  if (rc) return rc;
  if (ws_bytes < plan.peak || (plan.peak > 0 && !wsp))
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_GRAM)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return A->format == PSK_DENSE ? gram_dense(alpha, *A, beta, C, ws, as_stream(stream))
                                : gram_csr(alpha, *A, beta, C, ws, as_stream(stream));
}

int rownorms_sq(double alpha, const psk_mat *A, const double *B, int64_t k,
                double beta, double *x, void *wsp, size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if (k < 1) return fail(PSK_EINVAL, "k must be >= 1");
  if (!B || !x) return fail(PSK_EINVAL, "B and x must be non-NULL");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  rc = A->format == PSK_DENSE
           ? rownorms_dense(alpha, *A, nullptr, k, beta, nullptr, plan, nullptr)
           : rownorms_csr(alpha, *A, nullptr, k, beta, nullptr, plan, nullptr);
  if (rc) return rc;
  if (ws_bytes < plan.peak || (plan.peak > 0 && !wsp))
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_ROWNORMS)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return A->format == PSK_DENSE
             ? rownorms_dense(alpha, *A, B, k, beta, x, ws, as_stream(stream))
             : rownorms_csr(alpha, *A, B, k, beta, x, ws, as_stream(stream));
}

int psk_check(const psk_mat *A, int check_values, void *wsp, size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if (A->format == PSK_DENSE && !check_values) return PSK_OK;
  Arena plan;
  if ((rc = check_operand(*A, check_values != 0, plan, nullptr))) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_CHECK)");
  Arena ws = Arena::over(wsp, ws_bytes);
  return check_operand(*A, check_values != 0, ws, as_stream(stream));
}

int sketch_qr(const double *C, int64_t m, int64_t d, double *R, double *Rinv,
              void *wsp, size_t ws_bytes, void *stream) {
  if (d < 1 || m < d) return fail(PSK_EINVAL, "sketch_qr needs m >= d >= 1");
  if (!C || !R || !Rinv) return fail(PSK_EINVAL, "C, R and Rinv must be non-NULL");
  Arena plan;
  int rc = sketch_qr_impl(nullptr, m, d, nullptr, nullptr, plan, nullptr);
  if (rc) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_QR)");
  Arena ws = Arena::over(wsp, ws_bytes);
  return sketch_qr_impl(C, m, d, R, Rinv, ws, as_stream(stream));
}

int sketch_delta(const double *Chat, const double *C, int64_t m, int64_t d, double *delta,
                 void *wsp, size_t ws_bytes, void *stream) {
  if (d < 1 || m < d) return fail(PSK_EINVAL, "sketch_delta needs m >= d >= 1");
  if (!Chat || !C || !delta) return fail(PSK_EINVAL, "Chat, C and delta must be non-NULL");
  Arena plan;
  int rc = sketch_delta_impl(nullptr, nullptr, m, d, nullptr, plan, nullptr);
  if (rc) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_DELTA)");
  Arena ws = Arena::over(wsp, ws_bytes);
  return sketch_delta_impl(Chat, C, m, d, delta, ws, as_stream(stream));
}

int lsq_solve(const psk_mat *A, const double *b, double *x, const psk_lsq_opts *opts,
              psk_lsq_info *info, void *wsp, size_t ws_bytes, void *stream) {
  int rc = check_mat(A);
  if (rc) return rc;
  if (!opts || !b || !x) return fail(PSK_EINVAL, "opts, b and x must be non-NULL");
  const psk_lsq_opts &o = *opts;
  if (!o.Rinv) {
    if (o.m < A->d) return fail(PSK_EINVAL, "lsq_solve needs opts->m >= d");
    if ((rc = check_r(o.r))) return rc;
    if (o.r < o.m) return fail(PSK_EINVAL, "lsq_solve needs opts->r >= opts->m");
  }
  if (o.max_iter < 1 || o.check_every < 1 || o.refine < 0)
    return fail(PSK_EINVAL, "lsq_solve needs max_iter >= 1, check_every >= 1, refine >= 0");
  if (!o.Rinv && o.prec != PSK_PREC_F64 && o.prec != PSK_PREC_BF16 &&
      o.prec != PSK_PREC_FP8)
    return fail(PSK_EDTYPE, "opts->prec must be PSK_PREC_F64, PSK_PREC_BF16 or PSK_PREC_FP8");
  Arena plan;
  if ((rc = validate_csr(*A, plan, nullptr))) return rc;
  if ((rc = lsq_impl(*A, nullptr, nullptr, o, nullptr, plan, nullptr))) return rc;
  if (!wsp || ws_bytes < plan.peak)
    return fail(PSK_ENOMEM, "workspace smaller than psk_workspace_size(PSK_OP_LSQ)");
  Arena ws = Arena::over(wsp, ws_bytes);
  if ((rc = validate_csr(*A, ws, as_stream(stream)))) return rc;
  return lsq_impl(*A, b, x, o, info, ws, as_stream(stream));
}

}  // extern "C"
