// Internal interfaces between the C-ABI layer and the kernel files of libpsk.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/psk.h"
#include "common.hpp"

namespace psk {

// Bump allocator over the caller's workspace.  A default-constructed arena
// only measures (psk_workspace_size runs the same planning code).
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  size_t peak = 0;      // high-water mark (regions may be reused, see mark())
  bool measure = true;  // planning pass: hand out nothing, launch nothing
  static Arena over(void *p, size_t bytes) {
    Arena a;
    a.base = (char *)p;
    a.cap = bytes;
    a.measure = false;
    return a;
  }
  bool dry() const { return measure; }
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = measure ? nullptr : reinterpret_cast<T *>(base + off);
    off += count * sizeof(T);
    if (off > peak) peak = off;
    return p;
  }
  // Scratch taken after mark() can be released with release(mark) and
  // handed out again: all work of one call is ordered on one stream.
  size_t mark() const { return off; }
  void release(size_t m) { off = m; }
  bool ok() const { return measure || peak <= cap; }
};

inline size_t elem_size(int dtype) { return dtype == PSK_F64 ? 8 : 4; }

// Event bracket around a launch (or region) when timing is enabled:
//   { KTimer t("gauss_gemm", st); kernel<<<..., st>>>(...); }
bool timing_enabled();
int timing_begin(const char *name, hipStream_t st);
void timing_end(int slot, hipStream_t st);
struct KTimer {
  int slot;
  hipStream_t st;
  KTimer(const char *name, hipStream_t s, bool on = true) : slot(-1), st(s) {
    if (on && timing_enabled()) slot = timing_begin(name, s);
  }
  ~KTimer() {
    if (slot >= 0) timing_end(slot, st);
  }
};

// ---- CountSketch (k_sketch.hip) ---------------------------------------------
// Bins the rows of A by bucket: perm[j] (row | sign<<31) sorted by bucket,
// stable; bptr[b] .. bptr[b+1] is bucket b's range.  For CSR A only rows
// holding an entry are binned, so bptr[r] may be below n and perm is valid
// only below bptr[r].  Returns 0 or a status.
int cs_bin(const psk_mat &A, uint32_t r, uint64_t seed, Arena &ws, hipStream_t st,
           uint32_t **perm, uint32_t **bptr);
// Stable LSD radix sort (8-bit digits) of (key, val) pairs with keys < r;
// keys/vals are consumed (used as the first ping-pong buffers).  On return
// *skeys/*svals point at the sorted arrays; with ptr != NULL, ptr[0..r] gets
// the start of each key's run (ptr[r] = n).  With dn != NULL only the first
// dn[0] <= n pairs (a count on the device) are sorted.
int sort_pairs(uint32_t *keys, uint32_t *vals, int64_t n, uint32_t r, Arena &ws,
               hipStream_t st, uint32_t **skeys, uint32_t **svals, uint32_t *ptr,
               const uint32_t *dn = nullptr);
int cs_hash_export(int64_t row0, int64_t count, uint32_t r, uint64_t seed,
                   int32_t *h, int8_t *sign, hipStream_t st);
// S*A into SA (r x d row-major): each bucket's rows summed in FP64 in bin
// order, multiplied by scale, written in the dtype of A, or in FP64 with
// out_f64.  entries: bin entries in all (n for CountSketch, n s for an
// OSNAP; 0 means n), which sizes the split of long buckets.
int cs_apply(const psk_mat &A, uint32_t r, const uint32_t *perm,
             const uint32_t *bptr, void *SA, Arena &ws, hipStream_t st,
             bool out_f64 = false, double scale = 1.0, int64_t entries = 0);
// OSNAP with s non-zeros per row (block construction, s | r): bins of the
// n s (row, non-zero) pairs, as cs_bin (CSR A: of the rows holding an
// entry); the hash export writes count * s rows and signs, non-zero k of
// row row0 + i at [i s + k].
int osnap_bin(const psk_mat &A, uint32_t s, uint32_t r, uint64_t seed, Arena &ws,
              hipStream_t st, uint32_t **perm, uint32_t **bptr);
int osnap_hash_export(int64_t row0, int64_t count, uint32_t s, uint32_t r, uint64_t seed,
                      int32_t *h, int8_t *sign, hipStream_t st);
// Wavefronts per bucket cs_apply uses for n rows in r buckets (1 = one
// wavefront sums a whole bucket).
int cs_splits(int64_t n, int64_t r);
// In-place exclusive scan of L uint32 values (k_sketch.hip); sums: scratch of
// scan_plan.
int scan_plan(int64_t L, Arena &ws, uint32_t **sums);
void scan_run(uint32_t *data, int64_t L, uint32_t *sums, hipStream_t st);

// Argument checks shared by the entry points (abi.hip): 0 or a status.
int check_mat(const psk_mat *A);
int check_r(int64_t r);

// ---- operand validation (k_check.hip) ---------------------------------------
// One pass over CSR A's offsets and indices (and, with values, over the stored
// values of CSR or dense A), then one read of the result on the host (the
// stream is synchronised): PSK_EINVAL for a malformed CSR structure,
// PSK_ENONFINITE for a NaN or infinity, else 0.  A planning arena only
// reserves the result word.
int check_operand(const psk_mat &A, bool values, Arena &ws, hipStream_t st);
// check_operand of the structure alone, for CSR A (dense A: nothing), with
// its word released again; every entry point runs it before any kernel that
// walks A.
int validate_csr(const psk_mat &A, Arena &ws, hipStream_t st);
// Bits of the status word the factorizations write (an int in device
// memory, cleared by its owner): 1 a Cholesky pivot not positive, 2 a pivot
// or a checked result not finite.  flag_nonfinite ORs 2 into *flag when one
// of count FP64 values is NaN or infinite; factor_status turns the word read
// back into PSK_ENONFINITE (bit 2, first), PSK_ERANK with rank_msg, or 0.
void flag_nonfinite(const double *p, int64_t count, int *flag, hipStream_t st);
int factor_status(int h, const char *rank_msg);

// S*A and G*S*A end to end (binning, scatter, GEMM), abi.hip.
// S*A in the dtype of A (FP64 sums rounded once), or as the FP64 sums
int do_sketch_cs(const psk_mat &A, int64_t r, uint64_t seed, void *SA, Arena &ws,
                 hipStream_t st, bool out_f64 = false);
int do_sketch_gcs(const psk_mat &A, int64_t m, int64_t r, uint64_t seed, int prec,
                  void *C, Arena &ws, hipStream_t st);
// G*S*A (m > 0) or S*A (m == 0) with the OSNAP S of s non-zeros per row;
// s == 1 is do_sketch_gcs itself.
int do_sketch_osnap(const psk_mat &A, int64_t s, int64_t m, int64_t r, uint64_t seed,
                    int prec, void *C, Arena &ws, hipStream_t st);
// C = G*A (sketch_g): the Gaussian GEMM with A as operand (dense), or the
// sparse product over A's entries with one row per bucket (CSR)
int do_sketch_g(const psk_mat &A, int64_t m, uint64_t seed, int prec, double *C, Arena &ws,
                hipStream_t st);

// ---- Gaussian GEMM (k_gauss_gemm.hip) --------------------------------------
// C (m x d, FP64) = G (m x r) * SA (r x d, dtype sa_dtype), G generated.
int gauss_gemm(int64_t m, int64_t r, int64_t d, uint64_t seed, int prec,
               const void *SA, int sa_dtype, double *C, Arena &ws,
               hipStream_t st);

// The same product with bfloat16 operands (k_gauss_gemm_bf16.hip).
int gauss_gemm_bf16(int64_t m, int64_t r, int64_t d, uint64_t seed, const void *SA,
                    int sa_dtype, double *C, Arena &ws, hipStream_t st);
// For CSR A the BF16 product can start from the binned rows (perm, bptr of
// cs_bin) and form the limbs of S*A directly, without the r x d array; the
// result is the same bits.  bf16_csr_fusable tells when this path applies.
bool bf16_csr_fusable(const psk_mat &A, int64_t r);
int gauss_gemm_bf16_csr(int64_t m, int64_t r, const psk_mat &A, const uint32_t *perm,
                        const uint32_t *bptr, uint64_t seed, double *C, Arena &ws,
                        hipStream_t st);
// ... and with FP8 e4m3 operands, per-128-bucket E8M0 scales (k_gauss_gemm_fp8.hip).
int gauss_gemm_fp8(int64_t m, int64_t r, int64_t d, uint64_t seed, const void *SA,
                   int sa_dtype, double *C, Arena &ws, hipStream_t st);
// The FP8 product of CSR A from the binned rows (same bits, no r x d array).
bool fp8_csr_fusable(const psk_mat &A, int64_t r);
int gauss_gemm_fp8_csr(int64_t m, int64_t r, const psk_mat &A, const uint32_t *perm,
                       const uint32_t *bptr, uint64_t seed, double *C, Arena &ws,
                       hipStream_t st);

// The Gaussian product of CSR A over the nonzeros of S*A (k_gauss_sparse.hip),
// from the binned rows, in any of the three precisions; gauss_sparse_ok tells
// when it applies (S*A at most 1/32 dense, d <= 1023), gauss_sparse_pick when
// it is the kernel to use (FP8 keeps the fused dense FP8 GEMM unless A has
// fewer than r d / 512 nonzeros: above that its MFMA contraction costs less
// than the sparse product's per-nonzero updates).
// per_row: bin entries per row of A (1 for CountSketch, s for an OSNAP)
bool gauss_sparse_ok(const psk_mat &A, int64_t r, int64_t m, int64_t per_row = 1);
bool gauss_sparse_pick(const psk_mat &A, int64_t r, int64_t m, int prec, int64_t per_row = 1);
// the product's own limits (CSR, d <= 1023, sizes); gauss_gemm_sparse checks
// only these, the callers choose when it is worth taking
bool gauss_sparse_fits(const psk_mat &A, int64_t per_row = 1);
// one row per bucket, in row order, sign +1: the bins of S = identity
int identity_bins(int64_t n, Arena &ws, uint32_t **perm, uint32_t **bptr, hipStream_t st);
// per_row, sa_scale: the OSNAP's bins of n s (row, non-zero) pairs and its
// 1/sqrt(s), applied to each bucket's sum as S*A is formed
int gauss_gemm_sparse(int64_t m, int64_t r, const psk_mat &A, const uint32_t *perm,
                      const uint32_t *bptr, uint64_t seed, int prec, double *C, Arena &ws,
                      hipStream_t st, int64_t per_row = 1, double sa_scale = 1.0);

// ---- FP64 dense kernels (k_dense.hip) --------------------------------------
// C (d x d, out_dtype) = alpha * A^T A + beta * C for dense A.
int gram_dense(double alpha, const psk_mat &A, double beta, void *C, Arena &ws,
               hipStream_t st, bool out_f64 = false);
// x = alpha * rownorm^2(A B) + beta * x, dense A, B d x k FP64.
int rownorms_dense(double alpha, const psk_mat &A, const double *B, int64_t k,
                   double beta, double *x, Arena &ws, hipStream_t st);
// General FP64 product C = alpha*op(A)*op(B) + beta*C, all row-major.
int dgemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
          const double *A, int64_t lda, const double *B, int64_t ldb,
          double beta, double *C, int64_t ldc, Arena &ws, hipStream_t st);

// ---- CSR kernels (k_csr.hip) -----------------------------------------------
// out_f64: C is FP64 whatever the dtype of A (else the dtype of A)
int gram_csr(double alpha, const psk_mat &A, double beta, void *C, Arena &ws,
             hipStream_t st, bool out_f64 = false);
int rownorms_csr(double alpha, const psk_mat &A, const double *B, int64_t k,
                 double beta, double *x, Arena &ws, hipStream_t st);

// ---- small dense factorizations (k_chol.hip) -------------------------------
// flag_out (optional) receives the device address of an int set non-zero
// when a Cholesky pivot was not positive (numerically rank deficient C).
int sketch_qr_impl(const double *C, int64_t m, int64_t d, double *R,
                   double *Rinv, Arena &ws, hipStream_t st,
                   int **flag_out = nullptr);
// Upper Cholesky factor R of the SPD d x d matrix W (destroyed), W = R^T R,
// and X = R^{-1} (both written entirely, zero below the diagonal); *flag (a
// device int, 8-byte aligned, two ints cleared here) is set non-zero when a
// pivot was not positive.  d <= 4096.
int chol_factor(double *W, int64_t d, double *R, double *X, int *flag, Arena &ws,
                hipStream_t st);

// ---- direct solvers and exact leverage scores (k_direct.hip) ---------------
int leverage_gram_impl(const psk_mat &A, double *theta, Arena &ws, hipStream_t st);
int lsq_gram_impl(const psk_mat &A, const double *b, double *x, Arena &ws, hipStream_t st);
int lsq_sketch_solve_impl(const psk_mat &A, const double *b, double *x, int64_t m, int64_t r,
                          uint64_t seed, int prec, Arena &ws, hipStream_t st);

// ---- leverage scores from a sketch (k_leverage.hip) -------------------------
// theta_i = ||e_i^T A X||^2, X = R^{-1} (t == 0) or R^{-1} Pi (d x t), R from
// sketch_qr of G S A (m > 0) or S A (m == 0).  check_rank: synchronise the
// stream and return PSK_ERANK when a Cholesky pivot was not positive.
int leverage_sketch_impl(const psk_mat &A, int64_t m, int64_t r, int64_t t, uint64_t seed,
                         int prec, double *theta, bool check_rank, Arena &ws, hipStream_t st);
// The sketch as an FP64 operand of the factorizations: G S A (m > 0, m x d)
// or S A (m == 0, r x d; an FP32 S A is widened).
int sketch_f64(const psk_mat &A, int64_t m, int64_t r, uint64_t seed, int prec, double *C,
               Arena &ws, hipStream_t st);

// ---- perturbation of a sketch (k_delta.hip) ----------------------------------
// *delta (device) = ||(Chat - C) R^{-1}||_2, R from sketch_qr of C (m x d,
// m >= d, FP64 row-major).
int sketch_delta_impl(const double *Chat, const double *C, int64_t m, int64_t d, double *delta,
                      Arena &ws, hipStream_t st);
// the same with R^{-1} of C already at hand
int delta_from_factor(const double *Chat, const double *C, const double *Ri, int64_t m,
                      int64_t d, double *delta, Arena &ws, hipStream_t st);

// ---- column subset selection (k_css.hip) ------------------------------------
// cols[0..k): the first k pivots of the column-pivoted QR of the sketch.
int css_select_impl(const psk_mat &A, int64_t m, int64_t r, int64_t k, uint64_t seed, int prec,
                    int32_t *cols, Arena &ws, hipStream_t st);
// theta: exact leverage scores of A[:, cols] for those k columns (cols may be
// NULL: kept in the workspace).
int leverage_css_impl(const psk_mat &A, int64_t m, int64_t r, int64_t k, uint64_t seed, int prec,
                      double *theta, int32_t *cols, Arena &ws, hipStream_t st);

// ---- LSQR (k_lsqr.hip) -----------------------------------------------------
int lsq_impl(const psk_mat &A, const double *b, double *x,
             const psk_lsq_opts &o, psk_lsq_info *info, Arena &ws,
             hipStream_t st);

}  // namespace psk
