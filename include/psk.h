/*
 * psk.h -- C ABI of libpsk: randomized sketching of tall-and-skinny matrices
 * on one AMD Instinct MI355X (gfx950).
 *
 * Operations follow "pylspack: Parallel algorithms and data structures for
 * sketching, column subset selection, regression and leverage scores"
 * (Sobczyk & Gallopoulos, arXiv 2203.02798):
 *
 *   cs_hash      the CountSketch hash h(i), sigma_i          (Definition 3)
 *   sketch_cs    S*A                                         (Alg. bcs_multiply)
 *   sketch_gcs   G*S*A, G Gaussian scaled by 1/sqrt(m)       (Alg. countgauss_multiply,
 *                                                             csrcgs / rmcgs)
 *   gram         C <- alpha*A^T*A + beta*C                   (Alg. gram, csrrk)
 *   rownorms_sq  x <- alpha*||e_i^T A B||^2 + beta*x         (Alg. squared_row_norms,
 *                                                             csrsqn / rmsqn)
 *   sketch_qr    R and R^{-1} of a sketch C = Q*R            (the orthogonaliser of
 *                                                             Alg. ls_approximate_drineas
 *                                                             and least_squares_precondition)
 *   lsq_solve    min ||A x - b|| by sketch-and-precondition  (Alg. least_squares_precondition)
 *   leverage_sketch  approximate leverage scores, optionally    (Alg. ls_approximate_drineas)
 *                    through a JL matrix Pi
 *   css_select   k columns by a pivoted QR of the sketch     (Alg. cgrrqr)
 *   leverage_css leverage scores of the selected columns     (Alg. ls_hrn_exact)
 *   leverage_gram, lsq_gram, lsq_sketch_solve, sketch_g: section 4's direct
 *                    solvers and exact leverage scores, and Gaussian sketching
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrix/vector pointers are DEVICE pointers on the current HIP device,
 *   owned by the caller; the library never frees them and never allocates
 *   device memory.  Scratch space is passed in as (ws, ws_bytes); its minimum
 *   size comes from psk_workspace_size().  Its contents on entry do not matter.
 * - `stream` is a hipStream_t (NULL = the default stream).  A call on dense A
 *   only enqueues work on that stream and returns; outputs are valid once
 *   the stream has reached that point.  Three things synchronise the stream
 *   inside a call: the structure check of a CSR A (below), the rank and
 *   finiteness checks of the calls that factor (lsq_solve, lsq_sketch_solve,
 *   lsq_gram, leverage_gram, leverage_sketch, css_select, leverage_css) and
 *   lsq_solve's convergence tests.
 * - A CSR A is validated on the device before any kernel walks it: offsets
 *   from 0 to nnz, never decreasing, column indices in [0, d) (the CSR
 *   definition of Section 1).  One pass reads indptr and indices once; a
 *   malformed A returns PSK_EINVAL with nothing else enqueued.  A matrix
 *   flagged PSK_MAT_CHECKED (accepted by psk_check before) skips this pass.  The stored
 *   values are not part of this check (psk_check tests them on request).
 * - Non-finite input: NaN and infinities propagate through the sums and
 *   products of the stream-ordered calls (IEEE arithmetic) into their
 *   outputs.  The calls that factor a sketch or a Gram matrix return
 *   PSK_ENONFINITE when a pivot of the factorization, a squared row norm
 *   they produce or LSQR's residual estimate is not finite: A or b held a
 *   NaN or an infinity, or a sum overflowed.
 * - Every call returns PSK_OK (0) or a negative psk_status; on an argument
 *   error no work has been enqueued (argument checks happen first).  After
 *   PSK_EDEVICE, PSK_ERANK, PSK_ENONFINITE or PSK_ENOCONV the call's outputs
 *   are unspecified unless its comment says otherwise.  psk_last_error()
 *   gives a message for the calling thread.
 * - Results are deterministic: identical inputs give bit-identical outputs,
 *   independent of other work on the device.  No floating-point atomic
 *   touches global memory; reduction orders across workgroups and K splits
 *   are fixed by the shapes.  Inside one wavefront, CSR kernels add into a
 *   private LDS row (ds_add): the instruction order is fixed, and when
 *   several lanes of one instruction hit the same address (duplicate column
 *   indices, or short rows handled one per lane) the LDS unit applies them
 *   in its fixed lane order, which is repeatable on this hardware but not
 *   an ISA guarantee.
 * - Random quantities are pure functions of (seed, index) through
 *   Philox4x32-10 (Salmon et al., SC'11):
 *     hash of row i:   x = Philox(ctr=(i lo32, i hi32, 0, 0), key=(seed lo32, seed hi32)),
 *                      h(i) = floor((x1*2^32 + x0) * r / 2^64), sigma_i = x2 even ? +1 : -1;
 *     Gaussian G[a,b]: x = Philox(ctr=(q lo32, q hi32, a, 1), key as above), q = b div 4,
 *                      u_k = (x_k + 1/2) 2^-32, Box-Muller on (u0,u1) and (u2,u3) gives
 *                      z0..z3, G[a,b] = z_{b mod 4} / sqrt(m);
 *     JL matrix Pi[b,j] (leverage_sketch): the same with counter word 3 = 2 and
 *                      a = j, Pi[b,j] = z_{b mod 4} / sqrt(t).
 * - Limits: n < 2^31 rows, r < 2^31 buckets, CSR nnz < 2^62.
 */
#ifndef PSK_H
#define PSK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
typedef enum {
  PSK_OK = 0,
  PSK_EINVAL = -1,       /* bad argument (shape, pointer, range, descriptor) */
  PSK_EDTYPE = -2,       /* unsupported dtype / precision combination         */
  PSK_ENOMEM = -3,       /* workspace smaller than psk_workspace_size()       */
  PSK_EDEVICE = -4,      /* a HIP runtime call failed                         */
  PSK_ENOCONV = -5,      /* lsq_solve reached max_iter before its tolerance   */
  PSK_ERANK = -6,        /* sketch numerically rank deficient (R_jj tiny)     */
  PSK_EUNSUPPORTED = -7, /* shape outside the limits documented per call      */
  PSK_ENONFINITE = -8,   /* NaN or infinity in the input or a factorization   */
  PSK_PENDING = 1        /* psk_server_poll: the request has not finished yet */
} psk_status;

/* ---- matrix descriptor ------------------------------------------------- */
enum { PSK_DENSE = 0, PSK_CSR = 1 };   /* psk_mat.format */
enum { PSK_F64 = 0, PSK_F32 = 1 };     /* psk_mat.dtype  */

/* A tall matrix A (n x d).
 * Dense: row-major, element (i,j) at values[i*ld + j], ld >= d.
 * CSR:   0-based; row i holds entries indptr[i] .. indptr[i+1]-1 with column
 *        indices[k] in [0, d) and value values[k].  Columns inside a row may be
 *        in any order.  Duplicate columns inside a row are summed, but then
 *        bit-reproducibility of the affected outputs is not guaranteed.
 *        indptr[0] must be 0, indptr never decreasing, indptr[n] == nnz;
 *        every call checks this and the index range on the device before
 *        use (PSK_EINVAL), unless flags holds PSK_MAT_CHECKED.
 * flags: 0, or PSK_MAT_CHECKED for a CSR matrix that psk_check has accepted
 *        and whose indptr and indices have not changed since: the calls then
 *        skip their own structure check and the stream synchronisation it
 *        needs.  The flag is the caller's promise; a malformed matrix passed
 *        with it is read out of bounds.  Ignored for dense A.  Any other bit,
 *        or a nonzero reserved word, is PSK_EINVAL. */
enum { PSK_MAT_CHECKED = 1 };          /* psk_mat.flags  */
typedef struct psk_mat {
  int32_t format;          /* PSK_DENSE or PSK_CSR              */
  int32_t dtype;           /* PSK_F64 or PSK_F32                */
  int64_t n;               /* rows    (>= 1)                    */
  int64_t d;               /* columns (>= 1)                    */
  int64_t ld;              /* dense: row stride in elements     */
  int64_t nnz;             /* CSR: stored entries               */
  const void *values;      /* dense: >= (n-1)*ld+d elements; CSR: nnz elements */
  const int64_t *indptr;   /* CSR: n+1 row offsets              */
  const int32_t *indices;  /* CSR: nnz column indices           */
  uint32_t flags;          /* 0 or PSK_MAT_CHECKED              */
  uint32_t reserved;       /* 0                                 */
} psk_mat;

/* ---- precision of the Gaussian GEMM of sketch_gcs / lsq_solve ---------- */
enum {
  PSK_PREC_F64 = 0,   /* G and S*A in FP64, FP64 MFMA, FP64 accumulation      *
                       * (S*A of FP32 A is summed in FP64 from the exactly   *
                       * widened entries and used unrounded)                 */
  PSK_PREC_BF16 = 1,  /* G rounded to bfloat16, S*A split into two bfloat16   *
                       * limbs (hi + lo), BF16 MFMA with FP32 accumulation,   *
                       * FP64 reduction of the K-split partial products.      *
                       * Each value of G is the RNE rounding of the FP64      *
                       * normal (drawn in FP32, redrawn in FP64 where the     *
                       * FP32 value lies within 8 ulps of a rounding          *
                       * midpoint); entries of S*A must lie in the bfloat16   *
                       * range.                                               */
  PSK_PREC_FP8 = 2    /* G and S*A quantised to OCP FP8 e4m3 (RNE) with one   *
                       * power-of-two (E8M0) scale per block of 128 buckets:  *
                       * for S*A per column, exponent ceil(log2(amax/448));   *
                       * for G the fixed 2^-6 (every normal of the generator  *
                       * has |z| < 6.77 < 448 * 2^-6), each value the         *
                       * rounding of the FP64 normal as for BF16.  Scaled     *
                       * FP8 MFMA with FP32 accumulation, FP64 reduction of   *
                       * the K-split partial products.  Entries of S*A must   *
                       * stay below 448 * 2^127.                              */
};

/* ---- operations for psk_workspace_size --------------------------------- */
enum {
  PSK_OP_SKETCH_CS = 0,
  PSK_OP_SKETCH_GCS = 1,
  PSK_OP_GRAM = 2,
  PSK_OP_ROWNORMS = 3,
  PSK_OP_QR = 4,
  PSK_OP_LSQ = 5,
  PSK_OP_SKETCH_G = 6,
  PSK_OP_LEVERAGE_GRAM = 7,
  PSK_OP_LSQ_GRAM = 8,
  PSK_OP_LSQ_SKETCH = 9,
  PSK_OP_LEVERAGE_SKETCH = 10,
  PSK_OP_CSS = 11,
  PSK_OP_LEVERAGE_CSS = 12,
  PSK_OP_DELTA = 13,
  PSK_OP_CHECK = 14,
  PSK_OP_SKETCH_OSNAP = 15   /* k = s, the non-zeros per column */
};

/* Library version string (static storage). */
const char *psk_version(void);

/* Message describing the last error returned on the calling thread
 * (thread-local storage, valid until the next psk call on this thread). */
const char *psk_last_error(void);

/* Minimum workspace, in bytes, for one call of `op`.
 *   A    : the matrix the call will get (for PSK_OP_QR and PSK_OP_DELTA only
 *          A->n = m rows and A->d = d columns of the sketch are read);
 *   m, r : Gaussian rows and CountSketch buckets (SKETCH_*, LSQ,
 *          LSQ_SKETCH, LEVERAGE_SKETCH, CSS, LEVERAGE_CSS; SKETCH_G reads m
 *          only);
 *   k    : columns of B (ROWNORMS), columns t of Pi (LEVERAGE_SKETCH),
 *          columns selected (CSS, LEVERAGE_CSS), non-zeros s per column
 *          (SKETCH_OSNAP); for LSQ nonzero when the call will set
 *          opts->want_delta;
 *   prec : PSK_PREC_* (SKETCH_GCS, SKETCH_OSNAP, SKETCH_G, LSQ, LSQ_SKETCH,
 *          LEVERAGE_SKETCH, CSS, LEVERAGE_CSS).
 * For PSK_OP_LSQ, m == 0 sizes a call that passes its own opts->Rinv.
 * Arguments an op does not use are ignored. */
int psk_workspace_size(int op, const psk_mat *A, int64_t m, int64_t r,
                       int64_t k, int prec, size_t *bytes);

/* CountSketch hash of rows row0 .. row0+count-1 (Definition 3 of the paper;
 * the hash and sign are drawn as stated in the header comment).
 *   h    : count int32 buckets in [0, r)          (device, may be NULL)
 *   sign : count int8 signs in {+1, -1}           (device, may be NULL)
 * Errors: PSK_EINVAL if count < 0, row0 < 0, or r < 1 or r >= 2^31. */
int cs_hash(int64_t row0, int64_t count, int64_t r, uint64_t seed,
            int32_t *h, int8_t *sign, void *stream);

/* S*A: the r x d CountSketch of A (Algorithm bcs_multiply).
 *   SA : r x d row-major, leading dimension d, dtype of A (device, written
 *        entirely; rows of empty buckets are zero).
 * Row i of A is added to row h(i) of SA with sign sigma_i; the rows of one
 * bucket are summed in increasing row order in FP64 (FP32 entries widened
 * exactly) and the sum is rounded once to the dtype of A.  Every Gaussian
 * product of this library reads those FP64 sums before any rounding.
 * Errors: PSK_EINVAL (shapes, r < 1, NULL pointers), PSK_EUNSUPPORTED (CSR
 * with d > 20480), PSK_ENOMEM. */
int sketch_cs(const psk_mat *A, int64_t r, uint64_t seed, void *SA,
              void *ws, size_t ws_bytes, void *stream);

/* C = G*(S*A) (Algorithm countgauss_multiply; csrcgs / rmcgs), G the m x r
 * Gaussian matrix with entries of variance 1/m.
 *   m    : rows of G; m == 0 returns S*A as sketch_cs does.
 *   prec : PSK_PREC_F64, PSK_PREC_BF16 or PSK_PREC_FP8 (ignored when m == 0).
 *   C    : m x d row-major FP64 (m > 0), or r x d in the dtype of A (m == 0).
 * G is generated inside the GEMM and never stored.
 * Errors: as sketch_cs, plus PSK_EDTYPE for an unknown prec. */
int sketch_gcs(const psk_mat *A, int64_t m, int64_t r, uint64_t seed,
               int prec, void *C, void *ws, size_t ws_bytes, void *stream);

/* ---- OSNAP with s > 1 non-zeros per column ------------------------------
 * Section 2's introduction: CountSketch is the OSNAP with s = 1, and its
 * data structures and products carry over to any OSNAP.  This library
 * builds the block construction: the r rows of S form s blocks of r/s rows
 * (s must divide r), and column i has one non-zero in each block, so its s
 * non-zeros lie in s distinct rows; each equals sigma / sqrt(s).  Non-zero k
 * of column i (k = 0 .. s-1) is drawn like the CountSketch hash with k in
 * counter word 2:
 *   x = Philox(ctr=(i lo32, i hi32, k, 0), key=(seed lo32, seed hi32)),
 *   row = k (r/s) + floor((x1*2^32 + x0) * (r/s) / 2^64),
 *   sigma = x2 even ? +1 : -1.
 * s = 1 is the CountSketch of cs_hash / sketch_cs / sketch_gcs exactly.  Each
 * column of S has unit norm, so E[S^T S] = I. */

/* Rows and signs of the s non-zeros of columns row0 .. row0+count-1.
 *   h    : count*s int32 rows in [0, r), non-zero k of column row0+i at
 *          h[i*s + k]                                  (device, may be NULL)
 *   sign : count*s int8 signs in {+1, -1}, same layout (device, may be NULL)
 * Errors: PSK_EINVAL if count < 0, row0 < 0, r out of [1, 2^31), s < 1,
 * s > r, r not a multiple of s, or count * s >= 2^40. */
int osnap_hash(int64_t row0, int64_t count, int64_t s, int64_t r, uint64_t seed, int32_t *h,
               int8_t *sign, void *stream);

/* C = G*(S*A) (m > 0) or S*A (m == 0) with the OSNAP S of s non-zeros per
 * column (Algorithms bcs_multiply and countgauss_multiply with this S).  The
 * n*s (row, non-zero) pairs are binned by row of S exactly as sketch_cs bins
 * rows (stable, each row of S lists its columns in increasing order); each
 * row of S*A is the FP64 sum of its signed rows of A in that order times
 * 1/sqrt(s), rounded once to the output type.  G is the same matrix as in
 * sketch_gcs for (m, r, seed), applied to S*A as its FP64 operand in any of
 * the three precisions.
 *   s    : non-zeros per column, 1 <= s <= r, r % s == 0, n*s < 2^32.
 *   C    : m x d row-major FP64 (m > 0), or r x d in the dtype of A (m == 0).
 *   ws   : psk_workspace_size(PSK_OP_SKETCH_OSNAP, A, m, r, s, prec) bytes
 *          (the bins of n*s pairs; for m > 0 also S*A, r x d FP64).
 * s == 1 returns exactly what sketch_gcs returns.
 * Errors: as sketch_gcs, plus PSK_EINVAL for s out of range and
 * PSK_EUNSUPPORTED for n*s >= 2^32. */
int sketch_osnap(const psk_mat *A, int64_t s, int64_t m, int64_t r, uint64_t seed, int prec,
                 void *C, void *ws, size_t ws_bytes, void *stream);

/* C = G*A (section "Gaussian sketching", Algorithm gaussian_sketch; csrjlt),
 * G the m x n Gaussian matrix with entries of variance 1/m.  Column i of G
 * is the column sketch_gcs draws for bucket i (same seed), so sketch_g(A)
 * is sketch_gcs with S the n x n identity.
 *   m    : rows of G (1 <= m < 2^31).
 *   prec : PSK_PREC_F64, PSK_PREC_BF16 or PSK_PREC_FP8: the operand formats
 *          of sketch_gcs with A in the place of S*A (FP8 scale blocks: 128
 *          rows of A per column, 128 columns of G per row).
 *   C    : m x d row-major FP64 (device, written entirely; csrjlt returns
 *          the column-major layout, every result of this library is
 *          row-major).
 * Dense A: the Gaussian GEMM with A as its operand (its rows are copied to
 * a contiguous workspace first when ld > d).  CSR A: the product over the
 * stored entries of A (duplicates summed), 2 nnz(A) m flops, G drawn once.
 * Errors: PSK_EINVAL (shapes, m out of range, NULL pointers), PSK_EDTYPE
 * (prec), PSK_EUNSUPPORTED (CSR with d > 1023 or nnz >= 2^31), PSK_ENOMEM. */
int sketch_g(const psk_mat *A, int64_t m, uint64_t seed, int prec, double *C,
             void *ws, size_t ws_bytes, void *stream);

/* C <- alpha*A^T*A + beta*C (Algorithm gram; csrrk).  C is d x d row-major in
 * the dtype of A, both triangles written.  beta == 0 ignores C's previous
 * contents (NaN-safe).  Products are accumulated in FP64.
 * Errors: PSK_EINVAL, PSK_EUNSUPPORTED (CSR with d > 8192), PSK_ENOMEM. */
int gram(double alpha, const psk_mat *A, double beta, void *C,
         void *ws, size_t ws_bytes, void *stream);

/* x <- alpha*q + beta*x with q_i = ||e_i^T A B||^2 (Algorithm
 * squared_row_norms; csrsqn / rmsqn).
 *   B : d x k row-major FP64 (device).
 *   x : n FP64 (device, in/out; beta == 0 ignores its previous contents).
 * Dense A: fused product-and-norm (A*B is never stored).  CSR A: B*B^T is
 * formed first and the row sums run over pairs of each row's entries.
 * Computation in FP64.
 * Errors: PSK_EINVAL, PSK_EUNSUPPORTED (CSR with d > 8192), PSK_ENOMEM. */
int rownorms_sq(double alpha, const psk_mat *A, const double *B, int64_t k,
                double beta, double *x, void *ws, size_t ws_bytes,
                void *stream);

/* Validity of a matrix operand, as every call checks it and more: for CSR A
 * the structure of the CSR definition (Section 1 notation: indptr[0] == 0,
 * indptr never decreasing, indptr[n] == nnz, 0 <= indices[k] < d); with
 * check_values != 0 also every stored value (CSR) or every element
 * (dense, n x d at stride ld) finite.  One pass over indptr, indices (and
 * values) on `stream`, then a synchronisation to read the result.
 *   ws : psk_workspace_size(PSK_OP_CHECK) bytes (a result word).
 * Returns PSK_OK, PSK_EINVAL (malformed CSR; checked before values),
 * PSK_ENONFINITE (a NaN or an infinity), or as the descriptor checks of the
 * other calls.  Dense A with check_values == 0 returns PSK_OK at once. */
int psk_check(const psk_mat *A, int check_values, void *ws, size_t ws_bytes, void *stream);

/* R and R^{-1} of an FP64 sketch C (m x d row-major, m >= d): C = Q*R with R
 * upper triangular, diag(R) > 0.  Computed by shifted Cholesky-QR (three
 * passes), so Q is never returned.  R and Rinv are d x d row-major FP64
 * (strict lower triangles written as zero).
 * Errors: PSK_EINVAL (m < d, NULL pointers), PSK_EUNSUPPORTED (d > 4096),
 * PSK_ENOMEM.  Rank deficiency is reported by lsq_solve, not here. */
int sketch_qr(const double *C, int64_t m, int64_t d, double *R, double *Rinv,
              void *ws, size_t ws_bytes, void *stream);

/* delta = ||(Chat - C) R^{-1}||_2, the perturbation of a sketch Chat (a
 * reduced-precision one, say) against a sketch C of the same A, with R the
 * triangular factor of C = Q R (sketch_qr).  With Chat R^{-1} = Q + F the
 * singular values of Rhat R^{-1} lie in [1 - delta, 1 + delta], so for
 * delta < 1 the leverage scores of Algorithm ls_approximate_drineas from Chat
 * and from C differ by a factor in [(1 + delta)^-2, (1 - delta)^-2], and the
 * preconditioner of Algorithm least_squares_precondition from Chat keeps
 * cond(A Rhat^{-1}) within (1 + delta) / (1 - delta) of the one from C.
 *   Chat, C : m x d row-major FP64 (device), m >= d, C of full column rank.
 *   delta   : one FP64 (device, written).
 * ||F||_2 is the square root of the largest eigenvalue of F^T F, found by
 * twelve normalised squarings of F^T F and the Rayleigh quotient of the
 * dominant column: never above ||F||_2, and within about (s2/s1)^8192 of it
 * relatively (s1 >= s2 the two largest singular values of F).  The stream
 * is synchronised once (inside sketch_qr).
 * Workspace: psk_workspace_size(PSK_OP_DELTA, A with n = m and d).
 * Errors: PSK_EINVAL (m < d, NULL pointers), PSK_EUNSUPPORTED (d > 4096),
 * PSK_ENOMEM. */
int sketch_delta(const double *Chat, const double *C, int64_t m, int64_t d, double *delta,
                 void *ws, size_t ws_bytes, void *stream);

/* sketch_qr without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops and harnesses
 * that forbid allocation): the same computation and the same results as
 * sketch_qr, with the scratch in a static device array of
 * PSK_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until the
 * process ends (its address is looked up once per device, on the first call
 * there).  Nothing is allocated by the call.  Every call on a GPU uses that
 * GPU's one array: calls that overlap on one GPU (other threads, other
 * streams) race and must be serialised by the caller.  The array keeps the
 * last call's contents; the call sets every part it reads first.
 * Errors: as sketch_qr, plus PSK_EUNSUPPORTED when m x d needs more scratch
 * than PSK_NOALLOC_SCRATCH_BYTES (about 2 m d + 11 d^2 doubles: e.g. m = 2000,
 * d = 500 fits), PSK_EDEVICE if the array's address cannot be found. */
#define PSK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int sketch_qr_noalloc(const double *C, int64_t m, int64_t d, double *R, double *Rinv,
                      void *stream);

/* Options and report of lsq_solve. */
typedef struct psk_lsq_opts {
  const double *Rinv; /* optional d x d row-major FP64 R^{-1} of a   *
                       * sketch of A (device), e.g. from sketch_qr;  *
                       * when non-NULL the sketch and factorization  *
                       * are skipped and m, r, seed, prec ignored    */
  int64_t m;          /* Gaussian rows of the sketch (>= d)          */
  int64_t r;          /* CountSketch buckets (>= m)                  */
  uint64_t seed;
  int32_t prec;       /* PSK_PREC_* of the sketch GEMM               */
  int32_t max_iter;   /* LSQR iteration limit per solve (>= 1)       */
  int32_t refine;     /* refinement passes after the first solve     */
  int32_t check_every;/* iterations between convergence checks (>=1) */
  double atol;        /* stop when ||(AN)^T r|| <= atol*||AN||*||r|| */
  double btol;        /* or when ||r|| <= btol*||b||                  */
  double escalate_cond; /* prec BF16 / FP8: when the factor's        *
                       * diagonal ratio max|R_ii| / min|R_ii| (a    *
                       * lower estimate of cond(A)) exceeds this,    *
                       * the sketch is rebuilt in FP64 from the same *
                       * S*A before LSQR starts; 0 selects 1e4 for   *
                       * BF16 and 10 for FP8, a negative value never *
                       * escalates                                   */
  int32_t want_delta; /* prec BF16 / FP8, own sketch: also form the  *
                       * FP64 sketch of the same S*A and report the  *
                       * reduced sketch's delta (as sketch_delta) in *
                       * info->delta_est; costs an FP64 Gaussian     *
                       * product and two factorizations more         */
  int32_t reserved;
} psk_lsq_opts;

typedef struct psk_lsq_info {
  int32_t iters;      /* LSQR iterations, all passes                 */
  int32_t status;     /* PSK_OK or PSK_ENOCONV                        */
  double resid;       /* ||b - A x|| estimate from the recurrences   */
  double ne_resid;    /* ||(AN)^T r|| / (||AN||_F ||r||) estimate    */
  int32_t prec_used;  /* PSK_PREC_* of the sketch the preconditioner *
                       * came from (-1 with a caller's Rinv)          */
  int32_t reserved;
  double delta_est;   /* delta = ||(Chat - C) R^{-1}||_2 of the sketch *
                       * LSQR was preconditioned with against the FP64 *
                       * sketch (sketch_delta): 0 when that is the     *
                       * FP64 sketch (prec F64, or escalated), the     *
                       * measured value with want_delta, else NaN      */
} psk_lsq_info;

/* x = argmin ||A x - b|| by sketch-and-precondition (Algorithm
 * least_squares_precondition): C = G*S*A, R from sketch_qr(C), LSQR on the
 * operator A*R^{-1} (Paige & Saunders 1982) in FP64, x = R^{-1} y, then
 * `refine` passes that solve for the residual and add the correction.
 *   b : n FP64 (device);  x : d FP64 (device, output).
 * The call enqueues LSQR iterations in groups of check_every; each group's
 * convergence flag is copied to pinned host memory (a few pinned bytes per
 * concurrent solve, kept for the life of the process) and read while the
 * next group runs.  The call returns with the stream idle.
 * Errors: PSK_EINVAL, PSK_ENOMEM, PSK_ENOCONV (x still written), PSK_ERANK,
 * PSK_ENONFINITE (a pivot of the sketch's factorization, or LSQR's norms
 * read at a convergence test, not finite). */
int lsq_solve(const psk_mat *A, const double *b, double *x,
              const psk_lsq_opts *opts, psk_lsq_info *info,
              void *ws, size_t ws_bytes, void *stream);

/* theta_i ~ leverage score of row i (Algorithm ls_approximate_drineas):
 *   1. the sketch: S A (m == 0, the algorithm as stated; r >= d) or G S A
 *      (m > 0; d <= m < 2^31), as sketch_cs / sketch_gcs with this seed and,
 *      for m > 0, prec;
 *   2. R and R^{-1} of the sketch (sketch_qr; the triangular factor stands in
 *      for the paper's SVD: A R^{-1} and A V Sigma^{-1} differ by an
 *      orthogonal factor, so their row norms agree);
 *   3. t > 0: X = R^{-1} Pi with Pi the d x t Gaussian of variance 1/t drawn
 *      as stated in the header comment (row norms kept to within 1 +- eps
 *      for t = O(log n / eps^2); the dense row-norm product costs n d t
 *      multiply-adds instead of n d^2); t == 0: X = R^{-1};
 *   4. theta_i = ||e_i^T A X||^2 (rownorms_sq).
 * An FP32 S A (m == 0) is widened to FP64 before the factorization.
 *   theta : n FP64 (device, written).
 * The call synchronises the stream once, to read the factorization's pivot
 * flag.  Workspace: psk_workspace_size(PSK_OP_LEVERAGE_SKETCH, A, m, r, t,
 * prec); it holds the sketch and two copies of it for the QR passes.
 * Errors: PSK_EINVAL (shapes, m, r out of range, t < 0 or d * t >= 2^31,
 * NULL theta), PSK_EDTYPE
 * (prec, when m > 0), PSK_EUNSUPPORTED (d > 4096; as sketch_cs), PSK_ENOMEM,
 * PSK_ERANK (a Cholesky pivot of the factorization was not positive; theta
 * is still written), PSK_ENONFINITE (a pivot or a score not finite). */
int leverage_sketch(const psk_mat *A, int64_t m, int64_t r, int64_t t, uint64_t seed, int prec,
                    double *theta, void *ws, size_t ws_bytes, void *stream);

/* ---- column subset selection (section 4.1) -------------------------------
 * The sketch B is G S A (m > 0, d <= m < 2^31) or S A (m == 0, r >= d), as
 * sketch_gcs with this seed and prec (an FP32 S A is widened to FP64), and
 * 1 <= k <= d <= 4096.  The pivoted QR is the column-pivoted Householder QR
 * of Businger and Golub (as LAPACK geqp3): step j takes the remaining column
 * of B whose rows j .. end have the largest norm (lowest index on equal
 * norms; norms recomputed exactly at each step), and a Householder reflector
 * zeroes that column below row j in every remaining column.  One kernel
 * launch per step; B is copied to a column-major workspace first. */

/* cols[0..k) = the first k pivots of the pivoted QR of B, in order (Algorithm
 * cgrrqr: the "top-k" columns of A).
 *   cols : k int32 (device, written).
 * The sketch is checked for NaN and infinities first (one synchronisation).
 * Errors: PSK_EINVAL (shapes, k out of range, NULL cols), PSK_EDTYPE (prec,
 * when m > 0), PSK_EUNSUPPORTED (d > 4096; as sketch_cs), PSK_ENOMEM,
 * PSK_ENONFINITE (the sketch not finite; no pivot chosen). */
int css_select(const psk_mat *A, int64_t m, int64_t r, int64_t k, uint64_t seed, int prec,
               int32_t *cols, void *ws, size_t ws_bytes, void *stream);

/* theta_i = leverage score of row i of A[:, K], K = css_select(A, m, r, k,
 * seed, prec) (Algorithm ls_hrn_exact; exact for A when k = rank(A) = d):
 * the K x K block of the FP64 Gram matrix A^T A, its Cholesky factor R_K, and
 * theta_i = ||e_i^T A B||^2 with B (d x k) holding R_K^{-1} at the rows K.
 *   theta : n FP64 (device, written);  cols : k int32 (device, written) or
 *   NULL.
 * The call synchronises the stream once, to read the pivot flag.
 * Errors: as css_select, plus PSK_ERANK (A[:, K] numerically rank deficient;
 * theta still written), PSK_ENONFINITE (a pivot or a score not finite). */
int leverage_css(const psk_mat *A, int64_t m, int64_t r, int64_t k, uint64_t seed, int prec,
                 double *theta, int32_t *cols, void *ws, size_t ws_bytes, void *stream);

/* ---- direct solvers and exact leverage scores ---------------------------
 * Section 4's Gram-based and sketch-and-solve algorithms.  A triangular
 * factor stands in for the paper's SVD (A R^{-1} spans the column space of
 * A V Sigma^{-1} with orthonormal columns, so leverage scores and
 * least-squares solutions are the same); full column rank is assumed and a
 * Cholesky pivot that is not positive returns PSK_ERANK (the outputs are
 * still written).  These calls synchronise the stream once, to read that
 * pivot flag.  d <= 4096. */

/* theta_i = ||e_i^T A B^{-1/2}||^2, B = A^T A (Algorithm ls_direct): the
 * exact leverage scores of A, from the FP64 Gram matrix, its Cholesky factor
 * R and rownorms_sq(A, R^{-1}).  B squares the condition number: the scores
 * carry an error of about cond(A)^2 u.
 *   theta : n FP64 (device, written).
 * Errors: PSK_EINVAL, PSK_EUNSUPPORTED (d > 4096), PSK_ENOMEM, PSK_ERANK,
 * PSK_ENONFINITE (a pivot or a score not finite). */
int leverage_gram(const psk_mat *A, double *theta, void *ws, size_t ws_bytes, void *stream);

/* x = argmin ||A x - b|| = B^{-1} A^T b, B = A^T A (Algorithm
 * least_squares_gram): Cholesky B = R^T R, c = A^T b (row-block partials in
 * a fixed order), x = R^{-1} R^{-T} c.  Accurate to about cond(A)^2 u.
 *   b : n FP64 (device);  x : d FP64 (device, written).
 * Errors: PSK_EINVAL, PSK_EUNSUPPORTED (d > 4096), PSK_ENOMEM, PSK_ERANK,
 * PSK_ENONFINITE (a pivot or an entry of x not finite). */
int lsq_gram(const psk_mat *A, const double *b, double *x, void *ws, size_t ws_bytes,
             void *stream);

/* x = argmin ||G S A x - G S b|| (Algorithm least_squares_approx,
 * sketch-and-solve): the sketches of A and of b with the same seed (so the
 * same S and G), R from sketch_qr of A~ = G S A, and the corrected
 * semi-normal equations x = R^{-1} R^{-T} A~^T b~ plus one correction from
 * the residual b~ - A~ x.  The solution of the sketched problem, so an
 * approximation of the least-squares solution (its residual is within a
 * factor of about 1 + d / (m - d) of the optimum in expectation).
 *   m, r, seed, prec : as for sketch_gcs (d <= m <= 2^31 - 1, r >= 1).
 *   b : n FP64 (device);  x : d FP64 (device, written).
 * Errors: PSK_EINVAL (shapes, m < d), PSK_EDTYPE (prec), PSK_EUNSUPPORTED,
 * PSK_ENOMEM, PSK_ERANK, PSK_ENONFINITE (a pivot or an entry of x not
 * finite). */
int lsq_sketch_solve(const psk_mat *A, const double *b, double *x, int64_t m, int64_t r,
                     uint64_t seed, int prec, void *ws, size_t ws_bytes, void *stream);

/* ---- ceiling probes ------------------------------------------------------
 * Measurement kernels, not part of the method: they give the rates this
 * device sustains for the resources the path's kernels are bound by, so a
 * kernel's roofline fraction can be stated against the measured ceiling as
 * well as the datasheet peak.  Each call enqueues one kernel on `stream`;
 * the caller times it (e.g. with events on that stream). */
#define PSK_PROBE_BLOCKS 4096 /* workgroups (of 256 threads) of the arithmetic probes */

/* dst <- src, a grid-stride copy of 16-byte words (HBM: `bytes` read and
 * `bytes` written).  bytes > 0, a multiple of 16; src, dst 16-byte aligned
 * device pointers, not overlapping.  Errors: PSK_EINVAL. */
int psk_probe_copy(const void *src, void *dst, size_t bytes, void *stream);

/* iters x 8 v_mfma_f64_16x16x4f64 per wavefront on 8 independent register
 * accumulators: PSK_PROBE_BLOCKS * 4 * iters * 8 * 2048 FP64 flops.
 *   out : PSK_PROBE_BLOCKS * 256 doubles (device), one value per thread.
 * Errors: PSK_EINVAL (iters < 1, NULL out). */
int psk_probe_mfma_f64(int64_t iters, double *out, void *stream);

/* fmt PSK_PREC_BF16: iters x 8 v_mfma_f32_16x16x32_bf16 per wavefront
 * (PSK_PROBE_BLOCKS * 4 * iters * 8 * 16384 flops); PSK_PREC_FP8: iters x 8
 * v_mfma_scale_f32_16x16x128_f8f6f4 on e4m3 operands with unit scales
 * (PSK_PROBE_BLOCKS * 4 * iters * 8 * 65536 flops); FP32 accumulation.
 *   out : PSK_PROBE_BLOCKS * 256 floats (device).
 * Errors: PSK_EINVAL (iters < 1, NULL out), PSK_EDTYPE (fmt). */
int psk_probe_mfma_lowp(int fmt, int64_t iters, float *out, void *stream);

/* iters x 8 independent v_fma_f32 per lane: PSK_PROBE_BLOCKS * 256 * iters
 * * 8 VALU lane-operations.
 *   out : PSK_PROBE_BLOCKS * 256 floats (device), one value per thread.
 * Errors: PSK_EINVAL (iters < 1, NULL out). */
int psk_probe_valu_f32(int64_t iters, float *out, void *stream);

/* ---- request server (serving form) ---------------------------------------
 * Continuous batching of least-squares and leverage-score requests of
 * uneven n and d on one GPU.  `slots` host worker threads, each with its own
 * HIP stream (default priority), take requests in arrival order; a request
 * is admitted when a slot is free and its whole workspace fits in the
 * caller's device pool, which the server carves with a first-fit allocator,
 * so the workspace footprint of the requests in flight never exceeds
 * pool_bytes.  Admission is strictly first-in first-out.  Requests on
 * different slots run concurrently on the device; each request's result is
 * the same bit for bit as when it runs alone (its kernels read only its own
 * inputs and workspace).
 *
 * Requests:
 *   PSK_REQ_LSQ       x = argmin ||A x - b|| exactly as lsq_solve with
 *                     `opts` (out: x, d doubles);
 *   PSK_REQ_LEVERAGE  sketched leverage scores theta_i = ||e_i^T A R^{-1}||^2
 *                     with R from sketch_qr(sketch_gcs(A, opts.m, opts.r,
 *                     opts.seed, opts.prec)) (Algorithm
 *                     ls_approximate_drineas with QR; out: theta, n doubles).
 * A, b and out are device pointers owned by the caller and must stay valid
 * and unmodified until the request has completed (psk_server_wait or a
 * psk_server_poll that returns PSK_OK).  Times are seconds of a monotonic
 * host clock.  The server object is thread-safe. */
typedef struct psk_server psk_server;

typedef struct psk_server_opts {
  void *pool;          /* device memory for request workspaces, 256-byte  *
                        * aligned, owned by the caller, untouched by the   *
                        * caller while the server exists                   */
  size_t pool_bytes;
  int32_t slots;       /* requests on the device at once, 1 .. 64          */
} psk_server_opts;

enum { PSK_REQ_LSQ = 0, PSK_REQ_LEVERAGE = 1 };

typedef struct psk_request {
  int32_t op;          /* PSK_REQ_*                                         */
  psk_mat A;
  const double *b;     /* LSQ: n doubles (device)                           */
  double *out;         /* LSQ: x (d); LEVERAGE: theta (n) (device)           */
  psk_lsq_opts opts;   /* LSQ: as lsq_solve; LEVERAGE: m, r, seed, prec     */
} psk_request;

typedef struct psk_result {
  int32_t status;      /* PSK_OK or the status lsq_solve would return       */
  int32_t iters;       /* LSQ: LSQR iterations                              */
  double resid;        /* LSQ: as psk_lsq_info                              */
  double ne_resid;
  double t_submit;     /* submit, admission and completion times (s)        */
  double t_start;
  double t_end;
  int32_t prec_used;   /* LSQ: as psk_lsq_info; LEVERAGE: opts.prec         */
  int32_t reserved;
  double delta_est;    /* LSQ: as psk_lsq_info (opts.want_delta); LEVERAGE: *
                        * NaN                                                */
} psk_result;

typedef struct psk_server_stats_t {
  int64_t submitted, completed, queued;
  int32_t inflight, inflight_peak;   /* requests on the device (now, max)  */
  size_t pool_bytes, pool_used, pool_peak;
} psk_server_stats_t;

/* Create a server on the current HIP device.
 * Errors: PSK_EINVAL (slots, pool), PSK_EDEVICE. */
int psk_server_create(const psk_server_opts *opts, psk_server **server);
/* Queue a request (returns at once) and give it a ticket.
 * Errors: as lsq_solve's argument checks; PSK_ENOMEM if the request's
 * workspace is larger than the whole pool. */
int psk_server_submit(psk_server *server, const psk_request *req, int64_t *ticket);
/* Block until the request has finished; fills `result` and forgets the
 * ticket.  The request's own failure is reported in result->status. */
int psk_server_wait(psk_server *server, int64_t ticket, psk_result *result);
/* PSK_OK with `result` filled (ticket forgotten) if finished, PSK_PENDING if
 * not. */
int psk_server_poll(psk_server *server, int64_t ticket, psk_result *result);
int psk_server_stats(psk_server *server, psk_server_stats_t *stats);
/* Finish every queued request, stop the workers, destroy the streams. */
int psk_server_destroy(psk_server *server);

/* ---- kernel timing (diagnostics) ----------------------------------------
 * When enabled, the library brackets its main kernels (and a few multi-kernel
 * regions) with HIP events recorded on the stream each one is launched on.
 * Names: "check" (CSR structure / value check), "cs_bin" (hash + radix
 * binning region), "cs_scatter" (S*A), "gauss_gemm" (Gaussian GEMM kernel,
 * dense or sparse form), "gemm_reduce" (its K-split sum), "g_draw" (the FP8
 * codes of G), "sa_entries" / "sa_limbs" / "sa_quant" (the nonzeros of S*A
 * for the sparse product, in FP64, BF16 limbs or FP8), "cs_scatter_limbs" /
 * "cs_scatter_quant" (S*A of CSR A straight into BF16 limbs / FP8 codes),
 * "gram" (Gram kernel), "gram_reduce" (its slab sums), "rownorm" (row-norm
 * kernel), "sketch_qr" (whole factorization region), "sketch_delta" (the
 * perturbation estimate), "jl_normals" (the JL matrix), "qrcp" (column-
 * pivoted QR of css_select), "lsqr_pass" (one LSQR pass over A).
 * psk_timing_collect waits for the recorded events and returns the summed
 * elapsed milliseconds and launch count of one name (0 and 0 if unseen).
 * psk_timing_names lists the names seen so far, comma separated (static
 * storage, valid until the next timing call).  Not thread-safe against
 * concurrent psk calls that record events. */
int psk_timing_enable(int on);
/* Record only the brackets named in `names` (comma separated, e.g.
 * "gauss_gemm"); NULL or "" records all of them again.  Each bracket costs
 * two event creations and records on the host, so timing a whole pipeline
 * slows its host side; a filter keeps the overhead to the kernels that are
 * being measured. */
int psk_timing_only(const char *names);
int psk_timing_reset(void);
int psk_timing_collect(const char *name, double *total_ms, int64_t *launches);
const char *psk_timing_names(void);

#ifdef __cplusplus
}
#endif
#endif /* PSK_H */
