/*
 * rtri.h -- C ABI of the recursive triangular multiply / solve library for
 * AMD Instinct MI355X (gfx950).
 *
 * Operations (paper, Sec. 2.1):
 *   TRMM  eq. (1)  B := alpha * op(A) * B          side = RTRI_LEFT
 *         eq. (2)  B := alpha * B * op(A)          side = RTRI_RIGHT
 *   TRSM  eq. (3)  solve op(A) * X = alpha * B     side = RTRI_LEFT,  X overwrites B
 *         eq. (4)  solve X * op(A) = alpha * B     side = RTRI_RIGHT, X overwrites B
 *   op(A) = A, A^T or conj(A^T); for real data RTRI_CONJTRANS means A^T.
 *
 * Method (paper, Sec. 3.1-3.2): A is split at its midpoint into two triangular
 * diagonal blocks and one off-diagonal block; the call recurses on the two
 * diagonal blocks and applies the off-diagonal block as one GEMM update per
 * level, until a block is at most the leaf size, where a leaf kernel solves or
 * multiplies the diagonal block directly (Sec. 3.3).
 *
 * Conventions shared by every entry point
 *   - Column-major storage: element (i, j) of a matrix X with leading
 *     dimension ldx is X[i + j * ldx].
 *   - For side = LEFT, A is m-by-m; for side = RIGHT, A is n-by-n; B is m-by-n.
 *   - Only the triangle named by uplo is read.  With diag = RTRI_UNIT the
 *     diagonal of A is not read either (taken as 1).
 *   - A and B are DEVICE pointers, owned by the caller; the library never
 *     frees them.  A and B must not overlap.
 *   - Calls are asynchronous on the handle's stream: they return once the work
 *     is enqueued.  Argument errors are reported synchronously and leave B
 *     untouched.  Device-side errors surface as RTRI_ERR_HIP on a later call or
 *     on rtri_sync.
 *   - Quick return: m == 0 or n == 0 does nothing.  alpha == 0 sets B := 0
 *     without reading A (BLAS semantics).
 *   - A singular A (a zero diagonal entry with diag = NONUNIT) is not detected;
 *     IEEE infinities / NaNs propagate into B, as in the reference BLAS.
 *
 * Return codes
 *   0                 success
 *   -i (i = 1..12)    argument i of the BLAS-style argument list is invalid:
 *                     1 side, 2 uplo, 3 trans, 4 diag, 5 m < 0, 6 n < 0,
 *                     8 A == NULL, 9 lda < max(1, ka), 10 B == NULL,
 *                     11 ldb < max(1, m)   (ka = m for LEFT, n for RIGHT)
 *   RTRI_ERR_HANDLE   NULL or destroyed handle
 *   RTRI_ERR_HIP      a HIP runtime call failed (rtri_last_hip_error gives it)
 *   RTRI_ERR_NOMEM    device workspace could not be allocated
 *   RTRI_ERR_UNSUPPORTED  option or type combination not supported
 *   RTRI_ERR_TOO_LARGE    the problem does not fit the fixed scratch of
 *                         rtri_dtrsm_noalloc
 */
#ifndef RTRI_H
#define RTRI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { RTRI_LEFT = 0, RTRI_RIGHT = 1 };
enum { RTRI_LOWER = 0, RTRI_UPPER = 1 };
enum { RTRI_NOTRANS = 0, RTRI_TRANS = 1, RTRI_CONJTRANS = 2 };
enum { RTRI_NONUNIT = 0, RTRI_UNIT = 1 };
enum { RTRI_F64 = 0, RTRI_F32 = 1, RTRI_BF16 = 2, RTRI_F16 = 3,
       RTRI_I8 = 4 /* profile records only: the INT8 matrix-core product of rtri_dtrmm_ozaki */ };

enum {
    RTRI_OK = 0,
    RTRI_ERR_HANDLE = 1,
    RTRI_ERR_HIP = 2,
    RTRI_ERR_NOMEM = 3,
    RTRI_ERR_UNSUPPORTED = 4,
    RTRI_NOT_CONVERGED = 5,
    RTRI_ERR_INVALID = 6,
    RTRI_ERR_TOO_LARGE = 7
};

/* Tunable options (rtri_set_option / rtri_get_option). */
enum {
    RTRI_OPT_LEAF_F64 = 1,   /* leaf size for FP64 (16, 32, 64, 128 or 256; 0 = automatic).
                                16 and 32: substitution leaves; 64 and up: matrix-core leaves
                                that apply FP64 inverses of their 16 x 16 diagonal tiles */
    RTRI_OPT_LEAF_F32 = 2,   /* leaf size for FP32 (same values) */
    RTRI_OPT_GEMM_TILE = 3,  /* GEMM tile choice: 0 = automatic, 1 = 128x128 (4 wavefronts), 2 = 64x64,
                                3 = 128x128 (8 wavefronts) */
    RTRI_OPT_TRMM_LEAVES = 4, /* TRMM leaf schedule (leaves of 64 rows and more): 0 = automatic (all in one
                                launch below 8192 vectors, and always for rtri_trmm_ex), 1 = one launch per
                                leaf, in recursion order, each GEMM update its own launch, 2 = the panel is
                                copied to workspace (rtri_trmm_ex reads its 16-bit original instead), all
                                leaves run in one launch, then all GEMM updates in one grouped launch that
                                reads the copy (a workgroup owns a tile of the panel and applies its updates
                                deepest first).  The two agree bit for bit where they use the same tiles (FP64
                                / FP32 updates that do not split K); otherwise to within rounding. */
    RTRI_OPT_GEMM16_TILE = 5, /* 16-bit GEMM tiles: 0 = automatic, 1 = 128x128 (4 wavefronts, 16x16x32 MFMA),
                                2 = 256x256 (8 wavefronts, 32x32x16 MFMA) wherever both operands are
                                k-contiguous and 16-byte aligned (else 128x128), with both operands 16-bit,
                                M and N multiples of 256 and K of 32 loaded straight into LDS; 3 = the
                                256x256 tiles with register-staged loads only (bit for bit the results of 2).
                                Results may differ in the last bits between 1 and 2 (another accumulation
                                order). */
    RTRI_OPT_RESIDUAL = 6     /* residual product of the refined solves (rtri_dtrsm_mixed, factor solves):
                                0 = FP64 matrix cores (the FP64 recursive TRMM), 1 = exact INT8 products
                                (the method of rtri_dtrmm_ozaki; op(A)'s residue planes made once per call,
                                or kept by a factor) */
};

typedef struct rtri_handle rtri_handle;

/* Create a handle bound to a HIP stream (a hipStream_t passed as void*; NULL =
 * the null stream) on the current device.  *h receives the handle. */
int rtri_create(rtri_handle **h, void *hip_stream);

/* Release a handle and any device workspace it owns.  Waits for no work:
 * synchronise first if work using the handle may still be running. */
int rtri_destroy(rtri_handle *h);

/* Re-bind the handle to another stream (hipStream_t as void*). */
int rtri_set_stream(rtri_handle *h, void *hip_stream);

/* Block the host until all work enqueued through the handle has finished;
 * returns RTRI_ERR_HIP if any of it failed. */
int rtri_sync(rtri_handle *h);

/* Set / read a tunable option (RTRI_OPT_*).  Invalid values return -3. */
int rtri_set_option(rtri_handle *h, int option, int64_t value);
int rtri_get_option(rtri_handle *h, int option, int64_t *value);

/* Static description of a return code. */
const char *rtri_status_string(int status);

/* The hipError_t value behind the last RTRI_ERR_HIP returned on this handle. */
int rtri_last_hip_error(rtri_handle *h);

/* Triangular solve, eqs. (3)/(4): B := X with op(A) X = alpha B (LEFT) or
 * X op(A) = alpha B (RIGHT).  FP64 / FP32. */
int rtri_dtrsm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
               double alpha, const double *A, int64_t lda, double *B, int64_t ldb);
int rtri_strsm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
               float alpha, const float *A, int64_t lda, float *B, int64_t ldb);

/* Triangular multiply, eqs. (1)/(2): B := alpha op(A) B (LEFT) or
 * B := alpha B op(A) (RIGHT), in place.  FP64 / FP32.
 * Workspace of both (owned by the handle, grown on demand, freed by
 * rtri_destroy): the packed diagonal blocks; for a TRMM whose leaves run in one
 * launch, a copy of B (m x n); for factor orders above 1536 whose updates are
 * short of tiles (narrow panels), 80 MiB of split-K partial products. */
int rtri_dtrmm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
               double alpha, const double *A, int64_t lda, double *B, int64_t ldb);
int rtri_strmm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
               float alpha, const float *A, int64_t lda, float *B, int64_t ldb);

/* Complex (FP64 complex, interleaved real / imaginary parts) TRSM and TRMM,
 * eqs. (1)-(4) with op(A) = A (RTRI_NOTRANS), A^T (RTRI_TRANS) or conj(A^T)
 * (RTRI_CONJTRANS).  A and B hold complex elements (two doubles each); lda,
 * ldb count complex elements.  alpha points to two doubles (real,
 * imaginary) in host memory.  The same recursion as the real calls: its GEMM
 * updates run on the real FP64 matrix cores through the real 2x2-block
 * embedding of op(A) (a + bi -> [a -b; b a]), made once per call in the
 * handle's workspace (4 ka^2 doubles); leaves of at most 64 rows work in
 * complex arithmetic (division by Smith's method).  alpha multiplies B first
 * (alpha = 0: B := 0, A not read).  Side R is computed as side L on the
 * transpose of B (a copy in the workspace).  Codes as rtri_dtrsm, and -7 for
 * alpha == NULL. */
int rtri_ztrsm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, const double *alpha,
               const void *A, int64_t lda, void *B, int64_t ldb);
int rtri_ztrmm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, const double *alpha,
               const void *A, int64_t lda, void *B, int64_t ldb);

/* ---- call plans: one TRSM / TRMM planned once, replayed as a HIP graph ----- */

/* Plan one FP64 / FP32 TRSM (op 0, eqs. (3)/(4)) or TRMM (op 1, eqs. (1)/(2))
 * on fixed operands: the recursion is planned once and every kernel of the
 * call (pack pass, leaves, GEMM updates) is captured in a HIP graph with
 * workspace the plan owns (packed blocks and one split-K region), so a replay
 * (rtri_call_plan_run) is one graph launch on the handle's current stream,
 * with no host planning and no allocation.  Each replay computes what the
 * plain call (rtri_dtrsm ...) computes with the handle's options at creation
 * (a TRMM: with RTRI_OPT_TRMM_LEAVES = 1, the schedule a plan captures), bit
 * for bit, reading A and the current contents of B.  The handle must not have
 * a profile open.
 * Argument codes: -2 op, -3 dtype, then the codes of rtri_dtrsm shifted by
 * three (-4 side ... -14 ldb), -15 out NULL.  Blocking (captures and
 * instantiates the graph). */
typedef struct rtri_call_plan rtri_call_plan;
int rtri_call_plan_create(rtri_handle *h, int op, int dtype, int side, int uplo, int trans, int diag, int64_t m,
                          int64_t n, double alpha, const void *A, int64_t lda, void *B, int64_t ldb,
                          rtri_call_plan **plan);
/* Replay (asynchronous on the handle's stream). */
int rtri_call_plan_run(rtri_call_plan *plan);
/* Free a plan (waits for the handle's stream first). */
int rtri_call_plan_destroy(rtri_call_plan *plan);

/* FP64 TRMM from exact INT8 matrix-core products (the refined solve's residual
 * product, available on its own): B := alpha op(A) B (LEFT) or alpha B op(A)
 * (RIGHT), eqs. (1)/(2), in place, FP64-accurate.  Method: the modular form
 * of the Ozaki scheme.  Each line of op(A) and of B (rows of the left
 * operand, columns of the right one) is scaled by a power of two and rounded
 * to an integer of at most beta bits, beta = min(55, floor((125.19 - 2 -
 * log2 K) / 2)) for the order K (55 up to K = 8192, 54 up to 16384); the
 * exact integer product is formed from its residues modulo 16 pairwise
 * coprime moduli <= 256, each residue one INT8 GEMM with exact INT32
 * accumulation over op(A)'s triangle, and recovered by the Chinese remainder
 * theorem (Garner's algorithm, 128-bit integer evaluation, one rounding).
 * Error per entry: at most |alpha| (2^(e_i-beta-1) ||right_j||_1 +
 * 2^(f_j-beta-1) ||left_i||_1 + K 2^(e_i+f_j-2 beta-2)) plus two roundings,
 * where 2^e_i, 2^f_j bound the largest magnitude of row i of the left and
 * column j of the right operand; exact when the scaled entries are integers
 * and the result is representable.  Workspace (handle-owned, grown on
 * demand): 16 (ka' k' + n' k' + m' n') bytes (' = rounded up to 256 lines /
 * 128 entries).  Codes as rtri_dtrmm, and RTRI_ERR_UNSUPPORTED for an order
 * of 131072 or more. */
int rtri_dtrmm_ozaki(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                     double alpha, const double *A, int64_t lda, double *B, int64_t ldb);

/* FP64 TRSM that allocates nothing, for callers that cannot call hipMalloc
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, codes and results as rtri_dtrsm (bit for bit,
 * with the same handle options); the handle must have been created outside
 * such a region (rtri_create allocates no device memory).
 * Its workspace (the packed diagonal blocks and one region of split-K partial
 * products) is a fixed array of RTRI_NOALLOC_SCRATCH_MIB MiB of device memory
 * defined by the library: each GPU the library runs on holds one copy, from
 * the first rtri_create (or call) on that device until the process ends.  No
 * memory is allocated by the call, and nothing in the array needs clearing.
 * Limits and rules:
 *   - the packed blocks must fit 32 MiB (plan size: ka/leaf blocks of
 *     128 (leaf/16)(leaf/16 + 1) doubles, e.g. ka <= 29000 with 256-row
 *     leaves); larger problems return RTRI_ERR_TOO_LARGE without touching B;
 *   - calls that overlap in time on one GPU (on different streams or
 *     handles) share the array and race: serialise them;
 *   - a handle with an open profile returns RTRI_ERR_UNSUPPORTED. */
#define RTRI_NOALLOC_SCRATCH_MIB 48
int rtri_dtrsm_noalloc(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                       double alpha, const double *A, int64_t lda, double *B, int64_t ldb);

/* Per-kernel profile: while a profile is open, every kernel the handle
 * launches is bracketed by two HIP events recorded on the handle's stream, and
 * its algorithmic work is attributed to a kernel class.  rtri_profile_end waits
 * for the stream, fills out[] with one entry per class that ran (at most
 * max_out entries), sets *n_out, and closes the profile.
 *   flops: GEMM 2*M*N*K; leaf nb*nb*nvec (multiply-adds counted twice)
 *   bytes: the minimum HBM traffic of the launch (each operand read once,
 *          the output read and written once) */
enum {
    RTRI_KCLASS_GEMM = 0,        /* GEMM update (Sec. 3.1) */
    RTRI_KCLASS_LEAF_SOLVE = 1,  /* leaf triangular solve (Sec. 3.3) */
    RTRI_KCLASS_LEAF_MULT = 2,   /* leaf triangular multiply */
    RTRI_KCLASS_OTHER = 3,       /* fills, conversions, norms */
    RTRI_KCLASS_BATCHED = 4      /* one launch of a batch plan (flops: sum of ka^2 * vectors) */
};
typedef struct {
    int kclass;       /* RTRI_KCLASS_* */
    int dtype;        /* RTRI_F64 / RTRI_F32 / RTRI_BF16 / RTRI_F16: element type of the inputs */
    int64_t launches;
    double ms;        /* summed event-to-event duration of the launches */
    double flops;     /* summed algorithmic flops */
    double bytes;     /* summed algorithmic bytes */
} rtri_kernel_stat;
int rtri_profile_begin(rtri_handle *h);
int rtri_profile_end(rtri_handle *h, rtri_kernel_stat *out, int max_out, int *n_out);

/* The GEMM update of one recursion level (Sec. 3.1), callable on its own:
 *     C := beta * C + s * op(P) * op(Q),   op(P) M-by-K, op(Q) K-by-N, C M-by-N
 * op(P) = P (trans_p = RTRI_NOTRANS) or P^T (RTRI_TRANS); likewise op(Q).
 * dtype is RTRI_F64 or RTRI_F32 (all of P, Q, C; alpha-like scalars passed as
 * double and rounded to the element type), or RTRI_BF16 / RTRI_F16 (P and Q
 * 16-bit, C FP32, FP32 accumulation: the matrix-core tiles of the 16-bit and
 * mixed-precision paths, RTRI_OPT_GEMM16_TILE).  beta == 0 writes C without reading
 * it.  Device pointers; C must not overlap P or Q.  Asynchronous on the
 * handle's stream.
 * Argument codes: -2 dtype, -3 trans_p, -4 trans_q, -5 M < 0, -6 N < 0,
 * -7 K < 0, -9 P NULL, -10 ldp < max(1, rows of P), -11 Q NULL,
 * -12 ldq < max(1, rows of Q), -14 C NULL, -15 ldc < max(1, M). */
int rtri_gemm_update(rtri_handle *h, int dtype, int trans_p, int trans_q, int64_t M, int64_t N, int64_t K,
                     double s, const void *P, int64_t ldp, const void *Q, int64_t ldq, double beta, void *C,
                     int64_t ldc);

/* Triangular multiply with 16-bit inputs and FP32 accumulation, out of place
 * (eqs. (1)/(2) with the result in a separate matrix):
 *     C := alpha * op(A) * B   (LEFT)    or    C := alpha * B * op(A)   (RIGHT)
 * A and B are BF16 or FP16 (a_type == b_type, RTRI_BF16 or RTRI_F16); C is
 * FP32 (c_type == RTRI_F32), m-by-n with leading dimension ldc.  Every product
 * of two 16-bit values is exact in FP32 and the sums accumulate in FP32, so the
 * result is the FP32-accumulated product of the 16-bit inputs.  C must not
 * overlap A or B; A and B are not modified.  For side LEFT with trans N (or
 * RIGHT with trans T) the handle's workspace grows to hold a transposed copy
 * of A (order x ceil8(order) 16-bit elements), kept until rtri_destroy.
 * Argument codes: -1..-6 as for rtri_dtrmm, -8 A NULL, -9 lda, -10 B NULL,
 * -11 ldb < max(1, m), -12 C NULL, -13 ldc < max(1, m); RTRI_ERR_UNSUPPORTED
 * for any other type combination. */
int rtri_trmm_ex(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, float alpha,
                 const void *A, int a_type, int64_t lda, const void *B, int b_type, int64_t ldb, void *C,
                 int c_type, int64_t ldc);

/* Progress of a mixed-precision solve (host memory). */
typedef struct {
    int iters;              /* low-precision solves performed */
    int converged;          /* 1 if eta <= tol was reached */
    double eta;             /* normwise backward error of the returned X (max over vectors) */
    double anorm;           /* |op(A)|_inf (LEFT) or |op(A)|_1 (RIGHT) */
    double eta_hist[32];    /* eta after each correction */
} rtri_refine_info;

/* Mixed-precision TRSM with iterative refinement, eqs. (3)/(4) in FP64:
 * B := X with op(A) X = alpha B (LEFT) or X op(A) = alpha B (RIGHT), where
 * each correction D solves op(A) D = R / s (or D op(A) = R / s) recursively
 * with the GEMM updates run in gemm_type (RTRI_BF16 or RTRI_F32) MFMA with
 * FP32 accumulation and FP32 leaves, and the residual
 *     R = alpha B - op(A) X   (or alpha B - X op(A))
 * and the update X += s D are formed in FP64 (s is a power of two scaling R
 * into range).  The product op(A) X of the residual runs on the FP64 matrix
 * cores (the FP64 recursive TRMM) or, with RTRI_OPT_RESIDUAL = 1, from exact
 * INT8 products (the method of rtri_dtrmm_ozaki, FP64-accurate; its residue
 * planes of op(A) are made once per call).  Stops when the normwise backward error
 *     eta = max_v |R_v|inf / (anorm |X_v|inf + |alpha B_v|inf)
 * (v over columns for LEFT, rows for RIGHT) is <= tol, when eta fails to halve
 * from one correction to the next, or after max_iter (<= 32) corrections; B
 * always receives the last iterate.  Host-blocking: one 16-byte device-to-host
 * read per correction.  Returns RTRI_NOT_CONVERGED (B and *info still filled)
 * if tol was not reached.  info may be NULL.  Argument codes as rtri_dtrsm;
 * -13 gemm_type, -14 tol < 0, -15 max_iter not in 1..32. */
int rtri_dtrsm_mixed(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
                     const double *A, int64_t lda, double *B, int64_t ldb, int gemm_type, double tol,
                     int max_iter, rtri_refine_info *info);

/* ---- operations built on the recursive TRSM -------------------------------- */

/* Inverse of a triangular matrix, in place: the triangle of A named by uplo
 * (and its diagonal unless diag = RTRI_UNIT) is overwritten by that triangle
 * of inv(A); the other triangle is neither read nor written.  The midpoint
 * recursion of the TRSM (Sec. 3.1) with, for a lower triangle split at k,
 * inv([L11 0; L21 L22]) = [inv(L11) 0; -inv(L22) L21 inv(L11)  inv(L22)]: the
 * off-diagonal block by two recursive TRSMs (side R with L11 and alpha -1,
 * then side L with L22), then both halves recursively; diagonal blocks of at
 * most 64 rows are inverted by substitution, all in one launch (an upper
 * triangle mirrors this).  n^3/3 flops.  Codes: -2 uplo, -3 diag, -4 n < 0,
 * -5 A NULL, -6 lda < max(1, n). */
int rtri_dtrtri(rtri_handle *h, int uplo, int diag, int64_t n, double *A, int64_t lda);
int rtri_strtri(rtri_handle *h, int uplo, int diag, int64_t n, float *A, int64_t lda);

/* Solve S X = B (B n x nrhs, overwritten by X) with S = L L^T (uplo LOWER, L
 * the lower triangle of A) or S = U^T U (uplo UPPER): two recursive TRSMs, L
 * then L^T (U^T then U).  A is a Cholesky factor (non-unit diagonal).  Codes:
 * -2 uplo, -3 n < 0, -4 nrhs < 0, -5 A NULL, -6 lda < max(1, n), -7 B NULL,
 * -8 ldb < max(1, n). */
int rtri_dpotrs(rtri_handle *h, int uplo, int64_t n, int64_t nrhs, const double *A, int64_t lda, double *B,
                int64_t ldb);
int rtri_spotrs(rtri_handle *h, int uplo, int64_t n, int64_t nrhs, const float *A, int64_t lda, float *B, int64_t ldb);

/* Solve S X = B (trans N) or S^T X = B (trans T or C) (B n x nrhs, overwritten
 * by X) given P S = L U in LAPACK's packed form: LU holds the unit lower L
 * below its diagonal and U on and above it; ipiv (HOST memory, n entries,
 * 1-based) is the sequence of row interchanges (row i swapped with row
 * ipiv[i] - 1, in order).  trans N: the interchanges applied to B, then L,
 * then U; trans T: U^T, then L^T, then the interchanges undone.  The
 * workspace holds a copy of B while its rows are interchanged.  Codes: -2
 * trans, -3 n < 0, -4 nrhs < 0, -5 LU NULL, -6 lda < max(1, n), -7 ipiv NULL
 * or an entry outside 1..n, -8 B NULL, -9 ldb < max(1, n). */
int rtri_dgetrs(rtri_handle *h, int trans, int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                const int32_t *ipiv, double *B, int64_t ldb);
int rtri_sgetrs(rtri_handle *h, int trans, int64_t n, int64_t nrhs, const float *LU, int64_t lda, const int32_t *ipiv,
                float *B, int64_t ldb);

/* ---- factor objects: one triangular factor, many right-hand sides --------- */

/* A triangular factor A (order ka, the triangle named by uplo, diag as in
 * rtri_dtrsm) kept for repeated solves and multiplies against it, eqs. (1)-(4)
 * with A fixed.  The first call that needs them makes, and the factor then
 * keeps in device memory it owns:
 *   - the packed diagonal blocks each plan's leaves read (per op, side, trans,
 *     leaf size and precision), so later calls skip the pack pass;
 *   - for refined solves: the copy of A in the GEMM type (BF16 or FP32,
 *     transposed where the 16-bit GEMM wants it) and |op(A)| (per side and
 *     trans), so later calls skip the conversion and the norm; with
 *     RTRI_OPT_RESIDUAL = 1 also op(A)'s INT8 residue planes (per side and
 *     trans).
 * Results are bit for bit those of rtri_dtrsm / rtri_strsm / rtri_dtrmm /
 * rtri_strmm / rtri_dtrsm_mixed with the same handle options.
 * Parts are made on the calling handle's stream; a call on another stream
 * waits for them on the device.  Calls on one factor from several host
 * threads are safe (parts are made under a lock). */
typedef struct rtri_factor rtri_factor;

/* flags of rtri_factor_create */
enum { RTRI_FACTOR_COPY = 1 };   /* keep a copy of A (the caller may release A once create returns) */

/* Create a factor.  dtype RTRI_F64 or RTRI_F32 (the element type of A and of
 * every B used with it).  Without RTRI_FACTOR_COPY the factor reads the
 * caller's A (device memory) on every call: it must stay valid and unchanged
 * until rtri_factor_destroy.  With it, A is copied (ka x ka, blocking) into
 * memory the factor owns.  Codes: -2 uplo, -3 diag, -4 ka < 0, -5 dtype,
 * -6 A NULL, -7 lda < max(1, ka), -8 unknown flag, -9 out NULL. */
int rtri_factor_create(rtri_handle *h, int uplo, int diag, int64_t ka, int dtype, const void *A, int64_t lda,
                       unsigned flags, rtri_factor **f);

/* TRSM against the factor, eqs. (3)/(4): B := X with op(A) X = alpha B (LEFT,
 * B is ka x n) or X op(A) = alpha B (RIGHT, B is m x ka).  B is double* for
 * an FP64 factor, float* for an FP32 one (alpha rounded to it).
 *   precision RTRI_PREC_F64: the plain recursive solve in the factor's type
 *     (tol, max_iter, info ignored; info, if given, reports converged = 1);
 *   RTRI_PREC_MIXED_BF16 / RTRI_PREC_MIXED_F32 (FP64 factors only): the
 *     refined solve of rtri_dtrsm_mixed, host-blocking, returns
 *     RTRI_NOT_CONVERGED if tol was not reached (B and *info still filled).
 * Codes: -2 factor invalid, -3 side, -4 trans, -5 m (< 0, or != ka for LEFT),
 * -6 n (< 0, or != ka for RIGHT), -8 B NULL, -9 ldb < max(1, m),
 * -10 precision, -11 tol < 0, -12 max_iter not in 1..32;
 * RTRI_ERR_UNSUPPORTED for a refined solve on an FP32 factor. */
int rtri_factor_trsm(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, double alpha, void *B,
                     int64_t ldb, int precision, double tol, int max_iter, rtri_refine_info *info);

/* TRMM against the factor, eqs. (1)/(2): B := alpha op(A) B (LEFT) or
 * alpha B op(A) (RIGHT), in place.  Codes as rtri_factor_trsm (-2 .. -9). */
int rtri_factor_trmm(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, double alpha, void *B,
                     int64_t ldb);

/* Device bytes the factor holds (its copy of A and every part made so far). */
int rtri_factor_bytes(rtri_factor *f, int64_t *bytes);

/* Free the factor and everything it holds.  Waits for no work: synchronise
 * first if calls using it may still be running.  RTRI_ERR_INVALID for a NULL
 * or destroyed factor. */
int rtri_factor_destroy(rtri_factor *f);

/* Synthetic inputs for benchmarks and serving workloads (not part of the
 * method).  Fills an m-by-n column-major matrix X (device, ldx) with values
 * from Philox4x32-10 (Salmon et al., SC'11): element (i, j) uses counter
 * (i, j, id low word, id high word) and key (seed low word XOR stream, seed high
 * word); u = 53 bits of the first two output words (word 1 high) times 2^-53.
 *   kind 0: U(-1,1) = 2u - 1 everywhere
 *   kind 1: lower triangular, off-diagonal 2u - 1, diagonal param + u, zero above
 *   kind 2: upper triangular, likewise, zero below
 * dtype RTRI_F64 or RTRI_F32 (the FP64 value rounded to nearest).  Asynchronous
 * on the handle's stream.  Codes: -2 dtype, -3 kind, -7 m or n < 0, -10 X NULL,
 * -11 ldx < max(1, m). */
int rtri_synth_fill(rtri_handle *h, int dtype, int kind, uint64_t seed, uint32_t stream, uint64_t id, int64_t m,
                    int64_t n, double param, void *X, int64_t ldx);

/* Tuning.  dtype RTRI_F64 / RTRI_F32: time leaf sizes (16 / 32 / 64 / 128 /
 * 256) for TRSM and TRMM at factor orders 256, 512, ... up to max_order and 64
 * / 512 / 4096 / 16384 vectors (at most max_order); the GEMM tile (128x128 of
 * 4 or 8 wavefronts, or 64x64) at M = K = 64 ... min(max_order / 2, 8192) and
 * the same vector counts; and the batched kernel's leaf (32 or 64 rows) on a
 * mix of 200 problems of orders log-uniform on [16, min(1024, max_order)] and
 * 1..128 vectors.  dtype RTRI_BF16 / RTRI_F16: the 16-bit GEMM tile (128x128
 * or 256x256) at M = K = 256 ... min(max_order / 2, 8192) and 512 / 4096 /
 * 16384 vectors.  Synthetic inputs in device memory the call allocates and
 * frees; the winners are kept in the handle (rules for other dtypes are kept)
 * and, if db_path != NULL, written there as JSON.  Blocking.  Options set
 * with rtri_set_option still take precedence.  Codes: -2 dtype, -3 max_order
 * < 256; RTRI_ERR_INVALID if the file cannot be written.  If a timed run
 * fails, its code is returned and the handle keeps the rules it had. */
int rtri_tune(rtri_handle *h, int dtype, int64_t max_order, const char *db_path);

/* Load a tuning database written by rtri_tune into the handle (replacing any
 * earlier one).  A handle created while the environment variable RTRI_TUNE_DB
 * names such a file loads it automatically.  RTRI_ERR_INVALID if the file is
 * missing or malformed. */
int rtri_load_tuning(rtri_handle *h, const char *path);

/* The leaf size the handle would use for a TRSM (op = 0) or TRMM (op = 1) of
 * dtype RTRI_F64 / RTRI_F32 with a factor of order `order` against `nvec`
 * vectors: the option if set, else the loaded tuning rules, else 64 for
 * orders up to 1024 and 256 above.  Codes: -2 dtype, -3 op, -4 order or nvec
 * negative, -6 leaf NULL. */
int rtri_query_leaf(rtri_handle *h, int dtype, int op, int64_t order, int64_t nvec, int *leaf);

/* ---- batched independent problems (one persistent launch) ----------------- */

/* One problem of a batch: TRSM (op = 0, eqs. (3)/(4)) or TRMM (op = 1,
 * eqs. (1)/(2)), in place on B, with the same argument meaning as
 * rtri_dtrsm / rtri_dtrmm.  A and B are device pointers; problems of one batch
 * must not write overlapping B regions. */
typedef struct {
    int op, side, uplo, trans, diag;
    int64_t m, n;
    double alpha;
    const void *A;
    int64_t lda;
    void *B;
    int64_t ldb;
} rtri_batch_entry;

typedef struct rtri_batch_plan rtri_batch_plan;

/* Build a reusable plan for `count` problems of one element type (dtype
 * RTRI_F64 or RTRI_F32): every problem's recursion is laid out as an op list
 * (the splits and order of the single-call path with 64-row leaves, or 32-row
 * leaves when the handle would pick a leaf of at most 32 for an order-1024,
 * 64-vector problem (option or tuning rule); each result
 * is then bitwise what rtri_?trsm / rtri_?trmm give with the same leaf size,
 * which is their untuned choice for factor orders up to 1024), its
 * independent right-hand-side vectors are cut into chunks of 64, and the
 * chunks are queued longest first.  The plan owns device copies of these
 * tables and a captured hipGraph of the launch (a queue reset and one
 * persistent kernel whose workgroups pull chunks until the queue is empty).
 * entries is host memory and is not kept.  On an invalid entry returns its
 * argument code (as rtri_dtrsm, or -1 for op) and sets *bad_index (nullable);
 * RTRI_ERR_UNSUPPORTED for another dtype.  Blocking (uploads the tables). */
int rtri_batch_plan_create(rtri_handle *h, int dtype, int count, const rtri_batch_entry *entries,
                           rtri_batch_plan **plan, int *bad_index);

/* Launch the plan's graph on the handle's current stream (asynchronous).  The
 * problems read and write the A / B memory named at plan creation. */
int rtri_batch_plan_run(rtri_batch_plan *plan);

/* Number of work chunks in the plan (for reporting). */
int rtri_batch_plan_chunks(const rtri_batch_plan *plan, int64_t *chunks);

/* Free a plan (waits for its last launch). */
int rtri_batch_plan_destroy(rtri_batch_plan *plan);

/* One-shot convenience: create a plan, run it once without graph capture,
 * wait for it, destroy it. */
int rtri_batched(rtri_handle *h, int dtype, int count, const rtri_batch_entry *entries, int *bad_index);

/* ---- serving: continuous batching of solve / multiply requests ------------- */

enum { RTRI_PREC_F64 = 0, RTRI_PREC_MIXED_BF16 = 1, RTRI_PREC_MIXED_F32 = 2 };

typedef struct {
    int slots;              /* concurrent executors (a stream, a handle and a worker thread each), 1..16 */
    int64_t hbm_budget;     /* device bytes the server may hold: cached factors, right-hand sides, workspace */
    int max_batch;          /* most requests folded into one batched launch */
    int64_t small_max;      /* FP64 requests with factor order <= small_max join batched launches */
    uint64_t synth_seed;    /* seed of synthetic factors and right-hand sides (rtri_synth_fill) */
    int refine_requeue;     /* 0: a refined solve runs to the end in one turn of its slot; 1: it
                               re-enters the queue after each correction (see rtri_request) */
    int mixed_batch;        /* 1: a refined solve with FP32 updates and factor order
                               <= min(small_max, 256) opens a lockstep batch of the arrived requests of its kind when
                               another is waiting (else it runs alone): per round of corrections
                               one batched FP32 solve and one batched FP64 residual product over
                               the batch; results meet the same tolerance, not bitwise the alone
                               solve */
} rtri_server_cfg;

/* One request: a TRSM (op 0) or TRMM (op 1) with the argument meaning of
 * rtri_dtrsm / rtri_dtrmm, on a factor named by factor_id (order ka = m for
 * LEFT, n for RIGHT).  A factor registered with rtri_server_register_factor is
 * used as is; any other id names a synthetic factor (rtri_synth_fill kind
 * 1 / 2 by uplo, diagonal ka + U(0,1), stream 1, id = factor_id) generated on
 * the device on first use and cached (evicted least recently used when the
 * budget needs room; never while a request uses it).  The right-hand side is
 * synthetic (kind 0, stream 2, id = rhs_id).  precision selects the FP64 path
 * or the mixed-precision refined TRSM (TRSM only; tolerance 1e-12, at most 30
 * corrections).  With refine_requeue set, a refined solve runs one correction
 * per turn and re-enters the queue after each (its right-hand side and
 * iteration state stay on the device; any slot may run its next correction;
 * at most `slots` refined solves are started and unfinished at a time), so
 * slots serve other requests between its corrections; either way the
 * arithmetic, and so the result, is that of a refined solve run alone.  If result != NULL the
 * m-by-n result is copied there (host, column-major, ld = m) before the
 * request completes; the buffer must stay valid until then.  t_arrival is the
 * scheduled arrival time on the server clock; latency is measured from it. */
typedef struct {
    int op, side, uplo, trans, diag;
    int64_t m, n;
    double alpha;
    int precision;
    uint64_t factor_id;
    uint64_t rhs_id;
    double *result;
    double t_arrival;
} rtri_request;

typedef struct {
    uint64_t ticket;
    int status;             /* RTRI_OK, RTRI_NOT_CONVERGED, or an error code */
    int batched;            /* 1 if it ran inside a batched launch */
    int iters;              /* refinement corrections (mixed precision) */
    double eta;             /* refinement backward error (mixed precision), else 0 */
    double t_arrival, t_start, t_done;   /* server clock, seconds */
} rtri_completion;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t launches, batched_launches, batched_requests;
    int64_t factor_hits, factor_misses, evictions;
    int64_t hbm_in_use, hbm_peak;   /* device memory the server holds (factors and their factor objects'
                                       parts, right-hand sides, refined solves' iteration state, slot
                                       workspace), now and at most; admission also counts reservations for
                                       work not yet done (workspace growth, factor-object parts, upper
                                       bounds), which these exclude */
    double useful_flops;    /* sum of ka^2 * vectors over completed requests */
    int64_t refine_turns;   /* turns run by refined solves (one per solve, or with refine_requeue
                               one per correction, re-queued between them) */
} rtri_server_counters;

typedef struct rtri_server rtri_server;

/* Start a server on the current device.  Codes: -1 cfg NULL or out NULL,
 * -2 slots, -3 budget <= 0, -4 max_batch < 1. */
int rtri_server_create(const rtri_server_cfg *cfg, rtri_server **out);
/* Register a caller-owned FP64 factor (device memory, kept valid while the
 * server may use it; not counted against the budget, never evicted). */
int rtri_server_register_factor(rtri_server *s, uint64_t factor_id, int64_t ka, int uplo, const double *A,
                                int64_t lda);
/* Queue a request (thread safe, never blocks on the GPU); *ticket numbers it. */
int rtri_server_submit(rtri_server *s, const rtri_request *req, uint64_t *ticket);
/* Collect up to max completions (in completion order); *n receives the count. */
int rtri_server_poll(rtri_server *s, rtri_completion *out, int max, int *n);
/* Block until every submitted request has completed. */
int rtri_server_drain(rtri_server *s);
int rtri_server_stats(rtri_server *s, rtri_server_counters *out);
/* Seconds since the server started (the clock of t_arrival / t_done). */
double rtri_server_now(rtri_server *s);
/* Drain, stop the workers and free everything the server owns. */
int rtri_server_destroy(rtri_server *s);

#ifdef __cplusplus
}
#endif

#endif /* RTRI_H */
