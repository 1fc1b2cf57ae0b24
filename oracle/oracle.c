/*
 * oracle.c -- plain, slow FP64 CPU reference for triangular matrix multiply
 * (TRMM) and triangular solve (TRSM).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may link,
 * load or call this file; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header or constant
 * with the GPU library.
 *
 * What it computes (paper, Sec. 2.1):
 *   TRMM  eq. (1)  B := alpha * op(A) * B      (side = L)
 *         eq. (2)  B := alpha * B * op(A)      (side = R)
 *   TRSM  eq. (3)  op(A) * X = alpha * B       (side = L), X overwrites B
 *         eq. (4)  X * op(A) = alpha * B       (side = R), X overwrites B
 *   op(A) in {A, A^T, conj(A^T)}; for real data conj(A^T) = A^T.
 *   A is upper or lower triangular, unit or non-unit diagonal.
 *
 * These are the plain definitions, written out: a triple loop for TRMM and
 * row-by-row forward / back substitution for TRSM.  No blocking, no recursion,
 * no reordering: the paper's recursive splitting only reorders these sums.
 *
 * Conventions: column-major storage, element (i,k) of A at A[i + k*lda].
 * For side = L, A is m-by-m; for side = R, A is n-by-n; B is m-by-n.
 * Only the triangle named by uplo is read; with diag = unit the diagonal is
 * not read either.
 *
 * Codes: side 0=L 1=R; uplo 0=lower 1=upper; trans 0=N 1=T 2=C; diag 0=non-unit 1=unit.
 *
 * Error metrics (test-side definitions, not from the paper):
 *   TRSM  normwise backward error per column (Rigal-Gaches)
 *           eta_j = |alpha b_j - op(A) x_j|_inf / (|op(A)|_inf |x_j|_inf + |alpha| |b_j|_inf)
 *   TRMM  eta_j = |c^_j - c_j|_inf / (|alpha| |op(A)|_inf |b_j|_inf)
 *   For side = R a row x_i of X solves the transposed system op(A)^T x_i^T =
 *   alpha b_i^T, so rows take the place of columns and |op(A)^T|_inf =
 *   |op(A)|_1 (largest column sum) takes the place of |op(A)|_inf.
 *   Residuals and the reference TRMM product used for the metrics are summed
 *   with the compensated dot product Dot2 (Ogita, Rump, Oishi, SIAM J. Sci.
 *   Comput. 2005), so their own rounding error (about u^2 * cond) is far below
 *   the tolerances being checked.  side = R uses rows instead of columns.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no contraction: the error-free
 * transformations below rely on every + and * being rounded separately).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- element access (O1): t(i,k) is element (i,k) of op(A) ---------------- */

static inline double elem_opA(const double *A, int64_t lda, int trans, int64_t i, int64_t k)
{
    return trans == 0 ? A[i + k * lda] : A[k + i * lda];
}

/* op(A) is lower triangular when A is lower and not transposed, or upper and transposed */
static inline int eff_lower(int uplo, int trans)
{
    return (uplo == 0) != (trans != 0);
}

/* value of op(A)(i,k) for (i,k) inside the effective triangle (diagonal included) */
static inline double tri_val(const double *A, int64_t lda, int trans, int diag, int64_t i, int64_t k)
{
    if (i == k && diag == 1)
        return 1.0;
    return elem_opA(A, lda, trans, i, k);
}

/* ---- TRMM, eqs. (1) and (2) ------------------------------------------------ */

/*
 * side = L:  C(i,j) = alpha * sum_{k in tri(i)} op(A)(i,k) * B(k,j)
 * side = R:  C(i,j) = alpha * sum_{k in tri'(j)} B(i,k) * op(A)(k,j)
 * The product is formed in a temporary and then written over B.
 */
void oracle_trmm(int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                 double alpha, const double *A, int64_t lda, double *B, int64_t ldb)
{
    const int low = eff_lower(uplo, trans);
    if (m <= 0 || n <= 0)
        return;
    if (side == 0) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t j = 0; j < n; ++j) {
            double *c = (double *)malloc(sizeof(double) * (size_t)m);
            double *b = B + j * ldb;
            for (int64_t i = 0; i < m; ++i) {
                int64_t k0 = low ? 0 : i, k1 = low ? i : m - 1;
                double s = 0.0;
                for (int64_t k = k0; k <= k1; ++k)
                    s += tri_val(A, lda, trans, diag, i, k) * b[k];
                c[i] = alpha * s;
            }
            memcpy(b, c, sizeof(double) * (size_t)m);
            free(c);
        }
    } else {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < m; ++i) {
            double *c = (double *)malloc(sizeof(double) * (size_t)n);
            for (int64_t j = 0; j < n; ++j) {
                /* op(A)(k,j) is non-zero for k >= j (lower) or k <= j (upper) */
                int64_t k0 = low ? j : 0, k1 = low ? n - 1 : j;
                double s = 0.0;
                for (int64_t k = k0; k <= k1; ++k)
                    s += B[i + k * ldb] * tri_val(A, lda, trans, diag, k, j);
                c[j] = alpha * s;
            }
            for (int64_t j = 0; j < n; ++j)
                B[i + j * ldb] = c[j];
            free(c);
        }
    }
}

/* ---- TRSM, eqs. (3) and (4) ------------------------------------------------ */

/*
 * side = L, op(A) lower: for each column, rows i = 0..m-1 in order,
 *     x_i = (alpha b_i - sum_{k<i} op(A)(i,k) x_k) / op(A)(i,i)
 * side = L, op(A) upper: rows i = m-1..0, sum over k > i.
 * side = R solves X op(A) = alpha B one row of X at a time:
 *   op(A) upper: columns j = 0..n-1,   x_j = (alpha b_j - sum_{k<j} x_k op(A)(k,j)) / op(A)(j,j)
 *   op(A) lower: columns j = n-1..0,   sum over k > j.
 * No division when diag = unit.  Division is IEEE division (no reciprocal).
 */
void oracle_trsm(int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                 double alpha, const double *A, int64_t lda, double *B, int64_t ldb)
{
    const int low = eff_lower(uplo, trans);
    if (m <= 0 || n <= 0)
        return;
    if (side == 0) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t j = 0; j < n; ++j) {
            double *x = B + j * ldb;
            for (int64_t r = 0; r < m; ++r) {
                int64_t i = low ? r : m - 1 - r;
                int64_t k0 = low ? 0 : i + 1, k1 = low ? i - 1 : m - 1;
                double s = 0.0;
                for (int64_t k = k0; k <= k1; ++k)
                    s += elem_opA(A, lda, trans, i, k) * x[k];
                double v = alpha * x[i] - s;
                x[i] = (diag == 1) ? v : v / elem_opA(A, lda, trans, i, i);
            }
        }
    } else {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t r = 0; r < n; ++r) {
                int64_t j = low ? n - 1 - r : r;
                int64_t k0 = low ? j + 1 : 0, k1 = low ? n - 1 : j - 1;
                double s = 0.0;
                for (int64_t k = k0; k <= k1; ++k)
                    s += B[i + k * ldb] * elem_opA(A, lda, trans, k, j);
                double v = alpha * B[i + j * ldb] - s;
                B[i + j * ldb] = (diag == 1) ? v : v / elem_opA(A, lda, trans, j, j);
            }
        }
    }
}

/* ---- complex TRMM / TRSM, eqs. (1)-(4) with op(A) = A, A^T or conj(A^T) ----- */

/*
 * Complex matrices are stored interleaved (real part, then imaginary part) in
 * column-major order: element (i, k) of A is (A[2(i + k lda)], A[2(i + k lda) + 1]),
 * lda counted in complex elements.  Products use the textbook formula
 * (a + bi)(c + di) = (ac - bd) + (ad + bc)i; quotients use Smith's method
 * (Smith 1962: divide through by the larger part of the divisor).
 */
typedef struct {
    double re, im;
} cplx;

static inline cplx c_mul(cplx a, cplx b)
{
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

static inline cplx c_div(cplx a, cplx b)
{
    cplx r;
    if (fabs(b.re) >= fabs(b.im)) {
        double q = b.im / b.re, den = b.re + b.im * q;
        r.re = (a.re + a.im * q) / den;
        r.im = (a.im - a.re * q) / den;
    } else {
        double q = b.re / b.im, den = b.re * q + b.im;
        r.re = (a.re * q + a.im) / den;
        r.im = (a.im * q - a.re) / den;
    }
    return r;
}

static inline cplx c_ld(const double *X, int64_t i, int64_t j, int64_t ld)
{
    cplx r = {X[2 * (i + j * ld)], X[2 * (i + j * ld) + 1]};
    return r;
}

static inline void c_st(double *X, int64_t i, int64_t j, int64_t ld, cplx v)
{
    X[2 * (i + j * ld)] = v.re;
    X[2 * (i + j * ld) + 1] = v.im;
}

/* op(A)(i, k) for (i, k) inside the effective triangle: A(i, k), A(k, i) or conj(A(k, i)) */
static inline cplx ztri_val(const double *A, int64_t lda, int trans, int diag, int64_t i, int64_t k)
{
    if (i == k && diag == 1) {
        cplx one = {1.0, 0.0};
        return one;
    }
    cplx a = trans == 0 ? c_ld(A, i, k, lda) : c_ld(A, k, i, lda);
    if (trans == 2)
        a.im = -a.im;
    return a;
}

/* side L: C(i,j) = alpha sum_k op(A)(i,k) B(k,j);  side R: C(i,j) = alpha sum_k B(i,k) op(A)(k,j) */
void oracle_ztrmm(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha_re,
                  double alpha_im, const double *A, int64_t lda, double *B, int64_t ldb)
{
    const int low = eff_lower(uplo, trans);
    const cplx alpha = {alpha_re, alpha_im};
    if (m <= 0 || n <= 0)
        return;
    double *C = (double *)malloc(sizeof(double) * 2 * (size_t)(m * n));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            cplx s = {0.0, 0.0};
            if (side == 0) {
                int64_t k0 = low ? 0 : i, k1 = low ? i : m - 1;
                for (int64_t k = k0; k <= k1; ++k) {
                    cplx p = c_mul(ztri_val(A, lda, trans, diag, i, k), c_ld(B, k, j, ldb));
                    s.re += p.re;
                    s.im += p.im;
                }
            } else {
                int64_t k0 = low ? j : 0, k1 = low ? n - 1 : j;
                for (int64_t k = k0; k <= k1; ++k) {
                    cplx p = c_mul(c_ld(B, i, k, ldb), ztri_val(A, lda, trans, diag, k, j));
                    s.re += p.re;
                    s.im += p.im;
                }
            }
            c_st(C, i, j, m, c_mul(alpha, s));
        }
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i)
            c_st(B, i, j, ldb, c_ld(C, i, j, m));
    free(C);
}

/* substitution as oracle_trsm, in complex arithmetic */
void oracle_ztrsm(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha_re,
                  double alpha_im, const double *A, int64_t lda, double *B, int64_t ldb)
{
    const int low = eff_lower(uplo, trans);
    const cplx alpha = {alpha_re, alpha_im};
    if (m <= 0 || n <= 0)
        return;
    if (side == 0) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t r = 0; r < m; ++r) {
                int64_t i = low ? r : m - 1 - r;
                int64_t k0 = low ? 0 : i + 1, k1 = low ? i - 1 : m - 1;
                cplx s = {0.0, 0.0};
                for (int64_t k = k0; k <= k1; ++k) {
                    cplx p = c_mul(ztri_val(A, lda, trans, diag, i, k), c_ld(B, k, j, ldb));
                    s.re += p.re;
                    s.im += p.im;
                }
                cplx v = c_mul(alpha, c_ld(B, i, j, ldb));
                v.re -= s.re;
                v.im -= s.im;
                c_st(B, i, j, ldb, diag == 1 ? v : c_div(v, ztri_val(A, lda, trans, diag, i, i)));
            }
        }
    } else {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t r = 0; r < n; ++r) {
                int64_t j = low ? n - 1 - r : r;
                int64_t k0 = low ? j + 1 : 0, k1 = low ? n - 1 : j - 1;
                cplx s = {0.0, 0.0};
                for (int64_t k = k0; k <= k1; ++k) {
                    cplx p = c_mul(c_ld(B, i, k, ldb), ztri_val(A, lda, trans, diag, k, j));
                    s.re += p.re;
                    s.im += p.im;
                }
                cplx v = c_mul(alpha, c_ld(B, i, j, ldb));
                v.re -= s.re;
                v.im -= s.im;
                c_st(B, i, j, ldb, diag == 1 ? v : c_div(v, ztri_val(A, lda, trans, diag, j, j)));
            }
        }
    }
}

/* ---- TRTRI: inverse of a triangular matrix ---------------------------------- */

/*
 * In place: the triangle of A named by uplo (and its diagonal unless unit)
 * becomes the same triangle of inv(A).  Column j of the inverse is the
 * solution x of A x = e_j, by the substitution of oracle_trsm:
 *   lower: x_i = 0 for i < j;  for i = j..n-1:  x_i = (delta_ij - sum_{j<=k<i} a_ik x_k) / a_ii
 *   upper: x_i = 0 for i > j;  for i = j..0:    x_i = (delta_ij - sum_{i<k<=j} a_ik x_k) / a_ii
 * (no division when unit).  The columns are formed in a temporary from the
 * original A and written back at the end; the other triangle is not touched.
 */
void oracle_trtri(int uplo, int diag, int64_t n, double *A, int64_t lda)
{
    if (n <= 0)
        return;
    double *X = (double *)calloc((size_t)(n * n), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        double *x = X + j * n;
        if (uplo == 0) {
            for (int64_t i = j; i < n; ++i) {
                double s = 0.0;
                for (int64_t k = j; k < i; ++k)
                    s += A[i + k * lda] * x[k];
                double v = (i == j ? 1.0 : 0.0) - s;
                x[i] = (diag == 1) ? v : v / A[i + i * lda];
            }
        } else {
            for (int64_t i = j; i >= 0; --i) {
                double s = 0.0;
                for (int64_t k = i + 1; k <= j; ++k)
                    s += A[i + k * lda] * x[k];
                double v = (i == j ? 1.0 : 0.0) - s;
                x[i] = (diag == 1) ? v : v / A[i + i * lda];
            }
        }
    }
    for (int64_t j = 0; j < n; ++j) {
        int64_t i0 = uplo == 0 ? j : 0, i1 = uplo == 0 ? n - 1 : j;
        for (int64_t i = i0; i <= i1; ++i)
            if (i != j || diag != 1)
                A[i + j * lda] = X[i + j * n];
    }
    free(X);
}

/* ---- compensated arithmetic for the error metrics -------------------------- */

/* error-free transformations: a + b = s + e exactly, a * b = p + e exactly */
static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* running Dot2 accumulator: value = s + c */
typedef struct {
    double s, c;
} dot2_acc;

static inline void dot2_add_prod(dot2_acc *acc, double a, double b)
{
    double p, ep, s, es;
    two_prod(a, b, &p, &ep);
    two_sum(acc->s, p, &s, &es);
    acc->s = s;
    acc->c += ep + es;
}

static inline double dot2_value(const dot2_acc *acc)
{
    return acc->s + acc->c;
}

double oracle_opnorm_one(int uplo, int trans, int diag, int64_t ka, const double *A, int64_t lda);

/* |op(A)|_inf: largest absolute row sum of the effective triangle (unit diagonal counts as 1) */
double oracle_opnorm_inf(int uplo, int trans, int diag, int64_t ka, const double *A, int64_t lda)
{
    const int low = eff_lower(uplo, trans);
    double best = 0.0;
    for (int64_t i = 0; i < ka; ++i) {
        int64_t k0 = low ? 0 : i, k1 = low ? i : ka - 1;
        double s = 0.0;
        for (int64_t k = k0; k <= k1; ++k)
            s += fabs(tri_val(A, lda, trans, diag, i, k));
        if (s > best)
            best = s;
    }
    return best;
}

/* |op(A)|_1: largest absolute column sum */
double oracle_opnorm_one(int uplo, int trans, int diag, int64_t ka, const double *A, int64_t lda)
{
    const int low = eff_lower(uplo, trans);
    double best = 0.0;
    for (int64_t k = 0; k < ka; ++k) {
        int64_t i0 = low ? k : 0, i1 = low ? ka - 1 : k;
        double s = 0.0;
        for (int64_t i = i0; i <= i1; ++i)
            s += fabs(tri_val(A, lda, trans, diag, i, k));
        if (s > best)
            best = s;
    }
    return best;
}

/*
 * Compensated product  C = alpha * op(A) * B  (side L)  or  alpha * B * op(A)  (side R),
 * written to C (ldc), B untouched.  Used as the accurate reference for TRMM errors.
 */
void oracle_trmm_dot2(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
                      const double *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc)
{
    const int low = eff_lower(uplo, trans);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            dot2_acc acc = {0.0, 0.0};
            if (side == 0) {
                int64_t k0 = low ? 0 : i, k1 = low ? i : m - 1;
                for (int64_t k = k0; k <= k1; ++k)
                    dot2_add_prod(&acc, tri_val(A, lda, trans, diag, i, k), B[k + j * ldb]);
            } else {
                int64_t k0 = low ? j : 0, k1 = low ? n - 1 : j;
                for (int64_t k = k0; k <= k1; ++k)
                    dot2_add_prod(&acc, B[i + k * ldb], tri_val(A, lda, trans, diag, k, j));
            }
            /* alpha * (s + c): the product of alpha with the compensated sum */
            dot2_acc out = {0.0, 0.0};
            dot2_add_prod(&out, alpha, acc.s);
            dot2_add_prod(&out, alpha, acc.c);
            C[i + j * ldc] = dot2_value(&out);
        }
    }
}

/*
 * Compensated residual  R = alpha * B - op(A) * X  (side L)  or  alpha * B - X * op(A)  (side R),
 * written to R (ldr).
 */
void oracle_trsm_residual(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
                          const double *A, int64_t lda, const double *B, int64_t ldb,
                          const double *X, int64_t ldx, double *R, int64_t ldr)
{
    const int low = eff_lower(uplo, trans);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            dot2_acc acc = {0.0, 0.0};
            dot2_add_prod(&acc, alpha, B[i + j * ldb]);
            if (side == 0) {
                int64_t k0 = low ? 0 : i, k1 = low ? i : m - 1;
                for (int64_t k = k0; k <= k1; ++k)
                    dot2_add_prod(&acc, -tri_val(A, lda, trans, diag, i, k), X[k + j * ldx]);
            } else {
                int64_t k0 = low ? j : 0, k1 = low ? n - 1 : j;
                for (int64_t k = k0; k <= k1; ++k)
                    dot2_add_prod(&acc, -X[i + k * ldx], tri_val(A, lda, trans, diag, k, j));
            }
            R[i + j * ldr] = dot2_value(&acc);
        }
    }
}

/* |v|_inf over a strided vector */
static double vnorm_inf(const double *v, int64_t len, int64_t stride)
{
    double best = 0.0;
    for (int64_t t = 0; t < len; ++t) {
        double a = fabs(v[t * stride]);
        if (a > best || a != a)
            best = a;
    }
    return best;
}

/*
 * TRSM normwise backward error, maximum over the columns (side L) or rows
 * (side R) of the computed solution X.  Returns NaN if any term is NaN.
 */
double oracle_trsm_eta(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
                       const double *A, int64_t lda, const double *B, int64_t ldb,
                       const double *X, int64_t ldx)
{
    if (m <= 0 || n <= 0)
        return 0.0;
    int64_t ka = side == 0 ? m : n;
    double *R = (double *)malloc(sizeof(double) * (size_t)(m * n));
    oracle_trsm_residual(side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb, X, ldx, R, m);
    double an = side == 0 ? oracle_opnorm_inf(uplo, trans, diag, ka, A, lda)
                          : oracle_opnorm_one(uplo, trans, diag, ka, A, lda);
    int64_t nvec = side == 0 ? n : m;
    double worst = 0.0;
    for (int64_t v = 0; v < nvec; ++v) {
        double rn, xn, bn;
        if (side == 0) {
            rn = vnorm_inf(R + v * m, m, 1);
            xn = vnorm_inf(X + v * ldx, m, 1);
            bn = vnorm_inf(B + v * ldb, m, 1);
        } else {
            rn = vnorm_inf(R + v, n, m);
            xn = vnorm_inf(X + v, n, ldx);
            bn = vnorm_inf(B + v, n, ldb);
        }
        double den = an * xn + fabs(alpha) * bn;
        double e = den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
        if (e != e) {
            worst = NAN;
            break;
        }
        if (e > worst)
            worst = e;
    }
    free(R);
    return worst;
}

/*
 * TRMM normwise error of a computed product Chat against the compensated
 * reference, maximum over columns (side L) or rows (side R).
 */
double oracle_trmm_eta(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
                       const double *A, int64_t lda, const double *B, int64_t ldb,
                       const double *Chat, int64_t ldc)
{
    if (m <= 0 || n <= 0)
        return 0.0;
    int64_t ka = side == 0 ? m : n;
    double *C = (double *)malloc(sizeof(double) * (size_t)(m * n));
    oracle_trmm_dot2(side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb, C, m);
    double an = side == 0 ? oracle_opnorm_inf(uplo, trans, diag, ka, A, lda)
                          : oracle_opnorm_one(uplo, trans, diag, ka, A, lda);
    int64_t nvec = side == 0 ? n : m;
    double worst = 0.0;
    for (int64_t v = 0; v < nvec; ++v) {
        double dn = 0.0, bn;
        if (side == 0) {
            for (int64_t i = 0; i < m; ++i) {
                double d = fabs(Chat[i + v * ldc] - C[i + v * m]);
                if (d > dn || d != d)
                    dn = d;
            }
            bn = vnorm_inf(B + v * ldb, m, 1);
        } else {
            for (int64_t j = 0; j < n; ++j) {
                double d = fabs(Chat[v + j * ldc] - C[v + j * m]);
                if (d > dn || d != d)
                    dn = d;
            }
            bn = vnorm_inf(B + v, n, ldb);
        }
        double den = fabs(alpha) * an * bn;
        double e = den > 0.0 ? dn / den : (dn > 0.0 ? INFINITY : 0.0);
        if (e != e) {
            worst = NAN;
            break;
        }
        if (e > worst)
            worst = e;
    }
    free(C);
    return worst;
}

/* ---- complex error metrics (compensated real and imaginary parts) ---------- */

/* acc_re + i acc_im += a b, every real product and sum compensated */
static inline void zdot2_add_prod(dot2_acc *re, dot2_acc *im, cplx a, cplx b)
{
    dot2_add_prod(re, a.re, b.re);
    dot2_add_prod(re, -a.im, b.im);
    dot2_add_prod(im, a.re, b.im);
    dot2_add_prod(im, a.im, b.re);
}

static inline double c_abs(cplx z) { return hypot(z.re, z.im); }

/* |op(A)|_inf (rows) or |op(A)|_1 (columns, by_rows = 0), moduli of the effective triangle */
double oracle_zopnorm(int uplo, int trans, int diag, int64_t ka, const double *A, int64_t lda, int by_rows)
{
    const int low = eff_lower(uplo, trans);
    double best = 0.0;
    for (int64_t l = 0; l < ka; ++l) {
        double s = 0.0;
        if (by_rows) {
            int64_t k0 = low ? 0 : l, k1 = low ? l : ka - 1;
            for (int64_t k = k0; k <= k1; ++k)
                s += c_abs(ztri_val(A, lda, trans, diag, l, k));
        } else {
            int64_t i0 = low ? l : 0, i1 = low ? ka - 1 : l;
            for (int64_t i = i0; i <= i1; ++i)
                s += c_abs(ztri_val(A, lda, trans, diag, i, l));
        }
        if (s > best)
            best = s;
    }
    return best;
}

/* compensated R = alpha B - op(A) X (side L) or alpha B - X op(A) (side R); R has ld m */
void oracle_ztrsm_residual(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha_re,
                           double alpha_im, const double *A, int64_t lda, const double *B, int64_t ldb,
                           const double *X, int64_t ldx, double *R)
{
    const int low = eff_lower(uplo, trans);
    const cplx alpha = {alpha_re, alpha_im};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            dot2_acc re = {0.0, 0.0}, im = {0.0, 0.0};
            zdot2_add_prod(&re, &im, alpha, c_ld(B, i, j, ldb));
            if (side == 0) {
                int64_t k0 = low ? 0 : i, k1 = low ? i : m - 1;
                for (int64_t k = k0; k <= k1; ++k) {
                    cplx a = ztri_val(A, lda, trans, diag, i, k);
                    a.re = -a.re;
                    a.im = -a.im;
                    zdot2_add_prod(&re, &im, a, c_ld(X, k, j, ldx));
                }
            } else {
                int64_t k0 = low ? j : 0, k1 = low ? n - 1 : j;
                for (int64_t k = k0; k <= k1; ++k) {
                    cplx x = c_ld(X, i, k, ldx);
                    x.re = -x.re;
                    x.im = -x.im;
                    zdot2_add_prod(&re, &im, x, ztri_val(A, lda, trans, diag, k, j));
                }
            }
            cplx v = {dot2_value(&re), dot2_value(&im)};
            c_st(R, i, j, m, v);
        }
    }
}

/* compensated C = alpha op(A) B (side L) or alpha B op(A) (side R); C has ld m */
void oracle_ztrmm_dot2(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha_re,
                       double alpha_im, const double *A, int64_t lda, const double *B, int64_t ldb, double *C)
{
    const int low = eff_lower(uplo, trans);
    const cplx alpha = {alpha_re, alpha_im};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) {
            dot2_acc re = {0.0, 0.0}, im = {0.0, 0.0};
            if (side == 0) {
                int64_t k0 = low ? 0 : i, k1 = low ? i : m - 1;
                for (int64_t k = k0; k <= k1; ++k)
                    zdot2_add_prod(&re, &im, ztri_val(A, lda, trans, diag, i, k), c_ld(B, k, j, ldb));
            } else {
                int64_t k0 = low ? j : 0, k1 = low ? n - 1 : j;
                for (int64_t k = k0; k <= k1; ++k)
                    zdot2_add_prod(&re, &im, c_ld(B, i, k, ldb), ztri_val(A, lda, trans, diag, k, j));
            }
            /* alpha (s + c), with s + c the compensated sum of each part */
            cplx sh = {re.s, im.s}, cl = {re.c, im.c};
            dot2_acc ore = {0.0, 0.0}, oim = {0.0, 0.0};
            zdot2_add_prod(&ore, &oim, alpha, sh);
            zdot2_add_prod(&ore, &oim, alpha, cl);
            cplx v = {dot2_value(&ore), dot2_value(&oim)};
            c_st(C, i, j, m, v);
        }
    }
}

static double zvnorm_inf(const double *v, int64_t len, int64_t stride)
{
    double best = 0.0;
    for (int64_t t = 0; t < len; ++t) {
        cplx z = {v[2 * t * stride], v[2 * t * stride + 1]};
        double a = c_abs(z);
        if (a > best || a != a)
            best = a;
    }
    return best;
}

/* complex TRSM backward error (moduli in every norm), as oracle_trsm_eta */
double oracle_ztrsm_eta(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha_re,
                        double alpha_im, const double *A, int64_t lda, const double *B, int64_t ldb,
                        const double *X, int64_t ldx)
{
    if (m <= 0 || n <= 0)
        return 0.0;
    int64_t ka = side == 0 ? m : n;
    double *R = (double *)malloc(sizeof(double) * 2 * (size_t)(m * n));
    oracle_ztrsm_residual(side, uplo, trans, diag, m, n, alpha_re, alpha_im, A, lda, B, ldb, X, ldx, R);
    double an = oracle_zopnorm(uplo, trans, diag, ka, A, lda, side == 0);
    double aa = hypot(alpha_re, alpha_im);
    int64_t nvec = side == 0 ? n : m;
    double worst = 0.0;
    for (int64_t v = 0; v < nvec; ++v) {
        double rn, xn, bn;
        if (side == 0) {
            rn = zvnorm_inf(R + 2 * v * m, m, 1);
            xn = zvnorm_inf(X + 2 * v * ldx, m, 1);
            bn = zvnorm_inf(B + 2 * v * ldb, m, 1);
        } else {
            rn = zvnorm_inf(R + 2 * v, n, m);
            xn = zvnorm_inf(X + 2 * v, n, ldx);
            bn = zvnorm_inf(B + 2 * v, n, ldb);
        }
        double den = an * xn + aa * bn;
        double e = den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
        if (e != e) {
            worst = NAN;
            break;
        }
        if (e > worst)
            worst = e;
    }
    free(R);
    return worst;
}

/* complex TRMM normwise error of Chat against the compensated product */
double oracle_ztrmm_eta(int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha_re,
                        double alpha_im, const double *A, int64_t lda, const double *B, int64_t ldb,
                        const double *Chat, int64_t ldc)
{
    if (m <= 0 || n <= 0)
        return 0.0;
    int64_t ka = side == 0 ? m : n;
    double *C = (double *)malloc(sizeof(double) * 2 * (size_t)(m * n));
    oracle_ztrmm_dot2(side, uplo, trans, diag, m, n, alpha_re, alpha_im, A, lda, B, ldb, C);
    double an = oracle_zopnorm(uplo, trans, diag, ka, A, lda, side == 0);
    double aa = hypot(alpha_re, alpha_im);
    int64_t nvec = side == 0 ? n : m;
    double worst = 0.0;
    for (int64_t v = 0; v < nvec; ++v) {
        double dn = 0.0, bn;
        int64_t len = side == 0 ? m : n;
        for (int64_t t = 0; t < len; ++t) {
            int64_t i = side == 0 ? t : v, j = side == 0 ? v : t;
            cplx d = {Chat[2 * (i + j * ldc)] - C[2 * (i + j * m)], Chat[2 * (i + j * ldc) + 1] - C[2 * (i + j * m) + 1]};
            double a = c_abs(d);
            if (a > dn || a != a)
                dn = a;
        }
        bn = side == 0 ? zvnorm_inf(B + 2 * v * ldb, m, 1) : zvnorm_inf(B + 2 * v, n, ldb);
        double den = aa * an * bn;
        double e = den > 0.0 ? dn / den : (dn > 0.0 ? INFINITY : 0.0);
        if (e != e) {
            worst = NAN;
            break;
        }
        if (e > worst)
            worst = e;
    }
    free(C);
    return worst;
}

/* set the number of OpenMP threads for later calls (no effect without OpenMP) */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* number of OpenMP threads the oracle runs with (1 if built without OpenMP) */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
