// Complex TRSM / TRMM (FP64 complex, interleaved storage), eqs. (1)-(4) with
// op(A) = A, A^T or conj(A^T).
//
// Same midpoint recursion as the real path (Sec. 3.1).  The GEMM updates run
// on the real FP64 MFMA GEMM through the real embedding of op(A): a complex
// entry a + bi becomes the 2x2 block [a -b; b a], so a complex M x K block of
// op(A) becomes a real 2M x 2K block that multiplies the interleaved
// (re, im) rows of a complex K x N panel directly, viewed as a real 2K x N
// matrix with leading dimension 2 ldb.  This costs 8 M N K real flops, exactly
// the complex multiply-adds' own count.  The embedding of op(A)'s strict
// triangle is made once per call.  Leaves solve / multiply a diagonal block of
// at most 64 rows in complex arithmetic, one lane per right-hand-side vector.
//
// alpha (complex) is applied to B up front (both operations are linear in B),
// so the recursion runs with alpha = 1.  Side R is side L on the transpose:
// X op(A) = B  <=>  op(A)^T X^T = B^T, where op(A)^T is A^T, A or conj(A);
// B is transposed into workspace and back.
#include <cstring>

#include "handle.h"

using namespace rtri;

namespace {

constexpr int ZLEAF = 64;

struct zc {
    double re, im;
};

__device__ __forceinline__ zc zmul(zc a, zc b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
// a / b with b scaled by its larger part (Smith's method)
__device__ __forceinline__ zc zdiv(zc a, zc b)
{
    if (fabs(b.re) >= fabs(b.im)) {
        const double q = b.im / b.re, den = b.re + b.im * q;
        return {(a.re + a.im * q) / den, (a.im - a.re * q) / den};
    }
    const double q = b.re / b.im, den = b.re * q + b.im;
    return {(a.re * q + a.im) / den, (a.im * q - a.re) / den};
}

// op(A)(i, k) for the op given as (transposed, conjugated)
__device__ __forceinline__ zc zop(const double *A, int64_t lda, bool tr, bool cj, int64_t i, int64_t k)
{
    const int64_t off = tr ? 2 * (k + i * lda) : 2 * (i + k * lda);
    return {A[off], cj ? -A[off + 1] : A[off + 1]};
}

// Real embedding E (2 ka x 2 ka, leading dimension lde) of the strict
// effective triangle of op(A): E[2i + a][2k + b] = [re -im; im re][a][b] of
// op(A)(i, k).  One thread per entry (i, k) of op(A); entries outside the
// strict triangle are not written (the GEMM updates never read them).
__global__ void zembed_kernel(const double *__restrict__ A, int64_t lda, int64_t ka, bool tr, bool cj, bool low,
                              double *__restrict__ E, int64_t lde)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ka)
        return;
    for (int64_t k = blockIdx.y; k < ka; k += gridDim.y) {
        if (low ? i <= k : i >= k)
            continue;
        const zc z = zop(A, lda, tr, cj, i, k);
        double *c0 = E + 2 * i + (2 * k) * lde;
        double *c1 = c0 + lde;
        c0[0] = z.re;
        c0[1] = z.im;
        c1[0] = -z.im;
        c1[1] = z.re;
    }
}

// alpha * X in place (m x n complex, ld ldx); alpha == 0 writes zeros
__global__ void zscale_kernel(double *__restrict__ X, int64_t ldx, int64_t m, int64_t n, double ar, double ai)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m)
        return;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
        double *p = X + 2 * (i + j * ldx);
        if (ar == 0.0 && ai == 0.0) {
            p[0] = 0.0;
            p[1] = 0.0;
        } else {
            const zc v = zmul({ar, ai}, {p[0], p[1]});
            p[0] = v.re;
            p[1] = v.im;
        }
    }
}

// Y (n x m, ldy) = X^T (X m x n, ldx), complex, through a 32 x 32 LDS tile
__global__ __launch_bounds__(256) void ztranspose_kernel(const double *__restrict__ X, int64_t ldx, double *__restrict__ Y,
                                                         int64_t ldy, int64_t m, int64_t n)
{
    __shared__ double2 tile[32][33];
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = i0 + tx, j = j0 + r;
        if (i < m && j < n) {
            const double *p = X + 2 * (i + j * ldx);
            tile[r][tx] = make_double2(p[0], p[1]);
        }
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t j = j0 + tx, i = i0 + r;   // Y(j, i) = X(i, j)
        if (i < m && j < n) {
            const double2 v = tile[tx][r];
            double *p = Y + 2 * (j + i * ldy);
            p[0] = v.x;
            p[1] = v.y;
        }
    }
}

// Leaf on the diagonal block [d0, d0 + h) of op(A) against every column of
// the panel B (rows d0.., ldb): solve  op(A)_blk x = b  or multiply
// b := op(A)_blk b, in place.  The block is staged in LDS in op(A)'s
// orientation; each lane owns one column, its vector kept in LDS.
__global__ __launch_bounds__(64) void zleaf_kernel(const double *__restrict__ A, int64_t lda, bool tr, bool cj,
                                                   bool low, bool unit, bool solve, int64_t d0, int h,
                                                   double *__restrict__ B, int64_t ldb, int64_t n)
{
    __shared__ zc T[ZLEAF][ZLEAF + 1];
    __shared__ zc V[ZLEAF][64];
    const int t = threadIdx.x;
    for (int idx = t; idx < h * h; idx += 64) {
        const int i = idx % h, k = idx / h;
        // the effective triangle; a unit diagonal is not read
        const bool in = (low ? i >= k : i <= k) && !(unit && i == k);
        T[i][k] = in ? zop(A, lda, tr, cj, d0 + i, d0 + k) : zc{0.0, 0.0};
    }
    const int64_t j = (int64_t)blockIdx.x * 64 + t;
    const bool act = j < n;
    double *col = B + 2 * (d0 + j * ldb);
    if (act)
        for (int i = 0; i < h; ++i)
            V[i][t] = {col[2 * i], col[2 * i + 1]};
    __syncthreads();
    if (act) {
        if (solve) {
            for (int r = 0; r < h; ++r) {
                const int i = low ? r : h - 1 - r;
                zc s = {0.0, 0.0};
                const int k0 = low ? 0 : i + 1, k1 = low ? i : h;
                for (int k = k0; k < k1; ++k) {
                    const zc p = zmul(T[i][k], V[k][t]);
                    s.re += p.re;
                    s.im += p.im;
                }
                const zc v = {V[i][t].re - s.re, V[i][t].im - s.im};
                V[i][t] = unit ? v : zdiv(v, T[i][i]);
            }
        } else {
            // in place: lower from the last row up, upper from the first row down
            for (int r = 0; r < h; ++r) {
                const int i = low ? h - 1 - r : r;
                zc s = unit ? V[i][t] : zmul(T[i][i], V[i][t]);
                const int k0 = low ? 0 : i + 1, k1 = low ? i : h;
                for (int k = k0; k < k1; ++k) {
                    const zc p = zmul(T[i][k], V[k][t]);
                    s.re += p.re;
                    s.im += p.im;
                }
                V[i][t] = s;
            }
        }
        for (int i = 0; i < h; ++i) {
            col[2 * i] = V[i][t].re;
            col[2 * i + 1] = V[i][t].im;
        }
    }
}

struct ZPlan {
    const double *A;
    int64_t lda, ka, n;
    bool tr, cj, low, unit, solve, forward;
    const double *E;
    int64_t lde;
    double *B;
    int64_t ldb;
};

int zrec(rtri_handle *h, const ZPlan &p, int64_t d0, int64_t hh)
{
    hipError_t e;
    if (hh <= ZLEAF) {
        const dim3 grid((unsigned)((p.n + 63) / 64));
        e = timed(h, p.solve ? RTRI_KCLASS_LEAF_SOLVE : RTRI_KCLASS_LEAF_MULT, RTRI_F64, 4.0 * hh * hh * (double)p.n,
                  16.0 * (hh * (hh + 1) / 2.0 + 2.0 * hh * p.n), [&] {
                      zleaf_kernel<<<grid, dim3(64), 0, h->stream>>>(p.A, p.lda, p.tr, p.cj, p.low, p.unit, p.solve,
                                                                    d0, (int)hh, p.B, p.ldb, p.n);
                      return hipGetLastError();
                  });
        return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
    }
    const int64_t k = ZLEAF * ((hh + 2 * ZLEAF - 1) / (2 * ZLEAF));
    const int64_t b1 = d0, h1 = k, b2 = d0 + k, h2 = hh - k;
    const int64_t f0 = p.forward ? b1 : b2, fh = p.forward ? h1 : h2;
    const int64_t g0 = p.forward ? b2 : b1, gh = p.forward ? h2 : h1;
    int rc = zrec(h, p, f0, fh);
    if (rc != RTRI_OK)
        return rc;
    // solve:    B[second] -= op(A)[second, first] B[first]
    // multiply: B[first]  += op(A)[first, second] B[second] (second not yet overwritten)
    const int64_t t0 = p.solve ? g0 : f0, th = p.solve ? gh : fh;
    const int64_t s0 = p.solve ? f0 : g0, sh = p.solve ? fh : gh;
    GemmDesc g{};
    g.M = 2 * th;
    g.N = p.n;
    g.K = 2 * sh;
    g.beta = 1.0;
    g.s = p.solve ? -1.0 : 1.0;
    g.P = p.E + 2 * t0 + (2 * s0) * p.lde;
    g.ldp = p.lde;
    g.tp = false;
    g.Q = p.B + 2 * s0;
    g.ldq = 2 * p.ldb;
    g.tq = false;
    g.C = p.B + 2 * t0;
    g.ldc = 2 * p.ldb;
    e = timed(h, RTRI_KCLASS_GEMM, RTRI_F64, 2.0 * g.M * (double)g.N * g.K,
              8.0 * ((double)g.M * g.K + (double)g.K * g.N + 2.0 * g.M * g.N),
              [&] { return launch_gemm(DType::F64, g, 0, h->stream); });
    if (e != hipSuccess)
        return hip_fail(h, e);
    return zrec(h, p, g0, gh);
}

int zrun(rtri_handle *h, bool solve, int side, int uplo, int trans, int diag, int64_t m, int64_t n, const double *alpha,
         const void *Av, int64_t lda, void *Bv, int64_t ldb)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    // codes in BLAS argument order: 1..6, then alpha (7), then A, lda, B, ldb
    const int rc0 = check_args(side, uplo, trans, diag, m, n, Av, lda, Bv, ldb, false);
    if (rc0 < 0 && rc0 > -7)
        return rc0;
    if (alpha == nullptr)
        return -7;
    if (m > 0 && n > 0 && !(alpha[0] == 0.0 && alpha[1] == 0.0) && Av == nullptr)
        return -8;
    if (rc0 != 0)
        return rc0;
    if (m == 0 || n == 0)
        return RTRI_OK;
    const double *A = static_cast<const double *>(Av);
    double *B = static_cast<double *>(Bv);
    const double ar = alpha[0], ai = alpha[1];
    hipStream_t st = h->stream;
    const bool left = side == RTRI_LEFT;
    const int64_t ka = left ? m : n;
    hipError_t e;
    // alpha applied up front (alpha = 0: B := 0, A not read)
    if (!(ar == 1.0 && ai == 0.0)) {
        e = timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 32.0 * m * n, [&] {
            zscale_kernel<<<dim3((unsigned)((m + 255) / 256), (unsigned)std::min<int64_t>(n, 4096)), dim3(256), 0,
                            st>>>(B, ldb, m, n, ar, ai);
            return hipGetLastError();
        });
        if (e != hipSuccess)
            return hip_fail(h, e);
        if (ar == 0.0 && ai == 0.0)
            return RTRI_OK;
    }
    // side L acts with op(A) on the columns of B; side R with op(A)^T on the columns of B^T
    bool tr = trans != RTRI_NOTRANS, cj = trans == RTRI_CONJTRANS;
    double *P = B;
    int64_t ldp = ldb, nv = n;
    if (!left) {
        tr = !tr;
        e = ensure_ws(h, WS_ZT, (size_t)m * (size_t)n * 16);
        if (e == hipSuccess)
            e = timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 32.0 * m * n, [&] {
                ztranspose_kernel<<<dim3((unsigned)((m + 31) / 32), (unsigned)((n + 31) / 32)), dim3(256), 0, st>>>(
                    B, ldb, static_cast<double *>(h->ws[WS_ZT]), n, m, n);
                return hipGetLastError();
            });
        if (e != hipSuccess)
            return hip_fail(h, e);
        P = static_cast<double *>(h->ws[WS_ZT]);
        ldp = n;
        nv = m;
    }
    // op(A) as read by this side-L recursion is lower when (uplo L) != transposed
    const bool low = (uplo == RTRI_LOWER) != tr;
    ZPlan zp{};
    zp.A = A;
    zp.lda = lda;
    zp.ka = ka;
    zp.n = nv;
    zp.tr = tr;
    zp.cj = cj;
    zp.low = low;
    zp.unit = diag == RTRI_UNIT;
    zp.solve = solve;
    zp.forward = solve ? low : !low;
    zp.B = P;
    zp.ldb = ldp;
    zp.lde = ws_ld(2 * ka);
    if (ka > ZLEAF) {
        e = ensure_ws(h, WS_ZEMB, (size_t)(2 * ka) * (size_t)zp.lde * 8);
        if (e == hipSuccess)
            e = timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 8.0 * ka * ka + 16.0 * ka * ka, [&] {
                zembed_kernel<<<dim3((unsigned)((ka + 255) / 256), (unsigned)std::min<int64_t>(ka, 4096)), dim3(256),
                                0, st>>>(
                    A, lda, ka, tr, cj, low, static_cast<double *>(h->ws[WS_ZEMB]), zp.lde);
                return hipGetLastError();
            });
        if (e != hipSuccess)
            return hip_fail(h, e);
        zp.E = static_cast<const double *>(h->ws[WS_ZEMB]);
    }
    const int rc = zrec(h, zp, 0, ka);
    if (rc != RTRI_OK || left)
        return rc;
    e = timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 32.0 * m * n, [&] {
        ztranspose_kernel<<<dim3((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32)), dim3(256), 0, st>>>(
            P, n, B, ldb, n, m);
        return hipGetLastError();
    });
    return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
}

}  // namespace

extern "C" {

int rtri_ztrsm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, const double *alpha,
               const void *A, int64_t lda, void *B, int64_t ldb)
{
    return zrun(h, true, side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb);
}

int rtri_ztrmm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, const double *alpha,
               const void *A, int64_t lda, void *B, int64_t ldb)
{
    return zrun(h, false, side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb);
}

}  // extern "C"
