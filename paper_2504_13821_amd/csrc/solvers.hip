// Operations built on the recursive TRSM (the paper notes TRSM as the core of
// matrix inversion and of solving with LU and similar factorisations, Sec. 1):
//   rtri_?trtri  inverse of a triangular matrix, in place
//   rtri_?potrs  S X = B with S = L L^T or U^T U (two triangular solves)
//   rtri_?getrs  S X = B or S^T X = B with P S = L U (row interchanges and two
//                triangular solves)
//
// TRTRI uses the same midpoint recursion as the TRSM itself.  For a lower
// triangle split at k,
//     inv([L11 0; L21 L22]) = [inv(L11) 0; -inv(L22) L21 inv(L11)  inv(L22)],
// so the off-diagonal block is formed by two TRSMs against the ORIGINAL
// diagonal blocks (L21 := -L21 inv(L11): side R, alpha -1; then
// L21 := inv(L22) L21: side L), before the two halves are inverted
// recursively; an upper triangle mirrors this.  Every TRSM of the recursion
// reads only original diagonal blocks, so all base blocks (<= 64 rows) are
// inverted at the end, in one launch.
#include <cstring>
#include <vector>

#include "handle.h"

using namespace rtri;

namespace {

constexpr int TRTRI_BASE = 64;

// Inverse of every diagonal block of at most 64 rows (block b covers rows /
// columns [64 b, min(64 b + 64, n))).  One wavefront per block; lane j forms
// column j of the block's inverse by substitution against the block staged in
// LDS, then the named triangle (and the diagonal unless unit) is written back.
template <class T>
__global__ __launch_bounds__(64) void trtri_base_kernel(T *__restrict__ A, int64_t lda, int64_t n, bool lower,
                                                        bool unit)
{
    __shared__ T L[TRTRI_BASE][TRTRI_BASE + 1];
    __shared__ T X[TRTRI_BASE][TRTRI_BASE + 1];
    const int64_t d0 = (int64_t)blockIdx.x * TRTRI_BASE;
    const int h = (int)min<int64_t>(TRTRI_BASE, n - d0);
    const int t = threadIdx.x;
    T *blk = A + d0 + d0 * lda;
    for (int k = 0; k < h; ++k)
        if (t < h) {
            const bool in = lower ? t > k : t < k;
            L[t][k] = in ? blk[t + k * lda] : (t == k && !unit ? blk[t + k * lda] : T(0));
        }
    __syncthreads();
    const int j = t;
    if (j < h) {
        if (lower) {
            for (int i = 0; i < j; ++i)
                X[i][j] = T(0);
            for (int i = j; i < h; ++i) {
                T s = T(0);
                for (int k = j; k < i; ++k)
                    s = fmat(L[i][k], X[k][j], s);
                const T v = (i == j ? T(1) : T(0)) - s;
                X[i][j] = unit ? v : v / L[i][i];
            }
        } else {
            for (int i = h - 1; i > j; --i)
                X[i][j] = T(0);
            for (int i = j; i >= 0; --i) {
                T s = T(0);
                for (int k = i + 1; k <= j; ++k)
                    s = fmat(L[i][k], X[k][j], s);
                const T v = (i == j ? T(1) : T(0)) - s;
                X[i][j] = unit ? v : v / L[i][i];
            }
        }
    }
    __syncthreads();
    for (int k = 0; k < h; ++k)
        if (t < h) {
            const bool in = lower ? t > k : t < k;
            if (in || (t == k && !unit))
                blk[t + k * lda] = X[t][k];
        }
}

// dst row i = src row perm[i] (gather), or dst row perm[i] = src row i (scatter)
template <class T>
__global__ void permute_rows_kernel(const T *__restrict__ src, int64_t lds, T *__restrict__ dst, int64_t ldd,
                                    const int32_t *__restrict__ perm, int64_t m, int64_t n, bool gather)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= m || j >= n)
        return;
    const int64_t p = perm[i];
    if (gather)
        dst[i + j * ldd] = src[p + j * lds];
    else
        dst[p + j * ldd] = src[i + j * lds];
}

template <class T>
int trsm_call(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
              const T *A, int64_t lda, T *B, int64_t ldb)
{
    if (m == 0 || n == 0)
        return RTRI_OK;
    const DType t = sizeof(T) == 8 ? DType::F64 : DType::F32;
    return run_plan(h, plain_plan(h, t, true, side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb));
}

template <class T>
int trtri_rec(rtri_handle *h, bool lower, int diag, T *A, int64_t lda, int64_t d0, int64_t nn)
{
    if (nn <= TRTRI_BASE)
        return RTRI_OK;
    const int64_t k = TRTRI_BASE * ((nn + 2 * TRTRI_BASE - 1) / (2 * TRTRI_BASE));
    T *A11 = A + d0 + d0 * lda;
    T *A22 = A + (d0 + k) + (d0 + k) * lda;
    int rc;
    if (lower) {
        T *A21 = A + (d0 + k) + d0 * lda;   // (nn - k) x k
        rc = trsm_call<T>(h, RTRI_RIGHT, RTRI_LOWER, RTRI_NOTRANS, diag, nn - k, k, -1.0, A11, lda, A21, lda);
        if (rc == RTRI_OK)
            rc = trsm_call<T>(h, RTRI_LEFT, RTRI_LOWER, RTRI_NOTRANS, diag, nn - k, k, 1.0, A22, lda, A21, lda);
    } else {
        T *A12 = A + d0 + (d0 + k) * lda;   // k x (nn - k)
        rc = trsm_call<T>(h, RTRI_RIGHT, RTRI_UPPER, RTRI_NOTRANS, diag, k, nn - k, -1.0, A22, lda, A12, lda);
        if (rc == RTRI_OK)
            rc = trsm_call<T>(h, RTRI_LEFT, RTRI_UPPER, RTRI_NOTRANS, diag, k, nn - k, 1.0, A11, lda, A12, lda);
    }
    if (rc == RTRI_OK)
        rc = trtri_rec<T>(h, lower, diag, A, lda, d0, k);
    if (rc == RTRI_OK)
        rc = trtri_rec<T>(h, lower, diag, A, lda, d0 + k, nn - k);
    return rc;
}

template <class T>
int trtri(rtri_handle *h, int uplo, int diag, int64_t n, T *A, int64_t lda)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (uplo != RTRI_LOWER && uplo != RTRI_UPPER) return -2;
    if (diag != RTRI_NONUNIT && diag != RTRI_UNIT) return -3;
    if (n < 0) return -4;
    if (n > 0 && A == nullptr) return -5;
    if (lda < std::max<int64_t>(1, n)) return -6;
    if (n == 0)
        return RTRI_OK;
    const bool lower = uplo == RTRI_LOWER;
    int rc = trtri_rec<T>(h, lower, diag, A, lda, 0, n);
    if (rc != RTRI_OK)
        return rc;
    const int64_t nb = (n + TRTRI_BASE - 1) / TRTRI_BASE;
    const double fl = (double)n * TRTRI_BASE * TRTRI_BASE / 3.0;
    const hipError_t e = timed(h, RTRI_KCLASS_OTHER, sizeof(T) == 8 ? RTRI_F64 : RTRI_F32, fl,
                               (double)sizeof(T) * n * TRTRI_BASE, [&] {
                                   trtri_base_kernel<T><<<dim3((unsigned)nb), dim3(64), 0, h->stream>>>(
                                       A, lda, n, lower, diag == RTRI_UNIT);
                                   return hipGetLastError();
                               });
    return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
}

template <class T>
int potrs(rtri_handle *h, int uplo, int64_t n, int64_t nrhs, const T *A, int64_t lda, T *B, int64_t ldb)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (uplo != RTRI_LOWER && uplo != RTRI_UPPER) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (n > 0 && nrhs > 0 && A == nullptr) return -5;
    if (lda < std::max<int64_t>(1, n)) return -6;
    if (n > 0 && nrhs > 0 && B == nullptr) return -7;
    if (ldb < std::max<int64_t>(1, n)) return -8;
    // S = L L^T: L y = b, then L^T x = y;  S = U^T U: U^T y = b, then U x = y
    const int first = uplo == RTRI_LOWER ? RTRI_NOTRANS : RTRI_TRANS;
    const int second = uplo == RTRI_LOWER ? RTRI_TRANS : RTRI_NOTRANS;
    int rc = trsm_call<T>(h, RTRI_LEFT, uplo, first, RTRI_NONUNIT, n, nrhs, 1.0, A, lda, B, ldb);
    if (rc == RTRI_OK)
        rc = trsm_call<T>(h, RTRI_LEFT, uplo, second, RTRI_NONUNIT, n, nrhs, 1.0, A, lda, B, ldb);
    return rc;
}

template <class T>
int getrs(rtri_handle *h, int trans, int64_t n, int64_t nrhs, const T *LU, int64_t lda, const int32_t *ipiv, T *B,
          int64_t ldb)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (trans != RTRI_NOTRANS && trans != RTRI_TRANS && trans != RTRI_CONJTRANS) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (n > 0 && nrhs > 0 && LU == nullptr) return -5;
    if (lda < std::max<int64_t>(1, n)) return -6;
    if (n > 0 && ipiv == nullptr) return -7;
    for (int64_t i = 0; i < n; ++i)
        if (ipiv[i] < 1 || ipiv[i] > n)
            return -7;
    if (n > 0 && nrhs > 0 && B == nullptr) return -8;
    if (ldb < std::max<int64_t>(1, n)) return -9;
    if (n == 0 || nrhs == 0)
        return RTRI_OK;
    // the interchanges as one permutation: row i of P B is row perm[i] of B
    std::vector<int32_t> perm((size_t)n);
    for (int64_t i = 0; i < n; ++i)
        perm[(size_t)i] = (int32_t)i;
    bool any = false;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t p = ipiv[i] - 1;
        if (p != i) {
            std::swap(perm[(size_t)i], perm[(size_t)p]);
            any = true;
        }
    }
    const size_t es = sizeof(T);
    auto permute = [&](bool gather) -> hipError_t {
        // B -> copy, then the copy's rows back into B, gathered or scattered
        hipError_t e = ensure_ws(h, WS_ROWS, (size_t)n * (size_t)nrhs * es);
        if (e == hipSuccess)
            e = ensure_ws(h, WS_PERM, (size_t)n * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->ws[WS_PERM], perm.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice,
                               h->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(h->stream);   // the host vector is released on return
        if (e == hipSuccess)
            e = timed(h, RTRI_KCLASS_OTHER, es == 8 ? RTRI_F64 : RTRI_F32, 0.0, 4.0 * es * n * nrhs, [&] {
                hipError_t e2 = hipMemcpy2DAsync(h->ws[WS_ROWS], n * es, B, ldb * es, n * es, nrhs,
                                                 hipMemcpyDeviceToDevice, h->stream);
                if (e2 != hipSuccess)
                    return e2;
                const dim3 grid((unsigned)((n + 255) / 256), (unsigned)nrhs);
                permute_rows_kernel<T><<<grid, dim3(256), 0, h->stream>>>(
                    static_cast<const T *>(h->ws[WS_ROWS]), n, B, ldb, static_cast<const int32_t *>(h->ws[WS_PERM]),
                    n, nrhs, gather);
                return hipGetLastError();
            });
        return e;
    };
    int rc = RTRI_OK;
    if (trans == RTRI_NOTRANS) {
        // P S = L U:  S x = b  <=>  L U x = P b
        if (any) {
            const hipError_t e = permute(true);
            if (e != hipSuccess)
                return hip_fail(h, e);
        }
        rc = trsm_call<T>(h, RTRI_LEFT, RTRI_LOWER, RTRI_NOTRANS, RTRI_UNIT, n, nrhs, 1.0, LU, lda, B, ldb);
        if (rc == RTRI_OK)
            rc = trsm_call<T>(h, RTRI_LEFT, RTRI_UPPER, RTRI_NOTRANS, RTRI_NONUNIT, n, nrhs, 1.0, LU, lda, B, ldb);
    } else {
        // S^T x = b  <=>  U^T L^T (P x) = b
        rc = trsm_call<T>(h, RTRI_LEFT, RTRI_UPPER, RTRI_TRANS, RTRI_NONUNIT, n, nrhs, 1.0, LU, lda, B, ldb);
        if (rc == RTRI_OK)
            rc = trsm_call<T>(h, RTRI_LEFT, RTRI_LOWER, RTRI_TRANS, RTRI_UNIT, n, nrhs, 1.0, LU, lda, B, ldb);
        if (rc == RTRI_OK && any) {
            const hipError_t e = permute(false);
            if (e != hipSuccess)
                return hip_fail(h, e);
        }
    }
    return rc;
}

}  // namespace

extern "C" {

int rtri_dtrtri(rtri_handle *h, int uplo, int diag, int64_t n, double *A, int64_t lda)
{
    return trtri<double>(h, uplo, diag, n, A, lda);
}

int rtri_strtri(rtri_handle *h, int uplo, int diag, int64_t n, float *A, int64_t lda)
{
    return trtri<float>(h, uplo, diag, n, A, lda);
}

int rtri_dpotrs(rtri_handle *h, int uplo, int64_t n, int64_t nrhs, const double *A, int64_t lda, double *B,
                int64_t ldb)
{
    return potrs<double>(h, uplo, n, nrhs, A, lda, B, ldb);
}

int rtri_spotrs(rtri_handle *h, int uplo, int64_t n, int64_t nrhs, const float *A, int64_t lda, float *B, int64_t ldb)
{
    return potrs<float>(h, uplo, n, nrhs, A, lda, B, ldb);
}

int rtri_dgetrs(rtri_handle *h, int trans, int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                const int32_t *ipiv, double *B, int64_t ldb)
{
    return getrs<double>(h, trans, n, nrhs, LU, lda, ipiv, B, ldb);
}

int rtri_sgetrs(rtri_handle *h, int trans, int64_t n, int64_t nrhs, const float *LU, int64_t lda, const int32_t *ipiv,
                float *B, int64_t ldb)
{
    return getrs<float>(h, trans, n, nrhs, LU, lda, ipiv, B, ldb);
}

}  // extern "C"
