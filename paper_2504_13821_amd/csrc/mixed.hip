// Low-precision entry points built on the recursion driver:
//   rtri_trmm_ex      TRMM with 16-bit inputs, FP32 accumulation and output
//   rtri_dtrsm_mixed  FP64 TRSM by iterative refinement around a
//                     low-precision recursive solve (BF16 or FP32 GEMM updates)
//
// Refinement (classical mixed-precision iterative refinement, in the
// three-precision form: factor / solve precision, working precision FP64,
// residual precision FP64):
//     X = 0, R = alpha B
//     repeat:  s = 2^ceil(log2 max|R|)
//              D = s * LoSolve(fl32(R / s))       (recursive TRSM, GEMMs in BF16/FP32)
//              X = X + D                           (FP64)
//              R = alpha B - op(A) X               (FP64: X copied, TRMM'd, subtracted)
//              eta = max_v |R_v| / (anorm |X_v| + |alpha B_v|)
//     until eta <= tol, eta stops halving, or max_iter corrections.
#include <cmath>
#include <cstring>

#include "handle.h"

using namespace rtri;

namespace {

double from_bits(unsigned long long b)
{
    double d;
    static_assert(sizeof(d) == sizeof(b), "size");
    std::memcpy(&d, &b, sizeof d);
    return d;
}

}  // namespace

namespace rtri {

hipError_t launch_mixed_copy(rtri_handle *h, ElemT gt, bool ag_trans, int64_t ka, const double *A, int64_t lda,
                             void *Acopy, int64_t ldag)
{
    return timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 8.0 * ka * ka, [&] {
        return ag_trans ? launch_transpose_convert(gt, A, lda, Acopy, ldag, ka, ka, h->stream)
                        : launch_convert(ElemT::F64, gt, A, lda, Acopy, ldag, ka, ka, 1.0, h->stream);
    });
}

hipError_t launch_mixed_norm(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t ka, const double *A,
                             int64_t lda, unsigned long long *out)
{
    const bool left = side == RTRI_LEFT;
    const bool low = (uplo == RTRI_LOWER) != (tr != RTRI_NOTRANS);
    return timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 4.0 * ka * ka, [&] {
        // lines of op(A) (LEFT) or of op(A)^T (RIGHT): |op(A)|_inf or |op(A)|_1
        return launch_line_norm(A, lda, ka, left ? tr != RTRI_NOTRANS : tr == RTRI_NOTRANS, left ? low : !low,
                                diag == RTRI_UNIT, out, h->stream);
    });
}

PlanIn mixed_lo_plan(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n, ElemT gt,
                     const double *A, int64_t lda)
{
    const int64_t ka = side == RTRI_LEFT ? m : n;
    PlanIn lo{};
    lo.solve = true;
    lo.side = side;
    lo.uplo = uplo;
    lo.trans = tr;
    lo.diag = diag;
    lo.m = m;
    lo.n = n;
    lo.alpha = 1.0;
    lo.bt = DType::F32;
    lo.gt = gt;
    lo.ag_trans = mixed_ag_trans(gt, side, tr);
    lo.st = ElemT::F64;
    lo.As = A;
    lo.ldas = lda;
    lo.leaf = pick_leaf(h, DType::F32, true, ka, side == RTRI_LEFT ? n : m);
    lo.pack_slot = WS_PACK2;
    return lo;
}

PlanIn mixed_mul_plan(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n, const double *A,
                      int64_t lda)
{
    const int64_t ka = side == RTRI_LEFT ? m : n;
    PlanIn mul{};
    mul.solve = false;
    mul.side = side;
    mul.uplo = uplo;
    mul.trans = tr;
    mul.diag = diag;
    mul.m = m;
    mul.n = n;
    mul.alpha = 1.0;
    mul.bt = DType::F64;
    mul.gt = ElemT::F64;
    mul.Ag = reinterpret_cast<const char *>(A);
    mul.ldag = lda;
    mul.st = ElemT::F64;
    mul.As = A;
    mul.ldas = lda;
    mul.leaf = pick_leaf(h, DType::F64, false, ka, side == RTRI_LEFT ? n : m);
    mul.pack_slot = WS_PACK;
    return mul;
}

size_t refine_state_bytes(int64_t m, int64_t n)
{
    const size_t ln = (size_t)ws_ld(m) * (size_t)n;
    return ln * 4 + 4 * ln * 8 + 256;
}

void refine_state_place(RefineState &st, void *mem, int64_t m, int64_t n)
{
    const int64_t ld = ws_ld(m);
    const size_t ln = (size_t)ld * (size_t)n;
    char *p = static_cast<char *>(mem);
    st.ld = ld;
    st.X = reinterpret_cast<double *>(p);
    st.R0 = st.X + ln;
    st.R = st.R0 + ln;
    st.W = st.R + ln;
    st.sc = reinterpret_cast<unsigned long long *>(st.W + ln);
    st.D = reinterpret_cast<float *>(p + 4 * ln * 8 + 256);   // after the 4 scalars (kept 256-byte aligned)
}

// the loop's continuation test (the refinement's stopping rules)
static bool refine_more(const RefineState &st, int max_iter)
{
    return !st.converged && !st.stalled && st.iters < max_iter && st.rmax > 0.0 && std::isfinite(st.rmax);
}

hipError_t refine_begin_enqueue(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n,
                                double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                                const MixedPrep &prep, RefineState &st, unsigned long long *host4)
{
    hipStream_t st_ = h->stream;
    const int64_t ka = side == RTRI_LEFT ? m : n;
    const size_t mn = (size_t)m * (size_t)n;
    auto other = [&](double bytes, auto &&f) { return timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, bytes, f); };
    // |op(A)| (unless known), alpha B, max |R|
    hipError_t e = launch_zero_u64(st.sc, 4, st_);
    if (e == hipSuccess && !prep.have_anorm)
        e = launch_mixed_norm(h, side, uplo, tr, diag, ka, A, lda, st.sc + 2);
    if (e == hipSuccess)
        e = other(16.0 * mn, [&] { return launch_convert(ElemT::F64, ElemT::F64, B, ldb, st.R0, st.ld, m, n, alpha, st_); });
    // the first residual is alpha B itself (X = 0): it is read from R0, and the
    // first correction is assigned to X rather than added
    if (e == hipSuccess)
        e = other(8.0 * mn, [&] { return launch_max_abs(st.R0, st.ld, m, n, st.sc + 1, st_); });
    if (e == hipSuccess)
        e = hipMemcpyAsync(host4, st.sc, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st_);
    return e;
}

void refine_begin_finish(const unsigned long long *host4, double tol, int max_iter, rtri_refine_info *info,
                         const MixedPrep &prep, RefineState &st)
{
    st.anorm = prep.have_anorm ? prep.anorm : from_bits(host4[2]);
    st.rmax = from_bits(host4[1]);
    if (info != nullptr)
        info->anorm = st.anorm;
    st.oz = prep.oz_planes;
    st.eta = st.rmax == 0.0 ? 0.0 : INFINITY;
    st.eta_prev = INFINITY;
    st.iters = 0;
    st.converged = st.eta <= tol;
    st.stalled = false;
    st.done = !refine_more(st, max_iter);
}

int refine_begin(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n, double alpha,
                 const double *A, int64_t lda, const double *B, int64_t ldb, double tol, int max_iter,
                 rtri_refine_info *info, const MixedPrep &prep, RefineState &st)
{
    const int64_t ka = side == RTRI_LEFT ? m : n;
    unsigned long long host[4];
    hipError_t e = refine_begin_enqueue(h, side, uplo, tr, diag, m, n, alpha, A, lda, B, ldb, prep, st, host);
    if (e == hipSuccess)
        e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess)
        return hip_fail(h, e);
    refine_begin_finish(host, tol, max_iter, info, prep, st);
    // residual product from exact INT8 products: op(A)'s residue planes once
    if (h->residual == 1 && ozaki_nmod(ka) > 0 && st.oz == nullptr) {
        e = ensure_ws(h, WS_OZA, ozaki_factor_bytes(side, ka));
        if (e == hipSuccess)
            e = ozaki_split_factor(h, side, uplo, tr, diag, ka, A, lda, h->ws[WS_OZA]);
        if (e != hipSuccess)
            return hip_fail(h, e);
        st.oz = h->ws[WS_OZA];
    }
    return RTRI_OK;
}

hipError_t refine_step_convert(rtri_handle *h, int64_t m, int64_t n, RefineState &st)
{
    const size_t mn = (size_t)m * (size_t)n;
    st.scale = std::ldexp(1.0, (int)std::ceil(std::log2(st.rmax)));
    const double *Rk = st.iters == 0 ? st.R0 : st.R;
    return timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 12.0 * mn, [&] {
        return launch_convert(ElemT::F64, ElemT::F32, Rk, st.ld, st.D, st.ld, m, n, 1.0 / st.scale, h->stream);
    });
}

hipError_t refine_step_update(rtri_handle *h, int64_t m, int64_t n, RefineState &st)
{
    const size_t mn = (size_t)m * (size_t)n;
    // X += s D (X = s D the first time), and W = X for the residual's product (one pass)
    const bool assign = st.iters == 0;
    return timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, (assign ? 20.0 : 28.0) * mn, [&] {
        return launch_add_scaled(st.X, st.ld, st.D, st.ld, m, n, st.scale, assign, st.W, st.ld, h->stream);
    });
}

hipError_t refine_step_resid(rtri_handle *h, int side, int64_t m, int64_t n, RefineState &st,
                             unsigned long long *host2)
{
    const size_t mn = (size_t)m * (size_t)n;
    hipError_t e = launch_zero_u64(st.sc, 2, h->stream);
    if (e == hipSuccess)
        e = timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 32.0 * mn, [&] {
            return launch_resid_eta(st.R0, st.ld, st.W, st.ld, st.R, st.ld, st.X, st.ld, m, n, side == RTRI_LEFT,
                                    st.anorm, st.sc, h->stream);
        });
    if (e == hipSuccess)
        e = hipMemcpyAsync(host2, st.sc, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream);
    return e;
}

void refine_step_finish(const unsigned long long *host2, double tol, int max_iter, rtri_refine_info *info,
                        RefineState &st)
{
    st.eta = from_bits(host2[0]);
    st.rmax = from_bits(host2[1]);
    if (info != nullptr && st.iters < 32)
        info->eta_hist[st.iters] = st.eta;
    ++st.iters;
    if (st.eta <= tol)
        st.converged = true;
    else if (!(st.eta <= 0.5 * st.eta_prev))   // stagnation (or NaN)
        st.stalled = true;
    st.eta_prev = st.eta;
    st.done = !refine_more(st, max_iter);
}

int refine_step(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n, const double *A,
                int64_t lda, ElemT gt, double tol, int max_iter, rtri_refine_info *info, const MixedPrep &prep,
                RefineState &st)
{
    const int64_t ka = side == RTRI_LEFT ? m : n;
    const int64_t ld = st.ld;

    PlanIn lo = mixed_lo_plan(h, side, uplo, tr, diag, m, n, gt, A, lda);
    lo.B = reinterpret_cast<char *>(st.D);
    lo.ldb = ld;
    lo.Ag = static_cast<const char *>(prep.Acopy);
    lo.ldag = prep.ldag;
    lo.ag_trans = prep.ag_trans;
    if (prep.lo_pack != nullptr && prep.lo_leaf == lo.leaf)
        lo.packed = prep.lo_pack;
    lo.skip_pack = st.lo_packed;
    PlanIn mul = mixed_mul_plan(h, side, uplo, tr, diag, m, n, A, lda);
    mul.B = reinterpret_cast<char *>(st.W);
    mul.ldb = ld;
    if (prep.mul_pack != nullptr && prep.mul_leaf == mul.leaf)
        mul.packed = prep.mul_pack;
    mul.skip_pack = st.mul_packed;
    const bool int8_resid = h->residual == 1 && ozaki_nmod(ka) > 0 && st.oz != nullptr;

    hipError_t e = refine_step_convert(h, m, n, st);
    if (e != hipSuccess)
        return hip_fail(h, e);
    int rc = run_plan(h, lo);
    if (rc != RTRI_OK)
        return rc;
    st.lo_packed = true;
    e = refine_step_update(h, m, n, st);
    if (e != hipSuccess)
        return hip_fail(h, e);
    if (int8_resid) {
        rc = ozaki_product(h, side, uplo, tr, m, n, 1.0, st.oz, st.W, ld, st.W, ld);
    } else {
        rc = run_plan(h, mul);
        st.mul_packed = true;
    }
    if (rc != RTRI_OK)
        return rc;
    unsigned long long host[2];
    e = refine_step_resid(h, side, m, n, st, host);
    if (e == hipSuccess)
        e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess)
        return hip_fail(h, e);
    refine_step_finish(host, tol, max_iter, info, st);
    return RTRI_OK;
}

int refine_end(rtri_handle *h, int64_t m, int64_t n, double *B, int64_t ldb, rtri_refine_info *info,
               const RefineState &st)
{
    const size_t mn = (size_t)m * (size_t)n;
    // no correction made (alpha B is zero, or not finite): X = 0
    const hipError_t e =
        timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, (st.iters == 0 ? 8.0 : 16.0) * mn, [&] {
            return st.iters == 0 ? launch_fill(DType::F64, B, m, n, ldb, 0.0, h->stream)
                                 : launch_convert(ElemT::F64, ElemT::F64, st.X, st.ld, B, ldb, m, n, 1.0, h->stream);
        });
    if (e != hipSuccess)
        return hip_fail(h, e);
    if (info != nullptr) {
        info->iters = st.iters;
        info->converged = st.converged ? 1 : 0;
        info->eta = st.eta;
    }
    return st.converged ? RTRI_OK : RTRI_NOT_CONVERGED;
}

int mixed_core(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n, double alpha,
               const double *A, int64_t lda, double *B, int64_t ldb, ElemT gt, double tol, int max_iter,
               rtri_refine_info *info, const MixedPrep &prep)
{
    // the whole refinement on this handle: its state in the handle's workspace
    hipError_t e = ensure_ws(h, WS_REFINE, refine_state_bytes(m, n));
    if (e != hipSuccess)
        return hip_fail(h, e);
    RefineState st;
    refine_state_place(st, h->ws[WS_REFINE], m, n);
    int rc = refine_begin(h, side, uplo, tr, diag, m, n, alpha, A, lda, B, ldb, tol, max_iter, info, prep, st);
    while (rc == RTRI_OK && !st.done)
        rc = refine_step(h, side, uplo, tr, diag, m, n, A, lda, gt, tol, max_iter, info, prep, st);
    if (rc != RTRI_OK)
        return rc;
    return refine_end(h, m, n, B, ldb, info, st);
}

}  // namespace rtri

extern "C" {

int rtri_trmm_ex(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, float alpha,
                 const void *A, int a_type, int64_t lda, const void *B, int b_type, int64_t ldb, void *C,
                 int c_type, int64_t ldc)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    int rc = check_args(side, uplo, trans, diag, m, n, A, lda, B, ldb, alpha != 0.0f);
    if (rc != 0)
        return rc;
    if (m > 0 && n > 0 && C == nullptr)
        return -12;
    if (ldc < std::max<int64_t>(1, m))
        return -13;
    if (!((a_type == RTRI_BF16 || a_type == RTRI_F16) && b_type == a_type && c_type == RTRI_F32))
        return RTRI_ERR_UNSUPPORTED;
    if (m == 0 || n == 0)
        return RTRI_OK;
    const ElemT et = a_type == RTRI_BF16 ? ElemT::BF16 : ElemT::F16;
    hipError_t e;
    if (alpha == 0.0f) {
        e = timed(h, RTRI_KCLASS_OTHER, RTRI_F32, 0.0, 4.0 * m * n,
                  [&] { return launch_fill(DType::F32, C, m, n, ldc, 0.0, h->stream); });
        return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
    }
    // C = B widened to FP32 (exact), then C := alpha op(A) C in place
    e = timed(h, RTRI_KCLASS_OTHER, a_type, 0.0, 6.0 * m * n,
              [&] { return launch_convert(et, ElemT::F32, B, ldb, C, ldc, m, n, 1.0, h->stream); });
    if (e != hipSuccess)
        return hip_fail(h, e);
    // The 16-bit GEMM reads its triangle operand fastest with k contiguous: for
    // side L and trans N (or side R and trans T) its GEMM updates read a
    // transposed copy of A (handle workspace), as the refined solve does.
    const int tr = trans == RTRI_CONJTRANS ? RTRI_TRANS : trans;
    const bool left = side == RTRI_LEFT;
    const int64_t ka = left ? m : n;
    const bool ag_trans = left ? tr == RTRI_NOTRANS : tr != RTRI_NOTRANS;
    const void *Ag = A;
    int64_t ldag = lda;
    if (ag_trans) {
        ldag = ws_ld(ka);
        e = ensure_ws(h, WS_ACOPY, (size_t)ka * (size_t)ldag * 2);
        if (e == hipSuccess)
            e = timed(h, RTRI_KCLASS_OTHER, a_type, 0.0, 4.0 * ka * ka,
                      [&] { return launch_transpose16(A, lda, h->ws[WS_ACOPY], ldag, ka, ka, h->stream); });
        if (e != hipSuccess)
            return hip_fail(h, e);
        Ag = h->ws[WS_ACOPY];
    }
    PlanIn p{};
    p.solve = false;
    p.side = side;
    p.uplo = uplo;
    p.trans = tr;
    p.diag = diag;
    p.m = m;
    p.n = n;
    p.alpha = alpha;
    p.bt = DType::F32;
    p.B = static_cast<char *>(C);
    p.ldb = ldc;
    p.gt = et;
    p.Ag = static_cast<const char *>(Ag);
    p.ldag = ldag;
    p.ag_trans = ag_trans;
    p.Bsrc16 = static_cast<const char *>(B);   // the updates read the 16-bit original of C
    p.ldbsrc16 = ldb;
    p.st = et;
    p.As = A;
    p.ldas = lda;
    p.leaf = pick_leaf(h, DType::F32, false, side == RTRI_LEFT ? m : n, side == RTRI_LEFT ? n : m);
    p.pack_slot = WS_PACK;
    p.skip_pack = false;
    return run_plan(h, p);
}

int rtri_dtrsm_mixed(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
                     const double *A, int64_t lda, double *B, int64_t ldb, int gemm_type, double tol,
                     int max_iter, rtri_refine_info *info)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    int rc = check_args(side, uplo, trans, diag, m, n, A, lda, B, ldb, alpha != 0.0);
    if (rc != 0)
        return rc;
    if (gemm_type != RTRI_BF16 && gemm_type != RTRI_F32)
        return -13;
    if (!(tol >= 0.0))
        return -14;
    if (max_iter < 1 || max_iter > 32)
        return -15;
    if (info != nullptr)
        std::memset(info, 0, sizeof *info);
    if (m == 0 || n == 0 || alpha == 0.0) {
        if (info != nullptr)
            info->converged = 1;
        if (m == 0 || n == 0)
            return RTRI_OK;
        const hipError_t e = launch_fill(DType::F64, B, m, n, ldb, 0.0, h->stream);
        return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
    }
    const int64_t ka = side == RTRI_LEFT ? m : n;
    const int tr = trans == RTRI_CONJTRANS ? RTRI_TRANS : trans;
    const ElemT gt = gemm_type == RTRI_BF16 ? ElemT::BF16 : ElemT::F32;
    // once per call: the GEMM copy of A (the packed blocks and |op(A)| are
    // made by the core on its first use)
    MixedPrep prep;
    prep.ldag = ws_ld(ka);
    prep.ag_trans = mixed_ag_trans(gt, side, tr);
    hipError_t e = ensure_ws(h, WS_ACOPY, (size_t)ka * (size_t)prep.ldag * elem_size(gt));
    if (e == hipSuccess)
        e = launch_mixed_copy(h, gt, prep.ag_trans, ka, A, lda, h->ws[WS_ACOPY], prep.ldag);
    if (e != hipSuccess)
        return hip_fail(h, e);
    prep.Acopy = h->ws[WS_ACOPY];
    return mixed_core(h, side, uplo, tr, diag, m, n, alpha, A, lda, B, ldb, gt, tol, max_iter, info, prep);
}

}  // extern "C"
