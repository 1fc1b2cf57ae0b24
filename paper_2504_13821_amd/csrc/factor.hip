// Factor objects: one triangular factor A kept for many solves and multiplies
// against it (eqs. (1)-(4) with A fixed and B varying).
//
// A factor remembers A (the caller's memory, or its own copy) and keeps, the
// first time a call needs them, the pieces every later call against the same
// A would otherwise make again:
//   - the packed diagonal blocks of a plan (per op, side, trans, leaf size and
//     panel type: the leaves read them, the pack pass is skipped);
//   - for the refined solve, the copy of A in the GEMM type (BF16 or FP32,
//     transposed where the 16-bit GEMM wants it) and |op(A)| for the
//     backward error (per side and trans), and with the INT8 residual product
//     op(A)'s residue planes (per side and trans).
// Results are bit for bit those of the plain entry points with the same
// handle options: the same plans run on the same packed blocks.
//
// Parts are made on the calling handle's stream while the factor's lock is
// held, and an event marks each one ready; a call on another stream waits for
// that event on the device before using the part.
#include <cstring>
#include <deque>
#include <mutex>

#include "handle.h"

using namespace rtri;

namespace {

constexpr uint32_t FMAGIC = 0x72666163u;   // 'rfac'

enum PartKind { PART_PACK = 0, PART_COPY = 1, PART_NORM = 2, PART_OZAKI = 3 };

struct Part {
    int kind;
    int key[6];
    void *mem = nullptr;
    size_t bytes = 0;
    double value = 0.0;          // PART_NORM: |op(A)|
    hipEvent_t ready = nullptr;  // recorded on `stream` after the part was made
    hipStream_t stream = nullptr;
    bool pooled = false;         // allocated from a handle's memory pool on `stream`
};

}  // namespace

struct rtri_factor {
    uint32_t magic;
    int uplo, diag, dtype;
    int64_t ka;
    const void *A;
    int64_t lda;
    void *own;                   // the factor's copy of A (RTRI_FACTOR_COPY), freed with it
    size_t own_bytes;
    std::mutex mu;
    std::deque<Part> parts;      // a deque: references to parts stay valid as parts are added
};

namespace {

bool factor_valid(const rtri_factor *f) { return f != nullptr && f->magic == FMAGIC; }

size_t parts_bytes(const rtri_factor *f)
{
    size_t b = f->own_bytes;
    for (const Part &p : f->parts)
        b += p.bytes;
    return b;
}

hipError_t part_alloc(rtri_handle *h, Part &p, size_t bytes)
{
    p.bytes = std::max<size_t>(bytes, 256);
    p.stream = h->stream;
    if (h->mem_pool != nullptr) {
        p.pooled = true;
        return hipMallocFromPoolAsync(&p.mem, p.bytes, h->mem_pool, h->stream);
    }
    return hipMalloc(&p.mem, p.bytes);
}

void part_free(Part &p)
{
    if (p.mem != nullptr) {
        if (p.pooled)
            (void)hipFreeAsync(p.mem, p.stream);
        else
            (void)hipFree(p.mem);
    }
    if (p.ready != nullptr)
        (void)hipEventDestroy(p.ready);
    p.mem = nullptr;
    p.ready = nullptr;
}

// The part with this kind and key, made by make(part) on h's stream if the
// factor has none yet.  Must be called with f->mu held.  On return the
// handle's stream is ordered after the part's making.
template <class Make>
hipError_t get_part(rtri_handle *h, rtri_factor *f, int kind, const int (&key)[6], Make &&make, const Part **out)
{
    for (const Part &p : f->parts)
        if (p.kind == kind && std::memcmp(p.key, key, sizeof key) == 0) {
            *out = &p;
            return p.stream == h->stream ? hipSuccess : hipStreamWaitEvent(h->stream, p.ready, 0);
        }
    Part p;
    p.kind = kind;
    std::memcpy(p.key, key, sizeof key);
    hipError_t e = make(p);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&p.ready, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventRecord(p.ready, h->stream);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(h->stream);
        part_free(p);
        return e;
    }
    f->parts.push_back(p);
    *out = &f->parts.back();
    return hipSuccess;
}

// the packed diagonal blocks of plan q (q.As / q.st / q.bt / q.leaf / q.solve /
// side / trans decide them; q.packed is set on return)
hipError_t packed_blocks(rtri_handle *h, rtri_factor *f, PlanIn &q)
{
    const int key[6] = {q.solve ? 1 : 0, q.side, q.trans, q.leaf, (int)q.bt, (int)q.st};
    const Part *part = nullptr;
    hipError_t e = get_part(h, f, PART_PACK, key, [&](Part &p) {
        hipError_t e2 = part_alloc(h, p, plan_pack_bytes(q));
        return e2 == hipSuccess ? pack_plan(h, q, p.mem) : e2;
    }, &part);
    if (e == hipSuccess)
        q.packed = part->mem;
    return e;
}

int check_factor_call(const rtri_factor *f, int side, int trans, int64_t m, int64_t n, const void *B, int64_t ldb)
{
    if (side != RTRI_LEFT && side != RTRI_RIGHT) return -3;
    if (trans != RTRI_NOTRANS && trans != RTRI_TRANS && trans != RTRI_CONJTRANS) return -4;
    if (m < 0 || (side == RTRI_LEFT && m != f->ka)) return -5;
    if (n < 0 || (side == RTRI_RIGHT && n != f->ka)) return -6;
    if (m > 0 && n > 0 && B == nullptr) return -8;
    if (ldb < std::max<int64_t>(1, m)) return -9;
    return 0;
}

int plain_call(rtri_handle *h, rtri_factor *f, bool solve, int side, int trans, int64_t m, int64_t n, double alpha,
               void *B, int64_t ldb)
{
    const DType t = f->dtype == RTRI_F64 ? DType::F64 : DType::F32;
    if (alpha == 0.0) {
        const hipError_t e = launch_fill(t, B, m, n, ldb, 0.0, h->stream);
        return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
    }
    PlanIn q = plain_plan(h, t, solve, side, f->uplo, trans, f->diag, m, n, alpha, f->A, f->lda, B, ldb);
    {
        std::lock_guard<std::mutex> lk(f->mu);
        const hipError_t e = packed_blocks(h, f, q);
        if (e != hipSuccess)
            return hip_fail(h, e);
    }
    return run_plan(h, q);
}

}  // namespace

// What the refined solve needs from A, made once per factor (the copy of A in
// the GEMM type, the packed blocks of both plans, |op(A)|, the INT8 residue
// planes when that residual is selected) and kept in its parts.
static int refine_prep(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, int precision,
                       MixedPrep &prep)
{
    const int tr = trans == RTRI_CONJTRANS ? RTRI_TRANS : trans;
    const ElemT gt = precision == RTRI_PREC_MIXED_BF16 ? ElemT::BF16 : ElemT::F32;
    const double *A = static_cast<const double *>(f->A);
    prep.ldag = ws_ld(f->ka);
    prep.ag_trans = mixed_ag_trans(gt, side, tr);
    {
        std::lock_guard<std::mutex> lk(f->mu);
        const Part *part = nullptr;
        const int kcopy[6] = {(int)gt, prep.ag_trans ? 1 : 0, 0, 0, 0, 0};
        hipError_t e = get_part(h, f, PART_COPY, kcopy, [&](Part &p) {
            hipError_t e2 = part_alloc(h, p, (size_t)f->ka * (size_t)prep.ldag * elem_size(gt));
            return e2 == hipSuccess ? launch_mixed_copy(h, gt, prep.ag_trans, f->ka, A, f->lda, p.mem, prep.ldag) : e2;
        }, &part);
        if (e != hipSuccess)
            return hip_fail(h, e);
        prep.Acopy = part->mem;
        PlanIn lo = mixed_lo_plan(h, side, f->uplo, tr, f->diag, m, n, gt, A, f->lda);
        e = packed_blocks(h, f, lo);
        if (e != hipSuccess)
            return hip_fail(h, e);
        prep.lo_pack = lo.packed;
        prep.lo_leaf = lo.leaf;
        PlanIn mul = mixed_mul_plan(h, side, f->uplo, tr, f->diag, m, n, A, f->lda);
        e = packed_blocks(h, f, mul);
        if (e != hipSuccess)
            return hip_fail(h, e);
        prep.mul_pack = mul.packed;
        prep.mul_leaf = mul.leaf;
        const int knorm[6] = {side, tr, 0, 0, 0, 0};
        e = get_part(h, f, PART_NORM, knorm, [&](Part &p) {
            // the norm is read back once, into host memory
            hipError_t e2 = ensure_ws(h, WS_SCALARS, 64);
            unsigned long long *sc = e2 == hipSuccess ? static_cast<unsigned long long *>(h->ws[WS_SCALARS]) : nullptr;
            unsigned long long bits = 0;
            if (e2 == hipSuccess)
                e2 = launch_zero_u64(sc, 1, h->stream);
            if (e2 == hipSuccess)
                e2 = launch_mixed_norm(h, side, f->uplo, tr, f->diag, f->ka, A, f->lda, sc);
            if (e2 == hipSuccess)
                e2 = hipMemcpyAsync(&bits, sc, sizeof bits, hipMemcpyDeviceToHost, h->stream);
            if (e2 == hipSuccess)
                e2 = hipStreamSynchronize(h->stream);
            if (e2 == hipSuccess)
                std::memcpy(&p.value, &bits, sizeof bits);
            p.stream = h->stream;
            return e2;
        }, &part);
        if (e != hipSuccess)
            return hip_fail(h, e);
        prep.have_anorm = true;
        prep.anorm = part->value;
        if (h->residual == 1 && ozaki_nmod(f->ka) > 0) {
            const int koz[6] = {side, tr, 0, 0, 0, 0};
            e = get_part(h, f, PART_OZAKI, koz, [&](Part &p) {
                hipError_t e2 = part_alloc(h, p, ozaki_factor_bytes(side, f->ka));
                return e2 == hipSuccess ? ozaki_split_factor(h, side, f->uplo, tr, f->diag, f->ka, A, f->lda, p.mem)
                                        : e2;
            }, &part);
            if (e != hipSuccess)
                return hip_fail(h, e);
            prep.oz_planes = part->mem;
        }
    }
    return RTRI_OK;
}

namespace rtri {

int factor_refine_begin(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, double alpha,
                        const double *B, int64_t ldb, int precision, double tol, int max_iter, rtri_refine_info *info,
                        RefineState &st)
{
    MixedPrep prep;
    const int rc = refine_prep(h, f, side, trans, m, n, precision, prep);
    if (rc != RTRI_OK)
        return rc;
    const int tr = trans == RTRI_CONJTRANS ? RTRI_TRANS : trans;
    return refine_begin(h, side, f->uplo, tr, f->diag, m, n, alpha, static_cast<const double *>(f->A), f->lda, B, ldb,
                        tol, max_iter, info, prep, st);
}

int factor_refine_prep(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, int precision,
                       MixedPrep &prep)
{
    return refine_prep(h, f, side, trans, m, n, precision, prep);
}

int factor_refine_step(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, int precision,
                       double tol, int max_iter, rtri_refine_info *info, RefineState &st)
{
    MixedPrep prep;
    const int rc = refine_prep(h, f, side, trans, m, n, precision, prep);
    if (rc != RTRI_OK)
        return rc;
    const int tr = trans == RTRI_CONJTRANS ? RTRI_TRANS : trans;
    const ElemT gt = precision == RTRI_PREC_MIXED_BF16 ? ElemT::BF16 : ElemT::F32;
    return refine_step(h, side, f->uplo, tr, f->diag, m, n, static_cast<const double *>(f->A), f->lda, gt, tol,
                       max_iter, info, prep, st);
}

}  // namespace rtri

extern "C" {

int rtri_factor_create(rtri_handle *h, int uplo, int diag, int64_t ka, int dtype, const void *A, int64_t lda,
                       unsigned flags, rtri_factor **out)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (uplo != RTRI_LOWER && uplo != RTRI_UPPER) return -2;
    if (diag != RTRI_NONUNIT && diag != RTRI_UNIT) return -3;
    if (ka < 0) return -4;
    if (dtype != RTRI_F64 && dtype != RTRI_F32) return -5;
    if (ka > 0 && A == nullptr) return -6;
    if (lda < std::max<int64_t>(1, ka)) return -7;
    if ((flags & ~(unsigned)RTRI_FACTOR_COPY) != 0) return -8;
    if (out == nullptr) return -9;
    rtri_factor *f = new (std::nothrow) rtri_factor();
    if (f == nullptr)
        return RTRI_ERR_NOMEM;
    f->magic = FMAGIC;
    f->uplo = uplo;
    f->diag = diag;
    f->dtype = dtype;
    f->ka = ka;
    f->A = A;
    f->lda = lda;
    f->own = nullptr;
    f->own_bytes = 0;
    if ((flags & RTRI_FACTOR_COPY) != 0 && ka > 0) {
        const size_t es = dtype == RTRI_F64 ? 8 : 4;
        f->own_bytes = (size_t)ka * (size_t)ka * es;
        hipError_t e = hipMalloc(&f->own, f->own_bytes);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(f->own, ka * es, A, lda * es, ka * es, ka, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(h->stream);   // A may be released once this returns
        if (e != hipSuccess) {
            (void)hipFree(f->own);
            f->magic = 0;
            delete f;
            return hip_fail(h, e);
        }
        f->A = f->own;
        f->lda = ka;
    }
    *out = f;
    return RTRI_OK;
}

int rtri_factor_destroy(rtri_factor *f)
{
    if (!factor_valid(f))
        return RTRI_ERR_INVALID;
    f->magic = 0;
    for (Part &p : f->parts)
        part_free(p);
    if (f->own != nullptr)
        (void)hipFree(f->own);
    delete f;
    return RTRI_OK;
}

int rtri_factor_bytes(rtri_factor *f, int64_t *bytes)
{
    if (!factor_valid(f))
        return RTRI_ERR_INVALID;
    if (bytes == nullptr)
        return -2;
    std::lock_guard<std::mutex> lk(f->mu);
    *bytes = (int64_t)parts_bytes(f);
    return RTRI_OK;
}

int rtri_factor_trmm(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, double alpha, void *B,
                     int64_t ldb)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (!factor_valid(f))
        return -2;
    const int rc = check_factor_call(f, side, trans, m, n, B, ldb);
    if (rc != 0)
        return rc;
    if (m == 0 || n == 0)
        return RTRI_OK;
    return plain_call(h, f, false, side, trans, m, n, alpha, B, ldb);
}

int rtri_factor_trsm(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, double alpha, void *B,
                     int64_t ldb, int precision, double tol, int max_iter, rtri_refine_info *info)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (!factor_valid(f))
        return -2;
    int rc = check_factor_call(f, side, trans, m, n, B, ldb);
    if (rc != 0)
        return rc;
    if (precision != RTRI_PREC_F64 && precision != RTRI_PREC_MIXED_BF16 && precision != RTRI_PREC_MIXED_F32)
        return -10;
    if (precision != RTRI_PREC_F64 && f->dtype != RTRI_F64)
        return RTRI_ERR_UNSUPPORTED;
    if (precision != RTRI_PREC_F64) {
        if (!(tol >= 0.0)) return -11;
        if (max_iter < 1 || max_iter > 32) return -12;
    }
    if (info != nullptr)
        std::memset(info, 0, sizeof *info);
    if (m == 0 || n == 0 || precision == RTRI_PREC_F64 || alpha == 0.0) {
        if (info != nullptr)
            info->converged = 1;
        if (m == 0 || n == 0)
            return RTRI_OK;
        return plain_call(h, f, true, side, trans, m, n, alpha, B, ldb);
    }
    // refined solve: copy of A, packed blocks of both plans and |op(A)| from the factor
    MixedPrep prep;
    rc = refine_prep(h, f, side, trans, m, n, precision, prep);
    if (rc != RTRI_OK)
        return rc;
    const int tr = trans == RTRI_CONJTRANS ? RTRI_TRANS : trans;
    const ElemT gt = precision == RTRI_PREC_MIXED_BF16 ? ElemT::BF16 : ElemT::F32;
    const double *A = static_cast<const double *>(f->A);
    return mixed_core(h, side, f->uplo, tr, f->diag, m, n, alpha, A, f->lda, static_cast<double *>(B), ldb, gt, tol,
                      max_iter, info, prep);
}

}  // extern "C"
