// Call plans: one FP64 / FP32 TRSM or TRMM (eqs. (1)-(4)) on fixed operands,
// planned once and captured in a HIP graph, then replayed.  A single call
// re-plans its recursion on the host and launches one kernel per leaf and per
// GEMM update (plus the pack pass); a replay is one graph launch, which is
// what small and narrow problems (whose kernels take microseconds) need.
//
// The plan owns the workspace its kernels use (the packed diagonal blocks and
// one split-K region), so nothing is allocated or re-planned at replay and
// the handle's own workspace may grow or move freely afterwards.  The TRMM
// runs its per-leaf schedule (each update its own launch, all captured):
// that schedule needs no saved copy of the panel and no host-built tables.
// Replays compute exactly what the plain call computes with the same handle
// options (the same plan and kernels), bit for bit.
#include "handle.h"

struct rtri_call_plan {
    rtri_handle *h;
    void *ws;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

using namespace rtri;

extern "C" {

int rtri_call_plan_create(rtri_handle *h, int op, int dtype, int side, int uplo, int trans, int diag, int64_t m,
                          int64_t n, double alpha, const void *A, int64_t lda, void *B, int64_t ldb,
                          rtri_call_plan **out)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (out == nullptr)
        return -15;
    *out = nullptr;
    if (op != 0 && op != 1)
        return -2;
    if (dtype != RTRI_F64 && dtype != RTRI_F32)
        return -3;
    const int rc = check_args(side, uplo, trans, diag, m, n, A, lda, B, ldb, alpha != 0.0);
    if (rc != 0)
        return rc - 3;   // argument i of the BLAS list is argument i + 3 here
    if (h->profiling)    // a profile records events created on demand: not capturable
        return RTRI_ERR_UNSUPPORTED;
    const DType t = dtype == RTRI_F64 ? DType::F64 : DType::F32;
    rtri_call_plan *p = new (std::nothrow) rtri_call_plan();
    if (p == nullptr)
        return RTRI_ERR_NOMEM;
    p->h = h;
    PlanIn pl = plain_plan(h, t, op == 0, side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb);
    const bool work = m > 0 && n > 0 && alpha != 0.0;
    const size_t pack = work ? (plan_pack_bytes(pl) + 255) / 256 * 256 : 0;
    hipError_t e = hipMalloc(&p->ws, pack + SPLIT_REGION_BYTES);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(h, e);
    }
    pl.ext_pack = p->ws;
    pl.ext_split = static_cast<char *>(p->ws) + pack;
    // capture on a stream of the plan's own, the handle bound to it meanwhile
    hipStream_t saved = h->stream, cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    int prc = RTRI_OK;
    if (e == hipSuccess) {
        h->stream = cs;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            if (m > 0 && n > 0 && alpha == 0.0)
                prc = launch_fill(t, B, m, n, ldb, 0.0, cs) == hipSuccess ? RTRI_OK : RTRI_ERR_HIP;
            else if (work)
                prc = run_plan(h, pl);
            const hipError_t ee = hipStreamEndCapture(cs, &p->graph);
            if (e == hipSuccess)
                e = ee;
        }
        h->stream = saved;
    }
    if (e == hipSuccess && prc == RTRI_OK)
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (cs != nullptr)
        (void)hipStreamDestroy(cs);
    if (e != hipSuccess || prc != RTRI_OK) {
        if (p->exec)
            (void)hipGraphExecDestroy(p->exec);
        if (p->graph)
            (void)hipGraphDestroy(p->graph);
        (void)hipFree(p->ws);
        delete p;
        return prc != RTRI_OK ? prc : hip_fail(h, e);
    }
    *out = p;
    return RTRI_OK;
}

int rtri_call_plan_run(rtri_call_plan *p)
{
    if (p == nullptr || !handle_valid(p->h))
        return RTRI_ERR_HANDLE;
    const hipError_t e = hipGraphLaunch(p->exec, p->h->stream);
    return e == hipSuccess ? RTRI_OK : hip_fail(p->h, e);
}

int rtri_call_plan_destroy(rtri_call_plan *p)
{
    if (p == nullptr)
        return -1;
    if (handle_valid(p->h))
        (void)hipStreamSynchronize(p->h->stream);
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    (void)hipFree(p->ws);
    delete p;
    return RTRI_OK;
}

}  // extern "C"
