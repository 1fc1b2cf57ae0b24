// FP64 TRSM that allocates no device memory: the packed diagonal blocks and
// the split-K partial products live in a fixed array of device memory that
// this file defines (one copy per GPU, held until the process ends), instead
// of the handle's workspace, which grows with hipMalloc.
//
// Host code never passes `scratch` itself to a kernel (in host code the name
// is a host-side stand-in, not a device address): the device address of each
// GPU's copy comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is handed to the recursion.
#include <mutex>

#include "handle.h"

namespace {

constexpr size_t PACK_BYTES = (size_t)32 << 20;                         // packed diagonal blocks
constexpr size_t SCRATCH_BYTES = PACK_BYTES + rtri::SPLIT_REGION_BYTES;  // + one split-K region
static_assert(SCRATCH_BYTES == (size_t)RTRI_NOALLOC_SCRATCH_MIB << 20, "header states the scratch size");
static_assert(PACK_BYTES % 256 == 0, "split region stays 256-byte aligned");

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES];   // device address of scratch on each device (nullptr: not taken yet)

// the device address of the current device's scratch (taken on first use)
hipError_t scratch_ptr(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

namespace rtri {

// called by rtri_create with the handle's device current: takes the address
// there, so a later no-allocation call does no set-up (a failure is reported
// by that call, which tries again)
void noalloc_prepare()
{
    void *p = nullptr;
    (void)scratch_ptr(&p);
}

}  // namespace rtri

extern "C" int rtri_dtrsm_noalloc(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                                  double alpha, const double *A, int64_t lda, double *B, int64_t ldb)
{
    using namespace rtri;
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    const int rc = check_args(side, uplo, trans, diag, m, n, A, lda, B, ldb, alpha != 0.0);
    if (rc != 0)
        return rc;
    if (h->profiling)   // a profile records events created on demand
        return RTRI_ERR_UNSUPPORTED;
    if (m == 0 || n == 0)
        return RTRI_OK;
    if (alpha == 0.0) {
        const hipError_t e = launch_fill(DType::F64, B, m, n, ldb, 0.0, h->stream);
        return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
    }
    PlanIn p = plain_plan(h, DType::F64, true, side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb);
    if (plan_pack_bytes(p) > PACK_BYTES)
        return RTRI_ERR_TOO_LARGE;
    void *base = nullptr;
    const hipError_t e = scratch_ptr(&base);
    if (e != hipSuccess)
        return hip_fail(h, e);
    p.ext_pack = base;
    p.ext_split = static_cast<char *>(base) + PACK_BYTES;
    return run_plan(h, p);
}
