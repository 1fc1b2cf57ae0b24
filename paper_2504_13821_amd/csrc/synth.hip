// Synthetic inputs generated on the device (benchmark and serving workloads).
// Not part of the method: it only draws numbers.  Philox4x32-10 (Salmon,
// Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11):
// 10 rounds of two 32x32->64 multiplies with the published multipliers and
// key increments.  Element (i, j) of a matrix uses counter (i, j, id_lo, id_hi)
// and key (seed_lo ^ stream, seed_hi); its value takes the first two output
// words as one 53-bit uniform u in [0, 1).
#include "handle.h"

using namespace rtri;

namespace {

struct U4 {
    unsigned x, y, z, w;
};

__device__ __forceinline__ U4 philox(U4 c, unsigned k0, unsigned k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
        const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
        const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// kind: 0 dense U(-1,1); 1 lower, 2 upper triangular with off-diagonal
// U(-1,1), diagonal param + U(0,1), zero outside the triangle
template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(int kind, unsigned long long seed, unsigned stream,
                                                   unsigned long long id, int64_t m, int64_t n, double param, T *X,
                                                   int64_t ldx)
{
    const int64_t total = m * n;
    const unsigned k0 = (unsigned)seed ^ stream, k1 = (unsigned)(seed >> 32);
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % m, j = e / m;
        double v;
        const bool in_tri = kind == 0 || (kind == 1 ? i >= j : i <= j);
        if (!in_tri) {
            v = 0.0;
        } else {
            const U4 r = philox(U4{(unsigned)i, (unsigned)j, (unsigned)id, (unsigned)(id >> 32)}, k0, k1);
            const unsigned long long bits = ((unsigned long long)r.y << 32 | r.x) >> 11;
            const double u = (double)bits * 0x1.0p-53;
            v = (kind != 0 && i == j) ? param + u : 2.0 * u - 1.0;
        }
        X[i + j * ldx] = (T)v;
    }
}

}  // namespace

extern "C" int rtri_synth_fill(rtri_handle *h, int dtype, int kind, uint64_t seed, uint32_t stream, uint64_t id,
                               int64_t m, int64_t n, double param, void *X, int64_t ldx)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (dtype != RTRI_F64 && dtype != RTRI_F32)
        return -2;
    if (kind < 0 || kind > 2)
        return -3;
    if (m < 0 || n < 0)
        return -7;
    if (ldx < std::max<int64_t>(1, m))
        return -11;
    if (m == 0 || n == 0)
        return RTRI_OK;
    if (X == nullptr)
        return -10;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((m * n + 255) / 256, 8192));
    if (dtype == RTRI_F64)
        hipLaunchKernelGGL(fill_kernel<double>, dim3(grid), dim3(256), 0, h->stream, kind, (unsigned long long)seed,
                           stream, (unsigned long long)id, m, n, param, static_cast<double *>(X), ldx);
    else
        hipLaunchKernelGGL(fill_kernel<float>, dim3(grid), dim3(256), 0, h->stream, kind, (unsigned long long)seed,
                           stream, (unsigned long long)id, m, n, param, static_cast<float *>(X), ldx);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
}
