// Small element-wise kernels.
#include "common.h"

namespace rtri {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(T *B, int64_t m, int64_t n, int64_t ldb, T value)
{
    const int64_t total = m * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % m, j = e / m;
        B[i + j * ldb] = value;
    }
}

}  // namespace

hipError_t launch_fill(DType t, void *B, int64_t m, int64_t n, int64_t ldb, double value, hipStream_t st)
{
    if (m <= 0 || n <= 0)
        return hipSuccess;
    const int64_t total = m * n;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    if (t == DType::F64)
        hipLaunchKernelGGL(fill_kernel<double>, dim3(blocks), dim3(256), 0, st, static_cast<double *>(B), m, n, ldb,
                           value);
    else
        hipLaunchKernelGGL(fill_kernel<float>, dim3(blocks), dim3(256), 0, st, static_cast<float *>(B), m, n, ldb,
                           (float)value);
    return hipGetLastError();
}

}  // namespace rtri
