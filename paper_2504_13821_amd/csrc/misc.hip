// Element-wise kernels: fills, precision conversions, and the bookkeeping of
// the mixed-precision refinement (correction update, residual, norms).  All of
// them are bound by HBM bandwidth.  Matrix kernels use a 2-D grid (x: chunks of
// 4 x 256 rows, y: columns, striding when there are more columns than grid
// rows), so consecutive threads touch consecutive addresses and no thread
// divides indices.
#include "common.h"

namespace rtri {

namespace {

constexpr int NT = 256;

constexpr int RPT = 4;   // rows per thread of a matrix kernel

dim3 grid2d(int64_t m, int64_t n)
{
    return dim3((unsigned)((m + NT * RPT - 1) / (NT * RPT)), (unsigned)std::min<int64_t>(n, 65535));
}

// f(i, j) for every element of an m-by-n matrix (launched with grid2d)
template <class F> __device__ __forceinline__ void for_each_2d(int64_t m, int64_t n, F &&f)
{
    const int64_t i0 = (int64_t)blockIdx.x * (NT * RPT) + threadIdx.x;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            const int64_t i = i0 + t * NT;
            if (i < m)
                f(i, j);
        }
}

template <typename T>
__global__ __launch_bounds__(NT) void fill_kernel(T *B, int64_t m, int64_t n, int64_t ldb, T value)
{
    for_each_2d(m, n, [&](int64_t i, int64_t j) { B[i + j * ldb] = value; });
}

// ---- conversions ----

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float x)
{
    const unsigned u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return (unsigned short)((u >> 16) | 0x40u);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// FP64 -> FP32 rounded to odd: truncate, then set the last bit if anything was
// dropped.  A second rounding (to nearest even) to a format at least two bits
// narrower then equals a single correct rounding of the FP64 value.
__device__ __forceinline__ float f64_to_f32_odd(double x)
{
    float r = __double2float_rz(x);
    if ((double)r != x && x == x)
        r = __uint_as_float(__float_as_uint(r) | 1u);
    return r;
}

template <ElemT S> __device__ __forceinline__ double load_as_f64(const void *p, int64_t off);
template <> __device__ __forceinline__ double load_as_f64<ElemT::F64>(const void *p, int64_t off)
{
    return static_cast<const double *>(p)[off];
}
template <> __device__ __forceinline__ double load_as_f64<ElemT::F32>(const void *p, int64_t off)
{
    return static_cast<const float *>(p)[off];
}
template <> __device__ __forceinline__ double load_as_f64<ElemT::BF16>(const void *p, int64_t off)
{
    return __uint_as_float((unsigned)static_cast<const unsigned short *>(p)[off] << 16);
}
template <> __device__ __forceinline__ double load_as_f64<ElemT::F16>(const void *p, int64_t off)
{
    return (double)__builtin_bit_cast(_Float16, static_cast<const unsigned short *>(p)[off]);
}

template <ElemT D> __device__ __forceinline__ void store_from_f64(void *p, int64_t off, double v);
template <> __device__ __forceinline__ void store_from_f64<ElemT::F64>(void *p, int64_t off, double v)
{
    static_cast<double *>(p)[off] = v;
}
template <> __device__ __forceinline__ void store_from_f64<ElemT::F32>(void *p, int64_t off, double v)
{
    static_cast<float *>(p)[off] = (float)v;
}
template <> __device__ __forceinline__ void store_from_f64<ElemT::BF16>(void *p, int64_t off, double v)
{
    static_cast<unsigned short *>(p)[off] = f32_to_bf16_rne(f64_to_f32_odd(v));
}
template <> __device__ __forceinline__ void store_from_f64<ElemT::F16>(void *p, int64_t off, double v)
{
    const _Float16 h = (_Float16)f64_to_f32_odd(v);
    static_cast<unsigned short *>(p)[off] = __builtin_bit_cast(unsigned short, h);
}

// every value of the 16-bit and FP32 formats is exact in FP64 and the scale is a
// power of two or 1 at every call site, so going through FP64 adds no rounding
template <ElemT S, ElemT D>
__global__ __launch_bounds__(NT) void convert_kernel(const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t m,
                                                     int64_t n, double scale)
{
    for_each_2d(m, n, [&](int64_t i, int64_t j) {
        const double v = load_as_f64<S>(X, i + j * ldx);
        store_from_f64<D>(Y, i + j * ldy, scale == 1.0 ? v : scale * v);
    });
}

// Y = fl_D(X^T): X m-by-n FP64, Y n-by-m.  32x32 tiles pass through LDS so
// both the reads of X and the writes of Y are contiguous along columns.
template <ElemT D>
__global__ __launch_bounds__(NT) void transpose_convert_kernel(const double *X, int64_t ldx, void *Y, int64_t ldy,
                                                               int64_t m, int64_t n)
{
    __shared__ double t[32][33];
    const int64_t tiles_m = (m + 31) / 32;
    const int64_t i0 = (blockIdx.x % tiles_m) * 32, j0 = (blockIdx.x / tiles_m) * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 8 rows of threads
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = i0 + tx, j = j0 + r;
        t[r][tx] = (i < m && j < n) ? X[i + j * ldx] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t yi = j0 + tx, yj = i0 + r;   // Y(yi, yj) = X(yj, yi)
        if (yi < n && yj < m)
            store_from_f64<D>(Y, yi + yj * ldy, t[tx][r]);
    }
}

// Y = X^T for 16-bit X (m-by-n) and Y (n-by-m), through 32x32 LDS tiles as above
__global__ __launch_bounds__(NT) void transpose16_kernel(const unsigned short *X, int64_t ldx, unsigned short *Y,
                                                         int64_t ldy, int64_t m, int64_t n)
{
    __shared__ unsigned short t[32][33];
    const int64_t tiles_m = (m + 31) / 32;
    const int64_t i0 = (blockIdx.x % tiles_m) * 32, j0 = (blockIdx.x / tiles_m) * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = i0 + tx, j = j0 + r;
        t[r][tx] = (i < m && j < n) ? X[i + j * ldx] : (unsigned short)0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t yi = j0 + tx, yj = i0 + r;
        if (yi < n && yj < m)
            Y[yi + yj * ldy] = t[tx][r];
    }
}

template <ElemT S>
hipError_t convert_from(ElemT dst, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t m, int64_t n,
                        double scale, hipStream_t st)
{
    const dim3 g = grid2d(m, n);
    switch (dst) {
    case ElemT::F64: hipLaunchKernelGGL((convert_kernel<S, ElemT::F64>), g, dim3(NT), 0, st, X, ldx, Y, ldy, m, n, scale); break;
    case ElemT::F32: hipLaunchKernelGGL((convert_kernel<S, ElemT::F32>), g, dim3(NT), 0, st, X, ldx, Y, ldy, m, n, scale); break;
    case ElemT::BF16: hipLaunchKernelGGL((convert_kernel<S, ElemT::BF16>), g, dim3(NT), 0, st, X, ldx, Y, ldy, m, n, scale); break;
    case ElemT::F16: hipLaunchKernelGGL((convert_kernel<S, ElemT::F16>), g, dim3(NT), 0, st, X, ldx, Y, ldy, m, n, scale); break;
    }
    return hipGetLastError();
}

// ---- refinement bookkeeping ----

__device__ __forceinline__ unsigned long long ordered_bits(double v)
{
    // non-negative doubles order like their bit patterns; NaN maps above +inf
    return v != v ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(v);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, 64);
        v = (w > v || w != w) ? w : v;
    }
    return v;
}

__device__ __forceinline__ double nmax(double a, double b) { return (b > a || b != b) ? b : a; }

// butterfly sum over the wavefront (the same fixed order on every run)
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// max over a 256-thread workgroup; the result is valid in thread 0
__device__ __forceinline__ double block_max(double v, double *red)
{
    v = wave_max(v);
    if (threadIdx.x % 64 == 0)
        red[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        v = nmax(nmax(red[0], red[1]), nmax(red[2], red[3]));
    return v;
}

// grid of a reduction over an m-by-n matrix: about REDUCE_BLOCKS workgroups,
// so that each adds one atomic on the result (columns stride over grid rows)
constexpr int64_t REDUCE_BLOCKS = 2048;

dim3 grid2d_reduce(int64_t m, int64_t n)
{
    const int64_t gx = (m + NT * RPT - 1) / (NT * RPT);
    const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(n, REDUCE_BLOCKS / std::max<int64_t>(gx, 1)));
    return dim3((unsigned)gx, (unsigned)std::min<int64_t>(gy, 65535));
}

// X += s * D (X = s * D when assign: X is not read), and W = X when W is given
__global__ __launch_bounds__(NT) void add_scaled_kernel(double *X, int64_t ldx, const float *D, int64_t ldd, int64_t m,
                                                        int64_t n, double s, bool assign, double *W, int64_t ldw)
{
    for_each_2d(m, n, [&](int64_t i, int64_t j) {
        const double d = s * (double)D[i + j * ldd];
        const double x = assign ? d : X[i + j * ldx] + d;
        X[i + j * ldx] = x;
        if (W != nullptr)
            W[i + j * ldw] = x;
    });
}

// Vectors are columns.  Each wavefront takes columns j = w, w + W, ... (W
// wavefronts in the grid), its lanes running down the rows four loads deep;
// the workgroup's largest eta and |r| then go to memory in one atomic each.
__global__ __launch_bounds__(NT) void resid_cols_kernel(const double *R0, int64_t ld0, const double *W, int64_t ldw,
                                                        double *R, int64_t ldr, const double *X, int64_t ldx,
                                                        int64_t m, int64_t n, double anorm, unsigned long long *out)
{
    __shared__ double red[NT / 64];
    const int lane = threadIdx.x % 64;
    const int64_t nw = (int64_t)gridDim.x * (NT / 64);
    double eta_w = 0.0, rn_w = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * (NT / 64) + threadIdx.x / 64; j < n; j += nw) {
        const double *r0 = R0 + j * ld0, *w = W + j * ldw, *x = X + j * ldx;
        double *r = R + j * ldr;
        double rn = 0.0, xn = 0.0, bn = 0.0;
        for (int64_t i0 = lane; i0 < m; i0 += 4 * 64) {
            double b[4], wv[4], xv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t i = i0 + t * 64;
                b[t] = i < m ? r0[i] : 0.0;
                wv[t] = i < m ? w[i] : 0.0;
                xv[t] = i < m ? x[i] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t i = i0 + t * 64;
                const double rv = b[t] - wv[t];
                if (i < m)
                    r[i] = rv;
                rn = nmax(rn, fabs(rv));
                xn = nmax(xn, fabs(xv[t]));
                bn = nmax(bn, fabs(b[t]));
            }
        }
        rn = wave_max(rn);
        xn = wave_max(xn);
        bn = wave_max(bn);
        const double den = anorm * xn + bn;
        const double eta = den > 0.0 ? rn / den : (rn > 0.0 ? __builtin_inf() : (rn != rn ? rn : 0.0));
        eta_w = nmax(eta_w, eta);
        rn_w = nmax(rn_w, rn);
    }
    eta_w = block_max(eta_w, red);
    __syncthreads();
    rn_w = block_max(rn_w, red);
    if (threadIdx.x == 0) {
        atomicMax(out, ordered_bits(eta_w));
        atomicMax(out + 1, ordered_bits(rn_w));
    }
}

// Vectors are rows.  A workgroup of RESID_ROWS_NT threads takes 32 rows; its
// 32 row groups of threads split the columns (thread (r, q) reads columns
// q, q + 32, ...), so each load instruction of a wavefront reads two 256-byte
// column segments.  The partial maxima of a row are combined in LDS.
constexpr int RESID_ROWS_NT = 1024;
constexpr int RESID_ROWS = 32;

__global__ __launch_bounds__(RESID_ROWS_NT) void resid_rows_kernel(const double *R0, int64_t ld0, const double *W,
                                                                   int64_t ldw, double *R, int64_t ldr,
                                                                   const double *X, int64_t ldx, int64_t m, int64_t n,
                                                                   double anorm, unsigned long long *out)
{
    constexpr int NQ = RESID_ROWS_NT / RESID_ROWS;
    __shared__ double prn[RESID_ROWS_NT], pxn[RESID_ROWS_NT], pbn[RESID_ROWS_NT];
    const int r = threadIdx.x % RESID_ROWS, q = threadIdx.x / RESID_ROWS;
    const int64_t i = (int64_t)blockIdx.x * RESID_ROWS + r;
    double rn = 0.0, xn = 0.0, bn = 0.0;
    if (i < m) {
#pragma unroll 4
        for (int64_t j = q; j < n; j += NQ) {
            const double b = R0[i + j * ld0];
            const double rv = b - W[i + j * ldw];
            R[i + j * ldr] = rv;
            rn = nmax(rn, fabs(rv));
            xn = nmax(xn, fabs(X[i + j * ldx]));
            bn = nmax(bn, fabs(b));
        }
    }
    prn[threadIdx.x] = rn;
    pxn[threadIdx.x] = xn;
    pbn[threadIdx.x] = bn;
    __syncthreads();
    if (threadIdx.x < 64) {
        double eta = 0.0;
        rn = 0.0;
        if (threadIdx.x < RESID_ROWS && i < m) {
            xn = bn = 0.0;
            for (int k = 0; k < NQ; ++k) {
                rn = nmax(rn, prn[r + k * RESID_ROWS]);
                xn = nmax(xn, pxn[r + k * RESID_ROWS]);
                bn = nmax(bn, pbn[r + k * RESID_ROWS]);
            }
            const double den = anorm * xn + bn;
            eta = den > 0.0 ? rn / den : (rn > 0.0 ? __builtin_inf() : (rn != rn ? rn : 0.0));
        }
        eta = wave_max(eta);
        rn = wave_max(rn);
        if (threadIdx.x == 0) {
            atomicMax(out, ordered_bits(eta));
            atomicMax(out + 1, ordered_bits(rn));
        }
    }
}

// Line sums s_i = sum_k |M(i, k)| over the referenced part of line i, then
// their maximum.  M(i, k) = A[i + k*lda] (lines are rows of A) or, with
// mtrans, A[k + i*lda] (lines are columns); the referenced part is k <= i
// (mlower) or k >= i, and a unit diagonal counts as 1 without being read.
// A workgroup takes 16 lines.  Rows: thread (r, q) sums line r over
// k = k0 + q, k0 + q + 16, ... (each load instruction reads 128-byte row
// segments of four columns).  Columns: each wavefront sums four lines in turn,
// its lanes along k.  Partials are combined in a fixed order.
constexpr int NORM_LINES = 16;

__global__ __launch_bounds__(NT) void line_norm_kernel(const double *A, int64_t lda, int64_t ka, bool mtrans,
                                                       bool mlower, bool unit, unsigned long long *out)
{
    __shared__ double part[NT];
    const int tid = threadIdx.x;
    const int64_t l0 = (int64_t)blockIdx.x * NORM_LINES;
    if (!mtrans) {
        constexpr int NQ = NT / NORM_LINES;
        const int r = tid % NORM_LINES, q = tid / NORM_LINES;
        const int64_t i = l0 + r;
        double s = 0.0;
        if (i < ka) {
            const int64_t k0 = mlower ? 0 : i, k1 = mlower ? i : ka - 1;   // inclusive
#pragma unroll 4
            for (int64_t k = k0 + q; k <= k1; k += NQ)
                s += (k == i && unit) ? 1.0 : fabs(A[i + k * lda]);
        }
        part[tid] = s;
        __syncthreads();
        if (tid < NORM_LINES) {
            double v = 0.0;
            for (int k = 0; k < NQ; ++k)
                v += part[tid + k * NORM_LINES];
            part[tid] = v;   // only this thread reads slot tid < 16 from here on
        }
    } else {
        const int w = tid / 64, lane = tid % 64;
        constexpr int PER_WAVE = NORM_LINES / (NT / 64);
        for (int c = 0; c < PER_WAVE; ++c) {
            const int64_t i = l0 + w * PER_WAVE + c;
            double s = 0.0;
            if (i < ka) {
                const int64_t k0 = mlower ? 0 : i, k1 = mlower ? i : ka - 1;
                const double *col = A + i * lda;
#pragma unroll 4
                for (int64_t k = k0 + lane; k <= k1; k += 64)
                    s += (k == i && unit) ? 1.0 : fabs(col[k]);
            }
            s = wave_sum(s);
            if (lane == 0)
                part[w * PER_WAVE + c] = s;
        }
    }
    __syncthreads();
    if (tid < 64) {
        double v = tid < NORM_LINES ? part[tid] : 0.0;
        v = wave_max(v);
        if (tid == 0)
            atomicMax(out, ordered_bits(v));
    }
}

// launched on grid2d_reduce: one atomic per workgroup
__global__ __launch_bounds__(NT) void max_abs_kernel(const double *X, int64_t ldx, int64_t m, int64_t n,
                                                     unsigned long long *out)
{
    __shared__ double red[NT / 64];
    double v = 0.0;
    for_each_2d(m, n, [&](int64_t i, int64_t j) { v = nmax(v, fabs(X[i + j * ldx])); });
    v = block_max(v, red);
    if (threadIdx.x == 0)
        atomicMax(out, ordered_bits(v));
}

__global__ void zero_u64_kernel(unsigned long long *p, int count)
{
    for (int i = threadIdx.x; i < count; i += blockDim.x)
        p[i] = 0ull;
}

}  // namespace

hipError_t launch_fill(DType t, void *B, int64_t m, int64_t n, int64_t ldb, double value, hipStream_t st)
{
    if (m <= 0 || n <= 0)
        return hipSuccess;
    const dim3 g = grid2d(m, n);
    if (t == DType::F64)
        hipLaunchKernelGGL(fill_kernel<double>, g, dim3(NT), 0, st, static_cast<double *>(B), m, n, ldb, value);
    else
        hipLaunchKernelGGL(fill_kernel<float>, g, dim3(NT), 0, st, static_cast<float *>(B), m, n, ldb, (float)value);
    return hipGetLastError();
}

hipError_t launch_convert(ElemT src, ElemT dst, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t m,
                          int64_t n, double scale, hipStream_t st)
{
    if (m <= 0 || n <= 0)
        return hipSuccess;
    switch (src) {
    case ElemT::F64: return convert_from<ElemT::F64>(dst, X, ldx, Y, ldy, m, n, scale, st);
    case ElemT::F32: return convert_from<ElemT::F32>(dst, X, ldx, Y, ldy, m, n, scale, st);
    case ElemT::BF16: return convert_from<ElemT::BF16>(dst, X, ldx, Y, ldy, m, n, scale, st);
    case ElemT::F16: return convert_from<ElemT::F16>(dst, X, ldx, Y, ldy, m, n, scale, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_transpose_convert(ElemT dst, const double *X, int64_t ldx, void *Y, int64_t ldy, int64_t m,
                                    int64_t n, hipStream_t st)
{
    if (m <= 0 || n <= 0)
        return hipSuccess;
    const int64_t tiles = ((m + 31) / 32) * ((n + 31) / 32);
    if (tiles > INT32_MAX)
        return hipErrorInvalidValue;
    const dim3 g((unsigned)tiles);
    switch (dst) {
    case ElemT::F64: hipLaunchKernelGGL((transpose_convert_kernel<ElemT::F64>), g, dim3(NT), 0, st, X, ldx, Y, ldy, m, n); break;
    case ElemT::F32: hipLaunchKernelGGL((transpose_convert_kernel<ElemT::F32>), g, dim3(NT), 0, st, X, ldx, Y, ldy, m, n); break;
    case ElemT::BF16: hipLaunchKernelGGL((transpose_convert_kernel<ElemT::BF16>), g, dim3(NT), 0, st, X, ldx, Y, ldy, m, n); break;
    case ElemT::F16: hipLaunchKernelGGL((transpose_convert_kernel<ElemT::F16>), g, dim3(NT), 0, st, X, ldx, Y, ldy, m, n); break;
    }
    return hipGetLastError();
}

hipError_t launch_transpose16(const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t m, int64_t n, hipStream_t st)
{
    if (m <= 0 || n <= 0)
        return hipSuccess;
    const int64_t tiles = ((m + 31) / 32) * ((n + 31) / 32);
    if (tiles > INT32_MAX)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(transpose16_kernel, dim3((unsigned)tiles), dim3(NT), 0, st,
                       static_cast<const unsigned short *>(X), ldx, static_cast<unsigned short *>(Y), ldy, m, n);
    return hipGetLastError();
}

hipError_t launch_add_scaled(double *X, int64_t ldx, const float *D, int64_t ldd, int64_t m, int64_t n, double s,
                             bool assign, double *W, int64_t ldw, hipStream_t st)
{
    if (m <= 0 || n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(add_scaled_kernel, grid2d(m, n), dim3(NT), 0, st, X, ldx, D, ldd, m, n, s, assign, W, ldw);
    return hipGetLastError();
}

hipError_t launch_resid_eta(const double *R0, int64_t ld0, const double *W, int64_t ldw, double *R, int64_t ldr,
                            const double *X, int64_t ldx, int64_t m, int64_t n, bool by_cols, double anorm,
                            unsigned long long *out, hipStream_t st)
{
    if (m <= 0 || n <= 0)
        return hipSuccess;
    if (by_cols) {
        const int64_t blocks = std::min<int64_t>((n + NT / 64 - 1) / (NT / 64), REDUCE_BLOCKS);
        hipLaunchKernelGGL(resid_cols_kernel, dim3((unsigned)blocks), dim3(NT), 0, st, R0, ld0, W, ldw, R, ldr, X,
                           ldx, m, n, anorm, out);
    } else {
        const int64_t blocks = (m + RESID_ROWS - 1) / RESID_ROWS;
        if (blocks > INT32_MAX)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(resid_rows_kernel, dim3((unsigned)blocks), dim3(RESID_ROWS_NT), 0, st, R0, ld0, W, ldw,
                           R, ldr, X, ldx, m, n, anorm, out);
    }
    return hipGetLastError();
}

hipError_t launch_line_norm(const double *A, int64_t lda, int64_t ka, bool mtrans, bool mlower, bool unit,
                            unsigned long long *out, hipStream_t st)
{
    if (ka <= 0)
        return hipSuccess;
    const int64_t blocks = (ka + NORM_LINES - 1) / NORM_LINES;
    if (blocks > INT32_MAX)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(line_norm_kernel, dim3((unsigned)blocks), dim3(NT), 0, st, A, lda, ka, mtrans, mlower, unit,
                       out);
    return hipGetLastError();
}

hipError_t launch_max_abs(const double *X, int64_t ldx, int64_t m, int64_t n, unsigned long long *out,
                          hipStream_t st)
{
    if (m <= 0 || n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(max_abs_kernel, grid2d_reduce(m, n), dim3(NT), 0, st, X, ldx, m, n, out);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int count, hipStream_t st)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, p, count);
    return hipGetLastError();
}

}  // namespace rtri
