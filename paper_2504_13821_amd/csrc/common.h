// Internal declarations shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rtri.h"

namespace rtri {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// fused multiply-add in the operand type (the untyped builtin would promote float to double)
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ---------------------------------------------------------------------------
// GEMM update:  C(MxN) = beta * C + s * op(P)(MxK) * op(Q)(KxN), column-major.
// op(P)(i,k) = tp ? P[k + i*ldp] : P[i + k*ldp]
// op(Q)(k,j) = tq ? Q[j + k*ldq] : Q[k + j*ldq]
// beta == 0 means C is written without being read.
// ---------------------------------------------------------------------------
struct GemmDesc {
    int64_t M, N, K;
    double beta, s;
    const void *P;
    int64_t ldp;
    const void *Q;
    int64_t ldq;
    void *C;
    int64_t ldc;
    bool tp, tq;
};

// ---------------------------------------------------------------------------
// Leaf kernel on one diagonal block.  The block's effective matrix is
//     Mx(r, c) = mtrans ? A[c + r*lda] : A[r + c*lda],   0 <= r, c < nb,
// lower-triangular when mlower, else upper.  The panel holds nvec independent
// vectors of length nb: element d of vector v is B[d*sd + v*si].
//   solve:     Mx y = alpha * b   (y overwrites b)
//   multiply:  b := alpha * Mx b
// ---------------------------------------------------------------------------
struct LeafDesc {
    const void *A;
    int64_t lda;
    void *B;
    int64_t sd, si;
    int nb;
    int64_t nvec;
    bool mtrans, mlower, unit;
    double alpha;
};

enum class DType { F64, F32 };

hipError_t launch_gemm(DType t, const GemmDesc &g, int tile, hipStream_t st);
hipError_t launch_leaf(DType t, bool solve, int nbmax, const LeafDesc &l, hipStream_t st);
hipError_t launch_fill(DType t, void *B, int64_t m, int64_t n, int64_t ldb, double value, hipStream_t st);

}  // namespace rtri
