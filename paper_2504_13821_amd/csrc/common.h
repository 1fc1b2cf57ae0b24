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
// Diagonal blocks.  Block b covers rows / columns [b*nbmax, min((b+1)*nbmax, ka))
// of the effective matrix
//     Mx(r, c) = mtrans ? A[c + r*lda] : A[r + c*lda],
// lower-triangular when mlower, else upper.  The pack pass writes each block
// as a canonical lower triangle L, packed column by column (L(k,k) first, then
// L(k+1,k) ...; ascending columns for a solve, descending for a multiply),
// with L(i,k) = Mx(p(i), p(k)), p(i) = i (lower)
// or nb-1-i (upper); rows past the block's end and a unit diagonal become the
// identity.  Each packed block takes tri_elems(nbmax) = nbmax*(nbmax+1)/2 slots.
// ---------------------------------------------------------------------------
struct PackDesc {
    const void *A;      // A of the whole problem (element (0,0) of Mx)
    int64_t lda;
    int64_t ka;         // order of Mx
    bool mtrans, mlower, unit;
    void *out;          // nblocks * tri_elems(nbmax) elements
};

// Leaf kernel on one diagonal block against a panel of nvec independent
// vectors of length nb: element d (block order) of vector v is B[d*sd + v*si].
//   solve:     L y = alpha * b  in canonical order (y overwrites b)
//   multiply:  b := alpha * L b
struct LeafDesc {
    const void *Lp;     // this block's packed canonical triangle
    void *B;
    int64_t sd, si;
    int nb;
    int64_t nvec;
    bool mlower, unit;
    double alpha;
};

inline int64_t tri_elems(int nb) { return (int64_t)nb * (nb + 1) / 2; }

enum class DType { F64, F32 };

hipError_t launch_gemm(DType t, const GemmDesc &g, int tile, hipStream_t st);
hipError_t launch_pack(DType t, bool solve, int nbmax, const PackDesc &p, hipStream_t st);
hipError_t launch_leaf(DType t, bool solve, int nbmax, const LeafDesc &l, hipStream_t st);
hipError_t launch_fill(DType t, void *B, int64_t m, int64_t n, int64_t ldb, double value, hipStream_t st);

}  // namespace rtri
