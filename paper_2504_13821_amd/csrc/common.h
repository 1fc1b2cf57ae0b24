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
// identity.  Each packed block takes pack_elems(nbmax) slots.
// ---------------------------------------------------------------------------
struct PackDesc {
    const void *A;      // A of the whole problem (element (0,0) of Mx)
    int64_t lda;
    int64_t ka;         // order of Mx
    bool mtrans, mlower, unit;
    void *out;          // nblocks * pack_elems(nbmax) elements
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
    // ka > 0: every diagonal block of an order-ka factor in one launch
    // (matrix-core leaves only): block y covers elements [y nbmax, min((y+1)
    // nbmax, ka)); Lp and B then address block 0 and nb is ignored
    int64_t ka;
};

inline int64_t tri_elems(int nb) { return (int64_t)nb * (nb + 1) / 2; }
// Leaves of 64, 128 and 256 rows read a tiled packed form instead (see
// mleaf.hip): the 16 x 16 tiles of the lower triangle, row block by row
// block.
inline int64_t bpack_elems(int nbmax) { return (int64_t)128 * (nbmax / 16) * (nbmax / 16 + 1); }
inline int64_t pack_elems(int nbmax) { return nbmax <= 32 ? tri_elems(nbmax) : bpack_elems(nbmax); }

enum class DType { F64, F32 };
// element types of matrices in memory
enum class ElemT { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };
inline size_t elem_size(ElemT t) { return t == ElemT::F64 ? 8 : t == ElemT::F32 ? 4 : 2; }

// Split K of one FP64 / FP32 update: slices (>= 2) of kslice values along K,
// partial products in part (slices * ldpart * N elements of the panel type)
struct Split {
    int slices = 0;
    int64_t kslice = 0, ldpart = 0;
    void *part = nullptr;
};
constexpr int64_t SPLIT_MIN_K = 1024;   // shorter updates never split
// the split for an update with fewer 64x64 tiles than CUs and K >= SPLIT_MIN_K
// whose partials fit in cap bytes (slices = 0: none); part is left unset
Split plan_split(DType t, const GemmDesc &g, int tile, size_t cap);
hipError_t launch_gemm(DType t, const GemmDesc &g, int tile, hipStream_t st, const Split &sp = Split{});
// Several updates in one launch: workgroup b owns the 64x64 output tile
// tiles[b] and applies its entries (update desc, tile origin m0, n0 inside that
// update) in order, each exactly as a 64x64-tile launch of that update would.
// All updates share op flags (tp, tq); vec: every operand 16-byte aligned with
// leading dimensions a multiple of 16 bytes.  descs / ents / tiles in device memory.
struct GroupEntry {
    int desc;
    int m0, n0;
};
struct GroupTile {
    int first, count;
};
hipError_t launch_gemm_grouped(DType t, const GemmDesc *descs, const GroupEntry *ents, const GroupTile *tiles,
                               int ntiles, bool tp, bool tq, bool vec, hipStream_t st);
// 16-bit GEMM: P is 16-bit when p16 (else FP32), Q when q16 (at least one of
// them); C is FP32.  tile: 0 automatic, 1 128x128 tiles, 2 256x256 tiles where
// both operands are k-contiguous (tp && !tq) and 16-byte aligned (loaded
// straight into LDS when both are 16-bit, M and N are multiples of 256 and K
// of 32), 3 the 256x256 tiles with register-staged loads only
hipError_t launch_gemm16(bool bf16, bool p16, bool q16, const GemmDesc &g, hipStream_t st, int tile = 0);
// 16-bit updates in one launch, as launch_gemm_grouped with 256x256 tiles:
// every update 16-bit in both operands, tp && !tq, 16-byte aligned operands
// with leading dimensions a multiple of 8, tile origins multiples of 256.
// tiles_dma: full tiles whose entries all have beta = 1, one scale s and K a
// multiple of 32 (one accumulator, operands loaded straight into LDS); tiles:
// the rest (a launch of its own after the first)
hipError_t launch_gemm16_grouped(bool bf16, const GemmDesc *descs, const GroupEntry *ents, const GroupTile *tiles_dma,
                                 int n_dma, const GroupTile *tiles, int ntiles, hipStream_t st);
// pack diagonal blocks read from A of type src into packed triangles of type dst
hipError_t launch_pack(ElemT src, DType dst, bool solve, int nbmax, const PackDesc &p, hipStream_t st);
hipError_t launch_leaf(DType t, bool solve, int nbmax, const LeafDesc &l, hipStream_t st);
// matrix-core leaves (nbmax = 64, 128 or 256, mleaf.hip), called by launch_pack / launch_leaf
hipError_t launch_bpack(ElemT src, DType dst, bool solve, int nbmax, const PackDesc &p, hipStream_t st);
hipError_t launch_bleaf(DType t, bool solve, int nbmax, const LeafDesc &l, hipStream_t st);
// the leaf variants behind launch_bleaf, one translation unit each
hipError_t mleaf_launch_f64_solve(int nbmax, const LeafDesc &l, hipStream_t st);
hipError_t mleaf_launch_f64_mult(int nbmax, const LeafDesc &l, hipStream_t st);
hipError_t mleaf_launch_f32_solve(int nbmax, const LeafDesc &l, hipStream_t st);
hipError_t mleaf_launch_f32_mult(int nbmax, const LeafDesc &l, hipStream_t st);
hipError_t launch_fill(DType t, void *B, int64_t m, int64_t n, int64_t ldb, double value, hipStream_t st);

// ---- element-wise kernels (HBM-bound) ----
// Y = fl_dst(scale * X) for an m-by-n matrix (round to nearest even; FP64 -> BF16
// is rounded once, not through FP32)
hipError_t launch_convert(ElemT src, ElemT dst, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t m,
                          int64_t n, double scale, hipStream_t st);
// Y = fl_dst(X^T): X is m-by-n FP64, Y is n-by-m (rounded once, as launch_convert)
hipError_t launch_transpose_convert(ElemT dst, const double *X, int64_t ldx, void *Y, int64_t ldy, int64_t m,
                                    int64_t n, hipStream_t st);
// Y = X^T for 16-bit X (m-by-n) and Y (n-by-m), bit patterns copied
hipError_t launch_transpose16(const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t m, int64_t n, hipStream_t st);
// X += s * D, or X = s * D when assign (X is then not read)   (X FP64, D FP32);
// then W = X when W != nullptr
hipError_t launch_add_scaled(double *X, int64_t ldx, const float *D, int64_t ldd, int64_t m, int64_t n, double s,
                             bool assign, double *W, int64_t ldw, hipStream_t st);
// Refinement bookkeeping.  Vectors are columns (by_cols) or rows of the m-by-n
// matrices.  R = R0 - W; per vector v: eta_v = |R_v|inf / (anorm |X_v|inf + |R0_v|inf);
// out[0] = max_v eta_v, out[1] = max |R| (both as ordered bit patterns of
// non-negative doubles, combined with atomicMax; NaN propagates as +NaN bits).
hipError_t launch_resid_eta(const double *R0, int64_t ld0, const double *W, int64_t ldw, double *R, int64_t ldr,
                            const double *X, int64_t ldx, int64_t m, int64_t n, bool by_cols, double anorm,
                            unsigned long long *out, hipStream_t st);
// out[0] = max over lines of sum |Mx(line, k)| with Mx as in PackDesc (unit diagonal counts 1)
hipError_t launch_line_norm(const double *A, int64_t lda, int64_t ka, bool mtrans, bool mlower, bool unit,
                            unsigned long long *out, hipStream_t st);
// out[0] = max |X|
hipError_t launch_max_abs(const double *X, int64_t ldx, int64_t m, int64_t n, unsigned long long *out,
                          hipStream_t st);
hipError_t launch_zero_u64(unsigned long long *p, int count, hipStream_t st);

}  // namespace rtri
