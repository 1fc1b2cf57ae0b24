// Direct-to-LDS K loop of a 256x256 output tile on the matrix cores, shared
// by the 16-bit GEMM and the INT8 GEMM of the INT8-product residual.
//
// Both operands are k-contiguous lines in memory (rows of op(P), columns of
// op(Q)), 16-byte aligned, with leading dimensions a multiple of 16 bytes; a
// k-step is 64 bytes of k per line (32 16-bit values or 64 bytes), two MFMA
// sub-steps of 32 bytes.  The operand tiles go from memory straight into LDS
// (global_load_lds, 16 bytes per lane: a wavefront's instruction fills 1 KB
// of LDS, lane l at byte 16 l) with no register stage and no LDS store
// instructions, in four LDS stages: the loads of k-step kt + 3 are issued
// while step kt multiplies.  A stage line is 64 bytes (four 16-byte chunks);
// chunk c of line r sits at slot c ^ sw(r), sw(r) = r2 | (r1 ^ r3) << 1 (ri:
// bit i of r), so the fragment reads of 16 consecutive lines cover the 256
// bytes of the 64 banks once each, and those of 8 consecutive lines 128
// distinct bytes (each lane loads the chunk that belongs at its slot).  With
// sw(r) = (r >> 1) & 3 (distinct over 8 lines only) the counters showed a
// 2-way conflict on every fragment read.  Past the last k-step the last stage is
// loaded again into the stage just freed (never read), so every step waits
// for the same count of loads; the compiler's wait-count pass then keeps the
// three younger stages in flight (with a count that depended on the step, or
// a segment switch inside the pipeline, it waited for all of them).  Each
// step reads all its fragments first, then multiplies.
//
// Workgroup: 512 threads, eight wavefronts in a 2 x 4 grid of 128 x 64
// blocks, each 4 x 2 blocks of 32 x 32 MFMA tiles.  32 x 32 MFMA operand
// layout (lane l, h = l / 32, c = l % 32): A operand line c, bytes 16 h ..
// 16 h + 15 of the sub-step; B operand likewise.
#pragma once

#include "common.h"

namespace rtri {
namespace dma {

constexpr int TW = 256;                 // tile lines (rows and columns)
constexpr int NTW = 512;                // threads per workgroup
constexpr int LINE = 64;                // bytes of k per line and k-step
constexpr int STGB = TW * LINE;         // bytes per operand and stage

// slot swizzle of line r (see above)
__device__ __forceinline__ int swz(int r) { return ((r >> 2) & 1) | (((r >> 1) ^ (r >> 3)) & 1) << 1; }
typedef int v4i __attribute__((ext_vector_type(4)));   // 16 bytes

typedef __attribute__((address_space(3))) void lds_t;
typedef const __attribute__((address_space(1))) void gbl_t;

// The four stages (A at [0, STGB), B at [STGB, 2 STGB)) are distinct LDS
// arrays, so the compiler's wait-count pass can tell them apart.
#define RTRI_DMA_STAGES                                                                 \
    __shared__ __attribute__((aligned(1024))) char S0[2 * rtri::dma::STGB];            \
    __shared__ __attribute__((aligned(1024))) char S1[2 * rtri::dma::STGB];            \
    __shared__ __attribute__((aligned(1024))) char S2[2 * rtri::dma::STGB];            \
    __shared__ __attribute__((aligned(1024))) char S3[2 * rtri::dma::STGB]

// acc += op(P) op(Q) over nk k-steps for one K segment: P, Q the byte
// addresses of the tile's first line at its first k, ldp, ldq line strides
// in bytes; mma(a, b, c) one 32 x 32 MFMA on 16-byte fragments.  Steps go in
// straight-line groups of four (a remainder of up to three after them).
// Ends with no load in flight and a barrier, so the stages may be refilled.
template <class Acc, class Mma>
__device__ __forceinline__ void k_seg(const char *P, const char *Q, int64_t ldp, int64_t ldq, int nk,
                                      Acc (&acc)[4][2], char *S0, char *S1, char *S2, char *S3, Mma &&mma)
{
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int lr = lane & 31, lh = lane >> 5;
    if (nk <= 0)
        return;
    // this lane's loads: instruction i fills LDS lines 16 (8 i + wave) ..+15,
    // lane l line 16 (8 i + wave) + l / 4, slot l % 4
    const char *pa[2], *pb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int line = 16 * (8 * i + wave) + (lane >> 2);
        const int chk = ((lane & 3) ^ swz(line)) * 16;
        pa[i] = P + line * ldp + chk;
        pb[i] = Q + line * ldq + chk;
    }
    auto issue = [&](int kt, char *S) {
        const int64_t k0 = (int64_t)kt * LINE;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int seg = 8 * i + wave;
            __builtin_amdgcn_global_load_lds((gbl_t *)(pa[i] + k0), (lds_t *)(S + seg * 1024), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((gbl_t *)(pb[i] + k0), (lds_t *)(S + STGB + seg * 1024), 16, 0, 0);
        }
    };
    const int sw = swz(lr);   // fragment lines start at multiples of 32
    auto compute = [&](const char *S) {
        v4i fa[2][4], fb[2][2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int ch = ((2 * ks + lh) ^ sw) * 16;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                fa[ks][i] = *reinterpret_cast<const v4i *>(S + (wm * 128 + i * 32 + lr) * LINE + ch);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                fb[ks][j] = *reinterpret_cast<const v4i *>(S + STGB + (wn * 64 + j * 32 + lr) * LINE + ch);
        }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = mma(fa[ks][i], fb[ks][j], acc[i][j]);
        __builtin_amdgcn_sched_group_barrier(0x100, 12, 0);   // the LDS reads first
        __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);   // then the MFMAs
    };
    // step kt: its stage has landed (the three younger ones may be in flight),
    // every wavefront is done with the stage refilled now (step kt - 1's)
    auto step = [&](int kt, const char *Sc, char *Sn) {
        __builtin_amdgcn_s_waitcnt(0x0F78);   // vmcnt(8): 4 loads per stage per lane
        __builtin_amdgcn_s_barrier();
        issue(min(kt + 3, nk - 1), Sn);
        compute(Sc);
    };
    issue(0, S0);
    issue(min(1, nk - 1), S1);
    issue(min(2, nk - 1), S2);
    const int n4 = nk & ~3;
    for (int kt = 0; kt < n4; kt += 4) {
        step(kt, S0, S3);
        step(kt + 1, S1, S0);
        step(kt + 2, S2, S1);
        step(kt + 3, S3, S2);
    }
    if (n4 < nk)
        step(n4, S0, S3);
    if (n4 + 1 < nk)
        step(n4 + 1, S1, S0);
    if (n4 + 2 < nk)
        step(n4 + 2, S2, S1);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): no LDS write in flight past this point
    __builtin_amdgcn_s_barrier();
}

}  // namespace dma
}  // namespace rtri
