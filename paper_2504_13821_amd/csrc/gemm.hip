// GEMM update of the recursion (paper, Sec. 3.1: nearly all flops of the
// recursive TRMM / TRSM land in one GEMM per level):
//     C(MxN) = beta * C + s * op(P)(MxK) * op(Q)(KxN),   column-major
//
// CDNA4 design: 256-thread workgroups (4 wavefronts in a 2x2 grid), each
// wavefront owns a WMxWN block of C held in MFMA accumulators and built from
// 16x16 MFMA blocks (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32).  Operand
// tiles of BK values along K are staged through LDS with a two-slot ring so the
// global loads of step k+1 overlap the MFMAs of step k; each tile keeps its
// global layout in LDS (padded), so the copy is a straight coalesced move.
//
// MFMA 16x16x4 operand layout (lane l, g = l/16, c = l%16):
//   A operand: A[c][g]   B operand: B[g][c]
//   D: slot r (0..3) of the lane holds D[4g + r][c] (FP32) or D[g + 4r][c] (FP64)
// Within a BK = 16 step, MFMA number t (t = 0..3) of a wavefront feeds lane group
// g with k = 4g + t: any consistent assignment of k between the two operands
// gives the same sum, and this one lets each lane fetch its four k values of a
// row with 16-byte LDS reads.
#include "gemm_core.h"

namespace rtri {

namespace {

using namespace gk;

// Workgroup tile BM x BN; WM x WN wavefronts, each a (BM/WM) x (BN/WN) block
// made of 16 x 16 MFMA blocks.
// Two workgroups per CU: 2 wavefronts per SIMD with 4-wavefront tiles, 4 with
// 8-wavefront tiles (at most 128 registers each).
template <typename T, int BM, int BN, bool TP, bool TQ, bool VEC, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(WM * WN / 2))) void
gemm_kernel(GemmDesc g, int tiles_m, int tiles_n)
{
    constexpr bool KCA = TP, KCB = !TQ;
    __shared__ __attribute__((aligned(16))) T As[2 * lds_elems<T, BM, KCA>()];
    __shared__ __attribute__((aligned(16))) T Bs[2 * lds_elems<T, BN, KCB>()];

    // XCD-aware tile order: consecutive workgroup ids are dealt round-robin to
    // the 8 XCDs, so regroup them so each XCD walks a contiguous range of
    // tiles, then walk tiles in column bands of 8 tile rows for L2 reuse.
    const int ntiles = tiles_m * tiles_n;
    int bid = blockIdx.x;
    if ((ntiles & 7) == 0) {
        const int per = ntiles >> 3;
        bid = (bid & 7) * per + (bid >> 3);
    }
    constexpr int GROUP = 8;
    const int band = bid / (GROUP * tiles_n);
    const int first_m = band * GROUP;
    const int gsize = min(tiles_m - first_m, GROUP);
    const int in_band = bid - band * GROUP * tiles_n;
    const int tm = first_m + in_band % gsize;
    const int tn = in_band / gsize;
    // the 64x64 tile serves the short-K updates: FP64 reads C during the K loop
    gemm_tile<T, BM, BN, TP, TQ, VEC, WM, WN, BM == 64 && sizeof(T) == 8>(g, (int64_t)tm * BM, (int64_t)tn * BN,
                                                                           As, Bs);
}

template <typename T, int BM, int BN, int WM, int WN, bool TP, bool TQ>
hipError_t launch_t(const GemmDesc &g, bool vec, hipStream_t st)
{
    const int tm = (int)((g.M + BM - 1) / BM), tn = (int)((g.N + BN - 1) / BN);
    const dim3 grid((unsigned)(tm * tn)), block(64 * WM * WN);
    if (vec)
        hipLaunchKernelGGL((gemm_kernel<T, BM, BN, TP, TQ, true, WM, WN>), grid, block, 0, st, g, tm, tn);
    else
        hipLaunchKernelGGL((gemm_kernel<T, BM, BN, TP, TQ, false, WM, WN>), grid, block, 0, st, g, tm, tn);
    return hipGetLastError();
}

template <typename T, int BM, int BN, int WM = 2, int WN = 2>
hipError_t launch_tile(const GemmDesc &g, bool vec, hipStream_t st)
{
    if (!g.tp && !g.tq) return launch_t<T, BM, BN, WM, WN, false, false>(g, vec, st);
    if (g.tp && !g.tq) return launch_t<T, BM, BN, WM, WN, true, false>(g, vec, st);
    if (!g.tp && g.tq) return launch_t<T, BM, BN, WM, WN, false, true>(g, vec, st);
    return launch_t<T, BM, BN, WM, WN, true, true>(g, vec, st);
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

// tile: 1 = 128x128 (4 wavefronts), 2 = 64x64, 3 = 128x128 (8 wavefronts of
// 64x32), 0 = pick by problem size
hipError_t launch_gemm(DType t, const GemmDesc &g, int tile, hipStream_t st)
{
    if (g.M <= 0 || g.N <= 0)
        return hipSuccess;
    const int64_t w = t == DType::F64 ? 2 : 4;
    const bool vec = aligned16(g.P) && aligned16(g.Q) && g.ldp % w == 0 && g.ldq % w == 0;
    if (tile == 0) {
        // 128x128 tiles of 8 wavefronts (4 per SIMD with 2 workgroups per CU)
        // once they fill the chip's 512 workgroup slots; smaller problems run
        // 64x64 tiles (measured faster up to M = 256 at N = 16384)
        const int64_t big = ((g.M + 127) / 128) * ((g.N + 127) / 128);
        tile = big >= 512 ? 3 : 2;
    }
    if (t == DType::F64)
        return tile == 1   ? launch_tile<double, 128, 128>(g, vec, st)
               : tile == 3 ? launch_tile<double, 128, 128, 2, 4>(g, vec, st)
                           : launch_tile<double, 64, 64>(g, vec, st);
    return tile == 1   ? launch_tile<float, 128, 128>(g, vec, st)
           : tile == 3 ? launch_tile<float, 128, 128, 2, 4>(g, vec, st)
                       : launch_tile<float, 64, 64>(g, vec, st);
}

}  // namespace rtri
