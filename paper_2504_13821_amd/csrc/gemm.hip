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
//
// Split K (kslice > 0): grid row y computes the K range [y*kslice, (y+1)*kslice)
// into its own partial product part + y*ldpart*N (leading dimension ldpart,
// beta 0, s 1); split_reduce_kernel then forms C = beta*C + s*(sum of the
// partials in y order).
template <typename T, int BM, int BN, bool TP, bool TQ, bool VEC, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(WM * WN / 2))) void
gemm_kernel(GemmDesc g, int tiles_m, int tiles_n, int64_t kslice, T *part, int64_t ldpart)
{
    if (kslice > 0) {
        const int64_t k0 = (int64_t)blockIdx.y * kslice;
        const T *P = static_cast<const T *>(g.P), *Q = static_cast<const T *>(g.Q);
        g.P = P + (TP ? k0 : k0 * g.ldp);
        g.Q = Q + (TQ ? k0 * g.ldq : k0);
        g.K = min(kslice, g.K - k0);
        g.C = part + (int64_t)blockIdx.y * ldpart * g.N;
        g.ldc = ldpart;
        g.beta = 0.0;
        g.s = 1.0;
    }
    constexpr bool KCA = TP, KCB = !TQ;
    // FP32 64x64 tiles: two k-steps per LDS stage (same MFMA sequence)
    constexpr int KS = sizeof(T) == 4 && BM == 64 && BN == 64 ? 2 : 1;
    __shared__ __attribute__((aligned(16))) T As[2 * lds_elems<T, BM, KCA, KS>()];
    __shared__ __attribute__((aligned(16))) T Bs[2 * lds_elems<T, BN, KCB, KS>()];

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
    gemm_tile<T, BM, BN, TP, TQ, VEC, WM, WN, BM == 64 && sizeof(T) == 8, KS>(g, (int64_t)tm * BM,
                                                                               (int64_t)tn * BN, As, Bs);
}

// Grouped updates (launch_gemm_grouped): the workgroup's tile takes its
// updates one after another.  Each update's epilogue reads and writes the C
// entries its own lanes wrote in the previous update (same tile shape and
// origin), so no barrier beyond gemm_tile's own is needed between them.
template <typename T, bool TP, bool TQ, bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void grouped_kernel(
    const GemmDesc *descs, const GroupEntry *ents, const GroupTile *tiles)
{
    // FP32: two k-steps per LDS stage (a 64x64 FP32 k-step is too short to
    // cover one barrier and one prefetch)
    constexpr int KS = sizeof(T) == 4 ? 2 : 1;
    __shared__ __attribute__((aligned(16))) T As[2 * lds_elems<T, 64, TP, KS>()];
    __shared__ __attribute__((aligned(16))) T Bs[2 * lds_elems<T, 64, !TQ, KS>()];
    const GroupTile tl = tiles[blockIdx.x];
    for (int e = tl.first; e < tl.first + tl.count; ++e) {
        const GroupEntry en = ents[e];
        const GemmDesc g = descs[en.desc];
        gemm_tile<T, 64, 64, TP, TQ, VEC, 2, 2, sizeof(T) == 8, KS>(g, en.m0, en.n0, As, Bs);
    }
}

template <typename T, bool TP, bool TQ>
hipError_t launch_grouped_t(const GemmDesc *descs, const GroupEntry *ents, const GroupTile *tiles, int ntiles,
                            bool vec, hipStream_t st)
{
    if (vec)
        hipLaunchKernelGGL((grouped_kernel<T, TP, TQ, true>), dim3((unsigned)ntiles), dim3(256), 0, st, descs, ents,
                           tiles);
    else
        hipLaunchKernelGGL((grouped_kernel<T, TP, TQ, false>), dim3((unsigned)ntiles), dim3(256), 0, st, descs, ents,
                           tiles);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grouped_typed(const GemmDesc *descs, const GroupEntry *ents, const GroupTile *tiles, int ntiles,
                                bool tp, bool tq, bool vec, hipStream_t st)
{
    if (!tp && !tq) return launch_grouped_t<T, false, false>(descs, ents, tiles, ntiles, vec, st);
    if (tp && !tq) return launch_grouped_t<T, true, false>(descs, ents, tiles, ntiles, vec, st);
    if (!tp && tq) return launch_grouped_t<T, false, true>(descs, ents, tiles, ntiles, vec, st);
    return launch_grouped_t<T, true, true>(descs, ents, tiles, ntiles, vec, st);
}

// C = beta*C + s*(part_0 + part_1 + ... + part_{S-1}), partials added in order
template <typename T>
__global__ __launch_bounds__(256) void split_reduce_kernel(const T *part, int S, int64_t ldpart, int64_t M, int64_t N,
                                                           T *C, int64_t ldc, T beta, T s)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M)
        return;
    for (int64_t j = blockIdx.y; j < N; j += gridDim.y) {
        const T *p = part + i + j * ldpart;
        T acc = p[0];
        for (int y = 1; y < S; ++y)
            acc += p[(int64_t)y * ldpart * N];
        const T v = s * acc;
        T *c = C + i + j * ldc;
        *c = beta == T(0) ? v : fmat(beta, *c, v);
    }
}

template <typename T, int BM, int BN, int WM, int WN, bool TP, bool TQ>
hipError_t launch_t(const GemmDesc &g, bool vec, const Split &sp, hipStream_t st)
{
    const int tm = (int)((g.M + BM - 1) / BM), tn = (int)((g.N + BN - 1) / BN);
    const dim3 grid((unsigned)(tm * tn), (unsigned)std::max(1, sp.slices)), block(64 * WM * WN);
    T *part = static_cast<T *>(sp.part);
    if (vec)
        hipLaunchKernelGGL((gemm_kernel<T, BM, BN, TP, TQ, true, WM, WN>), grid, block, 0, st, g, tm, tn, sp.kslice,
                           part, sp.ldpart);
    else
        hipLaunchKernelGGL((gemm_kernel<T, BM, BN, TP, TQ, false, WM, WN>), grid, block, 0, st, g, tm, tn, sp.kslice,
                           part, sp.ldpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || sp.slices < 2)
        return e;
    const dim3 rg((unsigned)((g.M + 255) / 256), (unsigned)std::min<int64_t>(g.N, 65535));
    hipLaunchKernelGGL(split_reduce_kernel<T>, rg, dim3(256), 0, st, static_cast<const T *>(part), sp.slices,
                       sp.ldpart, g.M, g.N, static_cast<T *>(g.C), g.ldc, (T)g.beta, (T)g.s);
    return hipGetLastError();
}

template <typename T, int BM, int BN, int WM = 2, int WN = 2>
hipError_t launch_tile(const GemmDesc &g, bool vec, const Split &sp, hipStream_t st)
{
    if (!g.tp && !g.tq) return launch_t<T, BM, BN, WM, WN, false, false>(g, vec, sp, st);
    if (g.tp && !g.tq) return launch_t<T, BM, BN, WM, WN, true, false>(g, vec, sp, st);
    if (!g.tp && g.tq) return launch_t<T, BM, BN, WM, WN, false, true>(g, vec, sp, st);
    return launch_t<T, BM, BN, WM, WN, true, true>(g, vec, sp, st);
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int auto_tile(const GemmDesc &g)
{
    // 128x128 tiles of 8 wavefronts (4 per SIMD with 2 workgroups per CU) once
    // they fill the chip's 512 workgroup slots; smaller problems run 64x64
    // tiles (measured faster up to M = 256 at N = 16384)
    const int64_t big = ((g.M + 127) / 128) * ((g.N + 127) / 128);
    return big >= 512 ? 3 : 2;
}

}  // namespace

Split plan_split(DType t, const GemmDesc &g, int tile, size_t cap)
{
    Split sp{};
    if (g.M <= 0 || g.N <= 0 || g.K < SPLIT_MIN_K)
        return sp;
    if ((tile == 0 ? auto_tile(g) : tile) != 2)
        return sp;
    // an update short of tiles (fewer 64x64 tiles than CUs) with a long K:
    // aim at ~512 workgroups, slices of at least 512 along K (multiples of 64)
    const int64_t tiles = ((g.M + 63) / 64) * ((g.N + 63) / 64);
    if (tiles >= 256)
        return sp;
    const size_t es = t == DType::F64 ? 8 : 4;
    const int64_t ldpart = (g.M + 7) / 8 * 8;   // 16-byte aligned columns
    int64_t s = std::min<int64_t>({8, std::max<int64_t>(1, 512 / tiles), g.K / 512});
    while (s >= 2) {
        const int64_t ks = ((g.K + s - 1) / s + 63) / 64 * 64;
        const int64_t n = (g.K + ks - 1) / ks;
        if (n >= 2 && (size_t)n * (size_t)ldpart * (size_t)g.N * es <= cap) {
            sp.slices = (int)n;
            sp.kslice = ks;
            sp.ldpart = ldpart;
            return sp;
        }
        --s;
    }
    return sp;
}

namespace {

template <typename T>
hipError_t launch_typed(const GemmDesc &g, int tile, bool vec, const Split &sp, hipStream_t st)
{
    return tile == 1   ? launch_tile<T, 128, 128>(g, vec, sp, st)
           : tile == 3 ? launch_tile<T, 128, 128, 2, 4>(g, vec, sp, st)
                       : launch_tile<T, 64, 64>(g, vec, sp, st);
}

}  // namespace

hipError_t launch_gemm_grouped(DType t, const GemmDesc *descs, const GroupEntry *ents, const GroupTile *tiles,
                               int ntiles, bool tp, bool tq, bool vec, hipStream_t st)
{
    if (ntiles <= 0)
        return hipSuccess;
    return t == DType::F64 ? launch_grouped_typed<double>(descs, ents, tiles, ntiles, tp, tq, vec, st)
                           : launch_grouped_typed<float>(descs, ents, tiles, ntiles, tp, tq, vec, st);
}

// tile: 1 = 128x128 (4 wavefronts), 2 = 64x64, 3 = 128x128 (8 wavefronts of
// 64x32), 0 = pick by problem size.  A split (from plan_split, with sp.part
// set to at least slices * ldpart * N elements) runs 64x64 tiles over slices
// of K and a reduction pass.
hipError_t launch_gemm(DType t, const GemmDesc &g, int tile, hipStream_t st, const Split &sp)
{
    if (g.M <= 0 || g.N <= 0)
        return hipSuccess;
    const int64_t w = t == DType::F64 ? 2 : 4;
    const bool vec = aligned16(g.P) && aligned16(g.Q) && g.ldp % w == 0 && g.ldq % w == 0;
    Split s = sp;
    if (s.slices >= 2 && s.part != nullptr)
        tile = 2;
    else
        s = Split{};
    if (tile == 0)
        tile = auto_tile(g);
    return t == DType::F64 ? launch_typed<double>(g, tile, vec, s, st) : launch_typed<float>(g, tile, vec, s, st);
}

}  // namespace rtri
