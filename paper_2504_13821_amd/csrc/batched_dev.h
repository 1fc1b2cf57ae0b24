// Device side of the batched launch (see batched.hip): work-item layout and
// the persistent kernel, instantiated per element type and leaf size in
// batched_*.hip so the variants compile in parallel.
#pragma once

#include "gemm_core.h"
#include "leaf_core.h"
#include "mleaf_core.h"

namespace rtri {
namespace bk {

constexpr int NT = 256;

struct BOp {
    int kind;        // 0 leaf, 1 gemm, 2 zero the chunk (alpha == 0)
    int a0, a1, a2, a3;
    int use_alpha;   // leaf / TRSM gemm: scale by the problem's alpha (first touch) or by 1
};

struct BInst {
    const void *A;
    void *B;
    int64_t lda, ldb;
    int64_t m, n;
    double alpha;
    int op_begin, op_end;
    int solve, left, low, tr, unit;
};

struct BItem {
    int inst;
    int v0;
};

// ---- device ----

// 64-row leaves run on the matrix cores (canonical staging + A-operand tiles),
// 16/32-row leaves as one-lane-per-vector substitution in wavefront 0
// FP32 GEMM tiles stage two k-steps per LDS buffer (same MFMA sequence)
template <typename T> constexpr int gemm_ks() { return sizeof(T) == 4 ? 2 : 1; }

template <typename T, int NB>
struct Smem {
    static constexpr int GEMM =
        2 * gk::lds_elems<T, 64, true, gemm_ks<T>()>() + 2 * gk::lds_elems<T, 64, false, gemm_ks<T>()>() + 64;
    static constexpr int LEAF = NB == 64 ? lk::tri_n<64>() + mk::ntiles<64>() * mk::TE
                                         : lk::tri_n<NB>() + lk::WAVE * (NB + 1);
    static constexpr int N = GEMM > LEAF ? GEMM : LEAF;
};

template <typename T, bool TP, bool TQ>
__device__ __forceinline__ void run_gemm(const GemmDesc &g, T *smem)
{
    constexpr int EA = gk::lds_elems<T, 64, TP, gemm_ks<T>()>();
    T *As = smem;
    T *Bs = smem + 2 * EA;
    // an opaque copy of the thread index: the offsets derived from it are
    // recomputed here instead of being hoisted out of the persistent loop and
    // kept live for the whole kernel
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    for (int64_t m0 = 0; m0 < g.M; m0 += 64)
        for (int64_t n0 = 0; n0 < g.N; n0 += 64)
            gk::gemm_tile<T, 64, 64, TP, TQ, false, 2, 2, false, gemm_ks<T>()>(g, m0, n0, As, Bs, tid);
}

// The chunk's vectors [v0, v0 + 64) against one diagonal block of 64 rows, on
// the matrix cores: the same tiles (diagonal tiles inverted by the same FP64
// substitution) and the same MFMA sequence as the single-call 64-row leaf, so
// the results agree bit for bit.  Dg: 4 x 16 x 17 doubles of LDS.
template <typename T, bool SOLVE>
__device__ __forceinline__ void run_mleaf(const BInst &in, const BOp &op, int v0, T *smem, double *Dg)
{
    constexpr int NB = 64, NBK = NB / mk::RB;
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));   // see run_gemm
    const int d0 = op.a0, h = op.a1;
    // the chunk's panel first (lane = vector, MFMA accumulator layout), so its
    // loads are in flight while the block is staged
    using AccT = mk::Acc<T>;
    const bool mtrans = in.left ? in.tr != 0 : in.tr == 0;
    const bool mlower = in.left ? in.low != 0 : in.low == 0;
    const int lane = tid % 64;
    const int w = __builtin_amdgcn_readfirstlane(tid / 64);
    const int c = lane % 16, g = lane / 16;
    int64_t sd, si, nvec;
    T *B = static_cast<T *>(in.B);
    if (in.left) {
        B += d0;
        sd = 1;
        si = in.ldb;
        nvec = in.n;
    } else {
        B += (int64_t)d0 * in.ldb;
        sd = in.ldb;
        si = 1;
        nvec = in.m;
    }
    const int64_t vec = (int64_t)v0 + 16 * w + c;
    const bool act = vec < nvec;
    T *Bv = B + vec * si;
    typename AccT::V acc[NBK];
#pragma unroll
    for (int i = 0; i < NBK; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = mk::RB * i + 4 * g + r;
            const int dm = mlower ? row : h - 1 - row;
            acc[i][r] = (act && row < h) ? Bv[(int64_t)dm * sd] : T(0);
        }
    T *Ls = smem;                        // canonical block, ascending stream order
    T *Lt = smem + lk::tri_n<NB>();      // the 10 tiles in A-operand order
    lk::stage_block<sizeof(T) == 8 ? ElemT::F64 : ElemT::F32, T, NB, true, NT>(
        in.A, (int64_t)d0 + (int64_t)d0 * in.lda, in.lda, h, mtrans, mlower, in.unit != 0, Ls, tid);
    __syncthreads();
    auto canon = [&](int i, int k) { return Ls[lk::colstart<NB, true>(k) + (i - k)]; };
    if (tid < NBK * mk::RB) {
        const int j = tid / mk::RB, k = tid % mk::RB;
        double y[mk::RB];
        mk::diag_column<SOLVE>(
            k, [&](int m, int q) { return (double)canon(mk::RB * j + m, mk::RB * j + q); }, y);
#pragma unroll
        for (int m = 0; m < mk::RB; ++m)
            Dg[(j * mk::RB + m) * (mk::RB + 1) + k] = y[m];
    }
    __syncthreads();
    // a tile has NT = 256 entries: thread tid writes entry tid of every tile
    static_assert(mk::TE == NT, "one tile entry per thread");
    int m, kk;
    mk::tile_entry<T>(tid, m, kk);
    m = mk::lrow<T>(m);
    kk = mk::lrow<T>(kk);
#pragma unroll
    for (int p = 0; p < NBK; ++p)
#pragma unroll
        for (int k = 0; k <= p; ++k) {
            T v;
            if (k == p) {
                v = (T)Dg[(p * mk::RB + m) * (mk::RB + 1) + kk];
            } else {
                v = canon(mk::RB * p + m, mk::RB * k + kk);
                if (SOLVE)
                    v = -v;
            }
            Lt[mk::rb_tile(p, k) * mk::TE + tid] = v;
        }
    __syncthreads();

    const T alpha = T(op.use_alpha ? in.alpha : 1.0);
    if (SOLVE)
#pragma unroll
        for (int i = 0; i < NBK; ++i)
            acc[i] *= alpha;
    mk::leaf_rows<T, NB, SOLVE>(
        acc, lane, [&](int p, int k) -> const T * { return Lt + mk::rb_tile(p, k) * mk::TE; }, [](int) {},
        [&](int p, typename AccT::V x) {
            if (!SOLVE)
                x *= alpha;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = mk::RB * p + 4 * g + r;
                const int dm = mlower ? row : h - 1 - row;
                if (act && row < h)
                    Bv[(int64_t)dm * sd] = x[r];
            }
        },
        [](auto, auto) {});
    __syncthreads();
}

template <typename T, int NB, bool SOLVE>
__device__ __forceinline__ void run_leaf(const BInst &in, const BOp &op, int v0, T *smem)
{
    const int tid = threadIdx.x;
    const int d0 = op.a0, h = op.a1;
    T *Ls = smem;
    T *Ps = smem + lk::tri_n<NB>();
    // the block of op(A) (side L) or of op(A)^T (side R), see driver.hip
    const bool mtrans = in.left ? in.tr != 0 : in.tr == 0;
    const bool mlower = in.left ? in.low != 0 : in.low == 0;
    lk::stage_block<sizeof(T) == 8 ? ElemT::F64 : ElemT::F32, T, NB, SOLVE, NT>(
        in.A, (int64_t)d0 + (int64_t)d0 * in.lda, in.lda, h, mtrans, mlower, in.unit != 0, Ls, tid);
    __syncthreads();
    if (tid < lk::WAVE) {
        LeafDesc d{};
        d.nb = h;
        d.unit = in.unit != 0;
        d.mlower = mlower;
        d.alpha = op.use_alpha ? in.alpha : 1.0;
        T *B = static_cast<T *>(in.B);
        if (in.left) {
            B += d0;
            d.sd = 1;
            d.si = in.ldb;
            d.nvec = in.n;
        } else {
            B += (int64_t)d0 * in.ldb;
            d.sd = in.ldb;
            d.si = 1;
            d.nvec = in.m;
        }
        auto none = [] {};
        if (d.unit)
            lk::leaf_panel<T, NB, SOLVE, true>(d, B, Ls, Ps, v0, none);
        else
            lk::leaf_panel<T, NB, SOLVE, false>(d, B, Ls, Ps, v0, none);
    }
    __syncthreads();
}

// Three workgroups per CU (12 wavefronts): every op of an item is a chain of
// dependent memory round trips, so more resident items hide more latency
// (measured on the 4096-problem FP64 mix: 2.73 -> 2.57 ms).
template <typename T, int NB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void batched_kernel(
    const BInst *insts, const BItem *items, int nitems, const BOp *ops, unsigned *counter)
{
    __shared__ __attribute__((aligned(16))) T smem[Smem<T, NB>::N];
    __shared__ double Dg[NB == 64 ? 4 * 16 * 17 : 1];
    __shared__ int s_item;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0)
            s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);   // uniform: scalar loads of the tables
        __syncthreads();
        if (it >= nitems)
            return;   // every wave of the workgroup leaves together
        const BItem item = items[it];
        const BInst in = insts[item.inst];
        const int64_t nvec = in.left ? in.n : in.m;
        const int nv = (int)min<int64_t>(lk::WAVE, nvec - item.v0);
        for (int o = in.op_begin; o < in.op_end; ++o) {
            const BOp op = ops[o];
            if (op.kind == 0) {
                if constexpr (NB == 64) {
                    if (in.solve)
                        run_mleaf<T, true>(in, op, item.v0, smem, Dg);
                    else
                        run_mleaf<T, false>(in, op, item.v0, smem, Dg);
                } else {
                    if (in.solve)
                        run_leaf<T, NB, true>(in, op, item.v0, smem);
                    else
                        run_leaf<T, NB, false>(in, op, item.v0, smem);
                }
            } else if (op.kind == 1) {
                GemmDesc g{};
                const int t0 = op.a0, th = op.a1, s0 = op.a2, sh = op.a3;
                g.K = sh;
                if (in.solve) {
                    g.beta = op.use_alpha ? in.alpha : 1.0;
                    g.s = -1.0;
                } else {
                    g.beta = 1.0;
                    g.s = in.alpha;
                }
                const T *A = static_cast<const T *>(in.A);
                T *B = static_cast<T *>(in.B);
                if (in.left) {
                    g.M = th;
                    g.N = nv;
                    g.P = A + (in.tr ? s0 + (int64_t)t0 * in.lda : t0 + (int64_t)s0 * in.lda);
                    g.ldp = in.lda;
                    g.tp = in.tr != 0;
                    g.Q = B + s0 + (int64_t)item.v0 * in.ldb;
                    g.ldq = in.ldb;
                    g.C = B + t0 + (int64_t)item.v0 * in.ldb;
                    g.ldc = in.ldb;
                    if (in.tr)
                        run_gemm<T, true, false>(g, smem);
                    else
                        run_gemm<T, false, false>(g, smem);
                } else {
                    g.M = nv;
                    g.N = th;
                    g.P = B + item.v0 + (int64_t)s0 * in.ldb;
                    g.ldp = in.ldb;
                    g.Q = A + (in.tr ? t0 + (int64_t)s0 * in.lda : s0 + (int64_t)t0 * in.lda);
                    g.ldq = in.lda;
                    g.tq = in.tr != 0;
                    g.C = B + item.v0 + (int64_t)t0 * in.ldb;
                    g.ldc = in.ldb;
                    if (in.tr)
                        run_gemm<T, false, true>(g, smem);
                    else
                        run_gemm<T, false, false>(g, smem);
                }
                __syncthreads();   // the update's stores are read by the next op
            } else {
                T *B = static_cast<T *>(in.B);
                const int64_t rows = in.left ? in.m : nv, cols = in.left ? nv : in.n;
                T *base = in.left ? B + (int64_t)item.v0 * in.ldb : B + item.v0;
                for (int64_t e = tid; e < rows * cols; e += NT)
                    base[e % rows + (e / rows) * in.ldb] = T(0);
                __syncthreads();
            }
        }
    }
}

template <typename T, int NB>
hipError_t launch(unsigned grid, const BInst *insts, const BItem *items, int nitems, const BOp *ops, unsigned *counter,
                  hipStream_t st);
template <typename T, int NB>
const void *kernel_ptr();

#define RTRI_BATCHED_INSTANTIATE(T, NB)                                                                          \
    template <>                                                                                                \
    hipError_t launch<T, NB>(unsigned grid, const BInst *insts, const BItem *items, int nitems, const BOp *ops, \
                             unsigned *counter, hipStream_t st)                                                \
    {                                                                                                          \
        hipLaunchKernelGGL((batched_kernel<T, NB>), dim3(grid), dim3(NT), 0, st, insts, items, nitems, ops,     \
                           counter);                                                                           \
        return hipGetLastError();                                                                              \
    }                                                                                                          \
    template <>                                                                                                \
    const void *kernel_ptr<T, NB>()                                                                            \
    {                                                                                                          \
        return reinterpret_cast<const void *>(&batched_kernel<T, NB>);                                         \
    }

}  // namespace bk
}  // namespace rtri
