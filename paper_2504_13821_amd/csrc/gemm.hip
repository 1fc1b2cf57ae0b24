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
#include "common.h"

namespace rtri {

namespace {

constexpr int NT = 256;   // threads per workgroup
constexpr int BK = 16;

// Accumulator row held in slot r of lane group g: the FP32 instruction returns
// four consecutive rows per lane (4g + r), the FP64 one interleaves them (g + 4r).
template <typename T> struct Acc;
template <> struct Acc<double> {
    using V = double4_t;
    static __device__ inline V mfma(double a, double b, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int g, int r) { return g + 4 * r; }
};
template <> struct Acc<float> {
    using V = float4_t;
    static __device__ inline V mfma(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int g, int r) { return 4 * g + r; }
};

// LDS layout of an operand tile (R rows of M or N, BK along K) follows its
// layout in global memory, so the global -> LDS copy never transposes:
//   KC (k contiguous in memory):    Ls[row * SK + k],  SK = BK + pad
//   MC (rows contiguous in memory): Ls[k * SM + row],  SM = R + 16
// The paddings make the MFMA fragment reads bank-conflict free: 16-byte reads
// of k pairs in the KC layout, 8-byte reads of 16 consecutive rows per lane
// group (groups 1152 B apart) in the MC layout.
template <typename T> constexpr int lds_sk() { return sizeof(T) == 8 ? BK + 2 : BK + 4; }
template <int R> constexpr int lds_sm() { return R + 16; }
template <typename T, int R, bool KC> constexpr int lds_elems() { return KC ? R * lds_sk<T>() : BK * lds_sm<R>(); }

template <typename T, int R, bool KC>
__device__ __forceinline__ T lds_at(const T *ls, int row, int k)
{
    return KC ? ls[row * lds_sk<T>() + k] : ls[k * lds_sm<R>() + row];
}

// Loader of one operand tile (R rows of the M or N dimension, BK along K) into
// registers, then into LDS as Ls[row][k] (k contiguous, padded rows).
//   KC = true : element (row, k) at base[k + row*ld]   (k contiguous in memory)
//   KC = false: element (row, k) at base[row + k*ld]   (rows contiguous in memory)
template <typename T, int R, bool KC, bool VEC>
struct TileLoader {
    static constexpr int W = 16 / sizeof(T);               // elements per 16-byte load
    static constexpr int PER = R * BK / NT;                 // elements per thread
    static constexpr int NV = PER / W;                      // 16-byte loads per thread
    static_assert(PER % W == 0, "tile too small");
    T reg[PER];

    __device__ inline void coords(int v, int tid, int &row, int &k) const
    {
        const int e = v * NT + tid;                          // index of the W-vector
        if (KC) {
            k = (e % (BK / W)) * W;
            row = e / (BK / W);
        } else {
            row = (e % (R / W)) * W;
            k = e / (R / W);
        }
    }

    // full tile, no bounds checks
    __device__ inline void load_full(const T *base, int64_t ld, int tid)
    {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            int row, k;
            coords(v, tid, row, k);
            const T *p = KC ? base + k + (int64_t)row * ld : base + row + (int64_t)k * ld;
            if (VEC) {
                using V4 = int __attribute__((ext_vector_type(4)));
                V4 x = *reinterpret_cast<const V4 *>(p);
                const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
                for (int w = 0; w < W; ++w)
                    reg[v * W + w] = xs[w];
            } else {
#pragma unroll
                for (int w = 0; w < W; ++w)
                    reg[v * W + w] = p[w];
            }
        }
    }

    // edge tile: rows >= rlim or k >= klim read as zero
    __device__ inline void load_edge(const T *base, int64_t ld, int tid, int rlim, int klim)
    {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            int row, k;
            coords(v, tid, row, k);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const int rr = KC ? row : row + w;
                const int kk = KC ? k + w : k;
                T x = T(0);
                if (rr < rlim && kk < klim)
                    x = KC ? base[kk + (int64_t)rr * ld] : base[rr + (int64_t)kk * ld];
                reg[v * W + w] = x;
            }
        }
    }

    __device__ inline void store(T *lds, int tid) const
    {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            int row, k;
            coords(v, tid, row, k);
            T *dst = KC ? lds + row * lds_sk<T>() + k : lds + k * lds_sm<R>() + row;
#pragma unroll
            for (int w = 0; w < W; ++w)
                dst[w] = reg[v * W + w];
        }
    }
};

// Workgroup tile BM x BN; wavefront tile (BM/2) x (BN/2) made of FM x FN MFMA blocks.
template <typename T, int BM, int BN, bool TP, bool TQ, bool VEC>
__global__ __launch_bounds__(NT, 2) void gemm_kernel(GemmDesc g, int tiles_m, int tiles_n)
{
    constexpr int FM = BM / 32, FN = BN / 32;
    constexpr bool KCA = TP, KCB = !TQ;           // operand layouts (see lds_at)
    using AccT = Acc<T>;
    using V = typename AccT::V;
    __shared__ __attribute__((aligned(16))) T As[2][lds_elems<T, BM, KCA>()];
    __shared__ __attribute__((aligned(16))) T Bs[2][lds_elems<T, BN, KCB>()];

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

    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int wm = wave & 1, wn = wave >> 1;
    const int lc = lane % 16, lg = lane / 16;

    const T *P = static_cast<const T *>(g.P);
    const T *Q = static_cast<const T *>(g.Q);
    const int64_t ldp = g.ldp, ldq = g.ldq;
    // tile origins: op(P) rows m0.., op(Q) columns n0..
    const T *Pt = TP ? P + m0 * ldp : P + m0;
    const T *Qt = TQ ? Q + n0 : Q + n0 * ldq;
    const int rlim_m = (int)min<int64_t>(BM, g.M - m0);
    const int rlim_n = (int)min<int64_t>(BN, g.N - n0);
    const bool full_mn = rlim_m == BM && rlim_n == BN;

    TileLoader<T, BM, TP, VEC> la;
    TileLoader<T, BN, !TQ, VEC> lb;

    V acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = V{0, 0, 0, 0};

    const int64_t K = g.K;
    const int nk = (int)((K + BK - 1) / BK);

    auto load_step = [&](int kt) {
        const int64_t k0 = (int64_t)kt * BK;
        const T *pa = TP ? Pt + k0 : Pt + k0 * ldp;
        const T *pb = TQ ? Qt + k0 * ldq : Qt + k0;
        if (full_mn && k0 + BK <= K) {
            la.load_full(pa, ldp, tid);
            lb.load_full(pb, ldq, tid);
        } else {
            const int klim = (int)min<int64_t>(BK, K - k0);
            la.load_edge(pa, ldp, tid, rlim_m, klim);
            lb.load_edge(pb, ldq, tid, rlim_n, klim);
        }
    };

    if (nk > 0) {
        load_step(0);
        la.store(As[0], tid);
        lb.store(Bs[0], tid);
    }
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk)
            load_step(kt + 1);

        // fragments: lane (lc, lg) reads row (block*16 + lc), k = 4*lg .. 4*lg+3,
        // two k values at a time (one 16-byte read for FP64)
        const int ra = wm * (BM / 2) + lc, rbq = wn * (BN / 2) + lc;
#pragma unroll
        for (int t2 = 0; t2 < 4; t2 += 2) {
            T fa[FM][2], fb[FN][2];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                fa[i][0] = lds_at<T, BM, KCA>(As[cur], ra + i * 16, 4 * lg + t2);
                fa[i][1] = lds_at<T, BM, KCA>(As[cur], ra + i * 16, 4 * lg + t2 + 1);
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                fb[j][0] = lds_at<T, BN, KCB>(Bs[cur], rbq + j * 16, 4 * lg + t2);
                fb[j][1] = lds_at<T, BN, KCB>(Bs[cur], rbq + j * 16, 4 * lg + t2 + 1);
            }
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = AccT::mfma(fa[i][t], fb[j][t], acc[i][j]);
        }

        if (kt + 1 < nk) {
            la.store(As[cur ^ 1], tid);
            lb.store(Bs[cur ^ 1], tid);
        }
        __syncthreads();
    }

    // epilogue: slot r of lane (lc, lg) holds row AccT::row(lg, r), column lc of every 16x16 block
    T *C = static_cast<T *>(g.C);
    const int64_t ldc = g.ldc;
    const T beta = T(g.beta), s = T(g.s);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int rb = wm * (BM / 2) + i * 16;              // local row of the block
            const int cl = wn * (BN / 2) + j * 16 + lc;        // local column
            if (cl >= rlim_n)
                continue;
            T *cp = C + (m0 + rb) + (n0 + cl) * ldc;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = AccT::row(lg, r);
                if (rb + rr < rlim_m) {
                    const T v = s * acc[i][j][r];
                    cp[rr] = (g.beta == 0.0) ? v : fmat(beta, cp[rr], v);
                }
            }
        }
    }
}

template <typename T, int BM, int BN, bool TP, bool TQ>
hipError_t launch_t(const GemmDesc &g, bool vec, hipStream_t st)
{
    const int tm = (int)((g.M + BM - 1) / BM), tn = (int)((g.N + BN - 1) / BN);
    const dim3 grid((unsigned)(tm * tn));
    if (vec)
        hipLaunchKernelGGL((gemm_kernel<T, BM, BN, TP, TQ, true>), grid, dim3(NT), 0, st, g, tm, tn);
    else
        hipLaunchKernelGGL((gemm_kernel<T, BM, BN, TP, TQ, false>), grid, dim3(NT), 0, st, g, tm, tn);
    return hipGetLastError();
}

template <typename T, int BM, int BN>
hipError_t launch_tile(const GemmDesc &g, bool vec, hipStream_t st)
{
    if (!g.tp && !g.tq) return launch_t<T, BM, BN, false, false>(g, vec, st);
    if (g.tp && !g.tq) return launch_t<T, BM, BN, true, false>(g, vec, st);
    if (!g.tp && g.tq) return launch_t<T, BM, BN, false, true>(g, vec, st);
    return launch_t<T, BM, BN, true, true>(g, vec, st);
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

// tile: 1 = 128x128, 2 = 64x64, 0 = pick by problem size
hipError_t launch_gemm(DType t, const GemmDesc &g, int tile, hipStream_t st)
{
    if (g.M <= 0 || g.N <= 0)
        return hipSuccess;
    const int64_t w = t == DType::F64 ? 2 : 4;
    const bool vec = aligned16(g.P) && aligned16(g.Q) && g.ldp % w == 0 && g.ldq % w == 0;
    if (tile == 0) {
        // 128x128 tiles once they fill the chip (2 workgroups on each of the
        // 256 CUs) at least twice over; smaller problems run 64x64 tiles
        const int64_t big = ((g.M + 127) / 128) * ((g.N + 127) / 128);
        tile = big >= 1024 ? 1 : 2;
    }
    if (t == DType::F64)
        return tile == 1 ? launch_tile<double, 128, 128>(g, vec, st) : launch_tile<double, 64, 64>(g, vec, st);
    return tile == 1 ? launch_tile<float, 128, 128>(g, vec, st) : launch_tile<float, 64, 64>(g, vec, st);
}

}  // namespace rtri
