// Device-side building blocks of the GEMM update (see gemm.hip), shared with
// the batched kernel.
#pragma once

#include "common.h"

namespace rtri {
namespace gk {

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

// Rows inside a 16-row block are relabelled: the row that the MFMA calls m
// (tile row) is block row lrow(m).  Slot r of lane group g holds tile row
// Acc::row(g, r), hence block row 4g + r for both element types: a lane's four
// slots are four consecutive rows, which column-major data moves with 16-byte
// accesses.  Only the lane that supplies (or receives) a row changes, not the
// arithmetic of any entry.
template <typename T> __host__ __device__ constexpr int lrow(int m)
{
    return sizeof(T) == 8 ? 4 * (m % 4) + m / 4 : m;
}

// 16 bytes of T, and four consecutive elements from 16-byte aligned addresses
template <typename T> struct Vec16;
template <> struct Vec16<double> { using V = double __attribute__((ext_vector_type(2))); };
template <> struct Vec16<float> { using V = float __attribute__((ext_vector_type(4))); };
__device__ __forceinline__ double4_t ld4(const double *p)
{
    const auto *q = reinterpret_cast<const Vec16<double>::V *>(p);
    const auto a = q[0], b = q[1];
    return double4_t{a.x, a.y, b.x, b.y};
}
__device__ __forceinline__ float4_t ld4(const float *p) { return *reinterpret_cast<const float4_t *>(p); }
__device__ __forceinline__ void st4(double *p, double4_t v)
{
    auto *q = reinterpret_cast<Vec16<double>::V *>(p);
    q[0] = Vec16<double>::V{v.x, v.y};
    q[1] = Vec16<double>::V{v.z, v.w};
}
__device__ __forceinline__ void st4(float *p, float4_t v) { *reinterpret_cast<float4_t *>(p) = v; }

// LDS layout of an operand tile (R rows of M or N, BK along K) follows its
// layout in global memory, so the global -> LDS copy never transposes:
//   KC (k contiguous in memory):    Ls[row * SK + k],  SK = BK + pad
//   MC (rows contiguous in memory): Ls[k * SM + row],  SM = R + 16
// The paddings make the MFMA fragment reads bank-conflict free: 16-byte reads
// of k pairs in the KC layout, 8-byte reads of 16 consecutive rows per lane
// group (groups 1152 B apart) in the MC layout.
// A stage may hold KS consecutive k-steps (KS * BK values along K).
template <typename T, int KS = 1> constexpr int lds_sk() { return sizeof(T) == 8 ? KS * BK + 2 : KS * BK + 4; }
template <typename T, int R> constexpr int lds_sm() { return sizeof(T) == 8 ? R + 16 : R + 4; }
template <typename T, int R, bool KC, int KS = 1> constexpr int lds_elems()
{
    return KC ? R * lds_sk<T, KS>() : KS * BK * lds_sm<T, R>();
}

template <typename T, int R, bool KC, int KS = 1>
__device__ __forceinline__ T lds_at(const T *ls, int row, int k)
{
    return KC ? ls[row * lds_sk<T, KS>() + k] : ls[k * lds_sm<T, R>() + row];
}

// Loader of one operand tile (R rows of the M or N dimension, KS * BK along K) into
// registers, then into LDS as Ls[row][k] (k contiguous, padded rows).
//   KC = true : element (row, k) at base[k + row*ld]   (k contiguous in memory)
//   KC = false: element (row, k) at base[row + k*ld]   (rows contiguous in memory)
template <typename T, int R, bool KC, bool VEC, int NTH = NT, int KS = 1>
struct TileLoader {
    static constexpr int BKS = KS * BK;                     // k values per stage
    static constexpr int W = 16 / sizeof(T);               // elements per 16-byte load
    static constexpr int PER = R * BKS / NTH;               // elements per thread
    static constexpr int NV = PER / W;                      // 16-byte loads per thread
    static_assert(PER % W == 0, "tile too small");
    T reg[PER];

    __device__ inline void coords(int v, int tid, int &row, int &k) const
    {
        const int e = v * NTH + tid;                         // index of the W-vector
        if (KC) {
            k = (e % (BKS / W)) * W;
            row = e / (BKS / W);
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
            T *dst = KC ? lds + row * lds_sk<T, KS>() + k : lds + k * lds_sm<T, R>() + row;
#pragma unroll
            for (int w = 0; w < W; ++w)
                dst[w] = reg[v * W + w];
        }
    }
};

// One BM x BN tile of C at (m0, n0), computed by the 64*WM*WN threads of the
// workgroup, wavefronts in a WM x WN grid of (BM/WM) x (BN/WN) blocks.  As / Bs:
// two LDS slots each (lds_elems elements per slot).  Ends with a barrier, so
// the LDS slots may be reused right after it returns.
// CPF: read C during the K loop (one accumulator block per k-step, right after
// that step's operand loads) instead of in the epilogue, for short K where the
// epilogue's reads would otherwise follow all the MFMA work (FP64: the FP32
// k-step is too short to cover the read, measured slower there).
// KS: k-steps per LDS stage (one barrier and one prefetch per stage); the
// MFMA sequence, and so every result, is that of KS = 1.
template <typename T, int BM, int BN, bool TP, bool TQ, bool VEC, int WM = 2, int WN = 2, bool CPF = false,
          int KS = 1>
__device__ __forceinline__ void gemm_tile(const GemmDesc &g, int64_t m0, int64_t n0, T *As, T *Bs,
                                          int tid = threadIdx.x)
{
    constexpr int NTH = 64 * WM * WN;
    constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
    constexpr int BKS = KS * BK;
    constexpr bool KCA = TP, KCB = !TQ;           // operand layouts (see lds_at)
    constexpr int EA = lds_elems<T, BM, KCA, KS>(), EB = lds_elems<T, BN, KCB, KS>();
    using AccT = Acc<T>;
    using V = typename AccT::V;
    const int wave = tid / 64, lane = tid % 64;
    const int wm = wave % WM, wn = wave / WM;
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

    TileLoader<T, BM, TP, VEC, NTH, KS> la;
    TileLoader<T, BN, !TQ, VEC, NTH, KS> lb;

    V acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = V{0, 0, 0, 0};

    const int64_t K = g.K;
    const int nk = (int)((K + BKS - 1) / BKS);

    // C block (i, j) of this lane: rows 4*lg .. 4*lg+3 of its 16-row block
    T *C = static_cast<T *>(g.C);
    const int64_t ldc = g.ldc;
    const bool cvec = reinterpret_cast<uintptr_t>(C) % 16 == 0 && (ldc * (int64_t)sizeof(T)) % 16 == 0;
    auto cptr = [&](int i, int j, int wm_, int wn_, int lc_, int lg_) {
        return C + (m0 + wm_ * (BM / WM) + i * 16 + 4 * lg_) + (n0 + wn_ * (BN / WN) + j * 16 + lc_) * ldc;
    };
    // prefetched C blocks: block t = i * FN + j is requested during k-step t
    const bool pre = CPF && cvec && full_mn && g.beta != 0.0 && nk > FM * FN;
    V cpre[CPF ? FM : 1][CPF ? FN : 1];

    auto load_step = [&](int kt) {
        const int64_t k0 = (int64_t)kt * BKS;
        const T *pa = TP ? Pt + k0 : Pt + k0 * ldp;
        const T *pb = TQ ? Qt + k0 * ldq : Qt + k0;
        if (full_mn && k0 + BKS <= K) {
            la.load_full(pa, ldp, tid);
            lb.load_full(pb, ldq, tid);
        } else {
            const int klim = (int)min<int64_t>(BKS, K - k0);
            la.load_edge(pa, ldp, tid, rlim_m, klim);
            lb.load_edge(pb, ldq, tid, rlim_n, klim);
        }
    };

    if (nk > 0) {
        load_step(0);
        la.store(As, tid);
        lb.store(Bs, tid);
    }
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk)
            load_step(kt + 1);
        if (CPF && pre) {
#pragma unroll
            for (int t = 0; t < FM * FN; ++t)
                if (kt == t)
                    cpre[CPF ? t / FN : 0][CPF ? t % FN : 0] = ld4(cptr(t / FN, t % FN, wm, wn, lc, lg));
        }

        // fragments: lane (lc, lg) reads row (block*16 + lrow(lc)) of op(P), row
        // (block*16 + lc) of op(Q)^T, k = 4*lg .. 4*lg+3, two k values at a time
        // (one 16-byte read for FP64)
        const int ra = wm * (BM / WM) + lrow<T>(lc), rbq = wn * (BN / WN) + lc;
#pragma unroll
        for (int h = 0; h < KS; ++h) {
            // a k-step wholly past K adds nothing: skipped (uniform)
            if (h > 0 && (int64_t)kt * BKS + h * BK >= K)
                break;
#pragma unroll
            for (int t2 = 0; t2 < 4; t2 += 2) {
                T fa[FM][2], fb[FN][2];
                const int kk = h * BK + 4 * lg + t2;
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    fa[i][0] = lds_at<T, BM, KCA, KS>((As + cur * EA), ra + i * 16, kk);
                    fa[i][1] = lds_at<T, BM, KCA, KS>((As + cur * EA), ra + i * 16, kk + 1);
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    fb[j][0] = lds_at<T, BN, KCB, KS>((Bs + cur * EB), rbq + j * 16, kk);
                    fb[j][1] = lds_at<T, BN, KCB, KS>((Bs + cur * EB), rbq + j * 16, kk + 1);
                }
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            acc[i][j] = AccT::mfma(fa[i][t], fb[j][t], acc[i][j]);
            }
        }

        if (kt + 1 < nk) {
            int ts = tid;
            // The FP64 8-wavefront tile with both operands transposed sits one
            // register over its 128-register budget: there, recompute the LDS
            // offsets each step from an opaque copy of the thread index instead
            // of spilling one.  Elsewhere that recomputation costs more than it
            // saves (measured 3% at 8192x16384x8192), so the offsets stay live.
            if constexpr (sizeof(T) == 8 && WM * WN == 8 && TP && TQ)
                asm volatile("" : "+v"(ts));
            la.store(As + (cur ^ 1) * EA, ts);
            lb.store(Bs + (cur ^ 1) * EB, ts);
        }
        __syncthreads();
    }

    // epilogue: slot r of lane (lc, lg) holds row 4*lg + r, column lc of every
    // 16x16 block; C moves as one or two 16-byte accesses per lane and block when
    // aligned, else element by element (the same arithmetic either way).  The
    // lane's offsets are recomputed from an opaque copy of the thread index, so
    // none of them is kept live (or spilled) across the K loop.
    int te = tid;
    asm volatile("" : "+v"(te));
    const int lane_e = te % 64, wave_e = te / 64;
    const int wm_e = wave_e % WM, wn_e = wave_e / WM, lc_e = lane_e % 16, lg_e = lane_e / 16;
    const T beta = T(g.beta), s = T(g.s);
    // A lane with few blocks (64x64 tiles) reads all its C blocks before the
    // first store: one memory round trip instead of one per block (the stores
    // could alias the later reads as far as the compiler knows, so it would
    // not reorder them itself).  Same arithmetic as the general loop below.
    if constexpr (FM * FN <= 4) {
        if (cvec && full_mn && g.beta != 0.0 && !(CPF && pre)) {
            V cb[FM][FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    cb[i][j] = ld4(cptr(i, j, wm_e, wn_e, lc_e, lg_e));
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    V v = s * acc[i][j];
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        v[r] = fmat(beta, cb[i][j][r], v[r]);
                    st4(cptr(i, j, wm_e, wn_e, lc_e, lg_e), v);
                }
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int r0 = wm_e * (BM / WM) + i * 16 + 4 * lg_e;    // local row of slot 0
            const int cl = wn_e * (BN / WN) + j * 16 + lc_e;       // local column
            if (cl >= rlim_n)
                continue;
            T *cp = cptr(i, j, wm_e, wn_e, lc_e, lg_e);
            if (cvec && r0 + 4 <= rlim_m) {
                V v = s * acc[i][j];
                if (g.beta != 0.0) {
                    const V c = (CPF && pre) ? cpre[CPF ? i : 0][CPF ? j : 0] : ld4(cp);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        v[r] = fmat(beta, c[r], v[r]);
                }
                st4(cp, v);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r0 + r < rlim_m) {
                        const T v = s * acc[i][j][r];
                        cp[r] = (g.beta == 0.0) ? v : fmat(beta, cp[r], v);
                    }
                }
            }
        }
    }
}


}  // namespace gk
}  // namespace rtri
