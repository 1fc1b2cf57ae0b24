// The matrix-core leaf kernel (the design is described in mleaf.hip), kept in
// a header so the solve / multiply and FP64 / FP32 variants compile as
// separate translation units.
#pragma once

#include "common.h"
#include "mleaf_core.h"

namespace rtri {
namespace mleaf {

using mk::RB;
using mk::TE;
using mk::Vec16;

using gk::ld4;
using gk::st4;

// Memory schedule.  The packed triangle reaches LDS in rounds of one 16-byte
// load per thread (512 FP64 / 1024 FP32 consecutive packed elements, 2 or 4
// tiles).  A short prologue loads the rounds of row blocks 0..K and panel
// blocks 0..DB.  Every later round is written to LDS during the even phase
// before the barrier that precedes its row block (barriers stand before phase 0
// and before every odd phase, so one barrier covers two row blocks) and
// fetched into registers D phases before that; panel block q is requested
// during phase q - 1 - DB; row block p of the result is stored during phase
// p + 1.  Tile t sits in LDS slot t mod CAP; every write lands on a slot whose
// previous tile belongs to a row block that all wavefronts finished before
// the last barrier (checked at compile time).
//
// A wavefront issues in order, and a memory instruction that cannot issue
// stalls it; with one wavefront per SIMD that idles the matrix core.  So the
// memory operations of a phase are spread over the gaps between its MFMAs
// (at most a few per gap) instead of being issued in a burst.
template <typename T, int NB> struct LeafSched {
    static constexpr int NBK = NB / RB;
    static constexpr int NTILE = mk::ntiles<NB>();
    static constexpr int W = 16 / (int)sizeof(T);                  // elements per 16-byte load
    static constexpr int TPR = 256 * W / TE;                        // tiles per round
    static constexpr int NR = (NTILE + TPR - 1) / TPR;              // rounds
    static constexpr int CAP_MAX = 144 * 1024 / (TE * (int)sizeof(T));
    static constexpr int CAP = NTILE < CAP_MAX ? NTILE : CAP_MAX;   // LDS slots, in tiles
    static constexpr int PRO = 8;                                   // prologue budget, rounds
    static constexpr int D = 2;                                     // triangle fetch distance, phases
    static constexpr int DB = 2;                                    // panel fetch distance, phases
    static constexpr int min_i(int a, int b) { return a < b ? a : b; }
    static constexpr int rounds_upto(int k) { return (mk::rb_tile(k + 1, 0) + TPR - 1) / TPR; }
    static constexpr int prologue_rows()
    {
        int k = NBK - 1;
        while (k > 0 && (rounds_upto(k) > PRO || min_i(rounds_upto(k) * TPR, NTILE) > CAP))
            --k;
        return k;
    }
    static constexpr int K = prologue_rows();
    static constexpr bool STREAM = K < NBK - 1;
    static constexpr int need(int u) { return mk::tile_row(u * TPR); }
    static constexpr bool pro(int u) { return need(u) <= K; }
    // a barrier before phase 0 and, when streaming, before every odd phase:
    // rounds are written during even phases, for the next two row blocks
    static constexpr bool barrier_at(int p) { return p == 0 || (STREAM && p % 2 == 1); }
    static constexpr int wrow(int q) { return q % 2 == 1 ? q - 1 : q - 2; }        // write phase of row block q
    static constexpr int wphase(int u) { return pro(u) ? -1 : wrow(need(u)); }     // -1: prologue
    static constexpr int fphase(int u) { return pro(u) ? -1 : wrow(need(u)) - D; }
    // the last barrier at or before phase w (every wavefront has finished the
    // phases before it)
    static constexpr int last_barrier(int w)
    {
        while (w > 0 && !barrier_at(w))
            --w;
        return w;
    }
    static constexpr int bphase(int q) { return q - 1 - DB; }                     // < 0: prologue

    // operations of phase p, in issue order: fetches, the panel block, LDS
    // writes, the store of row block p - 1
    enum Kind { FETCH, BLOCK, WRITE, STORE, NONE };
    struct Op {
        int kind, arg;
    };
    static constexpr int nops(int p)
    {
        int n = 0;
        for (int u = 0; u < NR; ++u)
            n += (fphase(u) == p) + (wphase(u) == p);
        return n + (p + 1 + DB < NBK) + (p >= 1);
    }
    static constexpr Op op(int p, int i)
    {
        for (int u = 0; u < NR; ++u)
            if (fphase(u) == p && i-- == 0)
                return Op{FETCH, u};
        if (p + 1 + DB < NBK && i-- == 0)
            return Op{BLOCK, p + 1 + DB};
        for (int u = 0; u < NR; ++u)
            if (wphase(u) == p && i-- == 0)
                return Op{WRITE, u};
        if (p >= 1 && i-- == 0)
            return Op{STORE, p - 1};
        return Op{NONE, 0};
    }
    // operation i goes to the gap after MFMA i * 4 (p + 1) / nops(p) of the
    // phase's 4 (p + 1); first(p, s) is the first operation of gap s or later
    static constexpr int first(int p, int s)
    {
        const int n = nops(p), m = 4 * (p + 1);
        return (s * n + m - 1) / m;
    }
    static constexpr bool valid()
    {
        if (STREAM && K < D)
            return false;
        for (int u = 0; u < NR; ++u)
            for (int t = u * TPR; t < (u + 1) * TPR && t < NTILE; ++t) {
                if (pro(u)) {
                    if (t >= CAP)
                        return false;
                } else if (t >= CAP && mk::tile_row(t - CAP) > last_barrier(wphase(u)) - 1) {
                    // slot still read by a wavefront that has not passed the last barrier
                    return false;
                }
                if (!pro(u) && fphase(u) < 0)
                    return false;
                if (!pro(u)) {
                    // a barrier between the write and the first phase that reads it
                    bool ok = false;
                    for (int b = wphase(u) + 1; b <= need(u); ++b)
                        ok = ok || barrier_at(b);
                    if (!ok)
                        return false;
                }
            }
        return true;
    }
};

// VEC: the panel's vectors are contiguous (sd == 1), 16-byte aligned, and nb is
// a multiple of 4, so a lane's four rows of a tile move as one or two 16-byte
// accesses.
template <typename T, int NB, bool SOLVE, bool VEC>
__global__ __launch_bounds__(256, 1) void mleaf_kernel(LeafDesc d, const T *__restrict__ Lp, T *__restrict__ B)
{
    using S = LeafSched<T, NB>;
    static_assert(S::valid(), "leaf memory schedule");
    constexpr int NBK = S::NBK, NR = S::NR, CAP = S::CAP, W = S::W, TPR = S::TPR, DB = S::DB;
    constexpr int TOT = S::NTILE * TE;
    using V = typename Vec16<T>::V;
    using A4 = typename mk::Acc<T>::V;

    __shared__ __attribute__((aligned(16))) T Lr[CAP * TE];

    const int tid = threadIdx.x, lane = tid % 64;
    const int w = __builtin_amdgcn_readfirstlane(tid / 64);
    const int c = lane % 16, g = lane / 16;
    const int64_t vec = (int64_t)blockIdx.x * 64 + 16 * w + c;
    const bool act = vec < d.nvec;
    int nb = d.nb;
    if (d.ka > 0) {
        // one of all the diagonal blocks (blockIdx.y)
        const int64_t d0 = (int64_t)blockIdx.y * NB;
        nb = (int)min<int64_t>(NB, d.ka - d0);
        B += d0 * d.sd;
        Lp += (int64_t)blockIdx.y * TOT;
    }
    const bool mlower = d.mlower;
    T *Bv = B + vec * d.si;
    const T alpha = T(d.alpha);

    // thread tid carries elements [tid W, tid W + W) of every round: tile
    // u TPR + x of the round, offset o within it
    const int x = tid * W / TE, o = tid * W % TE;
    V st[NR];
    auto fetch = [&](int u) {
        if (u * TPR * TE + tid * W < TOT)
            st[u] = *reinterpret_cast<const V *>(Lp + (int64_t)u * TPR * TE + tid * W);
    };
    auto write = [&](int u) {
        if (u * TPR * TE + tid * W < TOT) {
            int slot = (u * TPR) % CAP + x;
            if (slot >= CAP)
                slot -= CAP;
            *reinterpret_cast<V *>(Lr + slot * TE + o) = st[u];
        }
    };

    // row block i of the panel: slot r of the lane holds row RB i + 4g + r
    A4 acc[NBK];
    A4 res;   // the last finished row block of the result, stored one phase later
    auto load_block = [&](int i) {
        if (VEC) {
            const int r0 = RB * i + 4 * g;
            A4 v = A4{0, 0, 0, 0};
            if (act && r0 < nb) {
                v = ld4(Bv + (mlower ? r0 : nb - 4 - r0));
                if (!mlower)
                    v = v.wzyx;
            }
            acc[i] = v;
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = RB * i + 4 * g + r;
                const int dm = mlower ? row : nb - 1 - row;
                acc[i][r] = (act && row < nb) ? Bv[(int64_t)dm * d.sd] : T(0);
            }
        }
    };
    auto store_block = [&](int i) {
        A4 v = res;
        if (!SOLVE)
            v *= alpha;
        if (VEC) {
            const int r0 = RB * i + 4 * g;
            if (act && r0 < nb)
                st4(Bv + (mlower ? r0 : nb - 4 - r0), mlower ? v : v.wzyx);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = RB * i + 4 * g + q;
                const int dm = mlower ? row : nb - 1 - row;
                if (act && row < nb)
                    Bv[(int64_t)dm * d.sd] = v[q];
            }
        }
    };

    mk::static_for<0, NR>([&](auto U) {
        if constexpr (S::pro(decltype(U)::value))
            fetch(U);
    });
    mk::static_for<0, (DB + 1 < NBK ? DB + 1 : NBK)>([&](auto I) { load_block(I); });
    mk::static_for<0, NR>([&](auto U) {
        if constexpr (S::pro(decltype(U)::value))
            write(U);
    });

    mk::leaf_rows<T, NB, SOLVE>(
        acc, lane, [&](int p, int k) -> const T * { return Lr + (mk::rb_tile(p, k) % CAP) * TE; },
        [&](auto P) {
            if constexpr (S::barrier_at(decltype(P)::value))
                __syncthreads();
            if (SOLVE)
                acc[decltype(P)::value] *= alpha;
        },
        [&](auto, A4 r) { res = r; },
        [&](auto P, auto Sx) {
            constexpr int p = decltype(P)::value, s = decltype(Sx)::value;
            mk::static_for<S::first(p, s), S::first(p, s + 1)>([&](auto I) {
                constexpr typename S::Op op = S::op(p, decltype(I)::value);
                if constexpr (op.kind == S::FETCH)
                    fetch(op.arg);
                else if constexpr (op.kind == S::BLOCK)
                    load_block(op.arg);
                else if constexpr (op.kind == S::WRITE)
                    write(op.arg);
                else if constexpr (op.kind == S::STORE)
                    store_block(op.arg);
            });
            // memory operations and MFMAs keep their places; LDS reads and
            // scalar / vector arithmetic may move across
            __builtin_amdgcn_sched_barrier(0x2 | 0x4 | 0x100);
        });
    store_block(NBK - 1);
}

template <typename T, bool SOLVE, int NB>
hipError_t launch_nb(const LeafDesc &l, hipStream_t st)
{
    const dim3 grid((unsigned)((l.nvec + 63) / 64), l.ka > 0 ? (unsigned)((l.ka + NB - 1) / NB) : 1u);
    const T *L = static_cast<const T *>(l.Lp);
    T *B = static_cast<T *>(l.B);
    const bool vec = l.sd == 1 && (l.ka > 0 ? l.ka : (int64_t)l.nb) % 4 == 0 &&
                     reinterpret_cast<uintptr_t>(B) % 16 == 0 && (l.si * (int64_t)sizeof(T)) % 16 == 0;
    if (vec)
        hipLaunchKernelGGL((mleaf_kernel<T, NB, SOLVE, true>), grid, dim3(256), 0, st, l, L, B);
    else
        hipLaunchKernelGGL((mleaf_kernel<T, NB, SOLVE, false>), grid, dim3(256), 0, st, l, L, B);
    return hipGetLastError();
}

// one element type and operation, every leaf size
template <typename T, bool SOLVE>
hipError_t launch(int nbmax, const LeafDesc &l, hipStream_t st)
{
    switch (nbmax) {
    case 64: return launch_nb<T, SOLVE, 64>(l, st);
    case 128: return launch_nb<T, SOLVE, 128>(l, st);
    case 256: return launch_nb<T, SOLVE, 256>(l, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mleaf
}  // namespace rtri
