// Device-side building blocks of the matrix-core leaves (see mleaf.hip), shared
// with the batched kernel so both compute every diagonal block with the same
// operations in the same order.
#pragma once

#include <type_traits>

#include "gemm_core.h"

namespace rtri {
namespace mk {

using gk::Acc;

// f(std::integral_constant<int, i>) for i = B .. E-1, in order: the index is a
// constant in every call whatever the unroller decides
template <int B, int E, class F> __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int RB = 16;    // rows / columns of a tile
constexpr int TE = 256;   // elements of a tile

using gk::Vec16;

// Tiles are numbered by row block: tile (p, k), k <= p, of row block p is
// number p (p + 1) / 2 + k (k == p: the diagonal tile).
__host__ __device__ constexpr int rb_tile(int p, int k) { return p * (p + 1) / 2 + k; }
template <int NB> __host__ __device__ constexpr int ntiles() { return (NB / RB) * (NB / RB + 1) / 2; }
// row block of tile t
__host__ __device__ constexpr int tile_row(int t)
{
    int p = 0;
    while (rb_tile(p + 1, 0) <= t)
        ++p;
    return p;
}

// Block rows are relabelled as in the GEMM (gk::lrow): slot r of lane group g
// of an accumulator tile holds block row 4g + r, so side-L panels move with
// 16-byte accesses.  Triangle tiles carry the same labelling on both indices,
// so the products are unchanged.
using gk::lrow;

// element (K slice t, lane) of a tile in A-operand order: 16-byte groups of W
// slices per lane
template <typename T> __host__ __device__ constexpr int tile_pos(int t, int lane)
{
    constexpr int W = 16 / (int)sizeof(T);
    return ((t / W) * 64 + lane) * W + t % W;
}
// inverse of tile_pos: the tile entry M[m][kk] (tile rows / columns) that
// position pos holds
template <typename T> __device__ __forceinline__ void tile_entry(int pos, int &m, int &kk)
{
    constexpr int W = 16 / (int)sizeof(T);
    const int q = pos / W;
    const int lane = q % 64, t = (q / 64) * W + pos % W;
    m = lane % 16;
    kk = Acc<T>::row(lane / 16, t);
}

// Column k of a 16 x 16 diagonal tile for the leaf: for a solve, column k of
// its inverse by forward substitution in FP64 (y_m = (e_k - sum_{q<m} T(m,q)
// y_q) / T(m,m), sums in ascending q); for a multiply, column k of the tile.
// tv(m, q) returns T(m, q) (m >= q) as a double.  Row m's reads are issued as
// one group and pinned there (arithmetic may move past them), so at most one
// row of the tile is in registers.
template <bool SOLVE, class TV> __device__ __forceinline__ void diag_column(int k, TV &&tv, double (&y)[RB])
{
#pragma unroll
    for (int m = 0; m < RB; ++m) {
        if (!SOLVE) {
            y[m] = m >= k ? tv(m, k) : 0.0;
            continue;
        }
        double row[RB];
#pragma unroll
        for (int q = 0; q <= m; ++q)
            row[q] = tv(m, q);
        __builtin_amdgcn_sched_barrier(0x7);
        double s = m == k ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < m; ++q)
            if (q >= k)
                s = __builtin_fma(-row[q], y[q], s);
        y[m] = m < k ? 0.0 : s / row[m];
    }
}

// The phases of one leaf over the accumulator tiles acc[0..NB/16) of a
// wavefront, one row block of 16 rows per phase, ascending.  tile(p, k)
// returns the LDS address of tile (p, k); sync(P) runs before phase p (P: p as
// a std::integral_constant); done(P, R) receives row block p of the result;
// mid(P, S) runs after MFMA s of phase p (S: s as an integral constant), so a
// caller can thread other work between the matrix instructions.
//   solve:     X_p = inv(T_pp) (B_p + sum_{k<p} (-L_pk) X_k), k ascending;
//              acc[p] becomes X_p
//   multiply:  R_p = T_pp B_p + sum_{k<p} L_pk B_k, k descending; acc keeps B
// Each result entry sees the same operations in the same order as in the
// column-oriented forms (solve: B_i += (-L_ij) X_j, j ascending, then
// X_i = inv(T_ii) B_i; multiply: B_i = T_ii B_i, then B_i += L_ij B_j, j
// descending), so the two agree bit for bit.  Row block p needs only B_0..B_p,
// so the panel can stream in while the first phases run, and each finished
// row block can be stored while the later ones are computed.
template <typename T, int NB, bool SOLVE, class Tile, class Sync, class Done, class Mid>
__device__ __forceinline__ void leaf_rows(typename Acc<T>::V (&acc)[NB / RB], int lane, Tile &&tile, Sync &&sync,
                                          Done &&done, Mid &&mid)
{
    constexpr int NBK = NB / RB;
    using A4 = typename Acc<T>::V;
    static_for<0, NBK>([&](auto P) {
        constexpr int p = decltype(P)::value;
        sync(P);
        // C + M X for the tile M (A-operand order) at Mt, one MFMA per K slice t;
        // X in accumulator layout serves as the B operand, K index g of slice t
        // labelled by tile row Acc::row(g, t).  S0: index of the first MFMA in the phase.
        auto mm = [&](const T *Mt, const A4 &X, A4 C, auto S0) {
            constexpr int W = 16 / (int)sizeof(T);
            T a[4];   // the lane's four A operands, read as 16-byte groups
            static_for<0, 4 / W>([&](auto J) {
                const auto v = *reinterpret_cast<const typename Vec16<T>::V *>(
                    Mt + tile_pos<T>(W * decltype(J)::value, lane));
#pragma unroll
                for (int e = 0; e < W; ++e)
                    a[W * decltype(J)::value + e] = v[e];
            });
            static_for<0, 4>([&](auto Tt) {
                constexpr int t = decltype(Tt)::value;
                C = Acc<T>::mfma(a[t], X[t], C);
                mid(P, std::integral_constant<int, decltype(S0)::value + t>{});
            });
            return C;
        };
        if constexpr (SOLVE) {
            static_for<0, p>([&](auto Kk) {
                constexpr int k = decltype(Kk)::value;
                acc[p] = mm(tile(p, k), acc[k], acc[p], std::integral_constant<int, 4 * k>{});
            });
            acc[p] = mm(tile(p, p), acc[p], A4{0, 0, 0, 0}, std::integral_constant<int, 4 * p>{});
            done(P, acc[p]);
        } else {
            A4 r = mm(tile(p, p), acc[p], A4{0, 0, 0, 0}, std::integral_constant<int, 0>{});
            static_for<0, p>([&](auto Jj) {
                constexpr int k = p - 1 - decltype(Jj)::value;
                r = mm(tile(p, k), acc[k], r, std::integral_constant<int, 4 * (p - k)>{});
            });
            done(P, r);
        }
    });
}

}  // namespace mk
}  // namespace rtri
