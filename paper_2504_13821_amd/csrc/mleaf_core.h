// Device-side building blocks of the matrix-core leaves (see mleaf.hip), shared
// with the batched kernel so both compute every diagonal block with the same
// operations in the same order.
#pragma once

#include "gemm_core.h"

namespace rtri {
namespace mk {

using gk::Acc;

constexpr int RB = 16;    // rows / columns of a tile
constexpr int TE = 256;   // elements of a tile

// first tile of column block c (tiles c..nbk-1 of that block follow in order)
__host__ __device__ constexpr int cb_tile(int nbk, int c) { return c * nbk - c * (c - 1) / 2; }
template <int NB> __host__ __device__ constexpr int ntiles() { return (NB / RB) * (NB / RB + 1) / 2; }

// element (K slice t, lane) of a tile in A-operand order: 16-byte groups of W
// slices per lane
template <typename T> __host__ __device__ constexpr int tile_pos(int t, int lane)
{
    constexpr int W = 16 / (int)sizeof(T);
    return ((t / W) * 64 + lane) * W + t % W;
}
// inverse of tile_pos: the tile entry M[m][kk] that position pos holds
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

// D = M * X + C for the tile M (A-operand order) at Mt; X in accumulator
// layout serves as the B operand, K index g of slice t labelled by row
// Acc::row(g, t)
template <typename T>
__device__ __forceinline__ typename Acc<T>::V tile_mm(const T *Mt, int lane, const typename Acc<T>::V &X,
                                                      typename Acc<T>::V C)
{
#pragma unroll
    for (int t = 0; t < 4; ++t)
        C = Acc<T>::mfma(Mt[tile_pos<T>(t, lane)], X[t], C);
    return C;
}

// The phases of one leaf over the accumulator tiles acc[0..NB/16) of a
// wavefront.  tile(s, ti) returns the LDS address of tile ti (0 = diagonal) of
// the column block used in phase s; sync(s) runs after phase s (s < NBK - 1).
//   solve, blocks ascending:   X_j = inv(T_jj) B_j;  B_i += (-L_ij) X_j  (i > j)
//   multiply, descending:      B_i += L_ij B_j  (i > j);  B_j = T_jj B_j
template <typename T, int NB, bool SOLVE, class Tile, class Sync>
__device__ __forceinline__ void leaf_phases(typename Acc<T>::V (&acc)[NB / RB], int lane, Tile &&tile, Sync &&sync)
{
    constexpr int NBK = NB / RB;
    using A4 = typename Acc<T>::V;
#pragma unroll
    for (int s = 0; s < NBK; ++s) {
        const int j = SOLVE ? s : NBK - 1 - s;
        if (SOLVE) {
            acc[j] = tile_mm<T>(tile(s, 0), lane, acc[j], A4{0, 0, 0, 0});
#pragma unroll
            for (int i = j + 1; i < NBK; ++i)
                acc[i] = tile_mm<T>(tile(s, i - j), lane, acc[j], acc[i]);
        } else {
#pragma unroll
            for (int i = j + 1; i < NBK; ++i)
                acc[i] = tile_mm<T>(tile(s, i - j), lane, acc[j], acc[i]);
            acc[j] = tile_mm<T>(tile(s, 0), lane, acc[j], A4{0, 0, 0, 0});
        }
        if (s + 1 < NBK)
            sync(s);
    }
}

}  // namespace mk
}  // namespace rtri
