// Matrix-core leaves for diagonal blocks of 64, 128 or 256 rows (paper, Sec. 3.3:
// the base case of the recursion handles one diagonal block against the panel
// of right-hand sides; the leaf size is a tuning parameter).
//
// Why not one lane per vector, as in the 16/32-row leaves: with the triangle in LDS,
// every lane-FMA pulls its (broadcast) triangle value through the LDS return
// path, 8 bytes per lane for FP64, so several wavefronts on a CU saturate LDS
// long before the FMA units.  Here the panel lives in MFMA accumulator tiles
// and the triangle feeds the A operand, one distinct value per lane, which
// cuts LDS traffic by the wave width.
//
// Layout.  A workgroup of 4 wavefronts takes 64 vectors; wavefront w owns
// vectors 16w .. 16w+15 for all NB rows, as NB/16 accumulator tiles of 16
// rows x 16 vectors (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32).  Lane
// (c, g) = (lane % 16, lane / 16) holds vector c, tile rows Acc::row(g, r) of a
// tile in slot r.  For K slice t an MFMA reads B[k = g][c] from lane (c, g);
// slot t of a tile holds exactly the tile rows {Acc::row(g, t)}, so a tile is
// the B operand of the next MFMA as it stands, with K index g of slice t
// labelled by tile row Acc::row(g, t).  The A operand (16 x 16 triangle tile
// M) then carries M[m][Acc::row(g, t)] in lane (m, g) for slice t; the pack
// pass writes every tile in that order.  Tile rows are a relabelling of the
// block's rows (mk::lrow) under which slot r of group g is block row 4g + r,
// so a lane's slots are consecutive rows of its vector.  No data moves between
// lanes, and the four wavefronts never wait on each other's results.
//
// Phases, one row block p of 16 rows each, ascending (mk::leaf_rows):
//   solve:     X_p = inv(T_pp) (B_p - sum_{k<p} L_pk X_k)
//   multiply:  B_p := T_pp B_p + sum_{k<p} L_pk B_k   (from the original B)
// inv(T_pp) is the exact-arithmetic inverse of the 16 x 16 diagonal tile,
// formed in FP64 by substitution in the pack pass and rounded once to the
// panel type; applying it as a product instead of 16 dependent divisions is
// the one difference from a substitution leaf (its error is bounded by
// cond(T_pp) u instead of a small multiple of u; the diagonal tiles of a
// triangle with a dominant diagonal have cond(T_pp) close to 1).  Row block p
// needs only the panel's row blocks 0..p, so the panel streams in behind the
// first phases and each finished row block is stored while later ones are
// computed; the packed triangle streams through LDS, its tiles numbered row
// block by row block (mk::rb_tile).  The kernel and its memory schedule are in
// mleaf_kernel.h; this file holds the pack pass and the dispatch.
#include "leaf_core.h"
#include "mleaf_core.h"

namespace rtri {

namespace {

using lk::ld_src;
using mk::RB;
using mk::TE;
using mk::tile_pos;

// Canonical block element L(i, k), i >= k, rounded to T (identity past nb and
// on a unit diagonal).
template <ElemT S, typename T>
__device__ __forceinline__ T canon(const PackDesc &p, int64_t base, int nb, int i, int k)
{
    if (i >= nb || k >= nb)
        return i == k ? T(1) : T(0);
    if (i == k && p.unit)
        return T(1);
    const int r = p.mlower ? i : nb - 1 - i;
    const int c = p.mlower ? k : nb - 1 - k;
    return (T)ld_src<S>(p.A, base + (p.mtrans ? c + (int64_t)r * p.lda : r + (int64_t)c * p.lda));
}

// One workgroup per row block i (blockIdx.y) of a diagonal block
// (blockIdx.x): the tiles (i, 0..i) in A-operand order, tiles numbered by row
// block (mk::rb_tile).
//   solve:    diagonal tile inv(T_ii), off-diagonal tiles -L_ij
//   multiply: diagonal tile T_ii,      off-diagonal tiles  L_ij
template <ElemT S, typename T, int NB, bool SOLVE>
__global__ __launch_bounds__(256) void mpack_kernel(PackDesc p)
{
    constexpr int NTILE = mk::ntiles<NB>();
    static_assert(TE == 256, "one tile entry per thread");
    __shared__ double Dg[RB][RB + 1];    // the diagonal tile (inverted for a solve), FP64
    const int i = blockIdx.y;
    const int64_t d0 = (int64_t)blockIdx.x * NB;
    const int nb = (int)min<int64_t>(NB, p.ka - d0);
    const int64_t base = d0 + d0 * p.lda;
    T *out = static_cast<T *>(p.out) + ((int64_t)blockIdx.x * NTILE + mk::rb_tile(i, 0)) * TE;
    const int tid = threadIdx.x;

    // thread k < 16: column k of the diagonal tile, inverted by forward
    // substitution for a solve (values rounded to T first, FP64 arithmetic)
    if (tid < RB) {
        double y[RB];
        mk::diag_column<SOLVE>(
            tid, [&](int m, int q) { return (double)canon<S, T>(p, base, nb, RB * i + m, RB * i + q); }, y);
#pragma unroll
        for (int m = 0; m < RB; ++m)
            Dg[m][tid] = y[m];
    }
    // the off-diagonal entries of this thread (tile entry tid of each tile) meanwhile
    int m, kk;
    mk::tile_entry<T>(tid, m, kk);
    const int bm = mk::lrow<T>(m), bk = mk::lrow<T>(kk);
    for (int j = 0; j < i; ++j) {
        T v = canon<S, T>(p, base, nb, RB * i + bm, RB * j + bk);
        out[j * TE + tid] = SOLVE ? -v : v;
    }
    __syncthreads();
    out[i * TE + tid] = (T)Dg[bm][bk];
}

template <ElemT S, typename T, int NB>
void mpack_nb(bool solve, const PackDesc &p, hipStream_t st)
{
    const dim3 grid((unsigned)((p.ka + NB - 1) / NB), NB / RB);
    if (solve)
        hipLaunchKernelGGL((mpack_kernel<S, T, NB, true>), grid, dim3(256), 0, st, p);
    else
        hipLaunchKernelGGL((mpack_kernel<S, T, NB, false>), grid, dim3(256), 0, st, p);
}

template <ElemT S, typename T>
hipError_t mpack_t(bool solve, int nbmax, const PackDesc &p, hipStream_t st)
{
    if (nbmax == 64)
        mpack_nb<S, T, 64>(solve, p, st);
    else if (nbmax == 128)
        mpack_nb<S, T, 128>(solve, p, st);
    else if (nbmax == 256)
        mpack_nb<S, T, 256>(solve, p, st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

static_assert(TE * mk::ntiles<64>() == 2560 && TE * mk::ntiles<128>() == 9216 && TE * mk::ntiles<256>() == 34816,
              "packed sizes match bpack_elems");

hipError_t launch_bpack(ElemT src, DType dst, bool solve, int nbmax, const PackDesc &p, hipStream_t st)
{
    if (p.ka <= 0)
        return hipSuccess;
    if (dst == DType::F64) {
        if (src != ElemT::F64)
            return hipErrorInvalidValue;
        return mpack_t<ElemT::F64, double>(solve, nbmax, p, st);
    }
    switch (src) {
    case ElemT::F64: return mpack_t<ElemT::F64, float>(solve, nbmax, p, st);
    case ElemT::F32: return mpack_t<ElemT::F32, float>(solve, nbmax, p, st);
    case ElemT::BF16: return mpack_t<ElemT::BF16, float>(solve, nbmax, p, st);
    case ElemT::F16: return mpack_t<ElemT::F16, float>(solve, nbmax, p, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_bleaf(DType t, bool solve, int nbmax, const LeafDesc &l, hipStream_t st)
{
    if (l.nvec <= 0 || (l.ka > 0 ? l.ka : (int64_t)l.nb) <= 0)
        return hipSuccess;
    if (l.ka <= 0 && l.nb > nbmax)
        return hipErrorInvalidValue;
    if (t == DType::F64)
        return solve ? mleaf_launch_f64_solve(nbmax, l, st) : mleaf_launch_f64_mult(nbmax, l, st);
    return solve ? mleaf_launch_f32_solve(nbmax, l, st) : mleaf_launch_f32_mult(nbmax, l, st);
}

}  // namespace rtri
