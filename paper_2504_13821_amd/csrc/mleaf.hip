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
// (c, g) = (lane % 16, lane / 16) holds vector c, rows Acc::row(g, r) of a
// tile in slot r.  For K slice t an MFMA reads B[k = g][c] from lane (c, g);
// slot t of a tile holds exactly the rows {Acc::row(g, t)}, so a tile is the B
// operand of the next MFMA as it stands, with K index g of slice t labelled by
// row Acc::row(g, t).  The A operand (16 x 16 triangle tile M) then carries
// M[m][Acc::row(g, t)] in lane (m, g) for slice t; the pack pass writes every
// tile in that order.  No data moves between lanes, and the four wavefronts
// never wait on each other.
//
// Solve, row blocks j ascending:  X_j = inv(T_jj) B_j;  B_i += (-L_ij) X_j, i > j.
// Multiply, j descending:         B_i += L_ij B_j (i > j);  B_j = T_jj B_j.
// inv(T_jj) is the exact-arithmetic inverse of the 16 x 16 diagonal tile,
// formed in FP64 by substitution in the pack pass and rounded once to the
// panel type; applying it as a product instead of 16 dependent divisions is
// the one difference from a substitution leaf (its error is bounded by
// cond(T_jj) u instead of a small multiple of u; the diagonal tiles of a
// triangle with a dominant diagonal have cond(T_jj) close to 1).
//
// The packed triangle streams through a three-slot LDS ring one column block
// (16 columns, tiles j..NB/16-1) at a time, two phases ahead of its use.
#include "leaf_core.h"
#include "mleaf_core.h"

namespace rtri {

namespace {

using lk::ld_src;
using mk::RB;
using mk::TE;
using mk::cb_tile;
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

// One workgroup per diagonal block: every tile in A-operand order.
//   solve:    diagonal tiles inv(T_jj), off-diagonal tiles -L_ij
//   multiply: diagonal tiles T_jj,      off-diagonal tiles  L_ij
template <ElemT S, typename T, int NB, bool SOLVE>
__global__ __launch_bounds__(256) void mpack_kernel(PackDesc p)
{
    constexpr int NBK = NB / RB;
    constexpr int NTILE = NBK * (NBK + 1) / 2;
    __shared__ double Dg[NBK][RB][RB + 1];    // diagonal tiles (inverted for a solve), FP64
    const int64_t d0 = (int64_t)blockIdx.x * NB;
    const int nb = (int)min<int64_t>(NB, p.ka - d0);
    const int64_t base = d0 + d0 * p.lda;
    T *out = static_cast<T *>(p.out) + (int64_t)blockIdx.x * NTILE * TE;
    const int tid = threadIdx.x;

    // thread (j, k): column k of diagonal tile j, inverted by forward
    // substitution for a solve (values rounded to T first, FP64 arithmetic)
    if (tid < NBK * RB) {
        const int j = tid / RB, k = tid % RB;
        double y[RB];
        mk::diag_column<SOLVE>(
            k, [&](int m, int q) { return (double)canon<S, T>(p, base, nb, RB * j + m, RB * j + q); }, y);
#pragma unroll
        for (int m = 0; m < RB; ++m)
            Dg[j][m][k] = y[m];
    }
    __syncthreads();

    for (int e = tid; e < NTILE * TE; e += 256) {
        const int tile = e / TE;
        int m, kk;
        mk::tile_entry<T>(e % TE, m, kk);
        int j = 0;
        while (j + 1 < NBK && cb_tile(NBK, j + 1) <= tile)
            ++j;
        const int i = j + (tile - cb_tile(NBK, j));
        T v;
        if (i == j) {
            v = (T)Dg[j][m][kk];
        } else {
            v = canon<S, T>(p, base, nb, RB * i + m, RB * j + kk);
            if (SOLVE)
                v = -v;
        }
        out[e] = v;
    }
}

template <typename T> struct Vec16;
template <> struct Vec16<double> { using V = double __attribute__((ext_vector_type(2))); };
template <> struct Vec16<float> { using V = float __attribute__((ext_vector_type(4))); };

template <typename T, int NB, bool SOLVE>
__global__ __launch_bounds__(256, 1) void mleaf_kernel(LeafDesc d, const T *__restrict__ Lp, T *__restrict__ B)
{
    constexpr int NBK = NB / RB;
    constexpr int SLOT = NBK * TE;                // elements of the largest column block
    constexpr int W = 16 / (int)sizeof(T);
    constexpr int NV = SLOT / (256 * W);          // 16-byte loads per thread per column block
    static_assert(NV * 256 * W == SLOT, "column block split");
    using V = typename Vec16<T>::V;
    using AccT = mk::Acc<T>;
    using A4 = typename AccT::V;

    __shared__ __attribute__((aligned(16))) T Lr[3 * SLOT];

    const int tid = threadIdx.x, lane = tid % 64;
    const int w = __builtin_amdgcn_readfirstlane(tid / 64);
    const int c = lane % 16, g = lane / 16;
    const int64_t vec = (int64_t)blockIdx.x * 64 + 16 * w + c;
    const bool act = vec < d.nvec;
    const int nb = d.nb;
    T *Bv = B + vec * d.si;

    auto cbk = [](int s) { return SOLVE ? s : NBK - 1 - s; };
    V pre0[NV], pre1[NV];
    auto gload = [&](int s, V(&dst)[NV]) {
        const int cc = cbk(s);
        const int cnt = (NBK - cc) * TE;
        const T *src = Lp + (int64_t)cb_tile(NBK, cc) * TE;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = (v * 256 + tid) * W;
            if (e < cnt)
                dst[v] = *reinterpret_cast<const V *>(src + e);
        }
    };
    auto lstore = [&](int s, const V(&src)[NV]) {
        const int cc = cbk(s);
        const int cnt = (NBK - cc) * TE;
        T *dst = Lr + (s % 3) * SLOT;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = (v * 256 + tid) * W;
            if (e < cnt)
                *reinterpret_cast<V *>(dst + e) = src[v];
        }
    };

    gload(0, pre0);
    if (NBK > 1)
        gload(1, pre1);

    A4 acc[NBK];
#pragma unroll
    for (int i = 0; i < NBK; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = RB * i + AccT::row(g, r);
            const int dm = d.mlower ? row : nb - 1 - row;
            acc[i][r] = (act && row < nb) ? Bv[(int64_t)dm * d.sd] : T(0);
        }
    const T alpha = T(d.alpha);
    if (SOLVE)
#pragma unroll
        for (int i = 0; i < NBK; ++i)
            acc[i] *= alpha;

    lstore(0, pre0);
    if (NBK > 1)
        lstore(1, pre1);
    if (NBK > 2)
        gload(2, pre0);
    __syncthreads();

    mk::leaf_phases<T, NB, SOLVE>(
        acc, lane, [&](int s, int ti) -> const T * { return Lr + (s % 3) * SLOT + ti * TE; },
        [&](int s) {
            if (s + 2 < NBK)
                lstore(s + 2, pre0);
            if (s + 3 < NBK)
                gload(s + 3, pre0);
            __syncthreads();
        });

    if (!SOLVE)
#pragma unroll
        for (int i = 0; i < NBK; ++i)
            acc[i] *= alpha;
#pragma unroll
    for (int i = 0; i < NBK; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = RB * i + AccT::row(g, r);
            const int dm = d.mlower ? row : nb - 1 - row;
            if (act && row < nb)
                Bv[(int64_t)dm * d.sd] = acc[i][r];
        }
}

template <typename T, int NB>
hipError_t mleaf_nb(bool solve, const LeafDesc &l, hipStream_t st)
{
    const dim3 grid((unsigned)((l.nvec + 63) / 64));
    const T *L = static_cast<const T *>(l.Lp);
    T *B = static_cast<T *>(l.B);
    if (solve)
        hipLaunchKernelGGL((mleaf_kernel<T, NB, true>), grid, dim3(256), 0, st, l, L, B);
    else
        hipLaunchKernelGGL((mleaf_kernel<T, NB, false>), grid, dim3(256), 0, st, l, L, B);
    return hipGetLastError();
}

template <ElemT S, typename T, int NB>
void mpack_nb(bool solve, const PackDesc &p, hipStream_t st)
{
    const unsigned nblk = (unsigned)((p.ka + NB - 1) / NB);
    if (solve)
        hipLaunchKernelGGL((mpack_kernel<S, T, NB, true>), dim3(nblk), dim3(256), 0, st, p);
    else
        hipLaunchKernelGGL((mpack_kernel<S, T, NB, false>), dim3(nblk), dim3(256), 0, st, p);
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
    if (l.nvec <= 0 || l.nb <= 0)
        return hipSuccess;
    if (l.nb > nbmax)
        return hipErrorInvalidValue;
    if (t == DType::F64) {
        switch (nbmax) {
        case 64: return mleaf_nb<double, 64>(solve, l, st);
        case 128: return mleaf_nb<double, 128>(solve, l, st);
        case 256: return mleaf_nb<double, 256>(solve, l, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (nbmax) {
    case 64: return mleaf_nb<float, 64>(solve, l, st);
    case 128: return mleaf_nb<float, 128>(solve, l, st);
    case 256: return mleaf_nb<float, 256>(solve, l, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace rtri
