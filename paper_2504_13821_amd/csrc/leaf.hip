// Substitution leaf kernels (diagonal blocks of 16 or 32 rows): triangular
// solve / multiply of one diagonal block against a panel of independent vectors
// (paper, Sec. 3.3).  Blocks of 64 rows and more run on the matrix cores
// (mleaf.hip); launch_pack / launch_leaf dispatch by block size.
//
// The paper's base TRSM gives each thread a row of one right-hand-side column
// and synchronises after every row.  On CDNA4 a wavefront is 64 lanes wide and
// has a large register file, so here each lane owns one whole vector (a column
// of B for side = L, a row of B for side = R) and keeps it in registers: the
// row-to-row dependency becomes a register dependency inside one lane and needs
// no barrier.  The panel is transposed through LDS so that both the global
// reads and writes are coalesced whichever side is solved.
//
// The diagonal block is wave-uniform data.  One pack pass per call writes every
// diagonal block in a canonical lower-triangular packed form (upper blocks with
// reversed row order, transposed blocks transposed), laid out in the order the
// leaf consumes it: column by column, diagonal entry first, ascending columns
// for the solve and descending for the multiply.  The leaf copies its block
// into LDS and streams it through a small register ring, issuing the broadcast
// LDS reads several chunks ahead of their use so their latency is hidden behind
// the FMAs of the chunks before.
//
// Solve (right-looking forward substitution, IEEE division by the diagonal):
//     b := alpha*b;  for k: x_k = b_k / L(k,k);  b_i -= L(i,k) x_k  (i > k)
// Multiply (descending, so every row still reads original values):
//     for k = nb-1..0: b_i += L(i,k) b_k (i > k);  b_k := L(k,k) b_k;   b := alpha*b
#include "leaf_core.h"

namespace rtri {

namespace {

using namespace lk;

// One workgroup per diagonal block: the canonical packed form read by the leaves.
template <ElemT S, typename T, int NB, bool ASC>
__global__ __launch_bounds__(256) void pack_kernel(PackDesc p)
{
    const int64_t d0 = (int64_t)blockIdx.x * NB;
    const int nb = (int)min<int64_t>(NB, p.ka - d0);
    T *out = static_cast<T *>(p.out) + (int64_t)blockIdx.x * tri_n<NB>();
    stage_block<S, T, NB, ASC, 256>(p.A, d0 + d0 * p.lda, p.lda, nb, p.mtrans, p.mlower, p.unit, out, threadIdx.x);
}

// One wavefront per 64 vectors of the panel.  The block's packed form is copied
// into LDS while the panel's loads are in flight.
template <typename T, int NB, bool SOLVE, bool UNIT>
__global__ __launch_bounds__(WAVE) void leaf_kernel(LeafDesc d, const T *__restrict__ L, T *__restrict__ B)
{
    __shared__ T Ps[WAVE * (NB + 1)];
    __shared__ __attribute__((aligned(16))) T Ls[tri_n<NB>()];
    const int lane = threadIdx.x;
    constexpr int TOT = tri_n<NB>();
    constexpr int PER = (TOT + WAVE - 1) / WAVE;
    T tv[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j)
        tv[j] = (j * WAVE + lane < TOT) ? L[j * WAVE + lane] : T(0);
    leaf_panel<T, NB, SOLVE, UNIT>(d, B, Ls, Ps, (int64_t)blockIdx.x * WAVE, [&] {
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (j * WAVE + lane < TOT)
                Ls[j * WAVE + lane] = tv[j];
    });
}

template <typename T, int NB>
hipError_t launch_nb(bool solve, const LeafDesc &l, hipStream_t st)
{
    const dim3 grid((unsigned)((l.nvec + WAVE - 1) / WAVE));
    const T *L = static_cast<const T *>(l.Lp);
    T *B = static_cast<T *>(l.B);
    if (solve) {
        if (l.unit)
            hipLaunchKernelGGL((leaf_kernel<T, NB, true, true>), grid, dim3(WAVE), 0, st, l, L, B);
        else
            hipLaunchKernelGGL((leaf_kernel<T, NB, true, false>), grid, dim3(WAVE), 0, st, l, L, B);
    } else {
        if (l.unit)
            hipLaunchKernelGGL((leaf_kernel<T, NB, false, true>), grid, dim3(WAVE), 0, st, l, L, B);
        else
            hipLaunchKernelGGL((leaf_kernel<T, NB, false, false>), grid, dim3(WAVE), 0, st, l, L, B);
    }
    return hipGetLastError();
}

template <ElemT S, typename T, int NB>
hipError_t pack_nb(bool solve, const PackDesc &p, hipStream_t st)
{
    const unsigned nblk = (unsigned)((p.ka + NB - 1) / NB);
    if (solve)
        hipLaunchKernelGGL((pack_kernel<S, T, NB, true>), dim3(nblk), dim3(256), 0, st, p);
    else
        hipLaunchKernelGGL((pack_kernel<S, T, NB, false>), dim3(nblk), dim3(256), 0, st, p);
    return hipGetLastError();
}

template <ElemT S, typename T>
hipError_t pack_t(bool solve, int nbmax, const PackDesc &p, hipStream_t st)
{
    switch (nbmax) {
    case 16: return pack_nb<S, T, 16>(solve, p, st);
    case 32: return pack_nb<S, T, 32>(solve, p, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_pack(ElemT src, DType dst, bool solve, int nbmax, const PackDesc &p, hipStream_t st)
{
    if (p.ka <= 0)
        return hipSuccess;
    if (nbmax >= 64)
        return launch_bpack(src, dst, solve, nbmax, p, st);
    if (dst == DType::F64) {
        if (src != ElemT::F64)
            return hipErrorInvalidValue;
        return pack_t<ElemT::F64, double>(solve, nbmax, p, st);
    }
    switch (src) {
    case ElemT::F64: return pack_t<ElemT::F64, float>(solve, nbmax, p, st);
    case ElemT::F32: return pack_t<ElemT::F32, float>(solve, nbmax, p, st);
    case ElemT::BF16: return pack_t<ElemT::BF16, float>(solve, nbmax, p, st);
    case ElemT::F16: return pack_t<ElemT::F16, float>(solve, nbmax, p, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_leaf(DType t, bool solve, int nbmax, const LeafDesc &l, hipStream_t st)
{
    if (l.ka > 0)   // all diagonal blocks in one launch: matrix-core leaves only
        return nbmax >= 64 ? launch_bleaf(t, solve, nbmax, l, st) : hipErrorInvalidValue;
    if (l.nvec <= 0 || l.nb <= 0)
        return hipSuccess;
    if (l.nb > nbmax)
        return hipErrorInvalidValue;
    if (nbmax >= 64)
        return launch_bleaf(t, solve, nbmax, l, st);
    if (t == DType::F64) {
        switch (nbmax) {
        case 16: return launch_nb<double, 16>(solve, l, st);
        case 32: return launch_nb<double, 32>(solve, l, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (nbmax) {
    case 16: return launch_nb<float, 16>(solve, l, st);
    case 32: return launch_nb<float, 32>(solve, l, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace rtri
