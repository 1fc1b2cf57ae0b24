// Leaf kernels: triangular solve / multiply of one diagonal block against a
// panel of independent vectors (paper, Sec. 3.3).
//
// The paper's base TRSM gives each thread a row of one right-hand-side column
// and synchronises after every row.  On CDNA4 a wavefront is 64 lanes wide and
// has a large register file, so here each lane owns one whole vector (a column
// of B for side = L, a row of B for side = R) and keeps it in registers: the
// row-to-row dependency becomes a register dependency inside one lane and needs
// no barrier.  The diagonal block is staged once per workgroup in LDS, in a
// canonical lower-triangular column-major layout, and read back as wave-uniform
// broadcasts.  Upper-triangular blocks are handled by reversing the row order
// (canonical row i <-> block row nb-1-i), transposed blocks by the order of the
// global reads, so one kernel covers every side / uplo / trans combination.
//
// Solve (right-looking forward substitution, IEEE division by the diagonal):
//     b := alpha*b;  for k: x_k = b_k / L(k,k);  b_i -= L(i,k) x_k  (i > k)
// Multiply (descending, so every row still reads original values):
//     for k = nb-1..0: b_i += L(i,k) b_k (i > k);  b_k := L(k,k) b_k;   b := alpha*b
#include "common.h"

namespace rtri {

namespace {

constexpr int WAVE = 64;

// packed canonical lower triangle, column-major: L(i,k), i >= k, at colstart(k) + (i - k)
template <int NB> __host__ __device__ constexpr int colstart(int k) { return k * NB - k * (k - 1) / 2; }
template <int NB> constexpr int tri_elems() { return NB * (NB + 1) / 2; }

template <typename T, int NB, bool SOLVE, bool UNIT>
__global__ __launch_bounds__(WAVE) void leaf_kernel(LeafDesc d)
{
    static_assert(NB <= WAVE, "one lane per block row when staging");
    constexpr int PS = NB + 1;                  // padded panel stride (odd: no bank conflicts)
    __shared__ T Ls[tri_elems<NB>()];           // the diagonal block, canonical lower
    __shared__ T Ps[WAVE * PS];                 // the panel: vector v, canonical row i at Ps[v*PS + i]

    const int lane = threadIdx.x;
    const int nb = d.nb;
    const T *A = static_cast<const T *>(d.A);
    const int64_t lda = d.lda;

    // stage the block: L(i,k) = Mx(p(i), p(k)) with p(i) = i (lower) or nb-1-i (upper);
    // rows beyond nb are padded with the identity so they are inert
    for (int k = 0; k < NB; ++k) {
        for (int i = k + lane; i < NB; i += WAVE) {
            T v = T(0);
            if (i == k) {
                v = T(1);
                if (!UNIT && i < nb) {
                    const int r = d.mlower ? i : nb - 1 - i;
                    v = A[r + (int64_t)r * lda];
                }
            } else if (i < nb) {
                const int r = d.mlower ? i : nb - 1 - i;
                const int c = d.mlower ? k : nb - 1 - k;
                v = d.mtrans ? A[c + (int64_t)r * lda] : A[r + (int64_t)c * lda];
            }
            Ls[colstart<NB>(k) + (i - k)] = v;
        }
    }

    // stage the panel with coalesced reads: lanes run along whichever of the two
    // panel dimensions is contiguous in memory
    const int64_t v0 = (int64_t)blockIdx.x * WAVE;
    const int nv = (int)min<int64_t>(WAVE, d.nvec - v0);
    T *B = static_cast<T *>(d.B);
    const bool along_d = d.sd == 1;
    for (int it = 0; it < (along_d ? WAVE : NB); ++it) {
        const int dd = along_d ? lane : it;      // element index in block order
        const int vv = along_d ? it : lane;      // vector index within this workgroup
        if (dd < nb && vv < nv) {
            const int ci = d.mlower ? dd : nb - 1 - dd;
            Ps[vv * PS + ci] = B[(v0 + vv) * d.si + (int64_t)dd * d.sd];
        }
    }
    __syncthreads();

    const T alpha = T(d.alpha);
    T b[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
        b[i] = (i < nb && lane < nv) ? Ps[lane * PS + i] : T(0);

    if (SOLVE) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
            b[i] *= alpha;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (!UNIT)
                b[k] = b[k] / Ls[colstart<NB>(k)];
            const T x = b[k];
#pragma unroll
            for (int i = k + 1; i < NB; ++i)
                b[i] = fmat(-Ls[colstart<NB>(k) + (i - k)], x, b[i]);
        }
    } else {
#pragma unroll
        for (int k = NB - 1; k >= 0; --k) {
            const T x = b[k];
#pragma unroll
            for (int i = k + 1; i < NB; ++i)
                b[i] = fmat(Ls[colstart<NB>(k) + (i - k)], x, b[i]);
            if (!UNIT)
                b[k] = Ls[colstart<NB>(k)] * x;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i)
            b[i] *= alpha;
    }

#pragma unroll
    for (int i = 0; i < NB; ++i)
        Ps[lane * PS + i] = b[i];
    __syncthreads();
    for (int it = 0; it < (along_d ? WAVE : NB); ++it) {
        const int dd = along_d ? lane : it;
        const int vv = along_d ? it : lane;
        if (dd < nb && vv < nv) {
            const int ci = d.mlower ? dd : nb - 1 - dd;
            B[(v0 + vv) * d.si + (int64_t)dd * d.sd] = Ps[vv * PS + ci];
        }
    }
}

template <typename T, int NB>
hipError_t launch_nb(bool solve, const LeafDesc &l, hipStream_t st)
{
    const dim3 grid((unsigned)((l.nvec + WAVE - 1) / WAVE));
    if (solve) {
        if (l.unit)
            hipLaunchKernelGGL((leaf_kernel<T, NB, true, true>), grid, dim3(WAVE), 0, st, l);
        else
            hipLaunchKernelGGL((leaf_kernel<T, NB, true, false>), grid, dim3(WAVE), 0, st, l);
    } else {
        if (l.unit)
            hipLaunchKernelGGL((leaf_kernel<T, NB, false, true>), grid, dim3(WAVE), 0, st, l);
        else
            hipLaunchKernelGGL((leaf_kernel<T, NB, false, false>), grid, dim3(WAVE), 0, st, l);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_leaf(DType t, bool solve, int nbmax, const LeafDesc &l, hipStream_t st)
{
    if (l.nvec <= 0 || l.nb <= 0)
        return hipSuccess;
    if (l.nb > nbmax)
        return hipErrorInvalidValue;
    if (t == DType::F64) {
        switch (nbmax) {
        case 16: return launch_nb<double, 16>(solve, l, st);
        case 32: return launch_nb<double, 32>(solve, l, st);
        case 64: return launch_nb<double, 64>(solve, l, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (nbmax) {
    case 16: return launch_nb<float, 16>(solve, l, st);
    case 32: return launch_nb<float, 32>(solve, l, st);
    case 64: return launch_nb<float, 64>(solve, l, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace rtri
