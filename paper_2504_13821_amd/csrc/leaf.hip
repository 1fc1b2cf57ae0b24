// Leaf kernels: triangular solve / multiply of one diagonal block against a
// panel of independent vectors (paper, Sec. 3.3).
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
#include "common.h"

namespace rtri {

namespace {

constexpr int WAVE = 64;

template <int NB> constexpr int tri_n() { return NB * (NB + 1) / 2; }
// start of column k in the stream: ascending columns (solve) or descending (multiply)
template <int NB, bool ASC> __host__ __device__ constexpr int colstart(int k)
{
    return ASC ? k * NB - k * (k - 1) / 2 : (NB - 1 - k) * (NB - k) / 2;
}

template <ElemT S> __device__ __forceinline__ double ld_src(const void *p, int64_t off);
template <> __device__ __forceinline__ double ld_src<ElemT::F64>(const void *p, int64_t off)
{
    return static_cast<const double *>(p)[off];
}
template <> __device__ __forceinline__ double ld_src<ElemT::F32>(const void *p, int64_t off)
{
    return static_cast<const float *>(p)[off];
}
template <> __device__ __forceinline__ double ld_src<ElemT::BF16>(const void *p, int64_t off)
{
    return __uint_as_float((unsigned)static_cast<const unsigned short *>(p)[off] << 16);
}
template <> __device__ __forceinline__ double ld_src<ElemT::F16>(const void *p, int64_t off)
{
    return (double)__builtin_bit_cast(_Float16, static_cast<const unsigned short *>(p)[off]);
}

// One workgroup per diagonal block.  The source may be narrower than the
// packed type (exact widening) or FP64 packed as FP32 (one rounding, to nearest).
template <ElemT S, typename T, int NB, bool ASC>
__global__ __launch_bounds__(256) void pack_kernel(PackDesc p)
{
    const int64_t d0 = (int64_t)blockIdx.x * NB;
    const int nb = (int)min<int64_t>(NB, p.ka - d0);
    const int64_t base = d0 + d0 * p.lda;
    T *out = static_cast<T *>(p.out) + (int64_t)blockIdx.x * tri_n<NB>();
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        const int i = e % NB, k = e / NB;
        if (i < k)
            continue;
        T v = (i == k) ? T(1) : T(0);
        if (i < nb && (i > k || !p.unit)) {
            const int r = p.mlower ? i : nb - 1 - i;
            const int c = p.mlower ? k : nb - 1 - k;
            v = (T)ld_src<S>(p.A, base + (p.mtrans ? c + (int64_t)r * p.lda : r + (int64_t)c * p.lda));
        }
        out[colstart<NB, ASC>(k) + (i - k)] = v;
    }
}

// Stream the packed block from LDS through a register ring of D chunks of CH
// values; chunk c + D is requested as soon as chunk c is used up.
template <typename T, int NB, bool SOLVE, bool UNIT>
__device__ __forceinline__ void leaf_compute(T (&b)[NB], const T *Ls)
{
    constexpr int TOT = tri_n<NB>();
    constexpr int CH = 8, D = 4;
    constexpr int NCH = (TOT + CH - 1) / CH;
    T ring[D][CH];
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
        for (int j = 0; j < CH; ++j)
            if (c < NCH && c * CH + j < TOT)
                ring[c][j] = Ls[c * CH + j];
    int f = 0;   // stream position (a compile-time constant once unrolled)
    T x = T(0), dk = T(1);
#pragma unroll
    for (int kk = 0; kk < NB; ++kk) {
        const int k = SOLVE ? kk : NB - 1 - kk;
        if (!SOLVE)
            x = b[k];
#pragma unroll
        for (int i = k; i < NB; ++i) {
            const T v = ring[(f / CH) % D][f % CH];
            if (i == k) {
                if (SOLVE) {
                    if (!UNIT)
                        b[k] = b[k] / v;
                    x = b[k];
                } else {
                    dk = v;
                }
            } else {
                b[i] = SOLVE ? fmat(-v, x, b[i]) : fmat(v, x, b[i]);
            }
            ++f;
            if (f % CH == 0) {
                const int c = f / CH - 1 + D;     // the chunk that reuses the slot just freed
                if (c < NCH) {
#pragma unroll
                    for (int j = 0; j < CH; ++j)
                        if (c * CH + j < TOT)
                            ring[c % D][j] = Ls[c * CH + j];
                }
                // keep the LDS reads where they are; arithmetic may move across
                __builtin_amdgcn_sched_barrier(0x7);
            }
        }
        if (!SOLVE && !UNIT)
            b[k] = dk * x;
    }
}

template <typename T, int NB, bool SOLVE, bool UNIT>
__global__ __launch_bounds__(WAVE) void leaf_kernel(LeafDesc d, const T *__restrict__ L, T *__restrict__ B)
{
    static_assert(NB <= WAVE, "one lane per block row when staging");
    constexpr int PS = NB + 1;                  // padded panel stride (odd: no bank conflicts)
    __shared__ T Ps[WAVE * PS];                 // the panel: vector v, canonical row i at Ps[v*PS + i]
    __shared__ __attribute__((aligned(16))) T Ls[tri_n<NB>()];   // the packed block, in stream order

    const int lane = threadIdx.x;
    const int nb = d.nb;

    // Stage the packed block (contiguous) and the panel into LDS.  All global
    // loads of both are issued before the first LDS store so that their
    // latencies overlap.  The panel is read coalesced: lanes run along
    // whichever of its two dimensions is contiguous in memory.
    constexpr int TOT = tri_n<NB>();
    constexpr int PER = (TOT + WAVE - 1) / WAVE;
    T tv[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j)
        tv[j] = (j * WAVE + lane < TOT) ? L[j * WAVE + lane] : T(0);

    const int64_t v0 = (int64_t)blockIdx.x * WAVE;
    const int nv = (int)min<int64_t>(WAVE, d.nvec - v0);
    const bool along_d = d.sd == 1;
    if (along_d) {
        // side L: lane = element of a column, one column per step
        const int dd = lane;
        const int ci = d.mlower ? dd : nb - 1 - dd;
        T pv[WAVE];
#pragma unroll
        for (int vv = 0; vv < WAVE; ++vv)
            pv[vv] = (dd < nb && vv < nv) ? B[(v0 + vv) * d.si + dd] : T(0);
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (j * WAVE + lane < TOT)
                Ls[j * WAVE + lane] = tv[j];
#pragma unroll
        for (int vv = 0; vv < WAVE; ++vv)
            if (dd < nb)
                Ps[vv * PS + ci] = pv[vv];
    } else {
        // side R: lane = one row of B, one column per step
        const int vv = lane;
        T pv[NB];
#pragma unroll
        for (int dd = 0; dd < NB; ++dd)
            pv[dd] = (dd < nb && vv < nv) ? B[(v0 + vv) * d.si + (int64_t)dd * d.sd] : T(0);
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (j * WAVE + lane < TOT)
                Ls[j * WAVE + lane] = tv[j];
#pragma unroll
        for (int dd = 0; dd < NB; ++dd)
            if (dd < nb)
                Ps[vv * PS + (d.mlower ? dd : nb - 1 - dd)] = pv[dd];
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
        leaf_compute<T, NB, true, UNIT>(b, Ls);
    } else {
        leaf_compute<T, NB, false, UNIT>(b, Ls);
#pragma unroll
        for (int i = 0; i < NB; ++i)
            b[i] *= alpha;
    }

#pragma unroll
    for (int i = 0; i < NB; ++i)
        Ps[lane * PS + i] = b[i];
    __syncthreads();
    if (along_d) {
        const int dd = lane;
        const int ci = d.mlower ? dd : nb - 1 - dd;
#pragma unroll
        for (int vv = 0; vv < WAVE; ++vv)
            if (dd < nb && vv < nv)
                B[(v0 + vv) * d.si + dd] = Ps[vv * PS + ci];
    } else {
        const int vv = lane;
#pragma unroll
        for (int dd = 0; dd < NB; ++dd)
            if (dd < nb && vv < nv)
                B[(v0 + vv) * d.si + (int64_t)dd * d.sd] = Ps[vv * PS + (d.mlower ? dd : nb - 1 - dd)];
    }
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
    case 64: return pack_nb<S, T, 64>(solve, p, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_pack(ElemT src, DType dst, bool solve, int nbmax, const PackDesc &p, hipStream_t st)
{
    if (p.ka <= 0)
        return hipSuccess;
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
