// Device-side building blocks of the leaf kernels (see leaf.hip), shared with
// the batched kernel.
#pragma once

#include "common.h"

namespace rtri {
namespace lk {

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

// Write one diagonal block (nb rows from element `base` of A) in canonical
// packed stream order to `out` (global or LDS), using the NTHR threads of the
// workgroup (tid = thread index).  L(i,k) = Mx(p(i), p(k)), p(i) = i (lower)
// or nb-1-i (upper); rows past nb and a unit diagonal become the identity.
// The source may be narrower than T (exact widening) or FP64 stored as FP32
// (one rounding, to nearest).  All of a thread's loads are issued before its
// first store, so one workgroup waits for one memory round trip, not one per
// element.
template <ElemT S, typename T, int NB, bool ASC, int NTHR>
__device__ __forceinline__ void stage_block(const void *A, int64_t base, int64_t lda, int nb, bool mtrans,
                                            bool mlower, bool unit, T *out, int tid)
{
    constexpr int PER = (NB * NB + NTHR - 1) / NTHR;
    T v[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = tid + t * NTHR;
        const int i = e % NB, k = e / NB;
        v[t] = (i == k) ? T(1) : T(0);
        if (e < NB * NB && i >= k && i < nb && (i > k || !unit)) {
            const int r = mlower ? i : nb - 1 - i;
            const int c = mlower ? k : nb - 1 - k;
            v[t] = (T)ld_src<S>(A, base + (mtrans ? c + (int64_t)r * lda : r + (int64_t)c * lda));
        }
    }
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = tid + t * NTHR;
        const int i = e % NB, k = e / NB;
        if (e < NB * NB && i >= k)
            out[colstart<NB, ASC>(k) + (i - k)] = v[t];
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

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront solves / multiplies the vectors [v0, v0 + 64) of a leaf panel
// (element d of vector v at B[d*sd + v*si]) against the block held in LDS at Ls
// in stream order.  Ps: this wavefront's LDS panel buffer (64 * (NB+1) elements).
// The panel's global loads are issued first; stage_tri() runs while they are in
// flight (the leaf kernel uses it to copy its block into Ls).
template <typename T, int NB, bool SOLVE, bool UNIT, class StageTri>
__device__ __forceinline__ void leaf_panel(const LeafDesc &d, T *__restrict__ B, const T *Ls, T *Ps, int64_t v0,
                                           StageTri &&stage_tri)
{
    static_assert(NB <= WAVE, "one lane per block row when staging");
    constexpr int PS = NB + 1;                  // padded panel stride (odd: no bank conflicts)
    const int lane = threadIdx.x % WAVE;
    const int nb = d.nb;

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
        stage_tri();
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
        stage_tri();
#pragma unroll
        for (int dd = 0; dd < NB; ++dd)
            if (dd < nb)
                Ps[vv * PS + (d.mlower ? dd : nb - 1 - dd)] = pv[dd];
    }
    wave_sync();

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
    wave_sync();
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


}  // namespace lk
}  // namespace rtri
