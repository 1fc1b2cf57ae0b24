// 16-bit GEMM update for the low-precision paths:
//     C(MxN) = beta * C + s * op(P)(MxK) * op(Q)(KxN)
// The triangular factor's block is stored in BF16 or FP16; the other operand
// (a block of the right-hand side) is 16-bit too or FP32, rounded to the 16-bit
// type (round to nearest even) on its way to LDS; C is FP32 and products
// accumulate in FP32 (v_mfma_f32_16x16x32_bf16 / _f16).
//
// Used by (a) the TRMM with 16-bit inputs, whose updates read the original
// 16-bit right-hand side (both operands 16-bit), and (b) the low-precision
// solve inside the mixed-precision TRSM, whose FP32 panel is rounded to BF16
// by design.
//
// Layout: 256-thread workgroups, 128x128 tiles, four 64x64 wavefront tiles of
// 16x16 MFMA blocks, BK = 64 (two MFMA k-steps per LDS stage).  Operand tiles
// are staged in LDS with k contiguous (rows padded to 72 elements, so the
// 16-byte fragment reads of 8 consecutive rows fall in distinct banks), two
// stages in LDS and two in registers: the global loads of step k + 2 are in
// flight while step k is multiplied, since one step of 16-bit MFMA work is too
// short to cover a memory round trip.  Registers hold the raw loaded values;
// the FP32 operand is rounded (v_cvt_pk_bf16_f32 / v_cvt_f16_f32, nearest
// even) when it is written to LDS.
//
// MFMA 16x16x32 operand layout (lane l, g = l/16, c = l%16): A operand row c,
// k = 8g..8g+7; B operand column c, k = 8g..8g+7; D: slot r holds D[4g + r][c].
#include <type_traits>

#include "common.h"
#include "dma_tile.h"

namespace rtri {

namespace {

constexpr int NT = 256;
constexpr int BK = 64;
constexpr int SK = BK + 8;   // padded LDS row (16-bit elements)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// float -> 16-bit pattern, round to nearest even (hardware conversion)
template <bool BF> __device__ __forceinline__ unsigned short to16(float x);
template <> __device__ __forceinline__ unsigned short to16<true>(float x)
{
    return __builtin_bit_cast(unsigned short, (__bf16)x);
}
template <> __device__ __forceinline__ unsigned short to16<false>(float x)
{
    return __builtin_bit_cast(unsigned short, (_Float16)x);
}

template <bool BF> __device__ __forceinline__ float4_t mfma16(u16x8 a, u16x8 b, float4_t c);
template <> __device__ __forceinline__ float4_t mfma16<true>(u16x8 a, u16x8 b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}
template <> __device__ __forceinline__ float4_t mfma16<false>(u16x8 a, u16x8 b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                  0, 0, 0);
}

typedef float float16_t __attribute__((ext_vector_type(16)));

// 32x32x16 MFMA (gfx950).  Lane l, h = l/32, c = l%32: A operand row c,
// k = 8h..8h+7; B operand column c, k = 8h..8h+7; D: slot 4q + r holds
// D[8q + 4h + r][c] (q, r = 0..3).
template <bool BF> __device__ __forceinline__ float16_t mfma32(u16x8 a, u16x8 b, float16_t c);
template <> __device__ __forceinline__ float16_t mfma32<true>(u16x8 a, u16x8 b, float16_t c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}
template <> __device__ __forceinline__ float16_t mfma32<false>(u16x8 a, u16x8 b, float16_t c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                  0, 0, 0);
}

// One R x BK operand tile: global -> registers (load), registers -> LDS as
// Ls[row * SK + k] (store).
//   SRC16: source is 16-bit (P); else FP32, rounded with to16 at the store (Q).
//   KC:    element (row, k) at base[k + row*ld]; else at base[row + k*ld].
//   VEC:   16-byte aligned base and ld (8 elements for 16-bit sources, 4 for
//          FP32): a full tile moves each 8-element chunk (contiguous in memory
//          in either layout) with 16-byte loads.
// Each thread moves NCH chunks of 8 elements; out-of-range elements are zero.
template <int R, bool SRC16, bool KC, bool BF, bool VEC>
struct Loader16 {
    static constexpr int W = 8;                 // elements per chunk
    static constexpr int NCH = R * BK / NT / W;  // 4 for R = 128
    u16x8 h[SRC16 ? NCH : 1];                    // raw 16-bit chunks
    float4_t f[SRC16 ? 1 : 2 * NCH];             // raw FP32 chunks (two halves each)

    __device__ inline void coords(int v, int tid, int &row, int &k) const
    {
        const int e = v * NT + tid;
        if (KC) {
            k = (e % (BK / W)) * W;
            row = e / (BK / W);
        } else {
            row = (e % (R / W)) * W;
            k = e / (R / W);
        }
    }

    __device__ inline void load(const void *base_, int64_t ld, int tid, int rlim, int klim, bool full)
    {
        if (VEC && full) {
#pragma unroll
            for (int v = 0; v < NCH; ++v) {
                int row, k;
                coords(v, tid, row, k);
                const int64_t off = KC ? k + (int64_t)row * ld : row + (int64_t)k * ld;
                if constexpr (SRC16) {
                    h[v] = *reinterpret_cast<const u16x8 *>(static_cast<const unsigned short *>(base_) + off);
                } else {
                    const float *fp = static_cast<const float *>(base_) + off;
                    f[2 * v] = *reinterpret_cast<const float4_t *>(fp);
                    f[2 * v + 1] = *reinterpret_cast<const float4_t *>(fp + 4);
                }
            }
            return;
        }
#pragma unroll
        for (int v = 0; v < NCH; ++v) {
            int row, k;
            coords(v, tid, row, k);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const int rr = KC ? row : row + w;
                const int kk = KC ? k + w : k;
                const int64_t off = KC ? kk + (int64_t)rr * ld : rr + (int64_t)kk * ld;
                const bool in = full || (rr < rlim && kk < klim);
                if constexpr (SRC16)
                    h[v][w] = in ? static_cast<const unsigned short *>(base_)[off] : (unsigned short)0;
                else
                    f[2 * v + w / 4][w % 4] = in ? static_cast<const float *>(base_)[off] : 0.0f;
            }
        }
    }

    __device__ inline u16x8 chunk(int v) const
    {
        if constexpr (SRC16) {
            return h[v];
        } else {
            u16x8 x;
#pragma unroll
            for (int w = 0; w < W; ++w)
                x[w] = to16<BF>(f[2 * v + w / 4][w % 4]);
            return x;
        }
    }

    __device__ inline void store(unsigned short *lds, int tid) const
    {
#pragma unroll
        for (int v = 0; v < NCH; ++v) {
            int row, k;
            coords(v, tid, row, k);
            const u16x8 x = chunk(v);
            if (KC) {   // 8 consecutive k of one row: one 16-byte LDS write
                *reinterpret_cast<u16x8 *>(lds + row * SK + k) = x;
                continue;
            }
#pragma unroll
            for (int w = 0; w < W; ++w)
                lds[(row + w) * SK + k] = x[w];
        }
    }
};

template <int BM, int BN, bool TP, bool TQ, bool BF, bool P16, bool Q16, bool VEC>
__global__ __launch_bounds__(NT, 2) void gemm16_kernel(GemmDesc g, int tiles_m, int tiles_n)
{
    constexpr int FM = BM / 32, FN = BN / 32;
    __shared__ __attribute__((aligned(16))) unsigned short As[2][BM * SK];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][BN * SK];

    const int ntiles = tiles_m * tiles_n;
    int bid = blockIdx.x;
    if ((ntiles & 7) == 0) {
        const int per = ntiles >> 3;
        bid = (bid & 7) * per + (bid >> 3);
    }
    constexpr int GROUP = 8;
    const int band = bid / (GROUP * tiles_n);
    const int first_m = band * GROUP;
    const int gsize = min(tiles_m - first_m, GROUP);
    const int in_band = bid - band * GROUP * tiles_n;
    const int tm = first_m + in_band % gsize;
    const int tn = in_band / gsize;

    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int wm = wave & 1, wn = wave >> 1;
    const int lc = lane % 16, lg = lane / 16;

    using PT = typename std::conditional<P16, unsigned short, float>::type;
    using QT = typename std::conditional<Q16, unsigned short, float>::type;
    const PT *P = static_cast<const PT *>(g.P);
    const QT *Q = static_cast<const QT *>(g.Q);
    const int64_t ldp = g.ldp, ldq = g.ldq;
    const PT *Pt = TP ? P + m0 * ldp : P + m0;
    const QT *Qt = TQ ? Q + n0 : Q + n0 * ldq;
    const int rlim_m = (int)min<int64_t>(BM, g.M - m0);
    const int rlim_n = (int)min<int64_t>(BN, g.N - n0);
    const bool full_mn = rlim_m == BM && rlim_n == BN;

    // two register stages per operand: step s lives in la[s & 1] / lb[s & 1]
    Loader16<BM, P16, TP, BF, VEC> la0, la1;
    Loader16<BN, Q16, !TQ, BF, VEC> lb0, lb1;

    float4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};

    const int64_t K = g.K;
    const int nk = (int)((K + BK - 1) / BK);
    auto load_step = [&](int kt, auto &la, auto &lb) {
        const int64_t k0 = (int64_t)kt * BK;
        const PT *pa = TP ? Pt + k0 : Pt + k0 * ldp;
        const QT *pb = TQ ? Qt + k0 * ldq : Qt + k0;
        const int klim = (int)min<int64_t>(BK, K - k0);
        const bool full = full_mn && klim == BK;
        la.load(pa, ldp, tid, rlim_m, klim, full);
        lb.load(pb, ldq, tid, rlim_n, klim, full);
    };
    auto multiply = [&](int buf) {
#pragma unroll
        for (int ks = 0; ks < BK / 32; ++ks) {
            u16x8 fa[FM], fb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                fa[i] = *reinterpret_cast<const u16x8 *>(
                    &As[buf][(wm * (BM / 2) + i * 16 + lc) * SK + ks * 32 + 8 * lg]);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                fb[j] = *reinterpret_cast<const u16x8 *>(
                    &Bs[buf][(wn * (BN / 2) + j * 16 + lc) * SK + ks * 32 + 8 * lg]);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = mfma16<BF>(fa[i], fb[j], acc[i][j]);
        }
    };
    // One step kt (its operands in LDS buffer kt & 1): issue the loads of step
    // kt + 2 into the register stage step kt held, multiply, then write step
    // kt + 1 (registers) to the other LDS buffer.  LA/LB: register stage of
    // kt (and kt + 2); LA1/LB1: that of kt + 1.
    auto step = [&](int kt, int buf, auto &LA, auto &LB, auto &LA1, auto &LB1) {
        if (kt + 2 < nk)
            load_step(kt + 2, LA, LB);
        multiply(buf);
        if (kt + 1 < nk) {
            LA1.store(As[buf ^ 1], tid);
            LB1.store(Bs[buf ^ 1], tid);
        }
        __syncthreads();
    };

    if (nk > 0) {
        load_step(0, la0, lb0);
        if (nk > 1)
            load_step(1, la1, lb1);
        la0.store(As[0], tid);
        lb0.store(Bs[0], tid);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
        step(kt, 0, la0, lb0, la1, lb1);
        if (kt + 1 < nk)
            step(kt + 1, 1, la1, lb1, la0, lb0);
    }

    float *C = static_cast<float *>(g.C);
    const int64_t ldc = g.ldc;
    const float beta = (float)g.beta, s = (float)g.s;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int rb = wm * (BM / 2) + i * 16;
            const int cl = wn * (BN / 2) + j * 16 + lc;
            if (cl >= rlim_n)
                continue;
            float *cp = C + (m0 + rb) + (n0 + cl) * ldc;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = 4 * lg + r;
                if (rb + rr < rlim_m) {
                    const float v = s * acc[i][j][r];
                    cp[rr] = (g.beta == 0.0) ? v : fmat(beta, cp[rr], v);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Wide tiles for large updates whose operands are both k-contiguous (op(P) =
// P^T, op(Q) = Q; the orientation the library's 16-bit copies are made in):
// 256x256 tiles of eight wavefronts (2 x 4, each a 128x64 tile of 32x32x16
// MFMA blocks), BK = 64, two LDS stages and one register stage (the loads of
// step k + 1 are in flight while step k multiplies; a step is 32 MFMAs per
// wavefront, long enough to cover an L2 round trip).  Each wavefront reads
// (128 + 64) x 16 operand elements from LDS per 8 MFMAs of 32x32x16, 1.5x
// fewer bytes per flop than the 64x64 wavefront tiles of the 128x128 kernel.
// The epilogue writes four consecutive rows of C per lane (16 bytes).
namespace wide {

constexpr int NTW = 512;
constexpr int TW = 256;   // tile rows and columns

// 256 x BK tile of a k-contiguous operand (element (row, k) at base[k + row*ld]):
// each thread moves 4 chunks of 8 consecutive k
template <bool SRC16, bool BF>
struct Loader {
    static constexpr int NCH = TW * BK / NTW / 8;   // 4
    u16x8 h[SRC16 ? NCH : 1];
    float4_t f[SRC16 ? 1 : 2 * NCH];

    __device__ inline void load(const void *base_, int64_t ld, int tid, int rlim, int klim, bool full)
    {
#pragma unroll
        for (int v = 0; v < NCH; ++v) {
            const int e = v * NTW + tid;
            const int row = e >> 3, k = (e & 7) * 8;
            const int64_t off = k + (int64_t)row * ld;
            if (full || (row < rlim && k + 8 <= klim)) {
                if constexpr (SRC16) {
                    h[v] = *reinterpret_cast<const u16x8 *>(static_cast<const unsigned short *>(base_) + off);
                } else {
                    const float *fp = static_cast<const float *>(base_) + off;
                    f[2 * v] = *reinterpret_cast<const float4_t *>(fp);
                    f[2 * v + 1] = *reinterpret_cast<const float4_t *>(fp + 4);
                }
            } else {
#pragma unroll
                for (int w = 0; w < 8; ++w) {
                    const bool in = row < rlim && k + w < klim;
                    if constexpr (SRC16)
                        h[v][w] = in ? static_cast<const unsigned short *>(base_)[off + w] : (unsigned short)0;
                    else
                        f[2 * v + w / 4][w % 4] = in ? static_cast<const float *>(base_)[off + w] : 0.0f;
                }
            }
        }
    }

    __device__ inline void store(unsigned short *lds, int tid) const
    {
#pragma unroll
        for (int v = 0; v < NCH; ++v) {
            const int e = v * NTW + tid;
            const int row = e >> 3, k = (e & 7) * 8;
            u16x8 x;
            if constexpr (SRC16) {
                x = h[v];
            } else {
#pragma unroll
                for (int w = 0; w < 8; ++w)
                    x[w] = to16<BF>(f[2 * v + w / 4][w % 4]);
            }
            *reinterpret_cast<u16x8 *>(lds + row * SK + k) = x;
        }
    }
};

// The operand tiles of one K segment: op(P) rows from P (= P^T: row m at
// P + m*ldp) and op(Q) columns from Q (column n at Q + n*ldq), K values.
struct WSeg {
    const void *P, *Q;
    int64_t ldp, ldq, K;
};

// The K loop of one 256x256 output tile by the workgroup's eight wavefronts:
// acc += op(P) op(Q) summed over a sequence of K segments, nk k-steps in all.
// next(sg) fills in the next segment; it is called in order, once per
// segment, when the segment's first k-step is loaded.  Ends with a barrier
// after the last k-step, so the LDS buffers may be reused at once.
template <bool BF, bool P16, bool Q16, class Next>
__device__ __forceinline__ void wide_k(Next &&next, int nk, int rlim_m, int rlim_n, float16_t (&acc)[4][2],
                                       unsigned short (*As)[TW * SK], unsigned short (*Bs)[TW * SK])
{
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int lr = lane & 31, lh = lane >> 5;

    using PT = typename std::conditional<P16, unsigned short, float>::type;
    using QT = typename std::conditional<Q16, unsigned short, float>::type;
    const bool full_mn = rlim_m == TW && rlim_n == TW;

    Loader<P16, BF> la;
    Loader<Q16, BF> lb;
    WSeg sg{};
    int sg_first = 0, sg_nk = 0;   // the segment being loaded: its first k-step and k-steps
    auto load_step = [&](int kt) {
        while (kt - sg_first >= sg_nk) {
            sg_first += sg_nk;
            next(sg);
            sg_nk = (int)((sg.K + BK - 1) / BK);
        }
        const int64_t k0 = (int64_t)(kt - sg_first) * BK;
        const int klim = (int)min<int64_t>(BK, sg.K - k0);
        const bool full = full_mn && klim == BK;
        la.load(static_cast<const PT *>(sg.P) + k0, sg.ldp, tid, rlim_m, klim, full);
        lb.load(static_cast<const QT *>(sg.Q) + k0, sg.ldq, tid, rlim_n, klim, full);
    };

    if (nk > 0) {
        load_step(0);
        la.store(As[0], tid);
        lb.store(Bs[0], tid);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk)
            load_step(kt + 1);
        const unsigned short *as = &As[buf][(wm * 128 + lr) * SK + 8 * lh];
        const unsigned short *bs = &Bs[buf][(wn * 64 + lr) * SK + 8 * lh];
#pragma unroll
        for (int ks = 0; ks < BK / 16; ++ks) {
            u16x8 fa[4], fb[2];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                fa[i] = *reinterpret_cast<const u16x8 *>(as + i * 32 * SK + ks * 16);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                fb[j] = *reinterpret_cast<const u16x8 *>(bs + j * 32 * SK + ks * 16);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = mfma32<BF>(fa[i], fb[j], acc[i][j]);
        }
        if (kt + 1 < nk) {
            la.store(As[buf ^ 1], tid);
            lb.store(Bs[buf ^ 1], tid);
        }
        __syncthreads();
    }
}

// C = beta C + s acc on a 256x256 tile at C (column-major, ldc) of which
// rlim_m x rlim_n entries exist; beta == 0: C is not read.  Each lane writes
// four consecutive rows of a column per 16 bytes (one access when aligned);
// the C reads of a row block are issued together, ahead of its stores.
__device__ __forceinline__ void wide_epilogue(const float16_t (&acc)[4][2], float *C, int64_t ldc, int rlim_m,
                                              int rlim_n, double beta_d, double s_d)
{
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int lr = lane & 31, lh = lane >> 5;
    const float beta = (float)beta_d, s = (float)s_d;
    const bool zero_beta = beta_d == 0.0;
    const bool cvec = rlim_m == TW && rlim_n == TW && (reinterpret_cast<uintptr_t>(C) & 15) == 0 && (ldc & 3) == 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (cvec) {
            float4_t o[2][4];
            if (!zero_beta) {
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        o[j][q] = *reinterpret_cast<const float4_t *>(
                            C + (wm * 128 + i * 32 + 8 * q + 4 * lh) + (wn * 64 + j * 32 + lr) * ldc);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float4_t v;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        v[r] = zero_beta ? s * acc[i][j][4 * q + r] : fmat(beta, o[j][q][r], s * acc[i][j][4 * q + r]);
                    *reinterpret_cast<float4_t *>(C + (wm * 128 + i * 32 + 8 * q + 4 * lh) +
                                                  (wn * 64 + j * 32 + lr) * ldc) = v;
                }
        } else {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int cl = wn * 64 + j * 32 + lr;
                if (cl >= rlim_n)
                    continue;
                float *cp = C + cl * ldc;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int rb = wm * 128 + i * 32 + 8 * q + 4 * lh;   // rows rb..rb+3
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (rb + r < rlim_m) {
                            const float v = s * acc[i][j][4 * q + r];
                            cp[rb + r] = zero_beta ? v : fmat(beta, cp[rb + r], v);
                        }
                    }
                }
            }
        }
    }
}

// One update on the 256x256 tile of C at (m0, n0).
template <bool BF, bool P16, bool Q16>
__device__ __forceinline__ void wide_tile(const GemmDesc &g, int64_t m0, int64_t n0, unsigned short (*As)[TW * SK],
                                          unsigned short (*Bs)[TW * SK])
{
    using PT = typename std::conditional<P16, unsigned short, float>::type;
    using QT = typename std::conditional<Q16, unsigned short, float>::type;
    const int rlim_m = (int)min<int64_t>(TW, g.M - m0);
    const int rlim_n = (int)min<int64_t>(TW, g.N - n0);
    float16_t acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                acc[i][j][r] = 0.0f;
    auto next = [&](WSeg &sg) {
        sg = WSeg{static_cast<const PT *>(g.P) + m0 * g.ldp, static_cast<const QT *>(g.Q) + n0 * g.ldq, g.ldp, g.ldq,
                  g.K};
    };
    wide_k<BF, P16, Q16>(next, (int)((g.K + BK - 1) / BK), rlim_m, rlim_n, acc, As, Bs);
    wide_epilogue(acc, static_cast<float *>(g.C) + m0 + n0 * g.ldc, g.ldc, rlim_m, rlim_n, g.beta, g.s);
}

// Tile of this workgroup in a tiles_m x tiles_n grid.  Blocks go round robin
// over the eight XCDs: give each XCD a contiguous range of tiles, then walk
// the tiles in bands of GROUP tile rows so that blocks in flight together
// share operand panels in L2.
__device__ __forceinline__ void tile_order(int tiles_m, int tiles_n, int &tm, int &tn)
{
    const int ntiles = tiles_m * tiles_n;
    int bid = blockIdx.x;
    if ((ntiles & 7) == 0) {
        const int per = ntiles >> 3;
        bid = (bid & 7) * per + (bid >> 3);
    }
    constexpr int GROUP = 4;
    const int band = bid / (GROUP * tiles_n);
    const int first_m = band * GROUP;
    const int gsize = min(tiles_m - first_m, GROUP);
    const int in_band = bid - band * GROUP * tiles_n;
    tm = first_m + in_band % gsize;
    tn = in_band / gsize;
}

template <bool BF, bool P16, bool Q16>
__global__ __launch_bounds__(NTW, 1) void gemm16w_kernel(GemmDesc g, int tiles_m, int tiles_n)
{
    __shared__ __attribute__((aligned(16))) unsigned short As[2][TW * SK];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][TW * SK];

    int tm, tn;
    tile_order(tiles_m, tiles_n, tm, tn);
    wide_tile<BF, P16, Q16>(g, (int64_t)tm * TW, (int64_t)tn * TW, As, Bs);
}

// Several updates in one launch (launch_gemm16_grouped): workgroup b owns a
// 256x256 tile of the output and applies its entries in order.  When every
// entry adds to the tile (beta = 1) with the same scale s, and all address the
// same C entries, the entries' products go into one accumulator, their K
// segments walked back to back, and C is read and written once:
//     C := C + s * sum_e op(P_e) op(Q_e)
// (rounded once instead of once per entry).  Otherwise each entry is applied
// as a launch of that update alone would.
template <bool BF>
__global__ __launch_bounds__(NTW, 1) void gemm16w_grouped_kernel(const GemmDesc *descs, const GroupEntry *ents,
                                                                 const GroupTile *tiles)
{
    __shared__ __attribute__((aligned(16))) unsigned short As[2][TW * SK];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][TW * SK];
    const GroupTile tl = tiles[blockIdx.x];
    if (tl.count <= 0)
        return;
    const GroupEntry e0 = ents[tl.first];
    const GemmDesc &g0 = descs[e0.desc];
    float *c0 = static_cast<float *>(g0.C) + e0.m0 + (int64_t)e0.n0 * g0.ldc;
    const int rm = (int)min<int64_t>(TW, g0.M - e0.m0), rn = (int)min<int64_t>(TW, g0.N - e0.n0);
    bool merge = g0.beta == 1.0;
    int64_t nk = 0;
    for (int e = tl.first; e < tl.first + tl.count; ++e) {
        const GroupEntry en = ents[e];
        const GemmDesc &g = descs[en.desc];
        merge = merge && g.beta == 1.0 && g.s == g0.s && g.ldc == g0.ldc &&
                static_cast<float *>(g.C) + en.m0 + (int64_t)en.n0 * g.ldc == c0 &&
                min<int64_t>(TW, g.M - en.m0) == rm && min<int64_t>(TW, g.N - en.n0) == rn;
        nk += (g.K + BK - 1) / BK;
    }
    if (merge) {
        float16_t acc[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    acc[i][j][r] = 0.0f;
        int idx = tl.first;
        auto next = [&](WSeg &sg) {
            const GroupEntry en = ents[idx++];
            const GemmDesc &g = descs[en.desc];
            sg = WSeg{static_cast<const unsigned short *>(g.P) + en.m0 * g.ldp,
                      static_cast<const unsigned short *>(g.Q) + en.n0 * g.ldq, g.ldp, g.ldq, g.K};
        };
        wide_k<BF, true, true>(next, (int)nk, rm, rn, acc, As, Bs);
        wide_epilogue(acc, c0, g0.ldc, rm, rn, 1.0, g0.s);
        return;
    }
    for (int e = tl.first; e < tl.first + tl.count; ++e) {
        const GroupEntry en = ents[e];
        wide_tile<BF, true, true>(descs[en.desc], en.m0, en.n0, As, Bs);
    }
}

// ---------------------------------------------------------------------------
// Full 256x256 tiles whose operands are both 16-bit (k-contiguous, 16-byte
// aligned, leading dimensions multiples of 8) with K a multiple of 32 in every
// segment: the operands go straight into LDS (dma_tile.h), 32 values of k
// per step.  Same MFMA sequence per accumulator as the register-staged
// tiles above.
constexpr int BKD = dma::LINE / 2;   // k per step

template <bool BF>
__device__ __forceinline__ void dma_seg16(const unsigned short *P, const unsigned short *Q, int64_t ldp, int64_t ldq,
                                          int nk, float16_t (&acc)[4][2], char *S0, char *S1, char *S2, char *S3)
{
    dma::k_seg(reinterpret_cast<const char *>(P), reinterpret_cast<const char *>(Q), 2 * ldp, 2 * ldq, nk, acc, S0,
               S1, S2, S3, [](dma::v4i a, dma::v4i b, float16_t c) {
                   return mfma32<BF>(__builtin_bit_cast(u16x8, a), __builtin_bit_cast(u16x8, b), c);
               });
}

// one update of full tiles: M, N multiples of 256, K a multiple of BKD
template <bool BF>
__global__ __launch_bounds__(NTW, 1) void gemm16d_kernel(GemmDesc g, int tiles_m, int tiles_n)
{
    RTRI_DMA_STAGES;
    int tm, tn;
    tile_order(tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * TW, n0 = (int64_t)tn * TW;
    float16_t acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                acc[i][j][r] = 0.0f;
    dma_seg16<BF>(static_cast<const unsigned short *>(g.P) + m0 * g.ldp,
                  static_cast<const unsigned short *>(g.Q) + n0 * g.ldq, g.ldp, g.ldq, (int)(g.K / BKD), acc, S0, S1,
                  S2, S3);
    wide_epilogue(acc, static_cast<float *>(g.C) + m0 + n0 * g.ldc, g.ldc, TW, TW, g.beta, g.s);
}

// grouped updates, tiles whose entries share one accumulator (the host lists
// here only full tiles whose entries all add with beta = 1 and one scale s,
// with K multiples of BKD): C := C + s * sum_e op(P_e) op(Q_e)
template <bool BF>
__global__ __launch_bounds__(NTW, 1) void gemm16d_grouped_kernel(const GemmDesc *descs, const GroupEntry *ents,
                                                                 const GroupTile *tiles)
{
    RTRI_DMA_STAGES;
    const GroupTile tl = tiles[blockIdx.x];
    if (tl.count <= 0)
        return;
    const GroupEntry e0 = ents[tl.first];
    const GemmDesc &g0 = descs[e0.desc];
    float16_t acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                acc[i][j][r] = 0.0f;
    for (int e = tl.first; e < tl.first + tl.count; ++e) {
        const GroupEntry en = ents[e];
        const GemmDesc &g = descs[en.desc];
        dma_seg16<BF>(static_cast<const unsigned short *>(g.P) + en.m0 * g.ldp,
                      static_cast<const unsigned short *>(g.Q) + en.n0 * g.ldq, g.ldp, g.ldq, (int)(g.K / BKD), acc,
                      S0, S1, S2, S3);
    }
    wide_epilogue(acc, static_cast<float *>(g0.C) + e0.m0 + (int64_t)e0.n0 * g0.ldc, g0.ldc, TW, TW, 1.0, g0.s);
}

}  // namespace wide

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// whether an update takes the wide tiles (tile: 0 automatic, 1 128x128, 2 wide
// where the operand layout allows): enough 256x256 tiles to keep most CUs
// busy, and a K long enough for the deeper tile to pay off
bool use_wide(const GemmDesc &g, int tile)
{
    if (tile == 1)
        return false;
    if (tile == 2 || tile == 3)
        return true;
    const int64_t tw = ((g.M + 255) / 256) * ((g.N + 255) / 256);
    return tw >= 96 && g.K >= 256;
}

template <bool TP, bool TQ, bool BF, bool P16, bool Q16>
hipError_t launch_t16(const GemmDesc &g, hipStream_t st, int tile)
{
    constexpr int BM = 128, BN = 128;
    const int tm = (int)((g.M + BM - 1) / BM), tn = (int)((g.N + BN - 1) / BN);
    // 16-byte chunks: 8 elements of a 16-bit operand, 4 of an FP32 one
    const int64_t lp = P16 ? 8 : 4, lq = Q16 ? 8 : 4;
    const bool vec = aligned16(g.P) && aligned16(g.Q) && g.ldp % lp == 0 && g.ldq % lq == 0;
    if constexpr (TP && !TQ) {
        if (vec && use_wide(g, tile)) {
            const int wm = (int)((g.M + 255) / 256), wn = (int)((g.N + 255) / 256);
            if constexpr (P16 && Q16) {
                if (tile != 3 && g.M % 256 == 0 && g.N % 256 == 0 && g.K % wide::BKD == 0) {
                    hipLaunchKernelGGL((wide::gemm16d_kernel<BF>), dim3((unsigned)(wm * wn)), dim3(wide::NTW), 0, st,
                                       g, wm, wn);
                    return hipGetLastError();
                }
            }
            hipLaunchKernelGGL((wide::gemm16w_kernel<BF, P16, Q16>), dim3((unsigned)(wm * wn)), dim3(wide::NTW), 0,
                               st, g, wm, wn);
            return hipGetLastError();
        }
    }
    if (vec)
        hipLaunchKernelGGL((gemm16_kernel<BM, BN, TP, TQ, BF, P16, Q16, true>), dim3((unsigned)(tm * tn)), dim3(NT),
                           0, st, g, tm, tn);
    else
        hipLaunchKernelGGL((gemm16_kernel<BM, BN, TP, TQ, BF, P16, Q16, false>), dim3((unsigned)(tm * tn)),
                           dim3(NT), 0, st, g, tm, tn);
    return hipGetLastError();
}

template <bool BF, bool P16, bool Q16>
hipError_t launch_bf(const GemmDesc &g, hipStream_t st, int tile)
{
    if (!g.tp && !g.tq) return launch_t16<false, false, BF, P16, Q16>(g, st, tile);
    if (g.tp && !g.tq) return launch_t16<true, false, BF, P16, Q16>(g, st, tile);
    if (!g.tp && g.tq) return launch_t16<false, true, BF, P16, Q16>(g, st, tile);
    return launch_t16<true, true, BF, P16, Q16>(g, st, tile);
}

template <bool BF>
hipError_t launch_types(bool p16, bool q16, const GemmDesc &g, hipStream_t st, int tile)
{
    if (p16 && q16)
        return launch_bf<BF, true, true>(g, st, tile);
    return p16 ? launch_bf<BF, true, false>(g, st, tile) : launch_bf<BF, false, true>(g, st, tile);
}

}  // namespace

hipError_t launch_gemm16_grouped(bool bf16, const GemmDesc *descs, const GroupEntry *ents, const GroupTile *tiles_dma,
                                 int n_dma, const GroupTile *tiles, int ntiles, hipStream_t st)
{
    if (n_dma > 0) {
        if (bf16)
            hipLaunchKernelGGL(wide::gemm16d_grouped_kernel<true>, dim3((unsigned)n_dma), dim3(wide::NTW), 0, st,
                               descs, ents, tiles_dma);
        else
            hipLaunchKernelGGL(wide::gemm16d_grouped_kernel<false>, dim3((unsigned)n_dma), dim3(wide::NTW), 0, st,
                               descs, ents, tiles_dma);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (ntiles <= 0)
        return hipSuccess;
    if (bf16)
        hipLaunchKernelGGL(wide::gemm16w_grouped_kernel<true>, dim3((unsigned)ntiles), dim3(wide::NTW), 0, st, descs,
                           ents, tiles);
    else
        hipLaunchKernelGGL(wide::gemm16w_grouped_kernel<false>, dim3((unsigned)ntiles), dim3(wide::NTW), 0, st,
                           descs, ents, tiles);
    return hipGetLastError();
}

hipError_t launch_gemm16(bool bf16, bool p16, bool q16, const GemmDesc &g, hipStream_t st, int tile)
{
    if (!p16 && !q16)
        return hipErrorInvalidValue;
    if (g.M <= 0 || g.N <= 0)
        return hipSuccess;
    return bf16 ? launch_types<true>(p16, q16, g, st, tile) : launch_types<false>(p16, q16, g, st, tile);
}

}  // namespace rtri
