// FP64-accurate triangular product op(A) * X (side L) or X * op(A) (side R)
// from exact INT8 matrix-core products: the residual product of the
// refined solve, computed without FP64 arithmetic in its inner loop.
//
// Method: the modular form of the Ozaki scheme (Ozaki, Uchino and Imamura,
// "Ozaki Scheme II: a GEMM-oriented emulation of floating-point matrix
// multiplication using an integer modular technique", 2025), restated:
//   1. Scale each line of the left operand P (its rows) and of the right
//      operand Q (its columns) by a power of two 2^(beta - e), where 2^e
//      bounds the line's largest magnitude, and round to integers:
//      P_int, Q_int with |entries| <= 2^beta.  The rounding moves each entry
//      by at most 2^(e - beta - 1) (the only approximation of the method).
//   2. The integer product Z = P_int Q_int (|Z| <= K 2^(2 beta)) is fixed by
//      its residues modulo 16 pairwise coprime moduli p_t <= 256 whose
//      product P (2^125.19) is at least 4 |Z| (Chinese remainder theorem);
//      beta = min(55, floor((log2 P - 2 - log2 K) / 2)), 55 up to K = 8192.
//      Residue t of Z is (P_int mod p_t)(Q_int mod p_t) mod p_t: one INT8
//      GEMM with exact INT32 accumulation per modulus (operands as symmetric
//      residues in [-128, 127]; K 128^2 < 2^31 for K < 2^17).
//   3. Z is recovered from its residues by Garner's mixed-radix algorithm
//      (exact small-integer arithmetic), evaluated by Horner's rule on 128-bit
//      integers (exact), converted to FP64 with one correct rounding and
//      scaled back by 2^(e_i + f_j - 2 beta).
// Triangular operands: entries outside op(A)'s triangle are zero residues, so
// every k range a tile multiplies may be cut at the triangle's edge.
//
// Kernels: split (FP64 lines -> 16 planes of int8 residues, lines
// k-contiguous, through an LDS tile so both source layouts read and write
// coalesced), the INT8 GEMM (256x256 tiles, eight wavefronts of 128x64,
// v_mfma_i32_32x32x32_i8, all moduli in one launch) writing residues of Z as
// bytes, and the reconstruction (Garner, one thread per four consecutive rows).
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "dma_tile.h"
#include "handle.h"

namespace rtri {
namespace oz {

typedef int int4_t __attribute__((ext_vector_type(4)));

constexpr int MAXMOD = 20;
// pairwise coprime, largest first (256 = 2^8; 255 = 3*5*17; 253 = 11*23;
// 247 = 13*19; the rest are primes)
__host__ __device__ constexpr int mod_at(int t)
{
    constexpr int M[MAXMOD] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227,
                               223, 211, 199, 197, 193, 191, 181, 179, 173, 167};
    return M[t];
}
constexpr int NMOD = 16;   // moduli used: their product P = 2^125.19 < 2^128
constexpr int BETA_MAX = 55;

// a modulo p in [0, p) for a 32-bit signed a (p a compile-time constant)
template <int P>
__device__ __forceinline__ int pmod(int a)
{
    const int r = a % P;
    return r < 0 ? r + P : r;
}

template <int P>
__device__ __forceinline__ signed char symres(int64_t v)
{
    // v = hi 2^32 + lo; 2^32 mod P folded in
    constexpr int T32 = (int)(((uint64_t)1 << 32) % (uint64_t)P);
    const int hi = (int)(v >> 32);
    const uint32_t lo = (uint32_t)v;
    const int r = pmod<P>(pmod<P>(hi) * T32 + (int)(lo % (uint32_t)P));
    return (signed char)(r > P / 2 ? r - P : r);
}

// ---------------------------------------------------------------------------
// Split: a matrix viewed as `lines` lines of K entries, entry (l, k) at
// src[k + l*ld] (kfast) or src[l + k*ld]; tri 1 keeps k <= l, tri 2 keeps
// k >= l (others are zero), unit puts 1 on the diagonal without reading it.
struct SplitDesc {
    const double *src;
    int64_t ld, lines, K;
    bool kfast, unit;
    int tri;
    int *exps;        // [lines_pad]: max |entry| of the line < 2^e (-1100 for a zero line)
    int8_t *out;      // plane t: out + t*plane; line l: + l*ldk
    int64_t ldk, plane;
    int nmod;
    int beta;         // bits kept: entries scaled below 2^beta
};

constexpr int ST = 64;   // split tile: 64 lines x 64 k

__device__ __forceinline__ double split_entry(const SplitDesc &d, int64_t l, int64_t k)
{
    if (l >= d.lines || k >= d.K)
        return 0.0;
    if (d.tri == 1 && k > l)
        return 0.0;
    if (d.tri == 2 && k < l)
        return 0.0;
    if (d.unit && k == l)
        return 1.0;
    return d.kfast ? d.src[k + l * d.ld] : d.src[l + k * d.ld];
}

// tile (l0, k0) into LDS, T[line][k] (pitch ST + 1); coalesced along the
// source's contiguous direction
__device__ __forceinline__ void split_tile(const SplitDesc &d, int64_t l0, int64_t k0, double (*T)[ST + 1])
{
    const int tid = threadIdx.x;
    const int a = tid % ST, b = tid / ST;   // a runs along memory
#pragma unroll 4
    for (int r = b; r < ST; r += 256 / ST) {
        if (d.kfast)
            T[r][a] = split_entry(d, l0 + r, k0 + a);
        else
            T[a][r] = split_entry(d, l0 + a, k0 + r);
    }
}

__global__ __launch_bounds__(256) void exps_init_kernel(int *exps, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        exps[i] = -1100;
}

__global__ __launch_bounds__(256) void split_exps_kernel(SplitDesc d)
{
    __shared__ double T[ST][ST + 1];
    const int64_t l0 = (int64_t)blockIdx.x * ST, k0 = (int64_t)blockIdx.y * ST;
    split_tile(d, l0, k0, T);
    __syncthreads();
    // 4 threads per line, 16 entries each
    const int tid = threadIdx.x;
    const int l = tid / 4, q = tid % 4;
    double mx = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c)
        mx = fmax(mx, fabs(T[l][q * 16 + c]));
    mx = fmax(mx, __shfl_xor(mx, 1));
    mx = fmax(mx, __shfl_xor(mx, 2));
    if (q == 0 && mx > 0.0 && l0 + l < d.lines) {
        int e;
        (void)frexp(mx, &e);   // mx < 2^e
        atomicMax(d.exps + l0 + l, e);
    }
}

template <int T0>
__device__ __forceinline__ void store_planes(const SplitDesc &d, const int64_t (&v)[16], int8_t *base)
{
    if constexpr (T0 < MAXMOD) {
        if (T0 < d.nmod) {
            constexpr int P = mod_at(T0);
            int w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t x = 0;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    x |= (uint32_t)(uint8_t)symres<P>(v[4 * q + c]) << (8 * c);
                w[q] = (int)x;
            }
            int4_t *dst = reinterpret_cast<int4_t *>(base + (int64_t)T0 * d.plane);
            *dst = int4_t{w[0], w[1], w[2], w[3]};
            store_planes<T0 + 1>(d, v, base);
        }
    }
}

__global__ __launch_bounds__(256) void split_planes_kernel(SplitDesc d)
{
    __shared__ double T[ST][ST + 1];
    const int64_t l0 = (int64_t)blockIdx.x * ST, k0 = (int64_t)blockIdx.y * ST;
    split_tile(d, l0, k0, T);
    __syncthreads();
    const int tid = threadIdx.x;
    const int l = tid / 4, q = tid % 4;   // 16 consecutive k of one line
    const int e = d.exps[l0 + l];
    int64_t v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const double x = T[l][q * 16 + c];
        // |x| < 2^e: the scaled value is below 2^beta in magnitude, an exact
        // power-of-two scaling; rint rounds to the nearest integer
        v[c] = e > -1100 ? (int64_t)rint(ldexp(x, d.beta - e)) : 0;
    }
    store_planes<0>(d, v, d.out + (l0 + l) * d.ldk + k0 + q * 16);
}

// ---------------------------------------------------------------------------
// INT8 GEMM over all moduli: residue plane t of Z = P_t Q_t^T (lines of P are
// rows of Z, lines of Q its columns), written as bytes in [0, p_t).
typedef int int16v __attribute__((ext_vector_type(16)));

constexpr int NTG = 512;
constexpr int TG = 256;              // tile lines (rows and columns of Z)
constexpr int BKB = 128;             // plane lines are zero-padded to a multiple of BKB bytes

struct GemmI8Desc {
    const int8_t *P, *Q;             // planes, lines k-contiguous, ldk bytes per line
    int64_t ldk, pplane, qplane;
    int64_t M, N, K;                 // logical sizes (M, N padded to TG in the planes)
    int tri;                         // 0 dense; 1 P lines keep k <= line; 2 P k >= line;
                                     // 3 Q lines keep k <= line; 4 Q k >= line
    uint8_t *res;                    // plane t at res + t*rplane, element (i, j) at i + j*ldr
    int64_t ldr, rplane;
};

__device__ __forceinline__ int16v mfma_i8(int4_t a, int4_t b, int16v c)
{
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(NTG, 1) void gemm_i8_kernel(GemmI8Desc g, int tiles_m, int tiles_n)
{
    RTRI_DMA_STAGES;

    const int ntiles = tiles_m * tiles_n;
    int bid = blockIdx.x;
    if ((ntiles & 7) == 0) {   // each XCD a contiguous range of tiles
        const int per = ntiles >> 3;
        bid = (bid & 7) * per + (bid >> 3);
    }
    constexpr int GROUP = 4;
    const int band = bid / (GROUP * tiles_n);
    const int first_m = band * GROUP;
    const int gsize = min(tiles_m - first_m, GROUP);
    const int in_band = bid - band * GROUP * tiles_n;
    const int tm = first_m + in_band % gsize;
    const int tn = in_band / gsize;
    const int t = blockIdx.y;   // modulus

    const int64_t m0 = (int64_t)tm * TG, n0 = (int64_t)tn * TG;
    // k range of this tile (the rest of the product is zero), in steps of
    // dma::LINE bytes; the planes' lines are zero-padded to a multiple of
    // BKB, so the last step may run past K
    int64_t kb = 0, ke = g.K;
    if (g.tri == 1) ke = min<int64_t>(g.K, m0 + TG);
    if (g.tri == 2) kb = m0;
    if (g.tri == 3) ke = min<int64_t>(g.K, n0 + TG);
    if (g.tri == 4) kb = n0;
    const int64_t sb = kb / dma::LINE, se = (ke + dma::LINE - 1) / dma::LINE;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int lr = lane & 31, lh = lane >> 5;

    int16v acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                acc[i][j][r] = 0;
    const int64_t k0 = sb * dma::LINE;
    dma::k_seg(reinterpret_cast<const char *>(g.P + (int64_t)t * g.pplane + m0 * g.ldk + k0),
               reinterpret_cast<const char *>(g.Q + (int64_t)t * g.qplane + n0 * g.ldk + k0), g.ldk, g.ldk,
               (int)(se - sb), acc, S0, S1, S2, S3,
               [](dma::v4i a, dma::v4i b, int16v c) { return mfma_i8(a, b, c); });

    // residues in [0, p): q = floor(acc / p) from a double quotient (|acc| < 2^31,
    // exact up to one unit, then corrected)
    const int p = mod_at(t);
    const double inv = 1.0 / (double)p;
    uint8_t *R = g.res + (int64_t)t * g.rplane;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t col = n0 + wn * 64 + j * 32 + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = m0 + wm * 128 + i * 32 + 8 * q + 4 * lh;   // four consecutive rows
                uint32_t w = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = acc[i][j][4 * q + r];
                    int rr = a - p * (int)floor((double)a * inv);
                    rr += rr < 0 ? p : 0;
                    rr -= rr >= p ? p : 0;
                    w |= (uint32_t)rr << (8 * r);
                }
                *reinterpret_cast<uint32_t *>(R + row + col * g.ldr) = w;
            }
        }
}

// ---------------------------------------------------------------------------
// Reconstruction: Z_ij from its N residues (Garner), then
//   W_ij = alpha * Z_ij * 2^(e_i + f_j - 2 beta)   (FP64)
struct GarnerDesc {
    const uint8_t *res;
    int64_t ldr, rplane;
    const int *erow, *ecol;
    int64_t M, N;
    double alpha;
    double *W;
    int64_t ldw;
    int beta2;        // 2 beta
};

// inverse of a modulo p (a, p coprime), by the extended Euclidean algorithm
__host__ __device__ constexpr int inv_mod(int a, int p)
{
    int t0 = 0, t1 = 1, r0 = p, r1 = a % p;
    while (r1 != 0) {
        const int q = r0 / r1;
        const int t2 = t0 - q * t1;
        t0 = t1;
        t1 = t2;
        const int r2 = r0 - q * r1;
        r0 = r1;
        r1 = r2;
    }
    return t0 < 0 ? t0 + p : t0;
}

// x mod P in [0, P) for an integer-valued float |x| < 2^16, exactly: the
// quotient estimate floor(x (1/P)) is off by at most one (its relative error
// is below 2^-22 and a remainder r != 0 keeps x / P at least 1/P from an
// integer), the fused multiply-add computes x - q P exactly (integers below
// 2^24), and one correction each way brings it into [0, P).  Full-rate FP32
// arithmetic in place of the quarter-rate 32-bit integer multiplies of a
// division by a constant.
template <int P>
__device__ __forceinline__ float fmodp(float x)
{
    const float q = __builtin_floorf(x * (1.0f / (float)P));
    float r = __builtin_fmaf(-q, (float)P, x);
    r = r < 0.0f ? r + (float)P : r;
    return r >= (float)P ? r - (float)P : r;
}

// digit T of the mixed-radix form: a_T = (((r_T - a_0) c_0T - a_1) c_1T - ...) mod p_T
// with c_sT = p_s^-1 mod p_T; digits and residues are integer-valued floats
// below 256, so every product (v - a_S) c_sT is an integer below 2^16 in
// magnitude, exact in FP32
template <int T, int S>
__device__ __forceinline__ float garner_step(float v, const float *a)
{
    if constexpr (S == T) {
        return v;
    } else {
        constexpr int P = mod_at(T);
        constexpr int C = inv_mod(mod_at(S) % P, P);
        return garner_step<T, S + 1>(fmodp<P>((v - a[S]) * (float)C), a);
    }
}

template <int N, int T>
__device__ __forceinline__ void garner_digits(const float *r, float *a)
{
    if constexpr (T < N) {
        a[T] = garner_step<T, 0>(r[T], a);
        garner_digits<N, T + 1>(r, a);
    }
}

// sum over t in [T0, T1) of d_t p_T0 ... p_(t-1) (Horner's rule from the top
// digit; the partial values stay below the product of those moduli, under
// 2^64 for eight of them)
template <int T0, int T1>
__device__ __forceinline__ uint64_t horner64(const uint32_t *d)
{
    uint64_t z = 0;
#pragma unroll
    for (int t = T1 - 1; t >= T0; --t)
        z = z * (uint64_t)mod_at(t) + d[t];
    return z;
}

// product of the moduli t in [T0, T1)
__host__ __device__ constexpr uint64_t mod_prod(int t0, int t1)
{
    uint64_t w = 1;
    for (int t = t0; t < t1; ++t)
        w *= (uint64_t)mod_at(t);
    return w;
}

template <int N>
__global__ __launch_bounds__(256) void garner_kernel(GarnerDesc d)
{
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    const int64_t j = blockIdx.y;
    if (i0 >= d.M)
        return;
    uint32_t w[N];
#pragma unroll
    for (int t = 0; t < N; ++t)
        w[t] = *reinterpret_cast<const uint32_t *>(d.res + t * d.rplane + i0 + j * d.ldr);
    const int fj = d.ecol[j];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + r;
        if (i >= d.M)
            break;
        float rr[N], a[N];
#pragma unroll
        for (int t = 0; t < N; ++t)
            rr[t] = (float)((w[t] >> (8 * r)) & 255u);
        garner_digits<N, 0>(rr, a);
        // Z' = a_0 + p_0 (a_1 + p_1 (...)) in [0, P); Z = Z' - P when the top
        // digit is in the upper half (|Z| < P/4 leaves no ambiguity).  The
        // negative case takes the digit complement: P - Z' = 1 + sum (p_t - 1 - a_t) W_t.
        // Exact 128-bit value (P < 2^128) as L + W_8 H, L and H the Horner
        // sums of digits 0..7 and 8..15 (each under 2^64), W_8 = p_0 ... p_7;
        // then one correctly rounded conversion to FP64 (the top 64
        // significant bits with a sticky bit for the rest), so an integer Z
        // representable in FP64 comes out exactly.
        static_assert(N == 16, "two halves of eight digits");
        const bool neg = 2.0f * a[N - 1] >= (float)mod_at(N - 1);
        uint32_t dg[N];
#pragma unroll
        for (int t = 0; t < N; ++t)
            dg[t] = (uint32_t)(neg ? (float)(mod_at(t) - 1) - a[t] : a[t]);
        constexpr uint64_t W8 = mod_prod(0, 8);
        const uint64_t lo = horner64<0, 8>(dg), hi = horner64<8, 16>(dg);
        uint64_t zl = hi * W8;
        uint64_t zh = __umul64hi(hi, W8);
        zl += lo;
        zh += zl < lo ? 1u : 0u;
        if (neg) {   // + 1 of the complement
            zl += 1u;
            zh += zl == 0u ? 1u : 0u;
        }
        double z;
        if (zh == 0u) {
            z = (double)zl;   // one rounding (the 64-bit conversion rounds once)
        } else {
            const int sh = 64 - __clzll((long long)zh);   // bits of zh; the value has 64 + sh bits
            uint64_t top = (zh << (64 - sh)) | (zl >> sh);
            top |= (zl << (64 - sh)) != 0u ? 1u : 0u;      // sticky: nothing below is lost to rounding
            z = ldexp((double)top, sh);
        }
        if (neg)
            z = -z;
        const int ei = d.erow[i];
        double out = 0.0;
        if (ei > -1100 && fj > -1100)
            out = d.alpha * ldexp(z, ei + fj - d.beta2);
        d.W[i + j * d.ldw] = out;
    }
}

template <int N>
hipError_t launch_garner_n(const GarnerDesc &d, hipStream_t st)
{
    const dim3 grid((unsigned)((d.M + 1023) / 1024), (unsigned)d.N);
    hipLaunchKernelGGL(garner_kernel<N>, grid, dim3(256), 0, st, d);
    return hipGetLastError();
}

}  // namespace oz

// ---------------------------------------------------------------------------
// host side

int ozaki_nmod(int64_t K)
{
    // exact INT32 sums: K * 128^2 < 2^31
    return K >= ((int64_t)1 << 17) ? 0 : oz::NMOD;
}

int ozaki_beta(int64_t K)
{
    // P = p_0 ... p_15 must reach 4 max |Z| = 4 K 2^(2 beta): beta as large as
    // that allows, at most BETA_MAX
    double lp = 0.0;
    for (int t = 0; t < oz::NMOD; ++t)
        lp += std::log2((double)oz::mod_at(t));
    const int b = (int)std::floor((lp - 2.0 - std::log2((double)std::max<int64_t>(K, 1))) / 2.0);
    return std::min(oz::BETA_MAX, b);
}

namespace {

inline int64_t rup(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// one operand's planes: lines padded to the GEMM tile, k to the GEMM step
struct OzOperand {
    int64_t lines, lines_pad, K, ldk, plane;
    size_t bytes() const { return exps_off() + (size_t)lines_pad * 4; }
    size_t exps_off() const { return (size_t)plane * (size_t)nmod; }
    int nmod;
};

OzOperand oz_operand(int64_t lines, int64_t K, int nmod)
{
    OzOperand o{};
    o.lines = lines;
    o.lines_pad = rup(std::max<int64_t>(lines, 1), oz::TG);
    o.K = K;
    o.ldk = rup(std::max<int64_t>(K, 1), oz::BKB);
    o.plane = o.lines_pad * o.ldk;
    o.nmod = nmod;
    return o;
}

hipError_t oz_split(const OzOperand &o, const double *src, int64_t ld, bool kfast, int tri, bool unit, void *mem,
                    hipStream_t st)
{
    oz::SplitDesc d{};
    d.src = src;
    d.ld = ld;
    d.lines = o.lines;
    d.K = o.K;
    d.kfast = kfast;
    d.unit = unit;
    d.tri = tri;
    d.out = static_cast<int8_t *>(mem);
    d.exps = reinterpret_cast<int *>(static_cast<char *>(mem) + o.exps_off());
    d.ldk = o.ldk;
    d.plane = o.plane;
    d.nmod = o.nmod;
    d.beta = ozaki_beta(o.K);
    hipLaunchKernelGGL(oz::exps_init_kernel, dim3((unsigned)((o.lines_pad + 255) / 256)), dim3(256), 0, st, d.exps,
                       o.lines_pad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const dim3 grid((unsigned)(o.lines_pad / oz::ST), (unsigned)(o.ldk / oz::ST));
    hipLaunchKernelGGL(oz::split_exps_kernel, grid, dim3(256), 0, st, d);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(oz::split_planes_kernel, grid, dim3(256), 0, st, d);
    return hipGetLastError();
}

}  // namespace

size_t ozaki_factor_bytes(int side, int64_t ka)
{
    (void)side;
    const int nmod = ozaki_nmod(ka);
    return oz_operand(ka, ka, nmod).bytes();
}

hipError_t ozaki_split_factor(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t ka, const double *A,
                              int64_t lda, void *mem)
{
    const int nmod = ozaki_nmod(ka);
    const OzOperand o = oz_operand(ka, ka, nmod);
    const bool low = (uplo == RTRI_LOWER) != (tr != RTRI_NOTRANS);   // op(A) lower
    bool kfast;
    int tri;
    if (side == RTRI_LEFT) {   // lines = rows i of op(A), entry (i, k) = op(A)(i, k)
        kfast = tr != RTRI_NOTRANS;
        tri = low ? 1 : 2;
    } else {                   // lines = columns j of op(A), entry (j, k) = op(A)(k, j)
        kfast = tr == RTRI_NOTRANS;
        tri = low ? 2 : 1;
    }
    return timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 4.0 * ka * ka + (double)nmod * o.plane,
                 [&] { return oz_split(o, A, lda, kfast, tri, diag == RTRI_UNIT, mem, h->stream); });
}

int ozaki_product(rtri_handle *h, int side, int uplo, int tr, int64_t m, int64_t n, double alpha, const void *Aplanes,
                  const double *X, int64_t ldx, double *W, int64_t ldw)
{
    const bool left = side == RTRI_LEFT;
    const int64_t ka = left ? m : n;
    const int nmod = ozaki_nmod(ka);
    if (nmod == 0)
        return RTRI_ERR_UNSUPPORTED;
    const bool low = (uplo == RTRI_LOWER) != (tr != RTRI_NOTRANS);
    const OzOperand oa = oz_operand(ka, ka, nmod);
    // the panel's lines: columns of X (side L, Z = op(A) X), rows of X (side R, Z = X op(A))
    const OzOperand ox = oz_operand(left ? n : m, ka, nmod);
    const int64_t Mpad = rup(m, oz::TG), Npad = rup(n, oz::TG);
    const size_t xbytes = ox.bytes();
    const size_t rbytes = (size_t)nmod * (size_t)Mpad * (size_t)Npad;
    hipError_t e = ensure_ws(h, WS_OZX, xbytes);
    if (e == hipSuccess)
        e = ensure_ws(h, WS_OZR, rbytes);
    if (e != hipSuccess)
        return hip_fail(h, e);
    void *xm = h->ws[WS_OZX];
    uint8_t *res = static_cast<uint8_t *>(h->ws[WS_OZR]);
    e = timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 16.0 * m * n + (double)nmod * ox.plane,
              [&] { return oz_split(ox, X, ldx, left, 0, false, xm, h->stream); });
    if (e != hipSuccess)
        return hip_fail(h, e);

    oz::GemmI8Desc g{};
    const int8_t *ap = static_cast<const int8_t *>(Aplanes);
    const int8_t *xp = static_cast<const int8_t *>(xm);
    g.P = left ? ap : xp;
    g.Q = left ? xp : ap;
    g.pplane = left ? oa.plane : ox.plane;
    g.qplane = left ? ox.plane : oa.plane;
    g.ldk = oa.ldk;
    g.M = m;
    g.N = n;
    g.K = ka;
    g.tri = left ? (low ? 1 : 2) : (low ? 4 : 3);
    g.res = res;
    g.ldr = Mpad;
    g.rplane = Mpad * Npad;
    const int tm = (int)(Mpad / oz::TG), tn = (int)(Npad / oz::TG);
    // useful work: the triangle's half of the dense product, per modulus
    const double ops = (double)nmod * (double)m * (double)n * (double)ka;
    e = timed(h, RTRI_KCLASS_GEMM, RTRI_I8, ops, (double)nmod * (oa.plane / 2 + ox.plane + (double)m * n), [&] {
        hipLaunchKernelGGL(oz::gemm_i8_kernel, dim3((unsigned)(tm * tn), (unsigned)nmod), dim3(oz::NTG), 0,
                           h->stream, g, tm, tn);
        return hipGetLastError();
    });
    if (e != hipSuccess)
        return hip_fail(h, e);

    oz::GarnerDesc d{};
    d.res = res;
    d.ldr = Mpad;
    d.rplane = Mpad * Npad;
    const int *ea = reinterpret_cast<const int *>(static_cast<const char *>(Aplanes) + oa.exps_off());
    const int *ex = reinterpret_cast<const int *>(static_cast<const char *>(xm) + ox.exps_off());
    d.erow = left ? ea : ex;
    d.ecol = left ? ex : ea;
    d.M = m;
    d.N = n;
    d.alpha = alpha;
    d.W = W;
    d.ldw = ldw;
    d.beta2 = 2 * ozaki_beta(ka);
    e = timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, (double)nmod * m * n + 8.0 * m * n,
              [&] { return oz::launch_garner_n<oz::NMOD>(d, h->stream); });
    return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
}

}  // namespace rtri

extern "C" int rtri_dtrmm_ozaki(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                                double alpha, const double *A, int64_t lda, double *B, int64_t ldb)
{
    using namespace rtri;
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    const int rc = check_args(side, uplo, trans, diag, m, n, A, lda, B, ldb, alpha != 0.0);
    if (rc != 0)
        return rc;
    if (m == 0 || n == 0)
        return RTRI_OK;
    hipError_t e;
    if (alpha == 0.0) {
        e = timed(h, RTRI_KCLASS_OTHER, RTRI_F64, 0.0, 8.0 * m * n,
                  [&] { return launch_fill(DType::F64, B, m, n, ldb, 0.0, h->stream); });
        return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
    }
    const int tr = trans == RTRI_CONJTRANS ? RTRI_TRANS : trans;
    const int64_t ka = side == RTRI_LEFT ? m : n;
    if (ozaki_nmod(ka) == 0)
        return RTRI_ERR_UNSUPPORTED;
    e = ensure_ws(h, WS_OZA, ozaki_factor_bytes(side, ka));
    if (e == hipSuccess)
        e = ozaki_split_factor(h, side, uplo, tr, diag, ka, A, lda, h->ws[WS_OZA]);
    if (e != hipSuccess)
        return hip_fail(h, e);
    // the panel's planes are made before the product overwrites B
    return ozaki_product(h, side, uplo, tr, m, n, alpha, h->ws[WS_OZA], B, ldb, B, ldb);
}
