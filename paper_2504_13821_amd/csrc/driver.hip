// Recursion driver and the core C ABI (include/rtri.h).
//
// The recursion (paper, Sec. 3.1-3.2) splits the triangular factor at its
// midpoint: two triangular diagonal blocks and one off-diagonal block.  It is
// written once, over the "dependency index" (rows of B for side = L, columns
// of B for side = R), and covers all sixteen side / uplo / trans cases and
// both diag values:
//
//   op(A) is effectively lower when (uplo == L) != (trans != N).
//   TRSM visits the blocks in dependency order: block 1 first when the solve
//   runs forward (side L with lower op(A), or side R with upper op(A)).
//   TRMM visits them in the opposite order, so its GEMM always reads the block
//   that has not been overwritten yet.
//
//   split h rows at k:  block 1 = [d0, d0+k),  block 2 = [d0+k, d0+h)
//   TRSM: first = rec(alpha); update: B_t = alpha*B_t - (off-diagonal) * X_s;
//         second = rec(1)              (alpha applied once, at first touch)
//   TRMM: first = rec(alpha); update: B_t += alpha * (off-diagonal) * B_s;
//         second = rec(alpha)
//   side L: C = B[t rows], P = op(A)[t, s], Q = B[s rows]
//   side R: C = B[t cols], P = B[s cols],    Q = op(A)[s, t]
//
// The split point is a multiple of the leaf size (half the block, rounded up),
// so every leaf but the last one is full and GEMM operands stay aligned.  The
// plan is a flat list of launches; one pack pass before it writes every
// diagonal block in the canonical form the leaf kernel reads.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "handle.h"

using namespace rtri;

namespace {

constexpr uint32_t MAGIC = 0x72747269u;  // 'rtri'

struct Op {
    bool gemm;
    int depth;   // recursion depth of the node that issued it
    GemmDesc g;
    LeafDesc l;
};

// whether op(A) reads the GEMM copy of A transposed: op(A)(r, c) is A(c, r)
// for trans = T, and a copy that holds A^T swaps the two readings
inline bool ag_tr(const PlanIn &p) { return (p.trans != RTRI_NOTRANS) != p.ag_trans; }

// pointer to op(A)[r0.., c0..] inside the GEMM copy of A
inline const char *tri_block(const PlanIn &p, int64_t r0, int64_t c0)
{
    const int64_t off = ag_tr(p) ? c0 + r0 * p.ldag : r0 + c0 * p.ldag;
    return p.Ag + off * (int64_t)elem_size(p.gt);
}

struct Planner {
    const PlanIn &p;
    size_t es;      // panel element size
    bool low;       // op(A) lower
    bool forward;   // block 1 before block 2
    std::vector<Op> ops;
    // where the GEMM updates of a TRMM read the original values of the other
    // block: the panel itself (one launch per leaf), or a copy of it taken
    // before all leaves run in one launch
    const char *src = nullptr;
    int64_t ldsrc = 0;
    size_t ses = 0;   // element size of src

    explicit Planner(const PlanIn &pr) : p(pr)
    {
        es = p.bt == DType::F64 ? 8 : 4;
        src = p.B;
        ldsrc = p.ldb;
        ses = es;
        if (!p.solve && p.Bsrc16 != nullptr) {
            src = p.Bsrc16;
            ldsrc = p.ldbsrc16;
            ses = 2;
        }
        low = (p.uplo == RTRI_LOWER) != (p.trans != RTRI_NOTRANS);
        const bool fwd_solve = p.side == RTRI_LEFT ? low : !low;
        forward = p.solve ? fwd_solve : !fwd_solve;
    }

    void leaf(int64_t d0, int64_t h, double alpha)
    {
        Op op{};
        op.gemm = false;
        LeafDesc &l = op.l;
        // offset of this block inside the packed workspace; rebased at launch
        l.Lp = reinterpret_cast<const void *>((intptr_t)((d0 / p.leaf) * pack_elems(p.leaf) * (int64_t)es));
        l.nb = (int)h;
        l.unit = p.diag == RTRI_UNIT;
        l.alpha = alpha;
        if (p.side == RTRI_LEFT) {
            // the block of op(A); vectors are columns of B
            l.mlower = low;
            l.B = p.B + d0 * (int64_t)es;
            l.sd = 1;
            l.si = p.ldb;
            l.nvec = p.n;
        } else {
            // x op(A) = alpha b  <=>  op(A)^T x^T = alpha b^T;  vectors are rows of B
            l.mlower = !low;
            l.B = p.B + d0 * p.ldb * (int64_t)es;
            l.sd = p.ldb;
            l.si = 1;
            l.nvec = p.m;
        }
        ops.push_back(op);
    }

    // B[t] = beta * B[t] + s * (off-diagonal block) x B[src]
    void update(int64_t t0, int64_t th, int64_t s0, int64_t sh, double beta, double s, int depth)
    {
        Op op{};
        op.gemm = true;
        op.depth = depth;
        GemmDesc &g = op.g;
        g.beta = beta;
        g.s = s;
        g.K = sh;
        const bool tr = ag_tr(p);
        if (p.side == RTRI_LEFT) {
            g.M = th;
            g.N = p.n;
            g.P = tri_block(p, t0, s0);
            g.ldp = p.ldag;
            g.tp = tr;
            g.Q = p.solve ? p.B + s0 * (int64_t)es : src + s0 * (int64_t)ses;
            g.ldq = p.solve ? p.ldb : ldsrc;
            g.tq = false;
            g.C = p.B + t0 * (int64_t)es;
        } else {
            g.M = p.m;
            g.N = th;
            g.P = p.solve ? p.B + s0 * p.ldb * (int64_t)es : src + s0 * ldsrc * (int64_t)ses;
            g.ldp = p.solve ? p.ldb : ldsrc;
            g.tp = false;
            g.Q = tri_block(p, s0, t0);
            g.ldq = p.ldag;
            g.tq = tr;
            g.C = p.B + t0 * p.ldb * (int64_t)es;
        }
        g.ldc = p.ldb;
        ops.push_back(op);
    }

    void rec(int64_t d0, int64_t h, double alpha, int depth = 0)
    {
        if (h <= p.leaf) {
            leaf(d0, h, alpha);
            return;
        }
        const int64_t a = p.leaf;
        const int64_t k = a * ((h + 2 * a - 1) / (2 * a));
        const int64_t b1 = d0, h1 = k, b2 = d0 + k, h2 = h - k;
        const int64_t f0 = forward ? b1 : b2, fh = forward ? h1 : h2;   // first block
        const int64_t g0 = forward ? b2 : b1, gh = forward ? h2 : h1;   // second block
        rec(f0, fh, alpha, depth + 1);
        if (p.solve) {
            update(g0, gh, f0, fh, alpha, -1.0, depth);   // B_second = alpha B_second - off * X_first
            rec(g0, gh, 1.0, depth + 1);
        } else {
            update(f0, fh, g0, gh, 1.0, alpha, depth);    // B_first += alpha * off * B_second (original)
            rec(g0, gh, alpha, depth + 1);
        }
    }
};

int dtype_code(ElemT t) { return (int)t; }

double gemm_flops(const GemmDesc &g) { return 2.0 * (double)g.M * (double)g.N * (double)g.K; }
double gemm_bytes(const GemmDesc &g, size_t esp, size_t esq, size_t esc)
{
    return (double)esp * g.M * g.K + (double)esq * g.K * g.N + (double)esc * (g.beta == 0.0 ? 1.0 : 2.0) * g.M * g.N;
}
double leaf_flops(const LeafDesc &l) { return (double)l.nb * l.nb * (double)l.nvec; }
double leaf_bytes(const LeafDesc &l, size_t es)
{
    return (double)es * ((double)l.nb * (l.nb + 1) / 2.0 + 2.0 * l.nb * (double)l.nvec);
}

}  // namespace

namespace rtri {

bool handle_valid(const rtri_handle *h) { return h != nullptr && h->magic == MAGIC; }

int hip_fail(rtri_handle *h, hipError_t e)
{
    h->last = e;
    return e == hipErrorOutOfMemory ? RTRI_ERR_NOMEM : RTRI_ERR_HIP;
}

hipError_t ensure_ws(rtri_handle *h, int slot, size_t bytes)
{
    if (bytes <= h->ws_bytes[slot])
        return hipSuccess;
    if (h->ws[slot] != nullptr) {
        hipError_t e = hipStreamSynchronize(h->stream);   // earlier work may still use it
        if (e != hipSuccess)
            return e;
        (void)hipFree(h->ws[slot]);
        h->ws[slot] = nullptr;
        h->ws_bytes[slot] = 0;
    }
    const size_t want = std::max<size_t>(bytes, (size_t)1 << 16);
    hipError_t e = hipMalloc(&h->ws[slot], want);
    if (e != hipSuccess) {
        h->ws[slot] = nullptr;
        return e;
    }
    h->ws_bytes[slot] = want;
    return hipSuccess;
}

hipError_t pool_event(rtri_handle *h, hipEvent_t *ev)
{
    if (h->pool_used == h->pool.size()) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess)
            return err;
        h->pool.push_back(e);
    }
    *ev = h->pool[h->pool_used++];
    return hipSuccess;
}

hipError_t timed_launch(rtri_handle *h, int kclass, int dtype, double flops, double bytes, hipError_t (*fn)(void *),
                        void *ctx)
{
    if (!h->profiling)
        return fn(ctx);
    ProfRec r{kclass, dtype, flops, bytes, nullptr, nullptr};
    hipError_t e = pool_event(h, &r.e0);
    if (e == hipSuccess)
        e = pool_event(h, &r.e1);
    if (e == hipSuccess)
        e = hipEventRecord(r.e0, h->stream);
    if (e != hipSuccess)
        return e;
    e = fn(ctx);
    if (e != hipSuccess)
        return e;
    e = hipEventRecord(r.e1, h->stream);
    if (e == hipSuccess)
        h->recs.push_back(r);
    return e;
}

int check_args(int side, int uplo, int trans, int diag, int64_t m, int64_t n, const void *A, int64_t lda,
               const void *B, int64_t ldb, bool need_a)
{
    if (side != RTRI_LEFT && side != RTRI_RIGHT) return -1;
    if (uplo != RTRI_LOWER && uplo != RTRI_UPPER) return -2;
    if (trans != RTRI_NOTRANS && trans != RTRI_TRANS && trans != RTRI_CONJTRANS) return -3;
    if (diag != RTRI_NONUNIT && diag != RTRI_UNIT) return -4;
    if (m < 0) return -5;
    if (n < 0) return -6;
    const int64_t ka = side == RTRI_LEFT ? m : n;
    if (m > 0 && n > 0 && need_a && A == nullptr) return -8;
    if (lda < std::max<int64_t>(1, ka)) return -9;
    if (m > 0 && n > 0 && B == nullptr) return -10;
    if (ldb < std::max<int64_t>(1, m)) return -11;
    return 0;
}

bool valid_leaf(int64_t v) { return v == 0 || v == 16 || v == 32 || v == 64 || v == 128 || v == 256; }

int pick_leaf(const rtri_handle *h, DType t, bool solve, int64_t ka, int64_t nvec)
{
    int leaf = t == DType::F64 ? h->leaf_f64 : h->leaf_f32;
    if (leaf == 0)
        leaf = tuned_leaf(h->tune, t == DType::F64 ? RTRI_F64 : RTRI_F32, solve, ka, nvec);
    if (leaf != 0)
        return leaf;
    // untuned: the 64-row leaf (also the batched kernel's) for small factors,
    // the matrix-core 256-row leaf above
    return ka <= 1024 ? 64 : 256;
}

// GEMM tile: the handle's option, else the tuning database's rule, else
// automatic (0).  A rule is measured at its bucket's largest size; a 128 x 128
// tile it names for an update that would leave CUs without a workgroup (fewer
// than 256 tiles, e.g. N far below the bucket's) falls back to automatic.
int pick_tile(const rtri_handle *h, int dtype, int64_t M, int64_t N)
{
    if (h->gemm_tile != 0)
        return h->gemm_tile;
    const int t = tuned_tile(h->tune, dtype, M, N);
    if ((t == 1 || t == 3) && ((M + 127) / 128) * ((N + 127) / 128) < 256)
        return 0;
    return t;
}

// GEMM updates with disjoint outputs and no mutual dependence, spread over
// the handle's auxiliary streams (one stays on the handle's stream);
// launch(g, stream) enqueues one update
template <class Launch>
hipError_t run_gemms_concurrent(rtri_handle *h, const std::vector<const GemmDesc *> &gs, Launch &&launch)
{
    // a fork / join across streams costs tens of microseconds: a few small
    // updates stay on the handle's stream, one after another (concurrent from
    // 8 updates, or from 2 of at least 1 GFLOP each)
    const bool big = !gs.empty() && 2.0 * (double)gs[0]->M * (double)gs[0]->N * (double)gs[0]->K >= 1e9;
    if (gs.size() < 2 || (gs.size() < 8 && !big)) {
        for (const GemmDesc *g : gs) {
            const hipError_t e = launch(*g, h->stream);
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    }
    hipError_t e = hipSuccess;
    if (!h->aux_ready) {
        for (int i = 0; i < 4 && e == hipSuccess; ++i)
            e = hipStreamCreateWithFlags(&h->aux[i], hipStreamNonBlocking);
        for (int i = 0; i < 5 && e == hipSuccess; ++i)
            e = hipEventCreateWithFlags(&h->aux_ev[i], hipEventDisableTiming);
        if (e != hipSuccess)
            return e;
        h->aux_ready = true;
    }
    const int na = (int)std::min<size_t>(4, gs.size() - 1);
    e = hipEventRecord(h->aux_ev[4], h->stream);
    for (int i = 0; i < na && e == hipSuccess; ++i)
        e = hipStreamWaitEvent(h->aux[i], h->aux_ev[4], 0);
    for (size_t j = 0; j < gs.size() && e == hipSuccess; ++j)
        e = launch(*gs[j], j == 0 ? h->stream : h->aux[(j - 1) % na]);
    for (int i = 0; i < na && e == hipSuccess; ++i) {
        e = hipEventRecord(h->aux_ev[i], h->aux[i]);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(h->stream, h->aux_ev[i], 0);
    }
    return e;
}

// All GEMM updates of a one-launch TRMM plan in one grouped launch: FP64 /
// FP32 panels in 64x64 tiles, 16-bit updates (both operands 16-bit) in
// 256x256 tiles.  The tables are built on the host, copied to the handle's
// workspace and read by the kernel.  Returns hipErrorNotSupported, with
// nothing launched, when 16-bit updates do not fit the 256x256 tiles (then
// the caller runs them depth by depth); sets h->last on other failures.
static hipError_t run_grouped(rtri_handle *h, const PlanIn &p, const std::vector<Op> &ops, DType bt)
{
    const size_t es = bt == DType::F64 ? 8 : 4;
    const bool g16 = p.gt == ElemT::BF16 || p.gt == ElemT::F16;
    const int64_t TS = g16 ? 256 : 64;   // output tile
    int maxd = -1;
    for (const Op &op : ops)
        if (op.gemm)
            maxd = std::max(maxd, op.depth);
    if (maxd < 0)
        return hipSuccess;
    std::vector<GemmDesc> descs;
    // the panel's TS x TS tiles, row tile r and column tile c at r + c * trows;
    // entries are collected per tile in the order the updates are visited
    const int64_t trows = (p.m + TS - 1) / TS, tcols = (p.n + TS - 1) / TS;
    std::vector<int> count((size_t)(trows * tcols), 0);
    std::vector<double> work((size_t)(trows * tcols), 0.0);
    struct Raw {
        int tile;
        GroupEntry e;
    };
    std::vector<Raw> raw;
    bool vec = true;
    bool tp = false, tq = false;
    double flops = 0.0, bytes = 0.0;
    for (int d = maxd; d >= 0; --d)
        for (const Op &op : ops) {
            if (!op.gemm || op.depth != d || op.g.M <= 0 || op.g.N <= 0)
                continue;
            const GemmDesc &g = op.g;
            const int idx = (int)descs.size();
            descs.push_back(g);
            tp = g.tp;
            tq = g.tq;
            const int64_t w = (int64_t)(16 / (g16 ? 2 : es));
            vec = vec && (reinterpret_cast<uintptr_t>(g.P) % 16 == 0) && (reinterpret_cast<uintptr_t>(g.Q) % 16 == 0) &&
                  g.ldp % w == 0 && g.ldq % w == 0;
            flops += gemm_flops(g);
            bytes += g16 ? gemm_bytes(g, 2, 2, 4) : gemm_bytes(g, es, es, es);
            // origin of this update's C inside the panel (a multiple of 64 in
            // both directions: leaf boundaries and the vector tiles; of 256 for
            // the 16-bit tiles, else they are not used)
            const int64_t off = (static_cast<const char *>(g.C) - p.B) / (int64_t)es;
            const int64_t r0 = off % p.ldb, c0 = off / p.ldb;
            if (g16 && (r0 % TS != 0 || c0 % TS != 0 || !g.tp || g.tq))
                return hipErrorNotSupported;
            for (int64_t n0 = 0; n0 < g.N; n0 += TS)
                for (int64_t m0 = 0; m0 < g.M; m0 += TS) {
                    const int t = (int)((r0 + m0) / TS + ((c0 + n0) / TS) * trows);
                    raw.push_back(Raw{t, GroupEntry{idx, (int)m0, (int)n0}});
                    ++count[(size_t)t];
                    work[(size_t)t] += (double)g.K;
                }
        }
    // 16-bit tiles whose updates can be loaded straight into LDS and share one
    // accumulator: full 256x256 tiles, every update adding (beta = 1) with
    // one scale, K a multiple of 32 (launch_gemm16_grouped)
    std::vector<char> dma(count.size(), g16 && h->gemm16_tile != 3 ? 1 : 0);
    std::vector<double> scale(count.size(), 0.0);
    std::vector<char> seen(count.size(), 0);
    if (g16)
        for (const Raw &r : raw) {
            const GemmDesc &g = descs[(size_t)r.e.desc];
            const size_t t = (size_t)r.tile;
            if (!seen[t]) {
                seen[t] = 1;
                scale[t] = g.s;
            }
            if (g.M - r.e.m0 < TS || g.N - r.e.n0 < TS || g.K % 32 != 0 || g.beta != 1.0 || g.s != scale[t])
                dma[t] = 0;
        }
    // tiles with updates, most work first (the direct-to-LDS ones before the
    // rest); entries grouped per tile, in visiting order (a counting sort keeps it)
    std::vector<int> order;
    for (int t = 0; t < (int)count.size(); ++t)
        if (count[(size_t)t] > 0)
            order.push_back(t);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (dma[(size_t)x] != dma[(size_t)y])
            return dma[(size_t)x] > dma[(size_t)y];
        return work[(size_t)x] > work[(size_t)y];
    });
    // The 64x64 tiles of a launch are mostly resident together (several
    // workgroups per CU), so where the dispatcher places them, not the order
    // they finish in, decides each CU's load.  Workgroup i lands on CU
    // i mod (CU count) when the launch fits: reversing every other round of
    // that many tiles gives each CU about the same work (a triangle's tiles
    // range from a few K steps to the whole order).
    if (!g16) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            for (size_t r0 = (size_t)cus; r0 < order.size(); r0 += 2 * (size_t)cus)
                std::reverse(order.begin() + (std::ptrdiff_t)r0,
                             order.begin() + (std::ptrdiff_t)std::min(order.size(), r0 + (size_t)cus));
    }
    std::vector<int> start(count.size(), 0);
    std::vector<GroupTile> tiles;
    tiles.reserve(order.size());
    int pos = 0, n_dma = 0;
    for (int t : order) {
        start[(size_t)t] = pos;
        tiles.push_back(GroupTile{pos, count[(size_t)t]});
        pos += count[(size_t)t];
        n_dma += dma[(size_t)t];
    }
    std::vector<GroupEntry> ents((size_t)pos);
    for (const Raw &r : raw)
        ents[(size_t)start[(size_t)r.tile]++] = r.e;
    if (g16 && !vec)
        return hipErrorNotSupported;
    const size_t bd = descs.size() * sizeof(GemmDesc), be = ents.size() * sizeof(GroupEntry),
                 bti = tiles.size() * sizeof(GroupTile);
    const size_t oe = (bd + 255) / 256 * 256, ot = oe + (be + 255) / 256 * 256;
    std::vector<char> host(ot + bti);
    std::memcpy(host.data(), descs.data(), bd);
    std::memcpy(host.data() + oe, ents.data(), be);
    std::memcpy(host.data() + ot, tiles.data(), bti);
    hipError_t e = ensure_ws(h, WS_GROUP, host.size());
    // pageable source: the copy is staged before the call returns, so the
    // host vector may go away at once
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->ws[WS_GROUP], host.data(), host.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        char *dev = static_cast<char *>(h->ws[WS_GROUP]);
        const GemmDesc *dd = reinterpret_cast<const GemmDesc *>(dev);
        const GroupEntry *de = reinterpret_cast<const GroupEntry *>(dev + oe);
        const GroupTile *dt = reinterpret_cast<const GroupTile *>(dev + ot);
        const int dcode = g16 ? dtype_code(p.gt) : bt == DType::F64 ? RTRI_F64 : RTRI_F32;
        e = timed(h, RTRI_KCLASS_GEMM, dcode, flops, bytes, [&] {
            return g16 ? launch_gemm16_grouped(p.gt == ElemT::BF16, dd, de, dt, n_dma, dt + n_dma,
                                               (int)tiles.size() - n_dma, h->stream)
                       : launch_gemm_grouped(bt, dd, de, dt, (int)tiles.size(), tp, tq, vec, h->stream);
        });
    }
    if (e != hipSuccess)
        h->last = e;
    return e;
}

bool trmm_one_launch(const rtri_handle *h, int leaf, int64_t ka, int64_t nvec)
{
    if (leaf < 64 || ka <= leaf)   // matrix-core leaves; a single leaf has no schedule to choose
        return false;
    if (h->trmm_leaves != 0)
        return h->trmm_leaves == 2;
    // one launch per leaf fills the chip from 8192 vectors on (128 workgroups
    // of 64 vectors); below that the leaves run on a few CUs one after another
    return nvec < 8192;
}

size_t plan_pack_bytes(const PlanIn &p)
{
    const int64_t ka = p.side == RTRI_LEFT ? p.m : p.n;
    const int64_t nblk = (ka + p.leaf - 1) / p.leaf;
    return (size_t)(nblk * pack_elems(p.leaf)) * (p.bt == DType::F64 ? 8 : 4);
}

hipError_t pack_plan(rtri_handle *h, const PlanIn &p, void *out)
{
    const int64_t ka = p.side == RTRI_LEFT ? p.m : p.n;
    const int64_t nblk = (ka + p.leaf - 1) / p.leaf;
    const size_t es = p.bt == DType::F64 ? 8 : 4;
    const bool low = (p.uplo == RTRI_LOWER) != (p.trans != RTRI_NOTRANS);
    PackDesc pk{};
    pk.A = p.As;
    pk.lda = p.ldas;
    pk.ka = ka;
    pk.unit = p.diag == RTRI_UNIT;
    if (p.side == RTRI_LEFT) {
        pk.mtrans = p.trans != RTRI_NOTRANS;
        pk.mlower = low;
    } else {
        pk.mtrans = p.trans == RTRI_NOTRANS;
        pk.mlower = !low;
    }
    pk.out = out;
    return timed(h, RTRI_KCLASS_OTHER, dtype_code(p.st), 0.0,
                 (double)elem_size(p.st) * ka * (double)p.leaf + (double)es * nblk * pack_elems(p.leaf),
                 [&] { return launch_pack(p.st, p.bt, p.solve, p.leaf, pk, h->stream); });
}

PlanIn plain_plan(rtri_handle *h, DType t, bool solve, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                  double alpha, const void *A, int64_t lda, void *B, int64_t ldb)
{
    PlanIn p{};
    p.solve = solve;
    p.side = side;
    p.uplo = uplo;
    p.trans = trans == RTRI_CONJTRANS ? RTRI_TRANS : trans;
    p.diag = diag;
    p.m = m;
    p.n = n;
    p.alpha = alpha;
    p.bt = t;
    p.B = static_cast<char *>(B);
    p.ldb = ldb;
    p.gt = t == DType::F64 ? ElemT::F64 : ElemT::F32;
    p.Ag = static_cast<const char *>(A);
    p.ldag = lda;
    p.st = p.gt;
    p.As = A;
    p.ldas = lda;
    p.leaf = pick_leaf(h, t, solve, side == RTRI_LEFT ? m : n, side == RTRI_LEFT ? n : m);
    p.pack_slot = WS_PACK;
    p.skip_pack = false;
    p.packed = nullptr;
    return p;
}

int run_plan(rtri_handle *h, const PlanIn &p)
{
    const int64_t ka = p.side == RTRI_LEFT ? p.m : p.n;
    if (p.m == 0 || p.n == 0)
        return RTRI_OK;
    const DType bt = p.bt;
    const size_t es = bt == DType::F64 ? 8 : 4;
    const int pcode = bt == DType::F64 ? RTRI_F64 : RTRI_F32;
    Planner pl(p);
    // TRMM with every leaf in one launch: the GEMM updates read the original
    // panel from a copy (m x n, leading dimension m), so the leaves may all run
    // first; every update sees the same operands as in recursion order
    const int64_t nvec_all = p.side == RTRI_LEFT ? p.n : p.m;
    // (a 16-bit TRMM's updates read the 16-bit original, so it needs no saved
    // copy and takes this schedule at any width: its updates then run as one
    // grouped launch of 256x256 tiles)
    const bool one = !p.solve && p.ext_split == nullptr &&
                     (trmm_one_launch(h, p.leaf, ka, nvec_all) ||
                      (p.Bsrc16 != nullptr && h->trmm_leaves != 1 && p.leaf >= 64 && ka > p.leaf));
    // a TRMM whose updates read the 16-bit original needs no saved copy
    const bool save = one && p.Bsrc16 == nullptr;
    if (save) {
        hipError_t e0 = ensure_ws(h, WS_SAVE, (size_t)p.m * (size_t)p.n * es);
        if (e0 != hipSuccess)
            return hip_fail(h, e0);
        pl.src = static_cast<const char *>(h->ws[WS_SAVE]);
        pl.ldsrc = p.m;
    }
    pl.rec(0, ka, p.alpha);

    // pack every diagonal block once into the canonical form the leaves read
    // (unless the plan brings its blocks packed already)
    if (p.packed == nullptr && !p.skip_pack) {
        hipError_t e0 = hipSuccess;
        if (p.ext_pack == nullptr)
            e0 = ensure_ws(h, p.pack_slot, plan_pack_bytes(p));
        if (e0 == hipSuccess)
            e0 = pack_plan(h, p, p.ext_pack != nullptr ? p.ext_pack : h->ws[p.pack_slot]);
        if (e0 != hipSuccess)
            return hip_fail(h, e0);
    }
    const char *pack_base = static_cast<const char *>(
        p.packed != nullptr ? p.packed : (p.ext_pack != nullptr ? p.ext_pack : h->ws[p.pack_slot]));
    for (Op &op : pl.ops)
        if (!op.gemm)
            op.l.Lp = pack_base + reinterpret_cast<intptr_t>(op.l.Lp);

    const bool g16 = p.gt == ElemT::BF16 || p.gt == ElemT::F16;
    const size_t ges = elem_size(p.gt);
    // updates short of tiles with a long K split K (partials in workspace, one
    // region per stream, since one depth's TRMM updates may run concurrently)
    bool any_split = false;
    if (!g16 && may_split(ka))
        for (const Op &op : pl.ops)
            if (op.gemm && plan_split(bt, op.g, pick_tile(h, pcode, op.g.M, op.g.N), SPLIT_REGION_BYTES).slices >= 2)
                any_split = true;
    if (any_split && p.ext_split == nullptr) {
        hipError_t e0 = ensure_ws(h, WS_SPLIT, SPLIT_WS_BYTES);
        if (e0 != hipSuccess)
            return hip_fail(h, e0);
    }
    auto split_region = [&](hipStream_t st) -> void * {
        if (p.ext_split != nullptr)
            return st == h->stream ? p.ext_split : nullptr;
        int r = 0;
        if (st != h->stream)
            for (int i = 0; i < 4; ++i)
                if (h->aux_ready && st == h->aux[i])
                    r = i + 1;
        if (r == 0 && st != h->stream)
            return nullptr;   // unknown stream: no split
        return static_cast<char *>(h->ws[WS_SPLIT]) + (size_t)r * SPLIT_REGION_BYTES;
    };
    // one GEMM update on a stream: 16-bit factor copy or panel-type MFMA tiles
    auto launch_update = [&](const GemmDesc &g, hipStream_t st) {
        if (g16) {
            // the factor's block is 16-bit; the panel operand too when a TRMM reads the 16-bit original
            const bool panel16 = !p.solve && p.Bsrc16 != nullptr;
            const bool left = p.side == RTRI_LEFT;
            const int t16 = h->gemm16_tile != 0 ? h->gemm16_tile : tuned_tile(h->tune, dtype_code(p.gt), g.M, g.N);
            return launch_gemm16(p.gt == ElemT::BF16, left || panel16, !left || panel16, g, st, t16);
        }
        const int tile = pick_tile(h, pcode, g.M, g.N);
        Split sp{};
        if (any_split) {
            sp = plan_split(bt, g, tile, SPLIT_REGION_BYTES);
            sp.part = sp.slices >= 2 ? split_region(st) : nullptr;
        }
        return launch_gemm(bt, g, tile, st, sp);
    };
    if (one) {
        hipError_t e = hipSuccess;
        if (save)
            e = timed(h, RTRI_KCLASS_OTHER, pcode, 0.0, 2.0 * es * p.m * p.n, [&] {
                return hipMemcpy2DAsync(h->ws[WS_SAVE], p.m * es, p.B, p.ldb * es, p.m * es, p.n,
                                        hipMemcpyDeviceToDevice, h->stream);
            });
        if (e != hipSuccess)
            return hip_fail(h, e);
        LeafDesc all{};
        double fl = 0.0, by = 0.0;
        for (const Op &op : pl.ops)
            if (!op.gemm) {
                if (all.nvec == 0) {
                    all = op.l;
                    all.B = p.B;   // block 0 starts at element 0 of the panel
                    all.Lp = pack_base;
                    all.nb = p.leaf;
                    all.ka = ka;
                }
                fl += leaf_flops(op.l);
                by += leaf_bytes(op.l, es);
            }
        e = timed(h, RTRI_KCLASS_LEAF_MULT, pcode, fl, by, [&] { return launch_leaf(bt, false, p.leaf, all, h->stream); });
        if (e != hipSuccess)
            return hip_fail(h, e);
    }
    if (one && (!g16 || p.Bsrc16 != nullptr)) {
        // The updates read only the saved panel (or the 16-bit original), and
        // each tile of the panel gets at most one update per depth, deepest
        // first in recursion order: one launch in which a workgroup owns a
        // tile and applies its updates in that order (tiles with the most
        // work first).  16-bit updates that do not fit the 256x256 tiles run
        // depth by depth below.
        const hipError_t e = run_grouped(h, p, pl.ops, bt);
        if (e == hipSuccess)
            return RTRI_OK;
        if (e != hipErrorNotSupported)
            return hip_fail(h, h->last);
    }
    if (one && !h->profiling) {
        // The updates read only the saved panel and each writes one row block,
        // which gets one update per depth, deepest first in recursion order: so
        // run the depths deepest first, the updates of one depth concurrently
        // on the auxiliary streams.
        int maxd = 0;
        for (const Op &op : pl.ops)
            if (op.gemm)
                maxd = std::max(maxd, op.depth);
        for (int d = maxd; d >= 0; --d) {
            std::vector<const GemmDesc *> gs;
            for (const Op &op : pl.ops)
                if (op.gemm && op.depth == d)
                    gs.push_back(&op.g);
            hipError_t e = run_gemms_concurrent(h, gs, launch_update);
            if (e != hipSuccess)
                return hip_fail(h, e);
        }
        return RTRI_OK;
    }
    for (const Op &op : pl.ops) {
        hipError_t e;
        if (one && !op.gemm)
            continue;
        if (op.gemm) {
            const bool left = p.side == RTRI_LEFT;
            const size_t pes = (p.solve || p.Bsrc16 == nullptr) ? es : 2;   // panel operand as read
            const double bytes = gemm_bytes(op.g, left ? ges : pes, left ? pes : ges, es);
            e = timed(h, RTRI_KCLASS_GEMM, g16 ? dtype_code(p.gt) : pcode, gemm_flops(op.g), bytes,
                      [&] { return launch_update(op.g, h->stream); });
        } else {
            e = timed(h, p.solve ? RTRI_KCLASS_LEAF_SOLVE : RTRI_KCLASS_LEAF_MULT, pcode, leaf_flops(op.l),
                      leaf_bytes(op.l, es), [&] { return launch_leaf(bt, p.solve, p.leaf, op.l, h->stream); });
        }
        if (e != hipSuccess)
            return hip_fail(h, e);
    }
    return RTRI_OK;
}

}  // namespace rtri

namespace {

int run(rtri_handle *h, DType t, bool solve, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
        double alpha, const void *A, int64_t lda, void *B, int64_t ldb)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    const int rc = check_args(side, uplo, trans, diag, m, n, A, lda, B, ldb, alpha != 0.0);
    if (rc != 0)
        return rc;
    if (m == 0 || n == 0)
        return RTRI_OK;
    const int dcode = t == DType::F64 ? RTRI_F64 : RTRI_F32;
    const size_t es = t == DType::F64 ? 8 : 4;
    if (alpha == 0.0) {
        hipError_t e = timed(h, RTRI_KCLASS_OTHER, dcode, 0.0, (double)es * m * n,
                             [&] { return launch_fill(t, B, m, n, ldb, 0.0, h->stream); });
        return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
    }
    return run_plan(h, plain_plan(h, t, solve, side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb));
}

}  // namespace

extern "C" {

int rtri_query_leaf(rtri_handle *h, int dtype, int op, int64_t order, int64_t nvec, int *leaf)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (dtype != RTRI_F64 && dtype != RTRI_F32)
        return -2;
    if (op != 0 && op != 1)
        return -3;
    if (order < 0 || nvec < 0)
        return -4;
    if (leaf == nullptr)
        return -6;
    *leaf = pick_leaf(h, dtype == RTRI_F64 ? DType::F64 : DType::F32, op == 0, order, nvec);
    return RTRI_OK;
}

int rtri_create(rtri_handle **out, void *stream)
{
    if (out == nullptr)
        return -1;
    rtri_handle *h = new (std::nothrow) rtri_handle();
    if (h == nullptr)
        return RTRI_ERR_NOMEM;
    h->magic = MAGIC;
    h->stream = static_cast<hipStream_t>(stream);
    h->leaf_f64 = 0;
    h->leaf_f32 = 0;
    h->gemm_tile = 0;
    h->trmm_leaves = 0;
    h->gemm16_tile = 0;
    h->residual = 0;
    h->tune = nullptr;
    h->last = hipSuccess;
    for (int i = 0; i < WS_COUNT; ++i) {
        h->ws[i] = nullptr;
        h->ws_bytes[i] = 0;
    }
    h->profiling = false;
    h->pool_used = 0;
    noalloc_prepare();   // the no-allocation entry point's scratch address on this device
    h->aux_ready = false;
    h->mem_pool = nullptr;
    // a tuning database named by the environment applies to every new handle
    if (const char *db = std::getenv("RTRI_TUNE_DB"))
        (void)load_tuning_file(h, db);
    *out = h;
    return RTRI_OK;
}

int rtri_destroy(rtri_handle *h)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    h->magic = 0;
    bool any = false;
    for (int i = 0; i < WS_COUNT; ++i)
        any = any || h->ws[i] != nullptr;
    if (any)
        (void)hipStreamSynchronize(h->stream);
    for (int i = 0; i < WS_COUNT; ++i)
        if (h->ws[i] != nullptr)
            (void)hipFree(h->ws[i]);
    for (hipEvent_t e : h->pool)
        (void)hipEventDestroy(e);
    if (h->aux_ready) {
        for (int i = 0; i < 4; ++i) {
            (void)hipStreamSynchronize(h->aux[i]);
            (void)hipStreamDestroy(h->aux[i]);
        }
        for (int i = 0; i < 5; ++i)
            (void)hipEventDestroy(h->aux_ev[i]);
    }
    tune_db_free(h->tune);
    delete h;
    return RTRI_OK;
}

int rtri_set_stream(rtri_handle *h, void *stream)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    h->stream = static_cast<hipStream_t>(stream);
    return RTRI_OK;
}

int rtri_sync(rtri_handle *h)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    hipError_t e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
}

int rtri_set_option(rtri_handle *h, int option, int64_t value)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    switch (option) {
    case RTRI_OPT_LEAF_F64:
        if (!valid_leaf(value)) return -3;
        h->leaf_f64 = (int)value;
        return RTRI_OK;
    case RTRI_OPT_LEAF_F32:
        if (!valid_leaf(value)) return -3;
        h->leaf_f32 = (int)value;
        return RTRI_OK;
    case RTRI_OPT_GEMM_TILE:
        if (value < 0 || value > 3) return -3;
        h->gemm_tile = (int)value;
        return RTRI_OK;
    case RTRI_OPT_TRMM_LEAVES:
        if (value < 0 || value > 2) return -3;
        h->trmm_leaves = (int)value;
        return RTRI_OK;
    case RTRI_OPT_GEMM16_TILE:
        if (value < 0 || value > 3) return -3;
        h->gemm16_tile = (int)value;
        return RTRI_OK;
    case RTRI_OPT_RESIDUAL:
        if (value < 0 || value > 1) return -3;
        h->residual = (int)value;
        return RTRI_OK;
    default:
        return -2;
    }
}

int rtri_get_option(rtri_handle *h, int option, int64_t *value)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (value == nullptr)
        return -3;
    switch (option) {
    case RTRI_OPT_LEAF_F64: *value = h->leaf_f64; return RTRI_OK;
    case RTRI_OPT_LEAF_F32: *value = h->leaf_f32; return RTRI_OK;
    case RTRI_OPT_GEMM_TILE: *value = h->gemm_tile; return RTRI_OK;
    case RTRI_OPT_TRMM_LEAVES: *value = h->trmm_leaves; return RTRI_OK;
    case RTRI_OPT_GEMM16_TILE: *value = h->gemm16_tile; return RTRI_OK;
    case RTRI_OPT_RESIDUAL: *value = h->residual; return RTRI_OK;
    default: return -2;
    }
}

const char *rtri_status_string(int s)
{
    if (s < 0) {
        static const char *names[] = {"invalid argument",        "invalid side",  "invalid uplo",
                                      "invalid trans",           "invalid diag",  "m < 0",
                                      "n < 0",                   "invalid alpha", "A is NULL",
                                      "lda too small",           "B is NULL",     "ldb too small",
                                      "invalid argument 12"};
        return (-s) <= 12 ? names[-s] : names[0];
    }
    switch (s) {
    case RTRI_OK: return "success";
    case RTRI_ERR_HANDLE: return "invalid handle";
    case RTRI_ERR_HIP: return "HIP runtime error";
    case RTRI_ERR_NOMEM: return "out of device memory";
    case RTRI_ERR_UNSUPPORTED: return "unsupported option or type combination";
    case RTRI_NOT_CONVERGED: return "iterative refinement did not converge";
    case RTRI_ERR_INVALID: return "invalid input";
    case RTRI_ERR_TOO_LARGE: return "problem exceeds the fixed scratch of the no-allocation entry point";
    default: return "unknown status";
    }
}

int rtri_last_hip_error(rtri_handle *h)
{
    if (!handle_valid(h))
        return -1;
    return (int)h->last;
}

int rtri_profile_begin(rtri_handle *h)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    h->recs.clear();
    h->pool_used = 0;
    h->profiling = true;
    return RTRI_OK;
}

int rtri_profile_end(rtri_handle *h, rtri_kernel_stat *out, int max_out, int *n_out)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (n_out == nullptr || (out == nullptr && max_out > 0))
        return -2;
    h->profiling = false;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess)
        return hip_fail(h, e);
    std::vector<rtri_kernel_stat> agg;
    for (const ProfRec &r : h->recs) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.e0, r.e1);
        if (e != hipSuccess)
            return hip_fail(h, e);
        rtri_kernel_stat *slot = nullptr;
        for (auto &a : agg)
            if (a.kclass == r.kclass && a.dtype == r.dtype)
                slot = &a;
        if (slot == nullptr) {
            agg.push_back(rtri_kernel_stat{r.kclass, r.dtype, 0, 0.0, 0.0, 0.0});
            slot = &agg.back();
        }
        slot->launches += 1;
        slot->ms += ms;
        slot->flops += r.flops;
        slot->bytes += r.bytes;
    }
    h->recs.clear();
    h->pool_used = 0;
    const int n = std::min<int>((int)agg.size(), std::max(0, max_out));
    for (int i = 0; i < n; ++i)
        out[i] = agg[i];
    *n_out = n;
    return RTRI_OK;
}

int rtri_dtrsm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
               const double *A, int64_t lda, double *B, int64_t ldb)
{
    return run(h, DType::F64, true, side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb);
}

int rtri_strsm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, float alpha,
               const float *A, int64_t lda, float *B, int64_t ldb)
{
    return run(h, DType::F32, true, side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb);
}

int rtri_dtrmm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, double alpha,
               const double *A, int64_t lda, double *B, int64_t ldb)
{
    return run(h, DType::F64, false, side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb);
}

int rtri_strmm(rtri_handle *h, int side, int uplo, int trans, int diag, int64_t m, int64_t n, float alpha,
               const float *A, int64_t lda, float *B, int64_t ldb)
{
    return run(h, DType::F32, false, side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb);
}

int rtri_gemm_update(rtri_handle *h, int dtype, int trans_p, int trans_q, int64_t M, int64_t N, int64_t K,
                     double s, const void *P, int64_t ldp, const void *Q, int64_t ldq, double beta, void *C,
                     int64_t ldc)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (dtype != RTRI_F64 && dtype != RTRI_F32 && dtype != RTRI_BF16 && dtype != RTRI_F16) return -2;
    if (trans_p != RTRI_NOTRANS && trans_p != RTRI_TRANS && trans_p != RTRI_CONJTRANS) return -3;
    if (trans_q != RTRI_NOTRANS && trans_q != RTRI_TRANS && trans_q != RTRI_CONJTRANS) return -4;
    if (M < 0) return -5;
    if (N < 0) return -6;
    if (K < 0) return -7;
    const bool tp = trans_p != RTRI_NOTRANS, tq = trans_q != RTRI_NOTRANS;
    const bool work = M > 0 && N > 0 && K > 0 && s != 0.0;
    if (work && P == nullptr) return -9;
    if (ldp < std::max<int64_t>(1, tp ? K : M)) return -10;
    if (work && Q == nullptr) return -11;
    if (ldq < std::max<int64_t>(1, tq ? N : K)) return -12;
    if (M > 0 && N > 0 && C == nullptr) return -14;
    if (ldc < std::max<int64_t>(1, M)) return -15;
    if (M == 0 || N == 0)
        return RTRI_OK;
    GemmDesc g{};
    g.M = M;
    g.N = N;
    g.K = work ? K : 0;
    g.s = s;
    g.beta = beta;
    g.P = P;
    g.ldp = ldp;
    g.tp = tp;
    g.Q = Q;
    g.ldq = ldq;
    g.tq = tq;
    g.C = C;
    g.ldc = ldc;
    if (dtype == RTRI_BF16 || dtype == RTRI_F16) {
        // 16-bit P and Q, FP32 C: the matrix-core tiles of the low-precision paths
        hipError_t e = timed(h, RTRI_KCLASS_GEMM, dtype, gemm_flops(g), gemm_bytes(g, 2, 2, 4), [&] {
            const int t16 = h->gemm16_tile != 0 ? h->gemm16_tile : tuned_tile(h->tune, dtype, g.M, g.N);
            return launch_gemm16(dtype == RTRI_BF16, true, true, g, h->stream, t16);
        });
        return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
    }
    const DType t = dtype == RTRI_F64 ? DType::F64 : DType::F32;
    const size_t es = t == DType::F64 ? 8 : 4;
    hipError_t e = timed(h, RTRI_KCLASS_GEMM, dtype, gemm_flops(g), gemm_bytes(g, es, es, es), [&] {
        const int tile = pick_tile(h, dtype, g.M, g.N);
        return launch_gemm(t, g, tile, h->stream);
    });
    return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
}

}  // extern "C"
