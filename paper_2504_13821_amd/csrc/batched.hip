// Batched independent TRSM / TRMM problems in one persistent launch.
//
// Each problem's recursion (the same midpoint splits, leaf size and visiting
// order as the single-call driver, see driver.hip) is laid out on the host as a
// short op list over its dependency index: leaf(d0, h) and gemm(t0, th, s0, sh).
// The right-hand-side vectors of a problem are independent, so a problem is cut
// into chunks of 64 vectors; a chunk is one work item.  Items are queued
// longest first (cost ka^2 * vectors), and every workgroup of the persistent
// grid pulls items from an atomic counter until the queue is empty, running
// the item's whole op list in-workgroup:
//   leaf: all 256 threads stage the diagonal block into LDS in the leaf's
//         canonical stream order, wavefront 0 solves / multiplies the chunk;
//   gemm: all 256 threads run 64x64 MFMA tiles of the update (gemm_core.h).
// Per element the arithmetic is the single-call path's (same GEMM k order,
// same leaf), so a problem's result does not depend on the batch around it.
#include <cstring>
#include <map>
#include <tuple>

#include "batched_dev.h"
#include "handle.h"

using namespace rtri;
using namespace rtri::bk;

namespace {

__global__ void reset_counter(unsigned *c) { *c = 0u; }

// ---- host ----

// op list of one recursion, relative to the problem (mirrors Planner::rec)
void gen_ops(std::vector<BOp> &out, int64_t d0, int64_t h, int leaf, bool solve, bool forward, bool alpha_first)
{
    if (h <= leaf) {
        out.push_back(BOp{0, (int)d0, (int)h, 0, 0, alpha_first ? 1 : 0});
        return;
    }
    const int64_t k = leaf * ((h + 2 * leaf - 1) / (2 * leaf));
    const int64_t b1 = d0, h1 = k, b2 = d0 + k, h2 = h - k;
    const int64_t f0 = forward ? b1 : b2, fh = forward ? h1 : h2;
    const int64_t g0 = forward ? b2 : b1, gh = forward ? h2 : h1;
    gen_ops(out, f0, fh, leaf, solve, forward, alpha_first);
    if (solve) {
        out.push_back(BOp{1, (int)g0, (int)gh, (int)f0, (int)fh, alpha_first ? 1 : 0});
        gen_ops(out, g0, gh, leaf, solve, forward, false);
    } else {
        out.push_back(BOp{1, (int)f0, (int)fh, (int)g0, (int)gh, 1});
        gen_ops(out, g0, gh, leaf, solve, forward, true);
    }
}

const void *pick_kernel(DType t, int nb)
{
    if (t == DType::F64)
        return nb == 32 ? kernel_ptr<double, 32>() : kernel_ptr<double, 64>();
    return nb == 32 ? kernel_ptr<float, 32>() : kernel_ptr<float, 64>();
}

hipError_t launch_batched(DType t, int nb, unsigned grid, const BInst *insts, const BItem *items, int nitems,
                          const BOp *ops, unsigned *counter, hipStream_t st)
{
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, st, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (t == DType::F64)
        return nb == 32 ? launch<double, 32>(grid, insts, items, nitems, ops, counter, st)
                        : launch<double, 64>(grid, insts, items, nitems, ops, counter, st);
    return nb == 32 ? launch<float, 32>(grid, insts, items, nitems, ops, counter, st)
                    : launch<float, 64>(grid, insts, items, nitems, ops, counter, st);
}

}  // namespace

struct rtri_batch_plan {
    rtri_handle *h;
    DType t;
    int nb;
    int nitems;
    unsigned grid;
    void *dmem;                  // insts | items | ops | counter
    BInst *insts;
    BItem *items;
    BOp *ops;
    unsigned *counter;
    hipGraph_t graph;
    hipGraphExec_t exec;
    double flops;
};

namespace {

struct Tables {
    DType t;
    int nb;
    std::vector<BInst> insts;
    std::vector<BItem> sorted;
    std::vector<BOp> ops;
    double flops;
};

// validate the entries and lay out instances, work items (longest first) and op lists
int build_tables(rtri_handle *h, int dtype, int count, const rtri_batch_entry *e, Tables &tb, int *bad_index)
{
    if (count < 0 || (count > 0 && e == nullptr))
        return -4;
    if (dtype != RTRI_F64 && dtype != RTRI_F32)
        return RTRI_ERR_UNSUPPORTED;
    const DType t = dtype == RTRI_F64 ? DType::F64 : DType::F32;
    // one leaf size per batch: the handle's leaf option decides if set (32 if
    // it picks at most 32 for an order-1024, 64-vector problem, else the
    // 64-row matrix-core leaf), else the tuning database's batched rule, else
    // the same choice from the handle's single-call policy
    const int opt = t == DType::F64 ? h->leaf_f64 : h->leaf_f32;
    const int tuned = opt == 0 ? tuned_batch_leaf(h->tune, dtype) : 0;
    const int nb = tuned != 0 ? tuned : (pick_leaf(h, t, true, 1024, 64) <= 32 ? 32 : 64);
    std::vector<BInst> &insts = tb.insts;
    std::vector<BItem> items;
    std::vector<BOp> &ops = tb.ops;
    std::vector<double> cost;
    std::map<std::tuple<int64_t, bool, bool, bool>, std::pair<int, int>> cache;
    double flops = 0.0;
    for (int i = 0; i < count; ++i) {
        const rtri_batch_entry &b = e[i];
        int rc = (b.op == 0 || b.op == 1) ? check_args(b.side, b.uplo, b.trans, b.diag, b.m, b.n, b.A, b.lda, b.B,
                                                       b.ldb, b.alpha != 0.0)
                                          : -1;
        if (rc == 0 && (b.m > INT32_MAX || b.n > INT32_MAX))
            rc = b.m > INT32_MAX ? -5 : -6;
        if (rc != 0) {
            if (bad_index != nullptr)
                *bad_index = i;
            return rc;
        }
        if (b.m == 0 || b.n == 0)
            continue;
        BInst in{};
        in.A = b.A;
        in.B = b.B;
        in.lda = b.lda;
        in.ldb = b.ldb;
        in.m = b.m;
        in.n = b.n;
        in.alpha = b.alpha;
        in.solve = b.op == 0;
        in.left = b.side == RTRI_LEFT;
        in.tr = b.trans != RTRI_NOTRANS;
        in.low = (b.uplo == RTRI_LOWER) != (in.tr != 0);
        in.unit = b.diag == RTRI_UNIT;
        const int64_t ka = in.left ? b.m : b.n;
        if (b.alpha == 0.0) {
            in.op_begin = (int)ops.size();
            ops.push_back(BOp{2, 0, 0, 0, 0, 0});
            in.op_end = (int)ops.size();
        } else {
            const bool fwd_solve = in.left ? in.low != 0 : in.low == 0;
            const bool forward = in.solve ? fwd_solve : !fwd_solve;
            const auto key = std::make_tuple(ka, (bool)in.solve, forward, true);
            auto it = cache.find(key);
            if (it == cache.end()) {
                const int begin = (int)ops.size();
                gen_ops(ops, 0, ka, nb, in.solve != 0, forward, true);
                it = cache.emplace(key, std::make_pair(begin, (int)ops.size())).first;
            }
            in.op_begin = it->second.first;
            in.op_end = it->second.second;
        }
        const int idx = (int)insts.size();
        insts.push_back(in);
        const int64_t nvec = in.left ? b.n : b.m;
        for (int64_t v0 = 0; v0 < nvec; v0 += lk::WAVE) {
            items.push_back(BItem{idx, (int)v0});
            cost.push_back((double)ka * ka * (double)std::min<int64_t>(lk::WAVE, nvec - v0));
        }
        flops += (double)ka * ka * (double)nvec;
    }
    // longest first
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i)
        order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    tb.sorted.resize(items.size());
    for (size_t i = 0; i < order.size(); ++i)
        tb.sorted[i] = items[order[i]];
    tb.t = t;
    tb.nb = nb;
    tb.flops = flops;
    return RTRI_OK;
}

// byte offsets of the three tables and the counter inside one device block
struct Layout {
    size_t items, ops, counter, total;
};
Layout layout_of(const Tables &tb)
{
    const size_t bi = tb.insts.size() * sizeof(BInst), bt = tb.sorted.size() * sizeof(BItem);
    const size_t bo = tb.ops.size() * sizeof(BOp);
    Layout L;
    L.items = (bi + 255) & ~(size_t)255;
    L.ops = L.items + ((bt + 255) & ~(size_t)255);
    L.counter = L.ops + ((bo + 255) & ~(size_t)255);
    L.total = L.counter + 256;
    return L;
}

hipError_t grid_for(DType t, int nb, int nitems, unsigned *grid)
{
    int dev = 0, cus = 256, per = 1;
    hipError_t err = hipGetDevice(&dev);
    if (err == hipSuccess)
        err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err == hipSuccess)
        err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pick_kernel(t, nb), NT, 0);
    *grid = (unsigned)std::max(1, std::min(nitems, cus * std::max(1, per)));
    return err;
}

int build_plan(rtri_handle *h, int dtype, int count, const rtri_batch_entry *e, rtri_batch_plan **out,
               int *bad_index, bool capture)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (out == nullptr)
        return -4;
    Tables tb;
    int rc = build_tables(h, dtype, count, e, tb, bad_index);
    if (rc != RTRI_OK)
        return rc;
    const DType t = tb.t;
    const int nb = tb.nb;
    const std::vector<BInst> &insts = tb.insts;
    const std::vector<BItem> &sorted = tb.sorted;
    const std::vector<BOp> &ops = tb.ops;
    const double flops = tb.flops;

    rtri_batch_plan *p = new (std::nothrow) rtri_batch_plan();
    if (p == nullptr)
        return RTRI_ERR_NOMEM;
    p->h = h;
    p->t = t;
    p->nb = nb;
    p->nitems = (int)sorted.size();
    p->flops = flops;
    const size_t bi = insts.size() * sizeof(BInst), bt = sorted.size() * sizeof(BItem), bo = ops.size() * sizeof(BOp);
    const size_t off_items = (bi + 255) & ~(size_t)255, off_ops = off_items + ((bt + 255) & ~(size_t)255);
    const size_t off_cnt = off_ops + ((bo + 255) & ~(size_t)255);
    hipError_t err = hipMalloc(&p->dmem, off_cnt + 256);
    if (err != hipSuccess) {
        delete p;
        return hip_fail(h, err);
    }
    char *base = static_cast<char *>(p->dmem);
    p->insts = reinterpret_cast<BInst *>(base);
    p->items = reinterpret_cast<BItem *>(base + off_items);
    p->ops = reinterpret_cast<BOp *>(base + off_ops);
    p->counter = reinterpret_cast<unsigned *>(base + off_cnt);
    if (bi)
        err = hipMemcpy(p->insts, insts.data(), bi, hipMemcpyHostToDevice);
    if (err == hipSuccess && bt)
        err = hipMemcpy(p->items, sorted.data(), bt, hipMemcpyHostToDevice);
    if (err == hipSuccess && bo)
        err = hipMemcpy(p->ops, ops.data(), bo, hipMemcpyHostToDevice);
    if (err == hipSuccess)
        err = grid_for(t, nb, p->nitems, &p->grid);
    p->graph = nullptr;
    p->exec = nullptr;
    if (err == hipSuccess && capture && p->nitems > 0) {
        hipStream_t cs;
        err = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (err == hipSuccess) {
            err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (err == hipSuccess) {
                hipError_t le = launch_batched(t, nb, p->grid, p->insts, p->items, p->nitems, p->ops, p->counter, cs);
                err = hipStreamEndCapture(cs, &p->graph);
                if (err == hipSuccess)
                    err = le;
            }
            if (err == hipSuccess)
                err = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
            (void)hipStreamDestroy(cs);
        }
    }
    if (err != hipSuccess) {
        if (p->exec)
            (void)hipGraphExecDestroy(p->exec);
        if (p->graph)
            (void)hipGraphDestroy(p->graph);
        (void)hipFree(p->dmem);
        delete p;
        return hip_fail(h, err);
    }
    *out = p;
    return RTRI_OK;
}

}  // namespace

namespace rtri {

void batch_scratch_free(BatchScratch &sc)
{
    if (sc.dev != nullptr)
        (void)hipFree(sc.dev);
    if (sc.host != nullptr)
        (void)hipHostFree(sc.host);
    sc = BatchScratch{};
}

int batch_run_async(rtri_handle *h, int dtype, int count, const rtri_batch_entry *e, BatchScratch &sc,
                    int *bad_index, double *flops)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    Tables tb;
    int rc = build_tables(h, dtype, count, e, tb, bad_index);
    if (rc != RTRI_OK)
        return rc;
    if (flops != nullptr)
        *flops = tb.flops;
    const int nitems = (int)tb.sorted.size();
    if (nitems == 0)
        return RTRI_OK;
    const Layout L = layout_of(tb);
    hipError_t err = hipSuccess;
    // the caller waits for the stream before the next call, so the staging can be reused
    if (L.total > sc.host_bytes) {
        if (sc.host != nullptr)
            (void)hipHostFree(sc.host);
        sc.host = nullptr;
        sc.host_bytes = 0;
        err = hipHostMalloc(&sc.host, L.total * 2, 0);
        if (err != hipSuccess)
            return hip_fail(h, err);
        sc.host_bytes = L.total * 2;
    }
    if (L.total > sc.dev_bytes) {
        if (sc.dev != nullptr)
            (void)hipFree(sc.dev);
        sc.dev = nullptr;
        sc.dev_bytes = 0;
        err = hipMalloc(&sc.dev, L.total * 2);
        if (err != hipSuccess)
            return hip_fail(h, err);
        sc.dev_bytes = L.total * 2;
    }
    char *hb = static_cast<char *>(sc.host);
    std::memcpy(hb, tb.insts.data(), tb.insts.size() * sizeof(BInst));
    std::memcpy(hb + L.items, tb.sorted.data(), tb.sorted.size() * sizeof(BItem));
    std::memcpy(hb + L.ops, tb.ops.data(), tb.ops.size() * sizeof(BOp));
    char *db = static_cast<char *>(sc.dev);
    err = hipMemcpyAsync(db, hb, L.counter, hipMemcpyHostToDevice, h->stream);
    unsigned grid = 1;
    if (err == hipSuccess)
        err = grid_for(tb.t, tb.nb, nitems, &grid);
    if (err == hipSuccess)
        err = timed(h, RTRI_KCLASS_BATCHED, dtype, tb.flops, 0.0, [&] {
            return launch_batched(tb.t, tb.nb, grid, reinterpret_cast<const BInst *>(db),
                                  reinterpret_cast<const BItem *>(db + L.items), nitems,
                                  reinterpret_cast<const BOp *>(db + L.ops), reinterpret_cast<unsigned *>(db + L.counter),
                                  h->stream);
        });
    return err == hipSuccess ? RTRI_OK : hip_fail(h, err);
}

}  // namespace rtri

extern "C" {

int rtri_batch_plan_create(rtri_handle *h, int dtype, int count, const rtri_batch_entry *entries,
                           rtri_batch_plan **plan, int *bad_index)
{
    return build_plan(h, dtype, count, entries, plan, bad_index, true);
}

int rtri_batch_plan_run(rtri_batch_plan *p)
{
    if (p == nullptr || !handle_valid(p->h))
        return RTRI_ERR_HANDLE;
    if (p->nitems == 0)
        return RTRI_OK;
    rtri_handle *h = p->h;
    hipError_t e = timed(h, RTRI_KCLASS_BATCHED, p->t == DType::F64 ? RTRI_F64 : RTRI_F32, p->flops, 0.0, [&] {
        if (p->exec != nullptr)
            return hipGraphLaunch(p->exec, h->stream);
        return launch_batched(p->t, p->nb, p->grid, p->insts, p->items, p->nitems, p->ops, p->counter, h->stream);
    });
    return e == hipSuccess ? RTRI_OK : hip_fail(h, e);
}

int rtri_batch_plan_chunks(const rtri_batch_plan *p, int64_t *chunks)
{
    if (p == nullptr || chunks == nullptr)
        return -1;
    *chunks = p->nitems;
    return RTRI_OK;
}

int rtri_batch_plan_destroy(rtri_batch_plan *p)
{
    if (p == nullptr)
        return -1;
    if (handle_valid(p->h))
        (void)hipStreamSynchronize(p->h->stream);
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    (void)hipFree(p->dmem);
    delete p;
    return RTRI_OK;
}

int rtri_batched(rtri_handle *h, int dtype, int count, const rtri_batch_entry *entries, int *bad_index)
{
    rtri_batch_plan *p = nullptr;
    int rc = build_plan(h, dtype, count, entries, &p, bad_index, false);
    if (rc != RTRI_OK)
        return rc;
    rc = rtri_batch_plan_run(p);
    hipError_t e = hipStreamSynchronize(h->stream);
    rtri_batch_plan_destroy(p);
    if (rc == RTRI_OK && e != hipSuccess)
        rc = hip_fail(h, e);
    return rc;
}

}  // extern "C"
