// Serving loop: continuous batching of TRSM / TRMM requests on one GPU.
//
// Requests become visible to the scheduler at their scheduled arrival time.
// Each slot (a worker thread with its own stream and handle) loops:
//   1. under the server lock, take work from the head of the arrival queue:
//      - a small FP64 request (factor order <= small_max) opens a batch: the
//        slot keeps taking small FP64 requests from the queue front, up to
//        max_batch, while their memory fits the budget;
//      - any other request (large, or mixed precision) runs alone; with
//        refine_requeue a refined (mixed-precision) solve runs one
//        correction per turn and re-enters the queue after each (its
//        right-hand side and iteration state stay on the device; everything
//        else it reads is the factor object's), so slots serve other
//        requests between its corrections and any slot may run its next one;
//        at most one refined solve per slot is started and unfinished;
//      - with mixed_batch, a small refined request with FP32 updates opens a
//        lockstep batch of such requests (execute_mixed_batch);
//      admission reserves the request's right-hand side and workspace and, for
//      a factor not resident yet, the factor itself; least-recently-used
//      factors nobody is using are evicted when the budget needs room.  A new
//      synthetic factor is allocated and generated on the admitting slot's
//      stream right away, and an event marks it ready for any other slot.
//   2. without the lock: wait for the factors' events, generate the
//      right-hand sides, run one batched launch (or, through the cached
//      factor's factor object, the single-call recursion or the
//      mixed-precision refined solve), copy requested results to the host,
//      wait for the stream.  A factor object keeps what the solves against its
//      factor share (packed diagonal blocks, the refined solve's GEMM-type copy
//      and |op(A)|), so only the first request on a factor makes them; it is
//      counted in the factor's memory and freed when the factor is evicted.
//   3. under the lock: release the reservations, record the completions.
// Several slots run at once, so requests arriving while others run are
// admitted as slots and memory free up, and their work overlaps on the device.
// Per request the arithmetic is the same alone or in any batch (the batched
// kernel reproduces the single-call path bit for bit).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "handle.h"

using namespace rtri;

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    uint64_t ticket;
    rtri_request r;
    int64_t ka;
    size_t rhs_bytes, ws_bytes;
    bool small;
    // a refined solve run in phases: one correction per turn, re-queued between
    bool refine = false;
    bool mixed_batch = false;   // a small refined solve with FP32 updates, run in a lockstep batch
    size_t state_bytes = 0;     // its iteration state (refine_state_bytes) and the padding before it
    int owner = -1;             // slot whose pool holds its buffers (set by the first turn)
    double *rhs = nullptr;      // right-hand side, then the solution, on the device
    void *state = nullptr;
    RefineState st;
    rtri_refine_info info{};
    double t_start = 0.0, t_requeue = 0.0;
};

// how far past the queue head a lockstep batch of small refined solves looks
// for members, and the largest factor order it takes (a larger problem walked
// by the batched kernel's workgroups holds the whole batch back)
constexpr int MIX_WINDOW = 512;
constexpr int64_t MIX_MAX_ORDER = 256;

// a refined solve's state follows its right-hand side in one block
size_t rhs_span(const Req &q)
{
    return (q.rhs_bytes + 255) & ~(size_t)255;
}

struct Factor {
    double *ptr = nullptr;
    int64_t ka = 0, lda = 0;
    int uplo = 0;
    size_t bytes = 0;
    int refs = 0;
    uint64_t last_use = 0;
    bool registered = false;
    int owner = -1;               // slot whose pool and stream hold a synthetic factor
    hipEvent_t ready = nullptr;   // recorded after generation (synthetic factors)
    rtri_factor *fo[2] = {nullptr, nullptr};   // factor objects on ptr, per diag (made at first admission)
    size_t part_bytes = 0;        // device memory the factor objects hold (counted in used)
};

struct Work {
    std::vector<Req> reqs;
    bool batched = false;
    bool mixed = false;       // a lockstep batch of small refined solves (batched is set too)
    bool cont = false;        // a later turn of a refined solve (admitted by its first)
    bool finished = true;     // a refined solve's turn completed it
    size_t ws_extra = 0;      // device memory reserved for the slot's workspace growth
    size_t part_extra = 0;    // reserved for parts a factor object may make (work run alone)
    size_t tables = 0;        // upper bound of the batch tables (batched work)
};

}  // namespace

struct rtri_server {
    rtri_server_cfg cfg;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> pending;
    std::deque<Req> cont;   // refined solves between corrections, in re-queue order
    int refining = 0;       // refined solves started and not finished (at most one per slot)
    std::unordered_map<uint64_t, Factor> factors;
    std::vector<rtri_completion> done;
    int64_t used = 0;       // held + reserved: what admission checks against the budget
    int64_t reserved = 0;   // reservations of work not yet done (workspace growth, factor-object parts)
    uint64_t next_ticket = 1, use_clock = 0;
    int64_t outstanding = 0;
    rtri_server_counters st{};
    bool stopping = false;
    Clock::time_point t0;
    struct Slot {
        std::thread th;
        int idx = 0;
        hipStream_t stream = nullptr;
        // Every device allocation of the slot (synthetic factors, right-hand
        // sides) comes from its own pool and is freed on its own stream, so
        // freed memory is only ever reused in that stream's order: no reuse
        // across the slots' streams, whatever the runtime would allow.
        hipMemPool_t pool = nullptr;
        rtri_handle *h = nullptr;
        BatchScratch sc;
        BatchScratch sc2;     // a lockstep refinement round's second batched launch (the residual products)
        size_t ws_held = 0;   // workspace the slot's handle keeps allocated (counted in used)
    };
    std::vector<Slot> slots;
};

namespace {

double now_s(const rtri_server *s) { return std::chrono::duration<double>(Clock::now() - s->t0).count(); }

size_t handle_ws_bytes(const rtri_handle *h)
{
    size_t b = 0;
    for (int i = 0; i < WS_COUNT; ++i)
        b += h->ws_bytes[i];
    return b;
}

constexpr size_t WS_MIN = (size_t)1 << 16;   // smallest workspace block a handle allocates

// upper bound of the workspace any handle may need for request r, whatever
// its leaf size (the largest packed form is the 256-row one)
size_t ws_bound(const rtri_request &r, int64_t ka, bool state_in_ws)
{
    const size_t mn = (size_t)r.m * (size_t)r.n;
    const size_t pack = (size_t)((ka + 255) / 256 + 1) * (size_t)pack_elems(256) + (size_t)ka * 136;
    // a TRMM (and the residual product of a mixed solve) may save its panel (mn * 8)
    const size_t split = may_split(ka) ? SPLIT_WS_BYTES : 0;
    if (r.precision == RTRI_PREC_F64)
        return 8 * pack + WS_MIN + (r.op == 1 ? mn * 8 + WS_MIN : 0) + split;
    // the iteration state: in the handle's workspace when the solve runs in one
    // turn, else the request's own (Req::state_bytes)
    const size_t state = state_in_ws ? refine_state_bytes(r.m, r.n) : 0;
    return (size_t)ka * (size_t)ws_ld(ka) * 4 + mn * 8 + 12 * pack + 10 * WS_MIN + split + state;
}

// device memory the slot's handle allocates to run q alone: for every
// workspace slot the request uses, what ensure_ws() would add
size_t alone_growth(const rtri_handle *h, const Req &q)
{
    const rtri_request &r = q.r;
    const int64_t nvec = r.side == RTRI_LEFT ? r.n : r.m;
    size_t need[WS_COUNT] = {};
    auto pack_bytes = [&](DType t, bool solve) {
        const int leaf = pick_leaf(h, t, solve, q.ka, nvec);
        return (size_t)((q.ka + leaf - 1) / leaf) * (size_t)pack_elems(leaf) * (t == DType::F64 ? 8 : 4);
    };
    // the panel copy of a TRMM that runs all its leaves in one launch
    auto save_bytes = [&] {
        const int leaf = pick_leaf(h, DType::F64, false, q.ka, nvec);
        return trmm_one_launch(h, leaf, q.ka, nvec) ? (size_t)r.m * (size_t)r.n * 8 : (size_t)0;
    };
    // split-K partials (an upper bound: allocated once some update of the plan splits)
    if (may_split(q.ka))
        need[WS_SPLIT] = SPLIT_WS_BYTES;
    // (the packed blocks and the refined solve's copy of A belong to the
    // factor object: part_growth below)
    (void)pack_bytes;
    if (r.precision == RTRI_PREC_F64) {
        if (r.op == 1)
            need[WS_SAVE] = save_bytes();
    } else {
        // the norm's scalars and the residual product's panel copy are the
        // handle's; so is the iteration state of a solve run in one turn (a
        // re-queued one holds its own: Req::state_bytes)
        need[WS_SCALARS] = 64;
        need[WS_SAVE] = save_bytes();
        if (q.refine && q.state_bytes == 0)
            need[WS_REFINE] = refine_state_bytes(r.m, r.n);
    }
    size_t g = 0;
    for (int i = 0; i < WS_COUNT; ++i)
        if (need[i] > h->ws_bytes[i])
            g += std::max(need[i], WS_MIN) - h->ws_bytes[i];
    return g;
}

// upper bound of the memory a factor object may add running q alone: the
// packed blocks of its plans and, for a refined solve, the GEMM-type copy of A
size_t part_growth(const rtri_handle *h, const Req &q)
{
    const rtri_request &r = q.r;
    const int64_t nvec = r.side == RTRI_LEFT ? r.n : r.m;
    auto pack_bytes = [&](DType t, bool solve) {
        const int leaf = pick_leaf(h, t, solve, q.ka, nvec);
        return (size_t)((q.ka + leaf - 1) / leaf) * (size_t)pack_elems(leaf) * (t == DType::F64 ? 8 : 4) + 256;
    };
    if (r.precision == RTRI_PREC_F64)
        return pack_bytes(DType::F64, r.op == 0);
    return (size_t)q.ka * (size_t)ws_ld(q.ka) * (r.precision == RTRI_PREC_MIXED_BF16 ? 2 : 4) +
           pack_bytes(DType::F32, true) + pack_bytes(DType::F64, false);
}

size_t factor_object_bytes(const Factor &f)
{
    size_t b = 0;
    for (rtri_factor *o : f.fo) {
        int64_t v = 0;
        if (o != nullptr && rtri_factor_bytes(o, &v) == RTRI_OK)
            b += (size_t)v;
    }
    return b;
}

// upper bound of one request's share of the batch tables (instance record,
// 64-vector work items, op list)
size_t batch_entry_bound(const Req &q)
{
    const int64_t nvec = q.r.side == RTRI_LEFT ? q.r.n : q.r.m;
    return 256 + 16 * (size_t)((nvec + 63) / 64) + 64 * (size_t)((q.ka + 31) / 32 + 2);
}

bool evict_one(rtri_server *s, hipStream_t st)
{
    auto victim = s->factors.end();
    for (auto it = s->factors.begin(); it != s->factors.end(); ++it) {
        const Factor &f = it->second;
        if (f.registered || f.refs > 0)
            continue;
        if (victim == s->factors.end() || f.last_use < victim->second.last_use)
            victim = it;
    }
    if (victim == s->factors.end())
        return false;
    Factor &f = victim->second;
    // no request uses it and every earlier user has completed on the host
    // side; the memory goes back to its owner's pool in the owner's stream order
    (void)st;
    for (rtri_factor *&o : f.fo)
        if (o != nullptr) {
            (void)rtri_factor_destroy(o);   // its parts go back to the pools of the slots that made them
            o = nullptr;
        }
    (void)hipFreeAsync(f.ptr, s->slots[f.owner].stream);
    if (f.ready != nullptr)
        (void)hipEventDestroy(f.ready);
    s->used -= (int64_t)(f.bytes + f.part_bytes);
    s->factors.erase(victim);
    s->st.evictions += 1;
    return true;
}

void complete_now(rtri_server *s, const Req &q, int status)
{
    rtri_completion c{};
    c.ticket = q.ticket;
    c.status = status;
    c.t_arrival = q.r.t_arrival;
    c.t_start = c.t_done = now_s(s);
    s->done.push_back(c);
    s->st.completed += 1;
    s->st.failed += 1;
    s->outstanding -= 1;
    s->cv.notify_all();   // drain() may be waiting for the last outstanding request
}

// Reserve what request q needs for slot `slot`; creates (and starts generating)
// a missing synthetic factor.  Returns false if it does not fit right now.
bool admit(rtri_server *s, rtri_server::Slot &slot, const Req &q, Work &w, bool batched, bool mixed = false)
{
    auto it = s->factors.find(q.r.factor_id);
    const bool have = it != s->factors.end();
    const size_t fbytes = have ? 0 : (size_t)q.ka * q.ka * 8;
    // workspace growth: exact for the handle, bounded for the batch tables
    // (the batched launch grows its scratch to twice the tables' size)
    size_t ws_extra = 0, tables = w.tables, part_extra = 0;
    if (batched) {
        tables += batch_entry_bound(q) + (w.reqs.empty() ? 1024 : 0);
        size_t grow = 2 * tables > slot.sc.dev_bytes ? 2 * tables - slot.sc.dev_bytes : 0;
        if (mixed) {
            // both launches of a round have their own scratch; the factor
            // object makes the GEMM-type copy and |op(A)| on first use
            grow += 2 * tables > slot.sc2.dev_bytes ? 2 * tables - slot.sc2.dev_bytes : 0;
            part_extra = part_growth(slot.h, q);
        }
        ws_extra = grow > w.ws_extra ? grow - w.ws_extra : 0;
    } else {
        ws_extra = alone_growth(slot.h, q);
        part_extra = part_growth(slot.h, q);
    }
    const int64_t need = (int64_t)(fbytes + q.rhs_bytes + q.state_bytes + ws_extra + part_extra);
    while (s->used + need > s->cfg.hbm_budget)
        if (!evict_one(s, slot.stream))
            return false;
    Factor *f;
    if (!have) {
        Factor nf;
        nf.ka = q.ka;
        nf.lda = q.ka;
        nf.uplo = q.r.uplo;
        nf.bytes = fbytes;
        nf.owner = slot.idx;
        hipError_t e = hipMallocFromPoolAsync((void **)&nf.ptr, fbytes, slot.pool, slot.stream);
        if (e == hipSuccess) {
            const int kind = q.r.uplo == RTRI_LOWER ? 1 : 2;
            int rc = rtri_synth_fill(slot.h, RTRI_F64, kind, s->cfg.synth_seed, 1u, q.r.factor_id, q.ka, q.ka,
                                     (double)q.ka, nf.ptr, q.ka);
            e = rc == RTRI_OK ? hipSuccess : hipErrorUnknown;
        }
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&nf.ready, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventRecord(nf.ready, slot.stream);
        if (e != hipSuccess)
            return false;
        it = s->factors.emplace(q.r.factor_id, nf).first;
        s->st.factor_misses += 1;
        s->used += (int64_t)fbytes;
    } else {
        s->st.factor_hits += 1;
    }
    f = &it->second;
    if ((!batched || mixed) && f->fo[q.r.diag] == nullptr) {
        // no device work: the object reads the factor in place
        if (rtri_factor_create(slot.h, f->uplo, q.r.diag, f->ka, RTRI_F64, f->ptr, f->lda, 0, &f->fo[q.r.diag]) !=
            RTRI_OK) {
            f->fo[q.r.diag] = nullptr;
            return false;
        }
    }
    f->refs += 1;
    f->last_use = ++s->use_clock;
    s->used += (int64_t)(q.rhs_bytes + q.state_bytes + ws_extra + part_extra);
    s->reserved += (int64_t)(ws_extra + part_extra);
    w.ws_extra += ws_extra;
    w.part_extra += part_extra;
    w.tables = tables;
    s->st.hbm_in_use = s->used - s->reserved;
    s->st.hbm_peak = std::max(s->st.hbm_peak, s->st.hbm_in_use);
    w.reqs.push_back(q);
    return true;
}

// a factor id already in the cache must describe the same factor
bool consistent(rtri_server *s, const Req &q)
{
    auto it = s->factors.find(q.r.factor_id);
    return it == s->factors.end() || (it->second.ka == q.ka && it->second.uplo == q.r.uplo);
}

// the next turn of the refined solve re-queued first, if any (any slot may
// run it: the previous turn ended with its stream synchronised)
static bool take_cont(rtri_server *s, Work &w)
{
    if (s->cont.empty())
        return false;
    w.reqs.push_back(s->cont.front());
    w.cont = true;
    s->cont.pop_front();
    return true;
}

// called with the lock held; fills w (possibly empty).  A refined solve's next
// turn goes before the pending head if it was re-queued before that arrived
// (arrival order), and whenever the head cannot be admitted now.
void take_work(rtri_server *s, rtri_server::Slot &slot, Work &w)
{
    const double t = now_s(s);
    if (!s->cont.empty() && (s->pending.empty() || s->pending.front().r.t_arrival > t ||
                             s->cont.front().t_requeue <= s->pending.front().r.t_arrival)) {
        take_cont(s, w);
        return;
    }
    while (!s->pending.empty() && s->pending.front().r.t_arrival <= t) {
        Req &head = s->pending.front();
        if (!consistent(s, head)) {
            complete_now(s, head, RTRI_ERR_INVALID);
            s->pending.pop_front();
            continue;
        }
        if ((int64_t)(head.ka * head.ka * 8 + head.rhs_bytes + head.state_bytes + head.ws_bytes) > s->cfg.hbm_budget) {
            complete_now(s, head, RTRI_ERR_NOMEM);
            s->pending.pop_front();
            continue;
        }
        break;
    }
    if (s->pending.empty() || s->pending.front().r.t_arrival > t) {
        take_cont(s, w);
        return;
    }
    const Req head = s->pending.front();
    // a lockstep batch pays only with company: another arrived request of its
    // kind among the next MIX_WINDOW; else the head runs alone (its state in
    // its own block, as with refine_requeue)
    bool mb = false;
    if (head.mixed_batch) {
        int seen = 0;
        for (auto it = std::next(s->pending.begin()); it != s->pending.end() && seen < MIX_WINDOW; ++it, ++seen) {
            if (it->r.t_arrival > t)
                break;
            if (it->mixed_batch && consistent(s, *it)) {
                mb = true;
                break;
            }
        }
    }
    if (head.refine && !mb && s->refining >= (int)s->slots.size()) {
        take_cont(s, w);   // finish a started refinement before starting another
        return;
    }
    if (!admit(s, slot, head, w, head.small || mb, mb)) {
        take_cont(s, w);
        return;
    }
    s->pending.pop_front();
    if (head.refine && !mb)
        s->refining += 1;
    if (!head.small && !mb)
        return;
    w.batched = true;
    w.mixed = mb;
    if (mb) {
        // the arrived requests of its kind among the next MIX_WINDOW join it,
        // in arrival order, ahead of the others in between
        int seen = 0;
        for (auto it = s->pending.begin();
             it != s->pending.end() && seen < MIX_WINDOW && (int)w.reqs.size() < s->cfg.max_batch; ++seen) {
            if (it->r.t_arrival > t)
                break;
            if (!it->mixed_batch || !consistent(s, *it)) {
                ++it;
                continue;
            }
            if (!admit(s, slot, *it, w, true, true))
                break;
            it = s->pending.erase(it);
        }
        return;
    }
    // continuous batching: more small FP64 requests that have arrived, in order
    while ((int)w.reqs.size() < s->cfg.max_batch && !s->pending.empty()) {
        const Req &q = s->pending.front();
        if (q.r.t_arrival > t || !q.small || !consistent(s, q))
            break;
        if (!admit(s, slot, q, w, true))
            break;
        s->pending.pop_front();
    }
}

void execute(rtri_server *s, rtri_server::Slot &slot, Work &w, std::vector<rtri_completion> &out)
{
    rtri_handle *h = slot.h;
    hipStream_t st = slot.stream;
    const double t_start = now_s(s);
    std::vector<double *> rhs(w.reqs.size(), nullptr);
    std::vector<const Factor *> fac(w.reqs.size(), nullptr);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (size_t i = 0; i < w.reqs.size(); ++i)
            fac[i] = &s->factors.at(w.reqs[i].r.factor_id);   // pinned by refs: the entry stays
    }
    std::vector<int> status(w.reqs.size(), RTRI_OK);
    std::vector<rtri_refine_info> info(w.reqs.size());
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < w.reqs.size() && e == hipSuccess; ++i) {
        const rtri_request &r = w.reqs[i].r;
        if (fac[i]->ready != nullptr)
            e = hipStreamWaitEvent(st, fac[i]->ready, 0);
        if (e == hipSuccess)
            e = hipMallocFromPoolAsync((void **)&rhs[i], w.reqs[i].rhs_bytes, slot.pool, st);
        if (e == hipSuccess && rtri_synth_fill(h, RTRI_F64, 0, s->cfg.synth_seed, 2u, r.rhs_id, r.m, r.n, 0.0, rhs[i],
                                               r.m) != RTRI_OK)
            e = hipErrorUnknown;
    }
    if (e == hipSuccess) {
        if (w.batched) {
            std::vector<rtri_batch_entry> be(w.reqs.size());
            for (size_t i = 0; i < w.reqs.size(); ++i) {
                const rtri_request &r = w.reqs[i].r;
                be[i] = rtri_batch_entry{r.op, r.side, r.uplo, r.trans, r.diag, r.m, r.n, r.alpha, fac[i]->ptr,
                                         fac[i]->lda, rhs[i], r.m};
            }
            int bad = -1;
            const int rc = batch_run_async(h, RTRI_F64, (int)be.size(), be.data(), slot.sc, &bad, nullptr);
            for (auto &x : status)
                x = rc;
        } else {
            const rtri_request &r = w.reqs[0].r;
            rtri_factor *fo = fac[0]->fo[r.diag];
            int rc;
            if (r.op == 1)
                rc = r.precision == RTRI_PREC_F64 ? rtri_factor_trmm(h, fo, r.side, r.trans, r.m, r.n, r.alpha, rhs[0], r.m)
                                                  : RTRI_ERR_UNSUPPORTED;
            else
                rc = rtri_factor_trsm(h, fo, r.side, r.trans, r.m, r.n, r.alpha, rhs[0], r.m, r.precision, 1e-12, 30,
                                      &info[0]);
            status[0] = rc;
        }
        for (size_t i = 0; i < w.reqs.size() && e == hipSuccess; ++i)
            if (w.reqs[i].r.result != nullptr && status[i] == RTRI_OK)
                e = hipMemcpyAsync(w.reqs[i].r.result, rhs[i], w.reqs[i].rhs_bytes, hipMemcpyDeviceToHost, st);
    }
    for (size_t i = 0; i < w.reqs.size(); ++i)
        if (rhs[i] != nullptr)
            (void)hipFreeAsync(rhs[i], st);
    const hipError_t se = hipStreamSynchronize(st);
    if (e == hipSuccess)
        e = se;
    const double t_done = now_s(s);
    for (size_t i = 0; i < w.reqs.size(); ++i) {
        rtri_completion c{};
        c.ticket = w.reqs[i].ticket;
        c.status = e != hipSuccess ? RTRI_ERR_HIP : status[i];
        c.batched = w.batched ? 1 : 0;
        c.iters = info[i].iters;
        c.eta = info[i].eta;
        c.t_arrival = w.reqs[i].r.t_arrival;
        c.t_start = t_start;
        c.t_done = t_done;
        out.push_back(c);
    }
}

// One turn of a refined solve: the first allocates its right-hand side
// from the slot's pool in its stream order (that slot is the owner), with
// refine_requeue the state in the same block (else it is the handle's
// workspace), generates the right-hand side and runs refine_begin; a turn
// then runs corrections to the end, or one with refine_requeue (each ends
// with a stream synchronisation, for the two scalars it reads back, so the
// next turn may run on any slot's stream).  When the refinement is done: X
// into the right-hand side, the result to the host, a synchronisation, then
// the block freed in the owner's stream order; the completion is recorded
// (w.finished).
void execute_refine(rtri_server *s, rtri_server::Slot &slot, Work &w, std::vector<rtri_completion> &out)
{
    rtri_handle *h = slot.h;
    hipStream_t st = slot.stream;
    Req &q = w.reqs[0];
    const rtri_request &r = q.r;
    constexpr double tol = 1e-12;
    constexpr int max_iter = 30;
    const Factor *fac;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        fac = &s->factors.at(r.factor_id);   // pinned by refs until the request completes
    }
    rtri_factor *fo = fac->fo[r.diag];
    hipError_t e = hipSuccess;
    int rc = RTRI_OK;
    if (!w.cont) {
        q.owner = slot.idx;
        q.t_start = now_s(s);
        if (fac->ready != nullptr)
            e = hipStreamWaitEvent(st, fac->ready, 0);
        const bool own = q.state_bytes != 0;
        if (e == hipSuccess)
            e = hipMallocFromPoolAsync((void **)&q.rhs, own ? rhs_span(q) + q.state_bytes : q.rhs_bytes, slot.pool,
                                       st);
        if (e == hipSuccess && !own)
            e = ensure_ws(h, WS_REFINE, refine_state_bytes(r.m, r.n));
        if (e == hipSuccess)
            q.state = own ? reinterpret_cast<char *>(q.rhs) + rhs_span(q) : h->ws[WS_REFINE];
        if (e == hipSuccess && rtri_synth_fill(h, RTRI_F64, 0, s->cfg.synth_seed, 2u, r.rhs_id, r.m, r.n, 0.0, q.rhs,
                                               r.m) != RTRI_OK)
            e = hipErrorUnknown;
        if (e == hipSuccess) {
            refine_state_place(q.st, q.state, r.m, r.n);
            rc = factor_refine_begin(h, fo, r.side, r.trans, r.m, r.n, r.alpha, q.rhs, r.m, r.precision, tol, max_iter,
                                     &q.info, q.st);
        }
    }
    while (e == hipSuccess && rc == RTRI_OK && !q.st.done) {
        rc = factor_refine_step(h, fo, r.side, r.trans, r.m, r.n, r.precision, tol, max_iter, &q.info, q.st);
        if (s->cfg.refine_requeue)
            break;
    }
    w.finished = e != hipSuccess || rc != RTRI_OK || q.st.done;
    if (!w.finished) {
        q.t_requeue = now_s(s);
        return;
    }
    if (e == hipSuccess && rc == RTRI_OK) {
        rc = refine_end(h, r.m, r.n, q.rhs, r.m, &q.info, q.st);
        if (r.result != nullptr && rc == RTRI_OK)
            e = hipMemcpyAsync(r.result, q.rhs, q.rhs_bytes, hipMemcpyDeviceToHost, st);
    }
    const hipError_t se = hipStreamSynchronize(st);
    if (e == hipSuccess)
        e = se;
    // nothing reads it any more: back to the owner's pool
    hipStream_t ost = q.owner >= 0 ? s->slots[q.owner].stream : st;
    if (q.rhs != nullptr)
        (void)hipFreeAsync(q.rhs, ost);
    q.rhs = nullptr;
    q.state = nullptr;
    rtri_completion c{};
    c.ticket = q.ticket;
    c.status = e != hipSuccess ? RTRI_ERR_HIP : rc;
    c.iters = q.info.iters;
    c.eta = q.info.eta;
    c.t_arrival = r.t_arrival;
    c.t_start = q.t_start;
    c.t_done = now_s(s);
    out.push_back(c);
}

// A lockstep batch of small refined solves with FP32 updates: each round of
// corrections is folded into two batched launches, the FP32 solves of every
// member still refining (against the factor objects' FP32 copies of A) and
// their FP64 residual products (against the FP64 factors); the element-wise
// phases run per member on the slot's stream, and one synchronisation per
// round reads every member's scalars.  A member's arithmetic is the batched
// kernel's: it meets the refined solve's tolerance, but is not bitwise the
// refined solve run alone.
void execute_mixed_batch(rtri_server *s, rtri_server::Slot &slot, Work &w, std::vector<rtri_completion> &out)
{
    rtri_handle *h = slot.h;
    hipStream_t st = slot.stream;
    const double t_start = now_s(s);
    constexpr double tol = 1e-12;
    constexpr int max_iter = 30;
    const size_t k = w.reqs.size();
    std::vector<const Factor *> fac(k, nullptr);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (size_t i = 0; i < k; ++i)
            fac[i] = &s->factors.at(w.reqs[i].r.factor_id);   // pinned by refs: the entry stays
    }
    auto trans_of = [](const rtri_request &r) { return r.trans == RTRI_CONJTRANS ? RTRI_TRANS : r.trans; };
    std::vector<MixedPrep> prep(k);
    std::vector<int> status(k, RTRI_OK);
    std::vector<unsigned long long> host(4 * k, 0);
    hipError_t e = hipSuccess;
    // each member: its block (right-hand side, then state), the right-hand
    // side, the factor object's parts, alpha B and max |alpha B|
    for (size_t i = 0; i < k && e == hipSuccess; ++i) {
        Req &q = w.reqs[i];
        const rtri_request &r = q.r;
        q.owner = slot.idx;
        if (fac[i]->ready != nullptr)
            e = hipStreamWaitEvent(st, fac[i]->ready, 0);
        if (e == hipSuccess)
            e = hipMallocFromPoolAsync((void **)&q.rhs, rhs_span(q) + q.state_bytes, slot.pool, st);
        if (e != hipSuccess)
            break;
        q.state = reinterpret_cast<char *>(q.rhs) + rhs_span(q);
        refine_state_place(q.st, q.state, r.m, r.n);
        if (rtri_synth_fill(h, RTRI_F64, 0, s->cfg.synth_seed, 2u, r.rhs_id, r.m, r.n, 0.0, q.rhs, r.m) != RTRI_OK) {
            e = hipErrorUnknown;
            break;
        }
        status[i] = factor_refine_prep(h, fac[i]->fo[r.diag], r.side, r.trans, r.m, r.n, r.precision, prep[i]);
        if (status[i] != RTRI_OK)
            continue;
        e = refine_begin_enqueue(h, r.side, r.uplo, trans_of(r), r.diag, r.m, r.n, r.alpha, fac[i]->ptr,
                                 fac[i]->lda, q.rhs, r.m, prep[i], q.st, &host[4 * i]);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e == hipSuccess)
        for (size_t i = 0; i < k; ++i)
            if (status[i] == RTRI_OK)
                refine_begin_finish(&host[4 * i], tol, max_iter, &w.reqs[i].info, prep[i], w.reqs[i].st);
    // rounds of corrections over the members still refining
    std::vector<size_t> act;
    std::vector<rtri_batch_entry> be;
    while (e == hipSuccess) {
        act.clear();
        for (size_t i = 0; i < k; ++i)
            if (status[i] == RTRI_OK && !w.reqs[i].st.done)
                act.push_back(i);
        if (act.empty())
            break;
        for (size_t x = 0; x < act.size() && e == hipSuccess; ++x)
            e = refine_step_convert(h, w.reqs[act[x]].r.m, w.reqs[act[x]].r.n, w.reqs[act[x]].st);
        // op(A32) D = R / s for every member: one batched FP32 launch
        be.clear();
        for (size_t i : act) {
            const Req &q = w.reqs[i];
            const rtri_request &r = q.r;
            be.push_back(rtri_batch_entry{0, r.side, r.uplo, trans_of(r), r.diag, r.m, r.n, 1.0, prep[i].Acopy,
                                          prep[i].ldag, q.st.D, q.st.ld});
        }
        int bad = -1;
        int rc = e == hipSuccess ? batch_run_async(h, RTRI_F32, (int)be.size(), be.data(), slot.sc, &bad, nullptr)
                                 : RTRI_OK;
        for (size_t x = 0; x < act.size() && e == hipSuccess && rc == RTRI_OK; ++x)
            e = refine_step_update(h, w.reqs[act[x]].r.m, w.reqs[act[x]].r.n, w.reqs[act[x]].st);
        // W := op(A) W in FP64 for every member: one batched launch
        be.clear();
        for (size_t i : act) {
            const Req &q = w.reqs[i];
            const rtri_request &r = q.r;
            be.push_back(rtri_batch_entry{1, r.side, r.uplo, trans_of(r), r.diag, r.m, r.n, 1.0, fac[i]->ptr,
                                          fac[i]->lda, q.st.W, q.st.ld});
        }
        if (e == hipSuccess && rc == RTRI_OK)
            rc = batch_run_async(h, RTRI_F64, (int)be.size(), be.data(), slot.sc2, &bad, nullptr);
        for (size_t x = 0; x < act.size() && e == hipSuccess && rc == RTRI_OK; ++x) {
            const size_t i = act[x];
            e = refine_step_resid(h, w.reqs[i].r.side, w.reqs[i].r.m, w.reqs[i].r.n, w.reqs[i].st, &host[4 * i]);
        }
        const hipError_t se = hipStreamSynchronize(st);   // also before the staging is reused
        if (e == hipSuccess)
            e = se;
        if (rc != RTRI_OK) {
            for (size_t i : act)
                status[i] = rc;
            break;
        }
        if (e == hipSuccess)
            for (size_t i : act)
                refine_step_finish(&host[4 * i], tol, max_iter, &w.reqs[i].info, w.reqs[i].st);
    }
    // X into the right-hand side, the results to the host
    for (size_t i = 0; i < k && e == hipSuccess; ++i) {
        Req &q = w.reqs[i];
        if (status[i] != RTRI_OK)
            continue;
        status[i] = refine_end(h, q.r.m, q.r.n, q.rhs, q.r.m, &q.info, q.st);
        if (q.r.result != nullptr && status[i] == RTRI_OK)
            e = hipMemcpyAsync(q.r.result, q.rhs, q.rhs_bytes, hipMemcpyDeviceToHost, st);
    }
    for (Req &q : w.reqs)
        if (q.rhs != nullptr) {
            (void)hipFreeAsync(q.rhs, st);
            q.rhs = nullptr;
            q.state = nullptr;
        }
    const hipError_t se = hipStreamSynchronize(st);
    if (e == hipSuccess)
        e = se;
    const double t_done = now_s(s);
    for (size_t i = 0; i < k; ++i) {
        const Req &q = w.reqs[i];
        rtri_completion c{};
        c.ticket = q.ticket;
        c.status = e != hipSuccess ? RTRI_ERR_HIP : status[i];
        c.batched = 1;
        c.iters = q.info.iters;
        c.eta = q.info.eta;
        c.t_arrival = q.r.t_arrival;
        c.t_start = t_start;
        c.t_done = t_done;
        out.push_back(c);
    }
}

void worker(rtri_server *s, int idx)
{
    rtri_server::Slot &slot = s->slots[idx];
    (void)hipSetDevice(s->device);
    std::vector<rtri_completion> out;
    for (;;) {
        Work w;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (s->stopping && s->pending.empty() && s->cont.empty())
                    return;
                take_work(s, slot, w);
                if (!w.reqs.empty())
                    break;
                if (!s->pending.empty() || !s->cont.empty()) {
                    const double wait = s->pending.empty() ? 0.0 : s->pending.front().r.t_arrival - now_s(s);
                    // not yet arrived, or waiting for memory: wake at the arrival or on any release
                    s->cv.wait_for(lk, std::chrono::duration<double>(wait > 0 ? std::min(wait, 0.01) : 0.001));
                } else {
                    s->cv.wait(lk);
                }
            }
        }
        out.clear();
        if (w.mixed)
            execute_mixed_batch(s, slot, w, out);
        else if (!w.batched && w.reqs[0].refine)
            execute_refine(s, slot, w, out);
        else
            execute(s, slot, w, out);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (size_t i = 0; i < w.reqs.size() && w.finished; ++i) {
                const Req &q = w.reqs[i];
                Factor &f = s->factors.at(q.r.factor_id);
                f.refs -= 1;
                s->used -= (int64_t)(q.rhs_bytes + q.state_bytes);
                const int64_t vecs = q.r.side == RTRI_LEFT ? q.r.n : q.r.m;
                if (out[i].status == RTRI_OK)
                    s->st.useful_flops += (double)q.ka * q.ka * (double)vecs;
                else
                    s->st.failed += 1;
            }
            // the slot keeps its largest workspace and batch scratch: count what it holds now
            const size_t held = handle_ws_bytes(slot.h) + slot.sc.dev_bytes + slot.sc2.dev_bytes;
            s->used += (int64_t)held - (int64_t)(slot.ws_held + w.ws_extra);
            slot.ws_held = held;
            // parts the factor objects made replace the reservation for them
            if (!w.batched || w.mixed) {
                std::vector<uint64_t> ids;
                for (const Req &q : w.reqs)
                    if (std::find(ids.begin(), ids.end(), q.r.factor_id) == ids.end())
                        ids.push_back(q.r.factor_id);
                for (uint64_t id : ids) {
                    Factor &f = s->factors.at(id);
                    const size_t now = factor_object_bytes(f);
                    s->used += (int64_t)now - (int64_t)f.part_bytes;
                    f.part_bytes = now;
                }
                s->used -= (int64_t)w.part_extra;
            }
            if (w.finished)
                s->st.completed += (int64_t)w.reqs.size();
            else
                s->cont.push_back(w.reqs[0]);   // its next correction, in re-queue order
            s->st.launches += 1;
            if (!w.batched && w.reqs[0].refine) {
                s->st.refine_turns += 1;
                if (w.finished)
                    s->refining -= 1;
            }
            if (w.batched) {
                s->st.batched_launches += 1;
                s->st.batched_requests += (int64_t)w.reqs.size();
            }
            s->reserved -= (int64_t)(w.ws_extra + w.part_extra);
            s->st.hbm_in_use = s->used - s->reserved;
            s->st.hbm_peak = std::max(s->st.hbm_peak, s->st.hbm_in_use);
            s->done.insert(s->done.end(), out.begin(), out.end());
            if (w.finished)
                s->outstanding -= (int64_t)w.reqs.size();
        }
        s->cv.notify_all();
    }
}

}  // namespace

extern "C" {

int rtri_server_create(const rtri_server_cfg *cfg, rtri_server **out)
{
    if (cfg == nullptr || out == nullptr)
        return -1;
    if (cfg->slots < 1 || cfg->slots > 16)
        return -2;
    if (cfg->hbm_budget <= 0)
        return -3;
    if (cfg->max_batch < 1)
        return -4;
    rtri_server *s = new (std::nothrow) rtri_server();
    if (s == nullptr)
        return RTRI_ERR_NOMEM;
    s->cfg = *cfg;
    s->t0 = Clock::now();
    hipError_t e = hipGetDevice(&s->device);
    s->slots.resize(cfg->slots);
    for (int i = 0; i < cfg->slots; ++i) {
        auto &sl = s->slots[i];
        sl.idx = i;
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess && rtri_create(&sl.h, sl.stream) != RTRI_OK)
            e = hipErrorOutOfMemory;
        if (e == hipSuccess) {
            hipMemPoolProps props{};
            props.allocType = hipMemAllocationTypePinned;
            props.handleTypes = hipMemHandleTypeNone;
            props.location.type = hipMemLocationTypeDevice;
            props.location.id = s->device;
            e = hipMemPoolCreate(&sl.pool, &props);
        }
        int off = 0;
        if (e == hipSuccess)
            e = hipMemPoolSetAttribute(sl.pool, hipMemPoolReuseAllowOpportunistic, &off);
        if (e == hipSuccess)
            e = hipMemPoolSetAttribute(sl.pool, hipMemPoolReuseAllowInternalDependencies, &off);
        if (e == hipSuccess)
            sl.h->mem_pool = sl.pool;   // factor objects' parts made by this slot come from its pool
    }
    if (e != hipSuccess) {
        for (auto &sl : s->slots) {
            if (sl.h)
                rtri_destroy(sl.h);
            if (sl.pool)
                (void)hipMemPoolDestroy(sl.pool);
            if (sl.stream)
                (void)hipStreamDestroy(sl.stream);
        }
        delete s;
        return RTRI_ERR_HIP;
    }
    for (int i = 0; i < cfg->slots; ++i)
        s->slots[i].th = std::thread(worker, s, i);
    *out = s;
    return RTRI_OK;
}

int rtri_server_register_factor(rtri_server *s, uint64_t id, int64_t ka, int uplo, const double *A, int64_t lda)
{
    if (s == nullptr)
        return -1;
    if (ka < 0)
        return -3;
    if (uplo != RTRI_LOWER && uplo != RTRI_UPPER)
        return -4;
    if (A == nullptr && ka > 0)
        return -5;
    if (lda < std::max<int64_t>(1, ka))
        return -6;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->factors.count(id))
        return RTRI_ERR_INVALID;
    Factor f;
    f.ptr = const_cast<double *>(A);
    f.ka = ka;
    f.lda = lda;
    f.uplo = uplo;
    f.registered = true;
    s->factors.emplace(id, f);
    return RTRI_OK;
}

int rtri_server_submit(rtri_server *s, const rtri_request *r, uint64_t *ticket)
{
    if (s == nullptr || r == nullptr)
        return -1;
    int rc = (r->op == 0 || r->op == 1) ? check_args(r->side, r->uplo, r->trans, r->diag, r->m, r->n,
                                                     (const void *)1, r->side == RTRI_LEFT ? r->m : r->n,
                                                     (const void *)1, std::max<int64_t>(1, r->m), false)
                                        : -2;
    if (rc != 0)
        return rc;
    if (r->precision < RTRI_PREC_F64 || r->precision > RTRI_PREC_MIXED_F32 || (r->precision != RTRI_PREC_F64 && r->op != 0))
        return RTRI_ERR_UNSUPPORTED;
    Req q;
    q.r = *r;
    q.ka = r->side == RTRI_LEFT ? r->m : r->n;
    q.rhs_bytes = (size_t)std::max<int64_t>(1, r->m * r->n) * 8;
    const bool requeue = s->cfg.refine_requeue != 0;
    q.small = r->precision == RTRI_PREC_F64 && q.ka <= s->cfg.small_max && r->m > 0 && r->n > 0;
    q.refine = r->precision != RTRI_PREC_F64 && r->op == 0 && r->alpha != 0.0 && r->m > 0 && r->n > 0;
    q.mixed_batch = s->cfg.mixed_batch != 0 && q.refine && r->precision == RTRI_PREC_MIXED_F32 &&
                    q.ka <= std::min<int64_t>(s->cfg.small_max, MIX_MAX_ORDER);
    const bool own_state = q.refine && (requeue || q.mixed_batch);
    q.state_bytes = own_state ? refine_state_bytes(r->m, r->n) + (rhs_span(q) - q.rhs_bytes) : 0;
    q.ws_bytes = ws_bound(*r, q.ka, q.refine && !own_state);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        q.ticket = s->next_ticket++;
        if (ticket != nullptr)
            *ticket = q.ticket;
        s->st.submitted += 1;
        s->outstanding += 1;
        if (r->m == 0 || r->n == 0) {
            rtri_completion c{};
            c.ticket = q.ticket;
            c.t_arrival = r->t_arrival;
            c.t_start = c.t_done = now_s(s);
            s->done.push_back(c);
            s->st.completed += 1;
            s->outstanding -= 1;
        } else {
            s->pending.push_back(q);
        }
    }
    s->cv.notify_all();
    return RTRI_OK;
}

int rtri_server_poll(rtri_server *s, rtri_completion *out, int max, int *n)
{
    if (s == nullptr || n == nullptr || (out == nullptr && max > 0))
        return -1;
    std::lock_guard<std::mutex> lk(s->mu);
    const int k = std::min<int>(std::max(0, max), (int)s->done.size());
    for (int i = 0; i < k; ++i)
        out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n = k;
    return RTRI_OK;
}

int rtri_server_drain(rtri_server *s)
{
    if (s == nullptr)
        return -1;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->outstanding == 0; });
    return RTRI_OK;
}

int rtri_server_stats(rtri_server *s, rtri_server_counters *out)
{
    if (s == nullptr || out == nullptr)
        return -1;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return RTRI_OK;
}

double rtri_server_now(rtri_server *s) { return s == nullptr ? 0.0 : now_s(s); }

int rtri_server_destroy(rtri_server *s)
{
    if (s == nullptr)
        return -1;
    rtri_server_drain(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv.notify_all();
    for (auto &sl : s->slots)
        if (sl.th.joinable())
            sl.th.join();
    for (auto &kv : s->factors) {
        for (rtri_factor *o : kv.second.fo)
            if (o != nullptr)
                (void)rtri_factor_destroy(o);
        if (!kv.second.registered && kv.second.ptr != nullptr)
            (void)hipFreeAsync(kv.second.ptr, s->slots[kv.second.owner].stream);
        if (kv.second.ready != nullptr)
            (void)hipEventDestroy(kv.second.ready);
    }
    for (auto &sl : s->slots)
        (void)hipStreamSynchronize(sl.stream);
    for (auto &sl : s->slots) {
        batch_scratch_free(sl.sc);
        batch_scratch_free(sl.sc2);
        rtri_destroy(sl.h);
        (void)hipMemPoolDestroy(sl.pool);
        (void)hipStreamDestroy(sl.stream);
    }
    delete s;
    return RTRI_OK;
}

}  // extern "C"
