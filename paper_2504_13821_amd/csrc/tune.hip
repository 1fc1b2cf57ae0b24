// Tuning: choose the leaf size (the recursion's cut-over, "a chosen
// threshold" in the paper, Sec. 3.1) and the GEMM tile shape by timing real
// shapes on the device, keep the winners as rules in a small JSON database,
// and consult them when a call does not fix the choice itself.
//
// Database (one file per architecture):
//   {"arch": "gfx950", "version": 1,
//    "leaf": [{"dtype": "f64", "op": "trsm", "ka_max": 1024, "n_max": 512, "leaf": 32}, ...],
//    "gemm_tile": [{"dtype": "f64", "m_max": 256, "n_max": 4096, "tile": 2}, ...,
//                  {"dtype": "bf16", "m_max": 2048, "n_max": 4096, "tile": 2}, ...],
//    "batched": [{"dtype": "f64", "leaf": 64}, ...]}
// A leaf rule covers factor orders up to ka_max and vector counts up to n_max
// (the smallest covering bucket wins; beyond the largest, the largest applies).
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

#include "handle.h"

using namespace rtri;

namespace rtri {

struct TuneDB {
    struct Leaf {
        int dtype, solve;
        int64_t ka_max, n_max;
        int leaf;
    };
    struct Tile {
        int dtype;
        int64_t m_max, n_max;
        int tile;
    };
    struct Batch {
        int dtype;
        int leaf;   // 32 or 64: the batched kernel's leaf
    };
    std::vector<Leaf> leaf;
    std::vector<Tile> tile;     // dtype F64 / F32: tiles 1..3; BF16 / F16: 16-bit tiles 1..2
    std::vector<Batch> batch;
};

namespace {

// ---- a minimal JSON reader for the database schema (objects, arrays, strings, numbers) ----
struct JVal {
    enum Kind { NUL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0;
    std::string str;
    std::vector<JVal> arr;
    std::map<std::string, JVal> obj;
};

struct JParser {
    const char *p, *end;
    bool ok = true;
    void ws()
    {
        while (p < end && std::isspace((unsigned char)*p))
            ++p;
    }
    bool eat(char c)
    {
        ws();
        if (p < end && *p == c) {
            ++p;
            return true;
        }
        return false;
    }
    std::string string_lit()
    {
        std::string s;
        if (!eat('"')) {
            ok = false;
            return s;
        }
        while (p < end && *p != '"') {
            if (*p == '\\' && p + 1 < end)
                ++p;
            s.push_back(*p++);
        }
        if (p < end)
            ++p;
        else
            ok = false;
        return s;
    }
    JVal value()
    {
        JVal v;
        ws();
        if (p >= end) {
            ok = false;
            return v;
        }
        if (*p == '{') {
            ++p;
            v.kind = JVal::OBJ;
            if (eat('}'))
                return v;
            do {
                std::string k = string_lit();
                if (!eat(':')) {
                    ok = false;
                    return v;
                }
                v.obj[k] = value();
            } while (ok && eat(','));
            if (!eat('}'))
                ok = false;
        } else if (*p == '[') {
            ++p;
            v.kind = JVal::ARR;
            if (eat(']'))
                return v;
            do {
                v.arr.push_back(value());
            } while (ok && eat(','));
            if (!eat(']'))
                ok = false;
        } else if (*p == '"') {
            v.kind = JVal::STR;
            v.str = string_lit();
        } else {
            char *q = nullptr;
            v.num = std::strtod(p, &q);
            if (q == p)
                ok = false;
            else
                v.kind = JVal::NUM;
            p = q;
        }
        return v;
    }
};

int dtype_of(const std::string &s)
{
    return s == "f64" ? RTRI_F64 : s == "f32" ? RTRI_F32 : s == "bf16" ? RTRI_BF16 : s == "f16" ? RTRI_F16 : -1;
}
const char *dtype_name(int d)
{
    return d == RTRI_F64 ? "f64" : d == RTRI_F32 ? "f32" : d == RTRI_BF16 ? "bf16" : "f16";
}
bool is16(int d) { return d == RTRI_BF16 || d == RTRI_F16; }

double num_of(const JVal &o, const char *k, bool &ok)
{
    auto it = o.obj.find(k);
    if (it == o.obj.end() || it->second.kind != JVal::NUM) {
        ok = false;
        return 0;
    }
    return it->second.num;
}
std::string str_of(const JVal &o, const char *k, bool &ok)
{
    auto it = o.obj.find(k);
    if (it == o.obj.end() || it->second.kind != JVal::STR) {
        ok = false;
        return "";
    }
    return it->second.str;
}

bool parse_db(const std::string &text, TuneDB &db)
{
    JParser jp{text.data(), text.data() + text.size()};
    JVal root = jp.value();
    if (!jp.ok || root.kind != JVal::OBJ)
        return false;
    bool ok = true;
    auto lr = root.obj.find("leaf");
    if (lr != root.obj.end() && lr->second.kind == JVal::ARR)
        for (const JVal &e : lr->second.arr) {
            TuneDB::Leaf r{dtype_of(str_of(e, "dtype", ok)), str_of(e, "op", ok) == "trsm" ? 1 : 0,
                           (int64_t)num_of(e, "ka_max", ok), (int64_t)num_of(e, "n_max", ok),
                           (int)num_of(e, "leaf", ok)};
            if (r.dtype < 0 || is16(r.dtype) || r.leaf == 0 || !valid_leaf(r.leaf))
                ok = false;
            db.leaf.push_back(r);
        }
    auto tr = root.obj.find("gemm_tile");
    if (tr != root.obj.end() && tr->second.kind == JVal::ARR)
        for (const JVal &e : tr->second.arr) {
            TuneDB::Tile r{dtype_of(str_of(e, "dtype", ok)), (int64_t)num_of(e, "m_max", ok),
                           (int64_t)num_of(e, "n_max", ok), (int)num_of(e, "tile", ok)};
            if (r.dtype < 0 || r.tile < 1 || r.tile > (is16(r.dtype) ? 2 : 3))
                ok = false;
            db.tile.push_back(r);
        }
    auto br = root.obj.find("batched");
    if (br != root.obj.end() && br->second.kind == JVal::ARR)
        for (const JVal &e : br->second.arr) {
            TuneDB::Batch r{dtype_of(str_of(e, "dtype", ok)), (int)num_of(e, "leaf", ok)};
            if (r.dtype < 0 || is16(r.dtype) || (r.leaf != 32 && r.leaf != 64))
                ok = false;
            db.batch.push_back(r);
        }
    return ok;
}

bool write_db(const char *path, const TuneDB &db)
{
    FILE *f = std::fopen(path, "w");
    if (f == nullptr)
        return false;
    std::fprintf(f, "{\"arch\": \"gfx950\", \"version\": 1,\n \"leaf\": [");
    for (size_t i = 0; i < db.leaf.size(); ++i) {
        const auto &r = db.leaf[i];
        std::fprintf(f, "%s\n  {\"dtype\": \"%s\", \"op\": \"%s\", \"ka_max\": %lld, \"n_max\": %lld, \"leaf\": %d}",
                     i ? "," : "", dtype_name(r.dtype), r.solve ? "trsm" : "trmm", (long long)r.ka_max,
                     (long long)r.n_max, r.leaf);
    }
    std::fprintf(f, "],\n \"gemm_tile\": [");
    for (size_t i = 0; i < db.tile.size(); ++i) {
        const auto &r = db.tile[i];
        std::fprintf(f, "%s\n  {\"dtype\": \"%s\", \"m_max\": %lld, \"n_max\": %lld, \"tile\": %d}", i ? "," : "",
                     dtype_name(r.dtype), (long long)r.m_max, (long long)r.n_max, r.tile);
    }
    std::fprintf(f, "],\n \"batched\": [");
    for (size_t i = 0; i < db.batch.size(); ++i)
        std::fprintf(f, "%s\n  {\"dtype\": \"%s\", \"leaf\": %d}", i ? "," : "", dtype_name(db.batch[i].dtype),
                     db.batch[i].leaf);
    std::fprintf(f, "]}\n");
    return std::fclose(f) == 0;
}

// the smallest bucket covering x, or the largest if none covers it
template <class R, class Get>
const R *pick_bucket(const std::vector<const R *> &c, int64_t x, Get get)
{
    const R *best = nullptr, *largest = nullptr;
    for (const R *r : c) {
        if (largest == nullptr || get(*r) > get(*largest))
            largest = r;
        if (get(*r) >= x && (best == nullptr || get(*r) < get(*best)))
            best = r;
    }
    return best ? best : largest;
}

}  // namespace

void tune_db_free(TuneDB *db) { delete db; }

int tuned_leaf(const TuneDB *db, int dtype, bool solve, int64_t ka, int64_t nvec)
{
    if (db == nullptr)
        return 0;
    std::vector<const TuneDB::Leaf *> c;
    for (const auto &r : db->leaf)
        if (r.dtype == dtype && r.solve == (solve ? 1 : 0))
            c.push_back(&r);
    if (c.empty())
        return 0;
    const TuneDB::Leaf *k = pick_bucket(c, ka, [](const TuneDB::Leaf &r) { return r.ka_max; });
    std::vector<const TuneDB::Leaf *> c2;
    for (const auto *r : c)
        if (r->ka_max == k->ka_max)
            c2.push_back(r);
    return pick_bucket(c2, nvec, [](const TuneDB::Leaf &r) { return r.n_max; })->leaf;
}

int tuned_tile(const TuneDB *db, int dtype, int64_t M, int64_t N)
{
    if (db == nullptr)
        return 0;
    std::vector<const TuneDB::Tile *> c;
    for (const auto &r : db->tile)
        if (r.dtype == dtype)
            c.push_back(&r);
    if (c.empty())
        return 0;
    const TuneDB::Tile *k = pick_bucket(c, M, [](const TuneDB::Tile &r) { return r.m_max; });
    std::vector<const TuneDB::Tile *> c2;
    for (const auto *r : c)
        if (r->m_max == k->m_max)
            c2.push_back(r);
    return pick_bucket(c2, N, [](const TuneDB::Tile &r) { return r.n_max; })->tile;
}

int tuned_batch_leaf(const TuneDB *db, int dtype)
{
    if (db == nullptr)
        return 0;
    for (const auto &r : db->batch)
        if (r.dtype == dtype)
            return r.leaf;
    return 0;
}

int load_tuning_file(rtri_handle *h, const char *path)
{
    FILE *f = std::fopen(path, "r");
    if (f == nullptr)
        return RTRI_ERR_INVALID;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0)
        text.append(buf, k);
    std::fclose(f);
    TuneDB *db = new (std::nothrow) TuneDB();
    if (db == nullptr)
        return RTRI_ERR_NOMEM;
    if (!parse_db(text, *db)) {
        delete db;
        return RTRI_ERR_INVALID;
    }
    delete h->tune;
    h->tune = db;
    return RTRI_OK;
}

}  // namespace rtri

namespace {

// median of `reps` event-timed runs of f, each after prep (untimed)
template <class Prep, class F>
float time_median(hipStream_t st, int reps, Prep &&prep, F &&f)
{
    std::vector<float> t;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    for (int r = 0; r <= reps; ++r) {
        prep();
        (void)hipEventRecord(a, st);
        f();
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        if (r > 0)   // the first run is a warm-up
            t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

}  // namespace

extern "C" {

int rtri_load_tuning(rtri_handle *h, const char *path)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (path == nullptr)
        return -2;
    return load_tuning_file(h, path);
}

namespace {

// 16-bit GEMM tiles (128x128 / 256x256) per (M = K, N), op(P) = P^T and
// op(Q) = Q: the layout the library's 16-bit copies are made in
int tune16(rtri_handle *h, int dtype, int64_t max_order, TuneDB &db)
{
    const int64_t max_n = std::min<int64_t>(std::max<int64_t>(max_order, 512), 16384);
    const int64_t kmax = std::min<int64_t>(std::max<int64_t>(max_order / 2, 256), 8192);
    void *P = nullptr, *Q = nullptr, *C = nullptr;
    hipError_t e = hipMalloc(&P, (size_t)kmax * kmax * 2);
    if (e == hipSuccess)
        e = hipMalloc(&Q, (size_t)kmax * max_n * 2);
    if (e == hipSuccess)
        e = hipMalloc(&C, (size_t)kmax * max_n * 4);
    // operands' values do not matter for timing: zeros
    if (e == hipSuccess)
        e = hipMemsetAsync(P, 0, (size_t)kmax * kmax * 2, h->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(Q, 0, (size_t)kmax * max_n * 2, h->stream);
    int rc = e == hipSuccess ? RTRI_OK : hip_fail(h, e);
    const int saved = h->gemm16_tile;
    for (int64_t mk = 256; mk <= kmax && rc == RTRI_OK; mk *= 2)
        for (int64_t n : {512, 4096, 16384}) {
            if (n > max_n || rc != RTRI_OK)
                continue;
            int best = 1;
            float best_ms = 1e30f;
            for (int tile : {1, 2}) {
                h->gemm16_tile = tile;
                int rr = RTRI_OK;
                const float ms = time_median(h->stream, 3, [] {}, [&] {
                    rr = rtri_gemm_update(h, dtype, RTRI_TRANS, RTRI_NOTRANS, mk, n, mk, 1.0, P, mk, Q, mk, 0.0, C,
                                          mk);
                });
                if (rr != RTRI_OK) {
                    rc = rr;
                    break;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = tile;
                }
            }
            db.tile.push_back(TuneDB::Tile{dtype, mk, n, best});
        }
    h->gemm16_tile = saved;
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(P);
    (void)hipFree(Q);
    (void)hipFree(C);
    return rc;
}

// the batched kernel's leaf (32 or 64 rows) on a mix like the batched
// workload: 200 problems, orders log-uniform on [16, min(1024, max_order)],
// 1..128 vectors, all on the top-left blocks of one lower factor A (lda lda),
// right-hand sides in disjoint column ranges of B (ldb)
int tune_batched(rtri_handle *h, int dtype, int64_t max_order, void *A, int64_t lda, void *B, int64_t ldb,
                 int64_t bcols, TuneDB &db)
{
    const size_t es = dtype == RTRI_F64 ? 8 : 4;
    std::vector<rtri_batch_entry> ents;
    uint64_t st = 0x9e3779b97f4a7c15ull;   // fixed host sequence (splitmix64)
    auto next = [&]() {
        st += 0x9e3779b97f4a7c15ull;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return (double)((z ^ (z >> 31)) >> 11) * 0x1.0p-53;
    };
    const double lmax = std::log((double)std::min<int64_t>(1024, max_order)), lmin = std::log(16.0);
    int64_t col = 0;
    for (int i = 0; i < 200; ++i) {
        const int64_t m = (int64_t)std::llround(std::exp(lmin + (lmax - lmin) * next()));
        const int64_t n = 1 + (int64_t)(next() * 128.0);
        if (col + n > bcols)
            break;
        rtri_batch_entry b{};
        b.op = 0;
        b.side = RTRI_LEFT;
        b.uplo = RTRI_LOWER;
        b.trans = RTRI_NOTRANS;
        b.diag = RTRI_NONUNIT;
        b.m = m;
        b.n = n;
        b.alpha = 1.0;
        b.A = A;
        b.lda = lda;
        b.B = static_cast<char *>(B) + (size_t)col * ldb * es;
        b.ldb = ldb;
        ents.push_back(b);
        col += n;
    }
    TuneDB *old = h->tune;
    TuneDB probe;
    h->tune = &probe;
    int best = 64, rc = RTRI_OK;
    float best_ms = 1e30f;
    for (int leaf : {32, 64}) {
        probe.batch.assign(1, TuneDB::Batch{dtype, leaf});
        rtri_batch_plan *plan = nullptr;
        int bad = -1;
        rc = rtri_batch_plan_create(h, dtype, (int)ents.size(), ents.data(), &plan, &bad);
        if (rc != RTRI_OK)
            break;
        int rr = RTRI_OK;
        const float ms = time_median(
            h->stream, 3,
            [&] {
                if (rr == RTRI_OK)
                    rr = rtri_synth_fill(h, dtype, 0, 77, 9, 1, max_order, bcols, 0.0, B, ldb);
            },
            [&] {
                if (rr == RTRI_OK)
                    rr = rtri_batch_plan_run(plan);
            });
        (void)rtri_batch_plan_destroy(plan);
        if (rr != RTRI_OK) {
            rc = rr;
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = leaf;
        }
    }
    h->tune = old;
    if (rc == RTRI_OK)
        db.batch.push_back(TuneDB::Batch{dtype, best});
    return rc;
}

}  // namespace

int rtri_tune(rtri_handle *h, int dtype, int64_t max_order, const char *db_path)
{
    if (!handle_valid(h))
        return RTRI_ERR_HANDLE;
    if (dtype != RTRI_F64 && dtype != RTRI_F32 && dtype != RTRI_BF16 && dtype != RTRI_F16)
        return -2;
    if (max_order < 256)
        return -3;
    if (dtype == RTRI_BF16 || dtype == RTRI_F16) {
        TuneDB db;
        if (h->tune != nullptr) {   // keep every other rule
            db = *h->tune;
            db.tile.erase(std::remove_if(db.tile.begin(), db.tile.end(),
                                         [&](const TuneDB::Tile &r) { return r.dtype == dtype; }),
                          db.tile.end());
        }
        const int rc = tune16(h, dtype, max_order, db);
        if (rc != RTRI_OK)
            return rc;   // the handle keeps the rules it had
        TuneDB *fresh = new (std::nothrow) TuneDB(db);
        if (fresh == nullptr)
            return RTRI_ERR_NOMEM;
        delete h->tune;
        h->tune = fresh;
        if (db_path != nullptr && !write_db(db_path, db))
            return RTRI_ERR_INVALID;
        return RTRI_OK;
    }
    const size_t es = dtype == RTRI_F64 ? 8 : 4;
    const int64_t max_n = std::min<int64_t>(max_order, 16384);
    void *A = nullptr, *B = nullptr, *C = nullptr;
    hipError_t e = hipMalloc(&A, (size_t)max_order * max_order * es);
    if (e == hipSuccess)
        e = hipMalloc(&B, (size_t)max_order * max_n * es);
    if (e == hipSuccess)
        e = hipMalloc(&C, (size_t)max_order * max_n * es);
    if (e != hipSuccess) {
        (void)hipFree(A);
        (void)hipFree(B);
        (void)hipFree(C);
        return hip_fail(h, e);
    }
    const int saved_f64 = h->leaf_f64, saved_f32 = h->leaf_f32, saved_tile = h->gemm_tile;
    TuneDB *old = h->tune;
    h->tune = nullptr;
    TuneDB db;
    if (old != nullptr)   // keep the other dtype's rules
        for (const auto &r : old->leaf)
            if (r.dtype != dtype)
                db.leaf.push_back(r);
    if (old != nullptr)
        for (const auto &r : old->tile)
            if (r.dtype != dtype)
                db.tile.push_back(r);
    if (old != nullptr)
        for (const auto &r : old->batch)
            if (r.dtype != dtype)
                db.batch.push_back(r);
    int rc = RTRI_OK;
    // leaf size per (op, order, vector count)
    for (int64_t ka = 256; ka <= max_order && rc == RTRI_OK; ka *= 2) {
        rc = rtri_synth_fill(h, dtype, 1, 77, 5, (uint64_t)ka, ka, ka, (double)ka, A, max_order);
        for (int64_t n : {64, 512, 4096, 16384}) {
            if (n > max_n || rc != RTRI_OK)
                continue;
            for (int solve = 1; solve >= 0; --solve) {
                int best = 64;
                float best_ms = 1e30f;
                for (int leaf : {16, 32, 64, 128, 256}) {
                    (dtype == RTRI_F64 ? h->leaf_f64 : h->leaf_f32) = leaf;
                    int rr = RTRI_OK;
                    const float ms = time_median(
                        h->stream, 3,
                        [&] {
                            if (rr == RTRI_OK)
                                rr = rtri_synth_fill(h, dtype, 0, 77, 6, 1, ka, n, 0.0, B, max_order);
                        },
                        [&] {
                            if (rr != RTRI_OK)
                                return;
                            if (dtype == RTRI_F64)
                                rr = solve ? rtri_dtrsm(h, 0, 0, 0, 0, ka, n, 1.0, (const double *)A, max_order,
                                                        (double *)B, max_order)
                                           : rtri_dtrmm(h, 0, 0, 0, 0, ka, n, 1.0, (const double *)A, max_order,
                                                        (double *)B, max_order);
                            else
                                rr = solve ? rtri_strsm(h, 0, 0, 0, 0, ka, n, 1.0f, (const float *)A, max_order,
                                                        (float *)B, max_order)
                                           : rtri_strmm(h, 0, 0, 0, 0, ka, n, 1.0f, (const float *)A, max_order,
                                                        (float *)B, max_order);
                        });
                    if (rr != RTRI_OK) {
                        rc = rr;
                        break;
                    }
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = leaf;
                    }
                }
                db.leaf.push_back(TuneDB::Leaf{dtype, solve, ka, n, best});
            }
        }
    }
    (dtype == RTRI_F64 ? h->leaf_f64 : h->leaf_f32) = dtype == RTRI_F64 ? saved_f64 : saved_f32;
    // GEMM tile per (M = K, N)
    for (int64_t mk = 64; mk <= std::min<int64_t>(max_order / 2, 8192) && rc == RTRI_OK; mk *= 2) {
        for (int64_t n : {64, 512, 4096, 16384}) {
            if (n > max_n)
                continue;
            int best = 1;
            float best_ms = 1e30f;
            for (int tile : {1, 2, 3}) {
                h->gemm_tile = tile;
                int rr = RTRI_OK;
                const float ms = time_median(
                    h->stream, 3, [] {},
                    [&] {
                        rr = rtri_gemm_update(h, dtype, 0, 0, mk, n, mk, -1.0, A, max_order, B, max_order, 1.0, C,
                                              max_order);
                    });
                if (rr != RTRI_OK) {
                    rc = rr;
                    break;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = tile;
                }
            }
            db.tile.push_back(TuneDB::Tile{dtype, mk, n, best});
        }
    }
    h->gemm_tile = saved_tile;
    // the batched kernel's leaf, with the single-call rules found above
    if (rc == RTRI_OK) {
        const int saved_leaf = dtype == RTRI_F64 ? h->leaf_f64 : h->leaf_f32;
        (dtype == RTRI_F64 ? h->leaf_f64 : h->leaf_f32) = 0;
        rc = rtri_synth_fill(h, dtype, 1, 77, 5, 1, max_order, max_order, (double)max_order, A, max_order);
        if (rc == RTRI_OK)
            rc = tune_batched(h, dtype, max_order, A, max_order, B, max_order, max_n, db);
        (dtype == RTRI_F64 ? h->leaf_f64 : h->leaf_f32) = saved_leaf;
    }
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(A);
    (void)hipFree(B);
    (void)hipFree(C);
    if (rc != RTRI_OK) {
        h->tune = old;   // a failed sweep leaves the rules the handle had
        return rc;
    }
    TuneDB *fresh = new (std::nothrow) TuneDB(db);
    if (fresh == nullptr) {
        h->tune = old;
        return RTRI_ERR_NOMEM;
    }
    delete old;
    h->tune = fresh;
    if (db_path != nullptr && !write_db(db_path, db))
        return RTRI_ERR_INVALID;
    return RTRI_OK;
}

}  // extern "C"
