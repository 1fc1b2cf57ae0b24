// Handle internals and the recursion plan interface shared by the host sources.
#pragma once

#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.h"

namespace rtri {

struct TuneDB;   // tuned leaf sizes and GEMM tiles (tune.hip)
void tune_db_free(TuneDB *db);
// 0 when the database has no rule for the case
int tuned_leaf(const TuneDB *db, int dtype, bool solve, int64_t ka, int64_t nvec);
int tuned_tile(const TuneDB *db, int dtype, int64_t M, int64_t N);   // dtype RTRI_BF16 / RTRI_F16: 16-bit tiles
int tuned_batch_leaf(const TuneDB *db, int dtype);
int load_tuning_file(rtri_handle *h, const char *path);

struct ProfRec {
    int kclass, dtype;
    double flops, bytes;
    hipEvent_t e0, e1;
};

// Device workspace slots owned by a handle, each grown on demand.
enum WsSlot {
    WS_PACK = 0,     // packed diagonal blocks of the current plan
    WS_PACK2,        // packed blocks kept across the refinement steps
    WS_ACOPY,        // converted copy of A (mixed precision)
    WS_REFINE,       // state of a refined solve run to the end (RefineState: X, R0, R, W, the FP32 panel)
    WS_SCALARS,      // small reduction results
    WS_SAVE,         // copy of a TRMM panel's original values (all leaves in one launch)
    WS_SPLIT,        // split-K partial products, one region per stream an update may run on
    WS_ROWS,         // copy of a right-hand side whose rows are interchanged (GETRS)
    WS_PERM,         // the row permutation of those interchanges
    WS_ZEMB,         // real embedding of a complex op(A) (2 ka x 2 ka)
    WS_ZT,           // transposed complex right-hand side (side R)
    WS_OZA,          // INT8 residue planes of op(A) (Ozaki-scheme product)
    WS_OZX,          // INT8 residue planes of the panel
    WS_OZR,          // residues of the integer product, one byte plane per modulus
    WS_GROUP,        // tables of a grouped update launch (descs, entries, tiles)
    WS_COUNT
};

// One recursive TRSM / TRMM to run: the panel B (FP64 or FP32), the
// triangular factor as read by the GEMM updates (same type as the panel, or a
// 16-bit copy), and the factor as read by the pack pass for the leaves.
struct PlanIn {
    bool solve;
    int side, uplo, trans, diag;   // trans already folded: 'C' -> 'T'
    int64_t m, n;
    double alpha;
    DType bt;                      // panel type (also the leaf arithmetic)
    char *B;
    int64_t ldb;
    ElemT gt;                      // type of the GEMM copy of A
    const char *Ag;
    int64_t ldag;
    bool ag_trans;                 // Ag holds A^T (column-major, ld ldag) instead of A
    ElemT st;                      // type of A as read by the pack pass
    const void *As;
    int64_t ldas;
    int leaf;
    int pack_slot;                 // workspace slot holding the packed blocks
    bool skip_pack;                // the packed blocks are already in pack_slot
    // packed blocks made earlier for this exact plan (a factor keeps them):
    // used in place of pack_slot, and no pack pass runs; nullptr otherwise
    const void *packed;
    // TRMM with a 16-bit GEMM copy of A: the original panel in that 16-bit type
    // (the panel B holds it widened), read by the GEMM updates in place of the
    // panel or its saved copy; nullptr otherwise
    const char *Bsrc16;
    int64_t ldbsrc16;
    // caller-supplied device workspace in place of the handle's slots (both
    // nullptr: the handle's own, grown on demand).  ext_pack receives the
    // packed blocks (plan_pack_bytes); ext_split is the split-K region of the
    // handle's stream (SPLIT_REGION_BYTES).  With ext_split set, updates on
    // other streams do not split, and a TRMM plan never saves its panel.
    void *ext_pack;
    void *ext_split;
};

}  // namespace rtri

struct rtri_handle {
    uint32_t magic;
    hipStream_t stream;
    int leaf_f64, leaf_f32, gemm_tile;
    int trmm_leaves;   // RTRI_OPT_TRMM_LEAVES: 0 automatic, 1 one launch per leaf, 2 all leaves in one launch
    int gemm16_tile;   // RTRI_OPT_GEMM16_TILE: 0 automatic, 1 128x128, 2 256x256 where the layout allows
    int residual;      // RTRI_OPT_RESIDUAL: refined solve's residual product, 0 FP64 MFMA, 1 INT8 (Ozaki)
    rtri::TuneDB *tune;
    hipError_t last;
    void *ws[rtri::WS_COUNT];
    size_t ws_bytes[rtri::WS_COUNT];
    // streams for independent GEMM updates (created on first use, default
    // priority) and the events that fork them from / join them to `stream`
    hipStream_t aux[4];
    hipEvent_t aux_ev[5];
    bool aux_ready;
    bool profiling;
    std::vector<rtri::ProfRec> recs;
    std::vector<hipEvent_t> pool;
    size_t pool_used;
    // memory pool for the parts of factors this handle prepares (a serving
    // slot's own pool, so freed blocks are reused only in its stream's order);
    // nullptr: plain hipMalloc / hipFree
    hipMemPool_t mem_pool;
};

namespace rtri {

bool handle_valid(const rtri_handle *h);
// takes the device address of the no-allocation entry point's scratch on the
// current device (once per device; failures are left to that entry point)
void noalloc_prepare();
int hip_fail(rtri_handle *h, hipError_t e);
hipError_t ensure_ws(rtri_handle *h, int slot, size_t bytes);
// leaf size: the handle's option, else the tuning database, else 64
bool valid_leaf(int64_t v);   // 0 (automatic), 16, 32, 64, 128 or 256
int pick_leaf(const rtri_handle *h, DType t, bool solve, int64_t ka, int64_t nvec);
// whether a TRMM with this leaf size runs all its leaves in one launch after
// saving the panel (workspace WS_SAVE, m x n elements)
bool trmm_one_launch(const rtri_handle *h, int leaf, int64_t ka, int64_t nvec);
// leading dimension of the refinement's workspace matrices and of the converted
// copy of A: rows rounded up to 8 elements, so every column starts on a 16-byte
// boundary and the GEMM kernels take their vector-load paths
inline int64_t ws_ld(int64_t rows) { return (rows + 7) / 8 * 8; }
// split-K workspace: one region for the handle's stream and one per auxiliary stream
constexpr size_t SPLIT_REGION_BYTES = (size_t)16 << 20;
constexpr int SPLIT_REGIONS = 5;
constexpr size_t SPLIT_WS_BYTES = SPLIT_REGION_BYTES * SPLIT_REGIONS;
// whether some update of an order-ka recursion may split K: the longest K is
// the top split, leaf * ceil(ka / (2 leaf)), which reaches SPLIT_MIN_K only
// for ka > 2 SPLIT_MIN_K - 2 leaf (leaf <= 256)
inline bool may_split(int64_t ka) { return ka > 2 * SPLIT_MIN_K - 512; }
int check_args(int side, int uplo, int trans, int diag, int64_t m, int64_t n, const void *A, int64_t lda,
               const void *B, int64_t ldb, bool need_a);
// enqueue a whole plan on the handle's stream (returns an RTRI_* status)
int run_plan(rtri_handle *h, const PlanIn &p);
// the packed diagonal blocks of a plan: their size in bytes, and the pack pass
// writing them to out (on the handle's stream)
size_t plan_pack_bytes(const PlanIn &p);
hipError_t pack_plan(rtri_handle *h, const PlanIn &p, void *out);
// the plan of a plain FP64 / FP32 TRSM or TRMM as the BLAS-style entry points
// build it (trans 'C' folded to 'T', leaf from the handle's policy)
PlanIn plain_plan(rtri_handle *h, DType t, bool solve, int side, int uplo, int trans, int diag, int64_t m, int64_t n,
                  double alpha, const void *A, int64_t lda, void *B, int64_t ldb);
// launch through f(); inside a profile, bracket it with events and record its work
hipError_t timed_launch(rtri_handle *h, int kclass, int dtype, double flops, double bytes, hipError_t (*fn)(void *),
                        void *ctx);

// What the refined solve needs from A besides A itself, made once per call by
// rtri_dtrsm_mixed or once per factor by a factor object (eqs. (3)/(4)):
struct MixedPrep {
    const void *Acopy = nullptr;    // A (or A^T when ag_trans) in the GEMM type, leading dimension ldag
    int64_t ldag = 0;
    bool ag_trans = false;
    const void *lo_pack = nullptr;  // packed FP32 solve blocks for leaf lo_leaf; nullptr: packed on first use
    const void *mul_pack = nullptr; // packed FP64 multiply blocks for leaf mul_leaf; nullptr: likewise
    int lo_leaf = 0, mul_leaf = 0;
    const void *oz_planes = nullptr; // op(A)'s INT8 residue planes (INT8-product residual); nullptr: made by the call
    bool have_anorm = false;        // anorm known (else computed by the call)
    double anorm = 0.0;             // |op(A)|_inf (side L) or |op(A)|_1 (side R)
};
// the GEMM copy's orientation: A^T where the 16-bit GEMM's triangle operand is
// then k-contiguous (side L with trans N, side R with trans T)
inline bool mixed_ag_trans(ElemT gt, int side, int tr)
{
    return gt == ElemT::BF16 && (side == RTRI_LEFT ? tr == RTRI_NOTRANS : tr != RTRI_NOTRANS);
}
// refined solve on checked arguments (m, n > 0, alpha != 0, trans 'C' folded)
int mixed_core(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n, double alpha,
               const double *A, int64_t lda, double *B, int64_t ldb, ElemT gt, double tol, int max_iter,
               rtri_refine_info *info, const MixedPrep &prep);
// The refinement in phases, so that a caller can run other work between its
// corrections (the serving loop re-queues refined requests once per
// correction): refine_begin (|op(A)|, R0 = alpha B, max |R0|), refine_step
// (one correction: low-precision solve, X update, residual and eta; one
// host read of two scalars), repeated until done, then refine_end (X into
// B).  The state's matrices (ld-padded m x n: X, R0, R, W in FP64, the FP32
// panel D, four scalars) live in refine_state_bytes(m, n) bytes of device
// memory given to refine_state_place; any handle with the same options may
// run any phase (the plans are rebuilt per phase).  Per element the
// arithmetic is that of mixed_core, which runs the phases back to back.
struct RefineState {
    float *D = nullptr;
    double *X = nullptr, *R0 = nullptr, *R = nullptr, *W = nullptr;
    unsigned long long *sc = nullptr;
    int64_t ld = 0;
    const void *oz = nullptr;   // op(A)'s INT8 residue planes (INT8-product residual)
    double anorm = 0.0, rmax = 0.0, eta = 0.0, eta_prev = 0.0;
    int iters = 0;
    bool converged = false, stalled = false, done = false;
    bool lo_packed = false, mul_packed = false;   // the plans' blocks packed (skip from now on)
    double scale = 1.0;   // this correction's power-of-two scale s (D = R / s)
};
size_t refine_state_bytes(int64_t m, int64_t n);
void refine_state_place(RefineState &st, void *mem, int64_t m, int64_t n);
int refine_begin(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n, double alpha,
                 const double *A, int64_t lda, const double *B, int64_t ldb, double tol, int max_iter,
                 rtri_refine_info *info, const MixedPrep &prep, RefineState &st);
int refine_step(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n, const double *A,
                int64_t lda, ElemT gt, double tol, int max_iter, rtri_refine_info *info, const MixedPrep &prep,
                RefineState &st);
int refine_end(rtri_handle *h, int64_t m, int64_t n, double *B, int64_t ldb, rtri_refine_info *info,
               const RefineState &st);
// The same phases split into what is enqueued on h's stream and the host
// halves that read the scalars back once the caller has synchronised it, for
// callers that run several refinements in lockstep (refine_begin and
// refine_step are these with their own solve, product and synchronisation):
//   begin: refine_begin_enqueue, sync, refine_begin_finish (host4: 4 words);
//   step:  refine_step_convert (D = R / s), the low-precision solve of D,
//          refine_step_update (X += s D, W = X), W := op(A) W in FP64,
//          refine_step_resid (R, eta, max |R|; host2: 2 words), sync,
//          refine_step_finish.
hipError_t refine_begin_enqueue(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n,
                                double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                                const MixedPrep &prep, RefineState &st, unsigned long long *host4);
void refine_begin_finish(const unsigned long long *host4, double tol, int max_iter, rtri_refine_info *info,
                         const MixedPrep &prep, RefineState &st);
hipError_t refine_step_convert(rtri_handle *h, int64_t m, int64_t n, RefineState &st);
hipError_t refine_step_update(rtri_handle *h, int64_t m, int64_t n, RefineState &st);
hipError_t refine_step_resid(rtri_handle *h, int side, int64_t m, int64_t n, RefineState &st,
                             unsigned long long *host2);
void refine_step_finish(const unsigned long long *host2, double tol, int max_iter, rtri_refine_info *info,
                        RefineState &st);
// the refined solve against a factor object in phases (factor.hip): arguments
// as rtri_factor_trsm checks them, m, n > 0, alpha != 0, a mixed precision;
// the factor's parts (copy of A, packed blocks, |op(A)|, residue planes) are
// made by the first phase that needs them
int factor_refine_begin(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, double alpha,
                        const double *B, int64_t ldb, int precision, double tol, int max_iter, rtri_refine_info *info,
                        RefineState &st);
int factor_refine_step(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, int precision,
                       double tol, int max_iter, rtri_refine_info *info, RefineState &st);
// the factor's parts a refined solve reads (GEMM-type copy, packed blocks,
// |op(A)|, residue planes), made if missing, for the split phases above
int factor_refine_prep(rtri_handle *h, rtri_factor *f, int side, int trans, int64_t m, int64_t n, int precision,
                       MixedPrep &prep);
// lines of op(A) (side L) or op(A)^T (side R) summed into out[0] (anorm)
hipError_t launch_mixed_norm(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t ka, const double *A,
                             int64_t lda, unsigned long long *out);
// the GEMM copy of A for the refined solve (conversion, transposed when ag_trans)
hipError_t launch_mixed_copy(rtri_handle *h, ElemT gt, bool ag_trans, int64_t ka, const double *A, int64_t lda,
                             void *Acopy, int64_t ldag);
// the two plans of the refined solve: low-precision solve on the FP32 panel D
// and the FP64 multiply of the residual on W (workspace pointers filled by the caller)
PlanIn mixed_lo_plan(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n, ElemT gt,
                     const double *A, int64_t lda);
PlanIn mixed_mul_plan(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t m, int64_t n, const double *A,
                      int64_t lda);

// FP64-accurate triangular product from INT8 matrix-core products (ozaki.hip):
// moduli used for inner dimension K (0: K beyond the method's range), and
// the bits beta kept of each scaled operand entry
int ozaki_nmod(int64_t K);
int ozaki_beta(int64_t K);
// device bytes of op(A)'s residue planes (and line exponents) for order ka
size_t ozaki_factor_bytes(int side, int64_t ka);
// op(A)'s planes into mem (ozaki_factor_bytes), on the handle's stream
hipError_t ozaki_split_factor(rtri_handle *h, int side, int uplo, int tr, int diag, int64_t ka, const double *A,
                              int64_t lda, void *mem);
// W := alpha op(A) X (side L) or alpha X op(A) (side R), m x n, from op(A)'s
// planes; X may equal W (its planes are made first).  RTRI_* status.
int ozaki_product(rtri_handle *h, int side, int uplo, int tr, int64_t m, int64_t n, double alpha, const void *Aplanes,
                  const double *X, int64_t ldx, double *W, int64_t ldw);

// Reusable staging for batched launches issued by a long-lived caller (a
// serving slot): pinned host tables and their device copy, grown on demand.
struct BatchScratch {
    void *dev = nullptr;
    size_t dev_bytes = 0;
    void *host = nullptr;
    size_t host_bytes = 0;
};
// Enqueue one batched launch on h's stream (no graph).  The caller must wait
// for the stream before reusing sc.  *flops (nullable) gets the useful flops.
int batch_run_async(rtri_handle *h, int dtype, int count, const rtri_batch_entry *e, BatchScratch &sc,
                    int *bad_index, double *flops);
void batch_scratch_free(BatchScratch &sc);

template <class F>
hipError_t timed(rtri_handle *h, int kclass, int dtype, double flops, double bytes, F &&f)
{
    using FF = std::remove_reference_t<F>;
    auto tramp = [](void *c) -> hipError_t { return (*static_cast<FF *>(c))(); };
    return timed_launch(h, kclass, dtype, flops, bytes, tramp, (void *)&f);
}

}  // namespace rtri
