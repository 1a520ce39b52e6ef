// sam_sequence.cpp -- a sequence of sources A_1..A_N mapped to the target A_0
// (Section 2: every map goes back to A_0), run as one HIP graph.
//
// Static mode (structure-only pattern, replan_each_run = 0): the pattern
// S((I + B)^p) and the plan are computed once at creation; a run is the
// numeric build and Frobenius residual of every map.
// Replanning mode (value-dependent sparsification, or replan_each_run = 1):
// a run recomputes, for every source, the sparsified pattern, the row sets,
// gather positions and buckets on the device, into buffers sized by the
// structural bound (the pattern of the unsparsified A_k contains every
// sparsified one), so no host synchronisation and no allocation is needed
// and the whole run is capturable.  Bucket sizes then stay on the device and
// every kernel variant launches with the bound grid.
#include "sam_host.hpp"

#include <climits>
#include <cstring>

using namespace samh;

// Replanning sequences: graph branches, each with its own scratch set.
constexpr int kBranches = 3;

struct sam_seq {
    sam_ctx* ctx = nullptr;
    int n = 0;
    int n_src = 0;
    int prec = 1;  // 0 FP64, 1 FP32 + refinement
    sam_pattern_spec spec{};
    bool replan = false;
    // B = S(A~_k) is A_k's own structure: nothing is dropped (no
    // sparsification) and every column of A_k holds its diagonal, so the
    // level expansion reads A_k's column lists directly
    bool b_is_a = false;
    const int *A0_cp = nullptr, *A0_ri = nullptr, *Ak_cp = nullptr, *Ak_ri = nullptr;
    const double* A0_val = nullptr;
    int nnzA = 0, nnzA0 = 0;
    // caller memory holding everything below
    void* mem = nullptr;
    size_t mem_bytes = 0;
    // structural pattern (the pattern of every map in static mode, the bound
    // otherwise) and its plan
    int *S_cp = nullptr, *S_ri = nullptr;
    int64_t nnzS = 0;
    PatternLevels levels;          // structural level sizes, longest columns, column pointers
    sam_plan* plan = nullptr;
    // replanning mode: every level of the pattern is written into slots laid
    // out like the structural level (levels.cp, p arrays of n+1), with its
    // column lengths beside it; only the final S_k is compacted (Sk_cp/Sk_ri).
    // kBranches sets of scratch and plan arrays: the symbolic work of the
    // next sources (set (k+1) % kBranches, ...) runs while the numeric build
    // of source k (set k % kBranches) still reads its plan.
    struct Scratch {
        sam_plan dplan;            // views into the sequence memory
        int *B_ri = nullptr, *B_cnt = nullptr, *L_ri[2] = {nullptr, nullptr}, *L_cnt[2] = {nullptr, nullptr},
            *F_ri = nullptr, *F_cnt = nullptr;
        int64_t* off = nullptr;
        void *stemp = nullptr, *btemp = nullptr;
        double* D = nullptr;
    };
    Scratch part[kBranches];
    std::vector<int*> Sk_cp, Sk_ri;
    // graph: source k runs on branch k mod kBranches, branch 0 being the
    // capture stream and the others side[] (parallel branches of the graph,
    // forked and joined by events)
    hipStream_t cap = nullptr;
    hipStream_t side[kBranches - 1] = {};
    std::vector<hipEvent_t> ev;    // fork, then one join per side stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> key;
};

namespace {

// Device-side buckets of replanning mode from the structural plan's: a
// sparsified column only shrinks, so it lands in its structural bucket or an
// earlier one, and the count of bucket b is at most the structural count of
// buckets >= b (the grid bound).  Buckets past the last one with a nonzero
// bound can receive no column and are left out of the table, which keeps the
// per-run bucket kernels short.
void bound_buckets(Combo& cb, const Combo& structural) {
    cb.variants = structural.variants;
    cb.tab = structural.tab;
    const std::vector<int>& sc = structural.counts;
    cb.counts.assign(sc.size(), 0);
    int suffix = 0;
    for (int b = (int)sc.size() - 1; b >= 0; --b) {
        suffix += sc[b];
        cb.counts[b] = suffix;
    }
    // a bucket whose class lies inside an earlier bucket's class never
    // receives a column (the first fitting bucket takes it): no launch
    for (int b = 1; b < (int)cb.counts.size(); ++b)
        for (int e = 0; e < b; ++e)
            if (cb.tab.max_rows[e] >= cb.tab.max_rows[b] && cb.tab.max_cols[e] >= cb.tab.max_cols[b]) {
                cb.counts[b] = 0;
                break;
            }
    int live = (int)cb.counts.size();
    while (live > 0 && cb.counts[(size_t)live - 1] == 0) --live;
    cb.counts.resize((size_t)live);
    cb.variants.resize(std::min(cb.variants.size(), (size_t)live));
    cb.tab.nb = std::min(cb.tab.nb, live);
    // every structural column fits the first class, and a sparsified column
    // only shrinks: no sort needed
    cb.identity = live == 1;
}

// Bucket bounds of every scratch set from the structural combination; the
// identity queue is written here (outside any capture) when one bucket lives.
sam_status set_bounds(sam_seq* q, hipStream_t s) {
    for (sam_seq::Scratch& R : q->part) {
        Combo& cb = R.dplan.combo[q->prec][0];
        bound_buckets(cb, q->plan->combo[q->prec][0]);
        if (cb.identity) HIP_TRY(q->ctx, samk::identity_queue(q->n, cb.queue, cb.bstart, s));
    }
    HIP_TRY(q->ctx, hipStreamSynchronize(s));
    return SAM_OK;
}

void drop_graph(sam_seq* q) {
    if (q->exec) (void)hipGraphExecDestroy(q->exec);
    if (q->graph) (void)hipGraphDestroy(q->graph);
    q->exec = nullptr;
    q->graph = nullptr;
    q->key.clear();
}

// Symbolic work for source k (replanning mode) into scratch set R: the
// pattern, row sets, gather positions and buckets.  A sparsified level is a
// subset of the structural one, column by column, so each level is written
// straight into the structural layout (one launch per level, no count pass);
// the final level is compacted by the positions kernel after one scan of its
// lengths, and the gathered entries of column j go to the structural offsets
// eoff[j] of the static plan.
sam_status enqueue_symbolic(sam_seq* q, int k, sam_seq::Scratch& R, const double* vals, hipStream_t s) {
    sam_ctx* ctx = q->ctx;
    const int n = q->n;
    const samk::SparsifySpec sp = to_sp(&q->spec);
    const int p = q->spec.power;
    const int* lcp = q->levels.cp;
    auto level_cp = [&](int lev) { return lcp + (size_t)lev * (n + 1); };
    int* Scp = q->Sk_cp[k];
    int* Sri = q->Sk_ri[k];
    // B = S(A~_k) plus the diagonal, in the slots of the structural B (whose
    // column pointers are A_k's when B is A_k's structure: its lists are
    // then read in place, lengths from the column pointers)
    int* b_ri = p == 1 ? R.F_ri : R.B_ri;
    int* b_cnt = p == 1 ? R.F_cnt : R.B_cnt;
    const bool direct = q->b_is_a && p > 1;
    if (!direct)
        HIP_TRY(ctx, samk::sparsify_slots(n, q->Ak_cp, q->Ak_ri, vals, sp, R.D, level_cp(0), b_ri, b_cnt, s));
    const int* Bq_ri = direct ? q->Ak_ri : R.B_ri;
    const int* Bq_cnt = direct ? nullptr : R.B_cnt;
    const int* cur_ri = direct ? q->Ak_ri : b_ri;
    const int* cur_cnt = direct ? nullptr : b_cnt;
    for (int lev = 1; lev < p; ++lev) {
        int* dri = lev == p - 1 ? R.F_ri : R.L_ri[lev & 1];
        int* dcnt = lev == p - 1 ? R.F_cnt : R.L_cnt[lev & 1];
        HIP_TRY(ctx, samk::expand_slots(n, level_cp(lev - 1), cur_cnt, cur_ri, level_cp(0), Bq_cnt, Bq_ri,
                                        level_cp(lev), dri, dcnt, q->levels.maxcol[(size_t)lev - 1],
                                        q->levels.maxcol[0], s));
        cur_ri = dri;
        cur_cnt = dcnt;
    }
    // compact column pointers of S_k, then row sets, gather positions and the
    // compact S_k in one pass, then the size buckets
    HIP_TRY(ctx, samk::scan_counts(R.F_cnt, n, R.off, Scp, nullptr, R.stemp, s));
    sam_plan* pl = &R.dplan;
    pl->S_cp = Scp;
    pl->S_ri = Sri;
    HIP_TRY(ctx, samk::plan_positions_slots(n, level_cp(p - 1), R.F_cnt, R.F_ri, Scp, Sri, q->Ak_cp, q->Ak_ri,
                                            q->A0_cp, q->A0_ri, pl->eoff, pl->nI, pl->posA, pl->posB,
                                            q->plan->max_cols, q->plan->max_len_A, s));
    Combo& cb = pl->combo[q->prec][0];
    if (!cb.identity)
        HIP_TRY(ctx, samk::bucket_sort(n, Scp, pl->nI, cb.tab, cb.queue, cb.bstart, nullptr, ctx->d_status, R.btemp,
                                       s));
    return SAM_OK;
}

// Replanning mode: source k's symbolic work and numeric build, in that order,
// on branch k mod kBranches, which also picks the scratch set: the capture
// stream for branch 0, side[b - 1] for branch b.  Every edge between the work
// of two sources is then an order within one stream (symbolic k after numeric
// k - kBranches, which used the same set), and the branches meet only at the
// fork and the join.  While one branch runs a numeric build (which holds most
// of the GPU's registers), the others' symbolic chains take whatever the
// build leaves free, and a symbolic chain's last kernel hands over to its
// build with no edge between branches.
sam_status enqueue_pipelined(sam_seq* q, const double* const* vals, void* const* M, double* res2, hipStream_t s) {
    sam_ctx* ctx = q->ctx;
    const int N = q->n_src;
    hipEvent_t fork = q->ev[0];
    HIP_TRY(ctx, hipEventRecord(fork, s));
    for (hipStream_t x : q->side) HIP_TRY(ctx, hipStreamWaitEvent(x, fork, 0));
    for (int k = 0; k < N; ++k) {
        const int b = k % kBranches;
        sam_seq::Scratch& R = q->part[b];
        hipStream_t x = b == 0 ? s : q->side[b - 1];
        sam_status st = enqueue_symbolic(q, k, R, vals[k], x);
        if (st) return st;
        st = run_numeric(&R.dplan, vals[k], q->A0_val, nullptr, 0.0, q->prec, 0, M[k], nullptr, res2 + k, x);
        if (st) return st;
    }
    for (int b = 1; b < kBranches; ++b) {
        HIP_TRY(ctx, hipEventRecord(q->ev[b], q->side[b - 1]));
        HIP_TRY(ctx, hipStreamWaitEvent(s, q->ev[b], 0));
    }
    return SAM_OK;
}

sam_status enqueue_run(sam_seq* q, const double* const* vals, void* const* M, double* res2, hipStream_t s) {
    if (q->replan) return enqueue_pipelined(q, vals, M, res2, s);
    for (int k = 0; k < q->n_src; ++k) {
        sam_status st = run_numeric(q->plan, vals[k], q->A0_val, nullptr, 0.0, q->prec, 0, M[k], nullptr,
                                    res2 + k, s);
        if (st) return st;
    }
    return SAM_OK;
}

// Sizes that fix a sequence's memory layout: the structural pattern's level
// sizes (from its count), and the bound nnz(S) x longest column of A_k for
// the gathered entries of a plan on it.
struct SeqDims {
    int n = 0, p = 1, nnzA = 0, nnzA0 = 0, longest = 0, n_src = 0, partcap = 0;
    bool replan = false;
    int64_t nnzS = 0, Ebound = 0;
    std::vector<int64_t> lev_nnz;
};

// Layout of a sequence's memory (q == null: measure only): the structural
// pattern's workspace (creation only), the structural S and its level column
// pointers, the plan, then (replanning) the per-source patterns and the
// scratch sets.  Returns the plan region through plan_mem / plan_bytes_out.
size_t seq_layout(Carve& cv, const SeqDims& d, sam_seq* q, PatternWs* pw, void** plan_mem, size_t* plan_sz) {
    const int n = d.n;
    pattern_ws_layout(cv, n, d.nnzA, d.longest, d.p, pw);
    int* S_cp = cv.take<int>((size_t)n + 1);
    int* S_ri = cv.take<int>((size_t)d.nnzS);
    int* lev = cv.take<int>((size_t)d.p * ((size_t)n + 1));
    const size_t pb = plan_bytes(n, d.Ebound, d.nnzA0, d.partcap);
    void* pm = cv.take<char>(pb);
    if (plan_mem) *plan_mem = pm;
    if (plan_sz) *plan_sz = pb;
    if (q) {
        q->S_cp = S_cp;
        q->S_ri = S_ri;
        q->levels.cp = lev;
    }
    if (!d.replan) return cv.off;
    auto lev_nnz = [&](int l) { return std::max<int64_t>(d.lev_nnz[(size_t)l], 1); };
    int64_t mid_max = 1;
    for (int l = 1; l + 1 < d.p; ++l) mid_max = std::max(mid_max, lev_nnz(l));
    for (int k = 0; k < d.n_src; ++k) {
        int* cp = cv.take<int>((size_t)n + 1);
        int* ri = cv.take<int>((size_t)d.nnzS);
        if (q) {
            q->Sk_cp.push_back(cp);
            q->Sk_ri.push_back(ri);
        }
    }
    for (int b = 0; b < kBranches; ++b) {
        sam_seq::Scratch dummy;
        sam_seq::Scratch& R = q ? q->part[b] : dummy;
        R.off = cv.take<int64_t>((size_t)n + 1);
        R.stemp = cv.take<char>(samk::scan_temp_bytes(n));
        R.btemp = cv.take<char>(samk::bucket_temp_bytes(n));
        R.D = cv.take<double>((size_t)n);
        R.B_ri = cv.take<int>((size_t)lev_nnz(0));
        R.B_cnt = cv.take<int>((size_t)n);
        for (int i = 0; i < 2; ++i) {
            R.L_ri[i] = cv.take<int>((size_t)mid_max);
            R.L_cnt[i] = cv.take<int>((size_t)n);
        }
        R.F_ri = cv.take<int>((size_t)lev_nnz(d.p - 1));
        R.F_cnt = cv.take<int>((size_t)n);
        sam_plan& pl = R.dplan;
        pl.nI = cv.take<int>((size_t)n);
        pl.posA = cv.take<unsigned char>((size_t)d.Ebound);
        pl.posB = cv.take<unsigned char>((size_t)d.nnzA0);
        Combo& cb = pl.combo[q ? q->prec : 0][0];
        cb.queue = cv.take<int>((size_t)n);
        cb.bstart = cv.take<int>(64);
        pl.colbuf = cv.take<double>((size_t)n);
        pl.partcap = d.partcap;
        pl.partbuf = cv.take<double>((size_t)d.partcap);
        pl.rtemp = cv.take<char>(samk::reduce_temp_bytes(std::max(n, d.partcap)));
    }
    return cv.off;
}

sam_status seq_args(sam_ctx* ctx, const sam_csc* A0, const sam_csc* Ak_struct, const sam_pattern_spec* spec,
                    int32_t n_src, int32_t prec) {
    sam_status st;
    if ((st = check_csc_args(ctx, A0, "A0", true))) return st;
    if ((st = check_csc_args(ctx, Ak_struct, "Ak_struct", false))) return st;
    if ((st = check_spec(ctx, spec))) return st;
    if (A0->n != Ak_struct->n) return fail(ctx, SAM_ERR_SHAPE, "A0 and Ak_struct differ in order");
    if (n_src < 1) return fail(ctx, SAM_ERR_ARG, "n_src must be >= 1 (got %d)", n_src);
    if (A0->n == 0) return fail(ctx, SAM_ERR_ARG, "empty matrices (n = 0): nothing to map");
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if (Ak_struct->nnz == 0 || A0->nnz == 0)
        return fail(ctx, SAM_ERR_ARG, "Ak and A0 must have stored entries (a nonsingular source has at least n)");
    return SAM_OK;
}

// Validates both structures and counts the structural pattern
// S((I + S(A_k))^p) in the pattern workspace w: fills d (all but the
// layout's own choices) and res.
sam_status seq_count(sam_ctx* ctx, const sam_csc* A0, const sam_csc* Ak_struct, const sam_pattern_spec* spec,
                     int32_t n_src, int32_t replan, const PatternWs& w, PatternLevels* levels, SeqDims* d,
                     PatternResult* res, hipStream_t s) {
    sam_status st;
    const int n = A0->n;
    if ((st = validate_csc(ctx, n, A0->nnz, A0->colptr, A0->rowind, "A0", s))) return st;
    if ((st = validate_csc(ctx, n, Ak_struct->nnz, Ak_struct->colptr, Ak_struct->rowind, "Ak_struct", s))) return st;
    sam_pattern_spec structural = *spec;
    structural.kind = SAM_SPARSIFY_NONE;
    sam_csc skel = *Ak_struct;
    skel.val = nullptr;
    if ((st = compute_pattern(ctx, &skel, &structural, w, res, s, levels))) return st;
    d->nnzS = res->nnz;
    d->lev_nnz = levels->nnz;
    d->Ebound = std::max<int64_t>(d->nnzS * (int64_t)d->longest, 1);
    d->n_src = n_src;
    d->replan = replan != 0 || spec->kind != SAM_SPARSIFY_NONE;
    return SAM_OK;
}

sam_status seq_dims_base(sam_ctx* ctx, const sam_csc* A0, const sam_csc* Ak_struct, const sam_pattern_spec* spec,
                         SeqDims* d, hipStream_t s) {
    d->n = A0->n;
    d->p = spec->power;
    d->nnzA = Ak_struct->nnz;
    d->nnzA0 = A0->nnz;
    d->partcap = partial_capacity(ctx);
    return host_colptr(ctx, Ak_struct->colptr, d->n, Ak_struct->nnz, "Ak_struct", &d->longest, s);
}

}  // namespace

extern "C" {

sam_status sam_sequence_size(sam_ctx* ctx, const sam_csc* A0, const sam_csc* Ak_struct, const sam_pattern_spec* spec,
                             int32_t n_src, int32_t prec, int32_t replan_each_run, void* ws, size_t ws_bytes,
                             size_t* bytes, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = seq_args(ctx, A0, Ak_struct, spec, n_src, prec))) return st;
    if (!bytes) return fail(ctx, SAM_ERR_ARG, "bytes is NULL");
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    SeqDims d;
    if ((st = seq_dims_base(ctx, A0, Ak_struct, spec, &d, s))) return st;
    Carve wc(ws);
    PatternWs w;
    pattern_ws_layout(wc, d.n, d.nnzA, d.longest, d.p, &w);
    if ((st = check_ws(ctx, ws, ws_bytes, wc.off, "pattern workspace"))) return st;
    PatternLevels levels;
    PatternResult res;
    if ((st = seq_count(ctx, A0, Ak_struct, spec, n_src, replan_each_run, w, &levels, &d, &res, s))) return st;
    Carve cv(nullptr);
    *bytes = seq_layout(cv, d, nullptr, nullptr, nullptr, nullptr);
    return SAM_OK;
}

sam_status sam_sequence_create(sam_ctx* ctx, const sam_csc* A0, const sam_csc* Ak_struct, const sam_pattern_spec* spec,
                               int32_t n_src, int32_t prec, int32_t replan_each_run, void* mem, size_t mem_bytes,
                               sam_seq** out, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    if (!out) return fail(ctx, SAM_ERR_ARG, "seq is NULL");
    *out = nullptr;
    sam_status st;
    if ((st = seq_args(ctx, A0, Ak_struct, spec, n_src, prec))) return st;
    if ((st = check_ws(ctx, mem, mem_bytes, 1, "sequence memory"))) return st;
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    const int n = A0->n;
    SeqDims d;
    if ((st = seq_dims_base(ctx, A0, Ak_struct, spec, &d, s))) return st;

    sam_seq* q = new (std::nothrow) sam_seq();
    if (!q) return fail(ctx, SAM_ERR_NOMEM, "host allocation failed");
    q->ctx = ctx;
    q->n = n;
    q->n_src = n_src;
    q->prec = prec == SAM_PREC_F32_REFINE ? 1 : 0;
    q->spec = *spec;
    q->A0_cp = A0->colptr;
    q->A0_ri = A0->rowind;
    q->A0_val = A0->val;
    q->nnzA0 = A0->nnz;
    q->Ak_cp = Ak_struct->colptr;
    q->Ak_ri = Ak_struct->rowind;
    q->nnzA = Ak_struct->nnz;
    q->mem = mem;
    q->mem_bytes = mem_bytes;
    auto bail = [&](sam_status code) {
        sam_sequence_destroy(q);
        return code;
    };

    // the structural pattern S((I + S(A_k))^p), the bound of every
    // sparsified one, counted in the workspace at the start of the memory
    Carve wc(mem);
    PatternWs w;
    pattern_ws_layout(wc, n, d.nnzA, d.longest, d.p, &w);
    if (wc.off > mem_bytes) return bail(fail(ctx, SAM_ERR_ARG, "sequence memory: %zu bytes given, more needed", mem_bytes));
    PatternResult res;
    // level column pointers: counted once without a copy target, then the
    // layout is known and the count is repeated with the copies
    PatternLevels probe;
    if ((st = seq_count(ctx, A0, Ak_struct, spec, n_src, replan_each_run, w, &probe, &d, &res, s))) return bail(st);
    q->replan = d.replan;
    Carve cv(mem);
    void* plan_mem = nullptr;
    size_t plan_sz = 0;
    const size_t need = seq_layout(cv, d, q, nullptr, &plan_mem, &plan_sz);
    if (need > mem_bytes)
        return bail(fail(ctx, SAM_ERR_ARG, "sequence memory: %zu bytes given, %zu needed", mem_bytes, need));
    {
        sam_pattern_spec structural = *spec;
        structural.kind = SAM_SPARSIFY_NONE;
        sam_csc skel = *Ak_struct;
        skel.val = nullptr;
        if ((st = compute_pattern(ctx, &skel, &structural, w, &res, s, &q->levels))) return bail(st);
        if (res.nnz != d.nnzS) return bail(fail(ctx, SAM_ERR_HIP, "structural pattern changed between two counts"));
        if ((st = pattern_fill(ctx, n, res, q->S_cp, q->S_ri, s))) return bail(st);
        q->nnzS = res.nnz;
        // B = A_k's structure plus the diagonal: as many entries as A_k
        // means no diagonal was added, and the level-0 column pointers are
        // A_k's (both ascending, the same rows)
        q->b_is_a = spec->kind == SAM_SPARSIFY_NONE && !q->levels.nnz.empty() &&
                    q->levels.nnz[0] == (int64_t)Ak_struct->nnz;
    }
    {
        sam_csc skel = *Ak_struct;
        skel.val = nullptr;
        sam_plan* pl = new (std::nothrow) sam_plan();
        if (!pl) return bail(fail(ctx, SAM_ERR_NOMEM, "host allocation failed"));
        q->plan = pl;
        if ((st = plan_init(ctx, pl, &skel, A0, q->S_cp, q->S_ri, q->nnzS, plan_mem, plan_sz, s))) return bail(st);
        if (pl->E > d.Ebound) return bail(fail(ctx, SAM_ERR_HIP, "gathered entries exceed their bound"));
    }
    if (!q->plan->combo[q->prec][0].ok)
        return bail(fail(ctx, SAM_ERR_UNSUPPORTED, "%s", q->plan->combo[q->prec][0].why.c_str()));

    if (q->replan) {
        for (sam_seq::Scratch& R : q->part) {
            sam_plan& dp = R.dplan;
            dp.ctx = ctx;
            dp.n = n;
            dp.nnzA = q->nnzA;
            dp.nnzA0 = q->nnzA0;
            dp.nnzS = q->nnzS;
            dp.E = q->plan->E;
            dp.max_cols = q->plan->max_cols;
            dp.max_len_A = q->plan->max_len_A;
            dp.Ak_cp = q->Ak_cp;
            dp.Ak_ri = q->Ak_ri;
            dp.A0_cp = q->A0_cp;
            dp.A0_ri = q->A0_ri;
            dp.eoff = q->plan->eoff;   // structural offsets of the gathered entries
            dp.combo[q->prec][0].ok = true;
            dp.device_counts = true;
        }
        for (hipStream_t& x : q->side)
            if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess)
                return bail(fail(ctx, SAM_ERR_HIP, "stream creation failed"));
        q->ev.assign(kBranches, nullptr);
        for (hipEvent_t& e : q->ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                return bail(fail(ctx, SAM_ERR_HIP, "event creation failed"));
    }
    if (hipStreamCreateWithFlags(&q->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(ctx, SAM_ERR_HIP, "stream creation failed"));
    if (q->replan) {
        sam_status st2 = set_bounds(q, s);
        if (st2) return bail(st2);
    }
    *out = q;
    return SAM_OK;
}

sam_status sam_sequence_destroy(sam_seq* q) {
    if (!q) return SAM_OK;
    if (q->ctx && q->ctx->device != SAM_NO_DEVICE) {
        (void)hipSetDevice(q->ctx->device);
        (void)hipDeviceSynchronize();
    }
    drop_graph(q);
    if (q->cap) (void)hipStreamDestroy(q->cap);
    for (hipStream_t x : q->side)
        if (x) (void)hipStreamDestroy(x);
    for (hipEvent_t e : q->ev)
        if (e) (void)hipEventDestroy(e);
    delete q->plan;   // host record: its arrays live in the sequence memory
    delete q;
    return SAM_OK;
}

sam_status sam_sequence_info(const sam_seq* q, int64_t* nnz_bound) {
    if (!q || !nnz_bound) return SAM_ERR_ARG;
    *nnz_bound = q->nnzS;
    return SAM_OK;
}

sam_status sam_sequence_pattern(sam_seq* q, int32_t k, int32_t* S_colptr, int32_t* S_rowind, int64_t* nnz_S,
                                sam_stream_t stream) {
    if (!q || !q->ctx) return SAM_ERR_ARG;
    sam_ctx* ctx = q->ctx;
    check_ctx(ctx);
    if (k < 0 || k >= q->n_src) return fail(ctx, SAM_ERR_ARG, "source index %d outside [0, %d)", k, q->n_src);
    if (!S_colptr || !nnz_S) return fail(ctx, SAM_ERR_ARG, "NULL argument");
    sam_status st = need_device(ctx);
    if (st) return st;
    hipStream_t s = S(stream);
    const int* cp = q->replan ? q->Sk_cp[k] : q->S_cp;
    const int* ri = q->replan ? q->Sk_ri[k] : q->S_ri;
    int last = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&last, cp + q->n, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    *nnz_S = last;
    HIP_TRY(ctx, hipMemcpyAsync(S_colptr, cp, (size_t)(q->n + 1) * 4, hipMemcpyDeviceToDevice, s));
    if (last > 0) {
        if (!S_rowind) return fail(ctx, SAM_ERR_ARG, "S_rowind is NULL");
        HIP_TRY(ctx, hipMemcpyAsync(S_rowind, ri, (size_t)last * 4, hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return SAM_OK;
}

sam_status sam_sequence_select(sam_seq* q, const int32_t* order, int32_t count, sam_stream_t stream) {
    if (!q || !q->ctx) return SAM_ERR_ARG;
    sam_ctx* ctx = q->ctx;
    check_ctx(ctx);
    bool ok = false;
    std::vector<const samk::NumericVariant*> vars = menu_subset(q->prec, 0, order, count, &ok);
    if (!ok) return fail(ctx, SAM_ERR_ARG, "variant order must list 1..%d valid menu indices", samk::kMaxBuckets);
    sam_status st = need_device(ctx);
    if (st) return st;
    if ((st = plan_select(q->plan, q->prec, vars, S(stream)))) return st;
    if (q->replan && (st = set_bounds(q, S(stream)))) return st;
    drop_graph(q);  // the next run captures the new launches
    return SAM_OK;
}

sam_status sam_sequence_run(sam_seq* q, const double* const* Ak_vals, void* const* M_vals, double* res2,
                            sam_stream_t stream) {
    if (!q || !q->ctx) return SAM_ERR_ARG;
    sam_ctx* ctx = q->ctx;
    check_ctx(ctx);
    if (!Ak_vals || !M_vals || !res2) return fail(ctx, SAM_ERR_ARG, "NULL argument");
    for (int k = 0; k < q->n_src; ++k)
        if (!Ak_vals[k] || !M_vals[k]) return fail(ctx, SAM_ERR_ARG, "NULL pointer for source %d", k);
    sam_status st = need_device(ctx);
    if (st) return st;
    std::vector<const void*> key;
    key.reserve(2 * q->n_src + 1);
    for (int k = 0; k < q->n_src; ++k) {
        key.push_back(Ak_vals[k]);
        key.push_back(M_vals[k]);
    }
    key.push_back(res2);
    if (!q->exec || key != q->key) {
        drop_graph(q);
        HIP_TRY(ctx, hipStreamBeginCapture(q->cap, hipStreamCaptureModeThreadLocal));
        st = enqueue_run(q, Ak_vals, M_vals, res2, q->cap);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(q->cap, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(ctx, SAM_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
        q->graph = g;
        e = hipGraphInstantiate(&q->exec, q->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(q);
            return fail(ctx, SAM_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        q->key = key;
    }
    HIP_TRY(ctx, hipGraphLaunch(q->exec, S(stream)));
    return SAM_OK;
}

}  // extern "C"
