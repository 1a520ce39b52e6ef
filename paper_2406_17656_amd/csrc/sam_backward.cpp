// sam_backward.cpp -- host side of the soft-weighted map's adjoint: the
// caller's workspace (staging of the per-column contributions and the row
// view of S), the backward launches per bucket, and the deterministic A_k
// value accumulation.
#include "sam_host.hpp"

#include <climits>

using namespace samh;

namespace {

struct BwdBufs {
    double* contrib;      // one per gathered entry, at the plan's eoff[j]
    int64_t* segoff;      // per S entry: where its column's contributions start
    int* ST_rowptr;       // row view of S: which columns j contain row l,
    int* ST_colind;       // ascending j
    int* ST_perm;
    int* rowcount;        // temporaries of the row view
    int* cursor;
    int64_t* off;
    void* stemp;
};

size_t bwd_layout(Carve& cv, int n, int64_t E, int64_t nnzS, BwdBufs* b) {
    BwdBufs x;
    x.contrib = cv.take<double>((size_t)E);
    x.segoff = cv.take<int64_t>((size_t)nnzS);
    x.ST_rowptr = cv.take<int>((size_t)n + 1);
    x.ST_colind = cv.take<int>((size_t)nnzS);
    x.ST_perm = cv.take<int>((size_t)nnzS);
    x.rowcount = cv.take<int>((size_t)std::max(n, 1));
    x.cursor = cv.take<int>((size_t)std::max(n, 1));
    x.off = cv.take<int64_t>((size_t)n + 1);
    x.stemp = cv.take<char>(samk::scan_temp_bytes(n));
    if (b) *b = x;
    return cv.off;
}

}  // namespace

extern "C" {

sam_status sam_backward_workspace_size(const sam_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return SAM_ERR_ARG;
    Carve cv(nullptr);
    *bytes = bwd_layout(cv, plan->n, plan->E, plan->nnzS, nullptr);
    return SAM_OK;
}

sam_status sam_backward_prepare(sam_plan* plan, void* ws, size_t ws_bytes, sam_stream_t stream) {
    if (!plan || !plan->ctx) return SAM_ERR_ARG;
    sam_ctx* ctx = plan->ctx;
    check_ctx(ctx);
    Carve cv(ws);
    BwdBufs b;
    sam_status st;
    if ((st = check_ws(ctx, ws, ws_bytes, bwd_layout(cv, plan->n, plan->E, plan->nnzS, &b), "backward workspace")))
        return st;
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    const int n = plan->n;
    plan->bwd_ws = nullptr;
    HIP_TRY(ctx, samk::fill_i32(b.rowcount, std::max(n, 1), 0, s));
    HIP_TRY(ctx, samk::fill_i32(b.cursor, std::max(n, 1), 0, s));
    HIP_TRY(ctx, samk::transpose_count(n, plan->S_cp, plan->S_ri, plan->nnzS, b.rowcount, s));
    HIP_TRY(ctx, samk::scan_counts(b.rowcount, n, b.off, b.ST_rowptr, nullptr, b.stemp, s));
    HIP_TRY(ctx, samk::transpose_fill(n, plan->S_cp, plan->S_ri, b.ST_rowptr, b.cursor, b.ST_colind, b.ST_perm, s));
    HIP_TRY(ctx, samk::transpose_sort_rows(n, b.ST_rowptr, b.ST_colind, b.ST_perm, s));
    plan->bwd_ws = ws;
    return SAM_OK;
}

sam_status sam_backward(sam_plan* plan, const double* Ak_val, const double* A0_val, const double* w, double mu,
                        double dL, int32_t prec, double* gAk, double* gA0, double* gw, double* loss, void* ws,
                        size_t ws_bytes, sam_stream_t stream) {
    if (!plan || !plan->ctx) return SAM_ERR_ARG;
    sam_ctx* ctx = plan->ctx;
    check_ctx(ctx);
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if ((plan->nnzA > 0 && (!Ak_val || !gAk)) || (plan->nnzA0 > 0 && (!A0_val || !gA0)))
        return fail(ctx, SAM_ERR_ARG, "value or gradient array is NULL");
    if (plan->nnzS > 0 && !w) return fail(ctx, SAM_ERR_ARG, "w is NULL");
    if (!(mu >= 0.0)) return fail(ctx, SAM_ERR_ARG, "mu must be >= 0 (got %g)", mu);
    Carve cv(ws);
    BwdBufs b;
    sam_status st;
    if ((st = check_ws(ctx, ws, ws_bytes, bwd_layout(cv, plan->n, plan->E, plan->nnzS, &b), "backward workspace")))
        return st;
    if (plan->bwd_ws != ws)
        return fail(ctx, SAM_ERR_ARG, "the backward workspace was not prepared for this plan (sam_backward_prepare)");
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    const int pi = prec == SAM_PREC_F32_REFINE ? 1 : 0;
    Combo& cb = plan->combo[pi][1];
    if (!cb.ok) return fail(ctx, SAM_ERR_UNSUPPORTED, "%s", cb.why.c_str());

    samk::NumericArgs a{};
    a.n = plan->n;
    a.nnzA = (uint32_t)plan->nnzA;
    a.nnzA0 = (uint32_t)plan->nnzA0;
    a.E = (uint32_t)plan->E;
    a.Ak_cp = plan->Ak_cp;
    a.Ak_v = Ak_val;
    a.A0_cp = plan->A0_cp;
    a.A0_v = A0_val;
    a.S_cp = plan->S_cp;
    a.S_ri = plan->S_ri;
    a.nI = plan->nI;
    a.eoff = plan->eoff;
    a.posA = plan->posA;
    a.posB = plan->posB;
    a.queue = cb.queue;
    a.bstart = cb.bstart;
    a.M = nullptr;
    a.col_res2 = plan->colbuf;
    a.status = ctx->d_status;
    a.w = w;
    a.mu = mu;
    a.dL = dL;
    a.contrib = b.contrib;
    a.segoff = b.segoff;
    a.gA0 = gA0;
    a.gw = gw;
    for (size_t k = 0; k < cb.variants.size(); ++k) {
        const int cnt = cb.counts[k];
        if (cnt <= 0) continue;
        const samk::NumericVariant* v = cb.variants[k];
        a.bucket = (int)k;
        int groups = (cnt + v->per_wave() - 1) / v->per_wave();
        int grid = std::min(groups, ctx->CUs * 16);
        if (grid >= 64) grid = grid / 8 * 8;
        HIP_TRY(ctx, v->launch_backward(a, grid, s));
    }
    HIP_TRY(ctx, samk::backward_scatter(plan->n, plan->Ak_cp, b.ST_rowptr, b.ST_perm, b.segoff, b.contrib, gAk, s));
    if (loss && plan->n > 0) HIP_TRY(ctx, samk::reduce_sum(plan->colbuf, plan->n, loss, plan->rtemp, s));
    return SAM_OK;
}

}  // extern "C"
