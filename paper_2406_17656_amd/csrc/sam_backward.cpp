// sam_backward.cpp -- host side of the soft-weighted map's adjoint: the
// staging buffers (allocated on the first call), the backward launches per
// bucket, and the deterministic A_k-value accumulation.
#include "sam_host.hpp"

#include <climits>

using namespace samh;

namespace {

struct BwdBufs {
    double* contrib;
    int64_t* segoff;
    int* ST_rowptr;
    int* ST_colind;
    int* ST_perm;
};

BwdBufs bwd_views(sam_plan* pl) {
    Carve cv(pl->bwd.p);
    BwdBufs b;
    b.contrib = cv.take<double>((size_t)std::max<int64_t>(pl->E, 1));
    b.segoff = cv.take<int64_t>((size_t)std::max<int64_t>(pl->nnzS, 1));
    b.ST_rowptr = cv.take<int>((size_t)pl->n + 1);
    b.ST_colind = cv.take<int>((size_t)std::max<int64_t>(pl->nnzS, 1));
    b.ST_perm = cv.take<int>((size_t)std::max<int64_t>(pl->nnzS, 1));
    return b;
}

// Staging for the contributions and the row view of S (which columns j
// contain row l, ascending j), built once per plan.
sam_status ensure_backward(sam_plan* pl, hipStream_t s) {
    sam_ctx* ctx = pl->ctx;
    if (pl->bwd.p) return SAM_OK;
    const int n = pl->n;
    const size_t nS = (size_t)std::max<int64_t>(pl->nnzS, 1);
    const size_t need = align256((size_t)std::max<int64_t>(pl->E, 1) * 8) + align256(nS * 8) +
                        align256(((size_t)n + 1) * 4) + 2 * align256(nS * 4) + 1024;
    HIP_TRY(ctx, grow(pl->bwd, need));
    BwdBufs b = bwd_views(pl);
    const size_t tneed = 2 * align256((size_t)std::max(n, 1) * 4) + align256(((size_t)n + 1) * 8) +
                         align256(samk::scan_temp_bytes(n)) + 512;
    HIP_TRY(ctx, grow(ctx->ws, tneed));
    Carve tw(ctx->ws.p);
    int* rowcount = tw.take<int>(std::max(n, 1));
    int* cursor = tw.take<int>(std::max(n, 1));
    int64_t* off = tw.take<int64_t>((size_t)n + 1);
    void* stemp = tw.take<char>(samk::scan_temp_bytes(n));
    HIP_TRY(ctx, hipMemsetAsync(rowcount, 0, (size_t)std::max(n, 1) * 4, s));
    HIP_TRY(ctx, hipMemsetAsync(cursor, 0, (size_t)std::max(n, 1) * 4, s));
    HIP_TRY(ctx, samk::transpose_count(n, pl->S_cp, pl->S_ri, pl->nnzS, rowcount, s));
    HIP_TRY(ctx, samk::scan_counts(rowcount, n, off, b.ST_rowptr, nullptr, stemp, s));
    HIP_TRY(ctx, samk::transpose_fill(n, pl->S_cp, pl->S_ri, b.ST_rowptr, cursor, b.ST_colind, b.ST_perm, s));
    HIP_TRY(ctx, samk::transpose_sort_rows(n, b.ST_rowptr, b.ST_colind, b.ST_perm, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return SAM_OK;
}

}  // namespace

extern "C" {

sam_status sam_backward(sam_plan* plan, const double* Ak_val, const double* A0_val, const double* w, double mu,
                        double dL, sam_precision prec, double* gAk, double* gA0, double* gw, double* loss,
                        sam_stream_t stream) {
    if (!plan || !plan->ctx) return SAM_ERR_ARG;
    sam_ctx* ctx = plan->ctx;
    check_ctx(ctx);
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if ((plan->nnzA > 0 && (!Ak_val || !gAk)) || (plan->nnzA0 > 0 && (!A0_val || !gA0)))
        return fail(ctx, SAM_ERR_ARG, "value or gradient array is NULL");
    if (plan->nnzS > 0 && !w) return fail(ctx, SAM_ERR_ARG, "w is NULL");
    if (!(mu >= 0.0)) return fail(ctx, SAM_ERR_ARG, "mu must be >= 0 (got %g)", mu);
    sam_status st = need_device(ctx);
    if (st) return st;
    hipStream_t s = S(stream);
    const int pi = prec == SAM_PREC_F32_REFINE ? 1 : 0;
    Combo& cb = plan->combo[pi][1];
    if (!cb.ok) return fail(ctx, SAM_ERR_UNSUPPORTED, "%s", cb.why.c_str());
    if ((st = ensure_backward(plan, s))) return st;
    BwdBufs b = bwd_views(plan);

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
