// sam_capi.cpp -- host implementation of the C ABI declared in include/sam.h:
// argument and structure validation, the context, patterns and plans in
// caller memory, and the launch sequence of the gfx950 kernels.
#include "sam_host.hpp"

#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>

using samk::BucketTable;
using samk::NumericArgs;
using samk::NumericVariant;
using namespace samh;

namespace samh {

sam_status fail(sam_ctx* ctx, sam_status st, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

sam_status check_ctx(sam_ctx* ctx) {
    if (!ctx) return SAM_ERR_ARG;
    ctx->err.clear();
    return SAM_OK;
}

sam_status need_device(sam_ctx* ctx) {
    if (ctx->device == SAM_NO_DEVICE)
        return fail(ctx, SAM_ERR_UNSUPPORTED, "context has no device (created with SAM_NO_DEVICE)");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(ctx, SAM_ERR_HIP, "hipSetDevice(%d): %s", ctx->device, hipGetErrorString(e));
    return SAM_OK;
}

sam_status check_csc_args(sam_ctx* ctx, const sam_csc* A, const char* name, bool need_val) {
    if (!A) return fail(ctx, SAM_ERR_ARG, "%s is NULL", name);
    if (A->n < 0 || A->nnz < 0) return fail(ctx, SAM_ERR_ARG, "%s: negative size (n=%d nnz=%d)", name, A->n, A->nnz);
    if (!A->colptr) return fail(ctx, SAM_ERR_ARG, "%s: colptr is NULL", name);
    if (A->nnz > 0 && !A->rowind) return fail(ctx, SAM_ERR_ARG, "%s: rowind is NULL", name);
    if (need_val && A->nnz > 0 && !A->val) return fail(ctx, SAM_ERR_ARG, "%s: val is NULL", name);
    return SAM_OK;
}

sam_status check_spec(sam_ctx* ctx, const sam_pattern_spec* spec) {
    if (!spec) return fail(ctx, SAM_ERR_ARG, "pattern spec is NULL");
    if (spec->kind < SAM_SPARSIFY_NONE || spec->kind > SAM_SPARSIFY_LFIL)
        return fail(ctx, SAM_ERR_ARG, "unknown sparsification kind %d", spec->kind);
    if (spec->power < 1) return fail(ctx, SAM_ERR_ARG, "power must be >= 1 (got %d)", spec->power);
    if (spec->kind == SAM_SPARSIFY_COLUMN && !(spec->tau >= 0.0 && spec->tau <= 1.0))
        return fail(ctx, SAM_ERR_ARG, "tau must lie in [0, 1] (got %g)", spec->tau);
    if (spec->kind == SAM_SPARSIFY_LFIL && spec->lfil < 1)
        return fail(ctx, SAM_ERR_ARG, "lfil must be >= 1 (got %d)", spec->lfil);
    if (spec->kind == SAM_SPARSIFY_GLOBAL && spec->global_scale != -1 && spec->global_scale != 1)
        return fail(ctx, SAM_ERR_ARG, "global_scale must be -1 or +1 (got %d)", spec->global_scale);
    return SAM_OK;
}

sam_status check_ws(sam_ctx* ctx, const void* ws, size_t ws_bytes, size_t need, const char* what) {
    if (ws_bytes < need)
        return fail(ctx, SAM_ERR_ARG, "%s: %zu bytes given, %zu needed", what, ws_bytes, need);
    if (need > 0 && !ws) return fail(ctx, SAM_ERR_ARG, "%s is NULL", what);
    if (((uintptr_t)ws & 255u) != 0) return fail(ctx, SAM_ERR_ARG, "%s is not 256-byte aligned", what);
    return SAM_OK;
}

samk::SparsifySpec to_sp(const sam_pattern_spec* spec) {
    samk::SparsifySpec sp;
    sp.kind = spec->kind;
    sp.thresh = spec->thresh;
    sp.global_scale = spec->global_scale;
    sp.tau = spec->tau;
    sp.lfil = spec->lfil;
    return sp;
}

sam_status host_colptr(sam_ctx* ctx, const int32_t* cp, int n, int64_t nnz, const char* name, int* longest,
                       hipStream_t s, std::vector<int>* keep) {
    std::vector<int> local;
    std::vector<int>& h = keep ? *keep : local;
    h.assign((size_t)n + 1, 0);
    HIP_TRY(ctx, hipMemcpyAsync(h.data(), cp, h.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (h[0] != 0 || h[(size_t)n] != nnz)
        return fail(ctx, SAM_ERR_UNSORTED, "%s: colptr[0] = %d and colptr[n] = %d, expected 0 and %lld", name, h[0],
                    h[(size_t)n], (long long)nnz);
    int most = 0;
    for (int j = 0; j < n; ++j) {
        const int len = h[(size_t)j + 1] - h[(size_t)j];
        if (len < 0) return fail(ctx, SAM_ERR_UNSORTED, "%s: colptr decreases at column %d", name, j);
        most = std::max(most, len);
    }
    if (longest) *longest = most;
    return SAM_OK;
}

sam_status validate_csc(sam_ctx* ctx, int n, int64_t nnz, const int32_t* cp, const int32_t* ri, const char* name,
                        hipStream_t s) {
    if (n == 0) return SAM_OK;
    int h = n;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_bad, &h, sizeof h, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, samk::check_csc(n, (int)nnz, cp, ri, ctx->d_bad, s));
    HIP_TRY(ctx, hipMemcpyAsync(&h, ctx->d_bad, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (h != n)
        return fail(ctx, SAM_ERR_UNSORTED,
                    "%s: invalid CSC structure at column %d (colptr not monotone or not ending at nnz, or rows "
                    "outside [0, n), unsorted or repeated)", name, h);
    return SAM_OK;
}

// ------------------------------------------------------------- patterns

int64_t level_bound(int n, int longest, int power) {
    const int64_t width = (int64_t)longest + 1;   // B adds the diagonal
    int64_t per = 1;
    for (int q = 0; q < power && per < n; ++q) per = std::min<int64_t>((int64_t)n, per * width);
    per = std::min<int64_t>(per, (int64_t)n);
    const int64_t b = per * (int64_t)n;
    return std::min<int64_t>(b, (int64_t)INT_MAX);
}

void pattern_ws_layout(Carve& cv, int n, int nnzA, int longest, int power, PatternWs* w) {
    PatternWs t;
    t.counts = cv.take<int>((size_t)n);
    t.off = cv.take<int64_t>((size_t)n + 1);
    t.stemp = cv.take<char>(samk::scan_temp_bytes(n));
    t.D = cv.take<double>((size_t)n);
    t.B_cp = cv.take<int>((size_t)n + 1);
    t.B_ri = cv.take<int>((size_t)nnzA + (size_t)n);
    t.flags = cv.take<int>(4);
    const int mids = power >= 3 ? std::min(power - 2, 2) : 0;
    t.Lcap = power >= 3 ? level_bound(n, longest, power - 1) : 0;
    for (int i = 0; i < mids; ++i) {
        t.L_cp[i] = cv.take<int>((size_t)n + 1);
        t.L_ri[i] = cv.take<int>((size_t)t.Lcap);
    }
    t.S_cp = cv.take<int>((size_t)n + 1);
    if (w) *w = t;
}

// Pattern pipeline: B = sparsify(A_k) (diagonal added), then p-1 times
// level <- expand(level, B).  Intermediate levels are stored in the
// workspace; the last is counted only.
sam_status compute_pattern(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, const PatternWs& w,
                           PatternResult* res, hipStream_t s, PatternLevels* levels) {
    const int n = Ak->n;
    const int p = spec->power;
    const size_t cp_bytes = (size_t)(n + 1) * 4;
    if (levels) {
        levels->nnz.clear();
        levels->maxcol.clear();
    }
    auto keep_level = [&](int lev, const int* cp) {
        return (levels && levels->cp)
                   ? hipMemcpyAsync(levels->cp + (size_t)lev * (n + 1), cp, cp_bytes, hipMemcpyDeviceToDevice, s)
                   : hipSuccess;
    };
    *res = PatternResult{};
    samk::SparsifySpec sp = to_sp(spec);
    const int init[3] = {0, n, 0};
    HIP_TRY(ctx, hipMemcpyAsync(w.flags, init, sizeof init, hipMemcpyHostToDevice, s));
    if (n == 0) {
        HIP_TRY(ctx, samk::fill_i32(w.B_cp, 1, 0, s));
        HIP_TRY(ctx, samk::fill_i32(w.S_cp, 1, 0, s));
        res->B_cp = w.B_cp;
        res->B_ri = w.B_ri;
        res->S_cp = p == 1 ? w.B_cp : w.S_cp;
        HIP_TRY(ctx, hipStreamSynchronize(s));
        return SAM_OK;
    }
    // total and longest column of the level just scanned
    auto level_facts = [&](int64_t* tot, int* maxc) {
        hipError_t e = hipMemcpyAsync(tot, w.off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(maxc, w.flags + 2, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    };
    HIP_TRY(ctx, samk::sparsify_count(n, Ak->colptr, Ak->rowind, Ak->val, sp, w.D, w.counts, s));
    HIP_TRY(ctx, samk::scan_counts(w.counts, n, w.off, w.B_cp, w.flags, w.stemp, s, w.flags + 2));
    HIP_TRY(ctx, samk::sparsify_fill(n, Ak->colptr, Ak->rowind, Ak->val, sp, w.D, w.B_cp, w.B_ri, s));
    HIP_TRY(ctx, keep_level(0, w.B_cp));
    int64_t nnzB = 0;
    int maxB = 0;
    HIP_TRY(ctx, level_facts(&nnzB, &maxB));
    if (levels) {
        levels->nnz.push_back(nnzB);
        levels->maxcol.push_back(maxB);
    }
    const int* cur_cp = w.B_cp;
    const int* cur_ri = w.B_ri;
    int cur_max = maxB;
    int64_t last_nnz = nnzB;
    for (int lev = 1; lev < p; ++lev) {
        HIP_TRY(ctx, samk::expand_count(n, cur_cp, cur_ri, w.B_cp, w.B_ri, w.counts, w.flags + 1, cur_max, s));
        HIP_TRY(ctx, samk::fill_i32(w.flags + 2, 1, 0, s));
        const bool last = lev == p - 1;
        int* dst_cp = last ? w.S_cp : w.L_cp[(lev - 1) & 1];
        HIP_TRY(ctx, samk::scan_counts(w.counts, n, w.off, dst_cp, w.flags, w.stemp, s, w.flags + 2));
        int64_t tot = 0;
        int tmax = 0;
        HIP_TRY(ctx, level_facts(&tot, &tmax));
        if (tot > INT_MAX)
            return fail(ctx, SAM_ERR_OVERFLOW, "pattern level %d has %lld entries (>= 2^31)", lev + 1, (long long)tot);
        HIP_TRY(ctx, keep_level(lev, dst_cp));
        if (levels) {
            levels->nnz.push_back(tot);
            levels->maxcol.push_back(tmax);
        }
        if (last) {
            res->last_cp = cur_cp;
            res->last_ri = cur_ri;
            res->last_max = cur_max;
            last_nnz = tot;
        } else {
            if (tot > w.Lcap)   // cannot happen: the bound holds for every pattern of this structure
                return fail(ctx, SAM_ERR_OVERFLOW, "pattern level %d exceeds its workspace bound", lev + 1);
            int* dst_ri = w.L_ri[(lev - 1) & 1];
            HIP_TRY(ctx, samk::expand_fill(n, cur_cp, cur_ri, w.B_cp, w.B_ri, dst_cp, dst_ri, cur_max, maxB, s));
            cur_cp = dst_cp;
            cur_ri = dst_ri;
            cur_max = tmax;
        }
    }
    int hflags[2] = {0, n};
    HIP_TRY(ctx, hipMemcpyAsync(hflags, w.flags, sizeof hflags, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (hflags[1] != n) return fail(ctx, SAM_ERR_UNSORTED, "column %d references a column index outside [0, n)", hflags[1]);
    if (hflags[0]) return fail(ctx, SAM_ERR_OVERFLOW, "pattern size does not fit in int32");
    res->nnz = last_nnz;
    res->B_cp = w.B_cp;
    res->B_ri = w.B_ri;
    res->maxB = maxB;
    res->S_cp = p == 1 ? w.B_cp : w.S_cp;
    return SAM_OK;
}

sam_status pattern_fill(sam_ctx* ctx, int n, const PatternResult& res, int* S_cp, int* S_ri, hipStream_t s) {
    HIP_TRY(ctx, hipMemcpyAsync(S_cp, res.S_cp, (size_t)(n + 1) * 4, hipMemcpyDeviceToDevice, s));
    if (res.nnz == 0) return SAM_OK;
    if (!res.last_cp) {   // power 1: S = B
        HIP_TRY(ctx, hipMemcpyAsync(S_ri, res.B_ri, (size_t)res.nnz * 4, hipMemcpyDeviceToDevice, s));
        return SAM_OK;
    }
    HIP_TRY(ctx, samk::expand_fill(n, res.last_cp, res.last_ri, res.B_cp, res.B_ri, S_cp, S_ri, res.last_max,
                                   res.maxB, s));
    return SAM_OK;
}

// ---------------------------------------------------------------- plans

BucketTable menu_table(int prec, int weighted, std::vector<const NumericVariant*>* variants) {
    int cnt = 0;
    const NumericVariant* menu = samk::numeric_menu(&cnt);
    BucketTable tab{};
    tab.nb = 0;
    tab.penalty_rows = weighted;
    for (int i = 0; i < cnt && tab.nb < samk::kMaxBuckets; ++i) {
        if (menu[i].prec != prec || menu[i].weighted != weighted) continue;
        tab.max_rows[tab.nb] = menu[i].max_rows();
        tab.max_cols[tab.nb] = menu[i].NC;
        if (variants) variants->push_back(&menu[i]);
        tab.nb++;
    }
    return tab;
}

BucketTable table_of(const std::vector<const NumericVariant*>& vars, int weighted) {
    BucketTable tab{};
    tab.nb = (int)std::min<size_t>(vars.size(), samk::kMaxBuckets);
    tab.penalty_rows = weighted;
    for (int b = 0; b < tab.nb; ++b) {
        tab.max_rows[b] = vars[b]->max_rows();
        tab.max_cols[b] = vars[b]->NC;
    }
    return tab;
}

sam_status plan_combo(sam_plan* pl, int prec, int weighted, hipStream_t s) {
    std::vector<const NumericVariant*> vars;
    menu_table(prec, weighted, &vars);
    return plan_combo_with(pl, prec, weighted, vars, s);
}

sam_status plan_combo_with(sam_plan* pl, int prec, int weighted, const std::vector<const NumericVariant*>& vars,
                           hipStream_t s) {
    sam_ctx* ctx = pl->ctx;
    Combo& cb = pl->combo[prec][weighted];
    cb.variants = vars;
    if (cb.variants.size() > (size_t)samk::kMaxBuckets) cb.variants.resize(samk::kMaxBuckets);
    BucketTable tab = table_of(cb.variants, weighted);
    cb.tab = tab;
    int* unfit_d = pl->flags;
    HIP_TRY(ctx, samk::fill_i32(unfit_d, 1, 0, s));
    HIP_TRY(ctx, samk::bucket_sort(pl->n, pl->S_cp, pl->nI, tab, cb.queue, cb.bstart, unfit_d, nullptr, pl->btemp, s));
    std::vector<int> hb(tab.nb + 1, 0);
    int unfit = 0;
    HIP_TRY(ctx, hipMemcpyAsync(hb.data(), cb.bstart, sizeof(int) * (tab.nb + 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(&unfit, unfit_d, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    cb.counts.resize(tab.nb);
    for (int b = 0; b < tab.nb; ++b) cb.counts[b] = hb[b + 1] - hb[b];
    cb.ok = unfit == 0;
    if (!cb.ok) {
        char buf[256];
        snprintf(buf, sizeof buf,
                 "%d columns exceed the largest kernel class for %s%s (max |I_j| = %d, max |J_j| = %d)", unfit,
                 prec ? "FP32+refine" : "FP64", weighted ? " weighted" : "", pl->max_rows, pl->max_cols);
        cb.why = buf;
    }
    return SAM_OK;
}

// Blocks of a numeric variant the GPU holds at once per CU (16 when the
// occupancy query failed).
int resident_blocks(const sam_ctx* ctx, const NumericVariant* v) {
    int cnt = 0;
    const NumericVariant* menu = samk::numeric_menu(&cnt);
    const ptrdiff_t i = v - menu;
    if (i >= 0 && i < (ptrdiff_t)ctx->resident.size() && ctx->resident[i] > 0) return ctx->resident[i];
    return 16;
}

int partial_capacity(const sam_ctx* ctx) {
    int most = 16;
    for (int r : ctx->resident) most = std::max(most, r);
    return samk::kMaxBuckets * ctx->CUs * most;
}

namespace {

struct PlanTemps {
    int* counts;
    int64_t* off;
    void* stemp;
};

void plan_temp_layout(Carve& cv, int n, PlanTemps* t) {
    PlanTemps x;
    x.counts = cv.take<int>((size_t)n);
    x.off = cv.take<int64_t>((size_t)n + 1);
    x.stemp = cv.take<char>(samk::scan_temp_bytes(n));
    if (t) *t = x;
}

// The plan's arrays (pl == null: measure only).
void plan_array_layout(Carve& cv, int n, int64_t E, int nnzA0, int partcap, sam_plan* pl) {
    sam_plan dummy;
    sam_plan* p = pl ? pl : &dummy;
    p->nI = cv.take<int>((size_t)n);
    p->eoff = cv.take<int64_t>((size_t)n + 1);
    p->posA = cv.take<unsigned char>((size_t)E);
    p->posB = cv.take<unsigned char>((size_t)nnzA0);
    for (int a = 0; a < 2; ++a)
        for (int w = 0; w < 2; ++w) {
            p->combo[a][w].queue = cv.take<int>((size_t)n);
            p->combo[a][w].bstart = cv.take<int>(64);
        }
    p->colbuf = cv.take<double>((size_t)n);
    p->partcap = partcap;
    p->partbuf = cv.take<double>((size_t)partcap);
    p->rtemp = cv.take<char>(samk::reduce_temp_bytes(std::max(n, partcap)));
    p->btemp = cv.take<char>(samk::bucket_temp_bytes(n));
    p->flags = cv.take<int>(4);
}

}  // namespace

size_t plan_bytes(int n, int64_t E, int nnzA0, int partcap) {
    Carve cv(nullptr);
    plan_temp_layout(cv, n, nullptr);
    plan_array_layout(cv, n, E, nnzA0, partcap, nullptr);
    return cv.off;
}

sam_status gathered_total(sam_ctx* ctx, int n, const int32_t* S_cp, const int32_t* S_ri, const int32_t* Ak_cp,
                          int64_t* E, hipStream_t s) {
    *E = 0;
    if (n == 0) return SAM_OK;
    unsigned long long h = 0;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_total, &h, sizeof h, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, samk::plan_gather_total(n, S_cp, S_ri, Ak_cp, ctx->d_total, s));
    HIP_TRY(ctx, read_back(ctx->d_total, &h, s));
    *E = (int64_t)h;
    return SAM_OK;
}

sam_status plan_init(sam_ctx* ctx, sam_plan* pl, const sam_csc* Ak, const sam_csc* A0, const int32_t* S_colptr,
                     const int32_t* S_rowind, int64_t nnz_S, void* mem, size_t mem_bytes, hipStream_t s) {
    const int n = Ak->n;
    pl->ctx = ctx;
    pl->n = n;
    pl->nnzA = Ak->nnz;
    pl->nnzA0 = A0->nnz;
    pl->nnzS = nnz_S;
    pl->Ak_cp = Ak->colptr;
    pl->Ak_ri = Ak->rowind;
    pl->A0_cp = A0->colptr;
    pl->A0_ri = A0->rowind;
    pl->S_cp = S_colptr;
    pl->S_ri = S_rowind;
    pl->mem = mem;
    pl->mem_bytes = mem_bytes;
    Carve cv(mem);
    PlanTemps t;
    plan_temp_layout(cv, n, &t);
    const size_t temps = cv.off;
    if (mem_bytes < temps) return fail(ctx, SAM_ERR_ARG, "plan memory: %zu bytes given, more needed", mem_bytes);

    std::vector<int> hcp;
    int longest = 0;
    sam_status st;
    if ((st = host_colptr(ctx, Ak->colptr, n, Ak->nnz, "Ak", &pl->max_len_A, s))) return st;
    if ((st = host_colptr(ctx, S_colptr, n, nnz_S, "S", &longest, s, &hcp))) return st;
    // pass 1: gathered entries per column -> eoff
    int64_t E = 0;
    if (n > 0) {
        HIP_TRY(ctx, samk::plan_gather_count(n, S_colptr, S_rowind, Ak->colptr, t.counts, s));
        HIP_TRY(ctx, samk::scan_counts(t.counts, n, t.off, nullptr, nullptr, t.stemp, s));
        HIP_TRY(ctx, read_back(t.off + n, &E, s));
    }
    pl->E = E;
    // the numeric kernels address A_k, A_0 and the gathered positions with
    // 32-bit byte offsets
    if ((int64_t)Ak->nnz * 8 > (int64_t)UINT32_MAX || (int64_t)A0->nnz * 8 > (int64_t)UINT32_MAX ||
        E > (int64_t)UINT32_MAX)
        return fail(ctx, SAM_ERR_UNSUPPORTED,
                    "nnz(A_k) = %d, nnz(A_0) = %d, gathered entries = %lld: the numeric kernels need "
                    "nnz < 2^29 and fewer than 2^32 gathered entries (split the columns)",
                    Ak->nnz, A0->nnz, (long long)E);
    plan_array_layout(cv, n, E, A0->nnz, partial_capacity(ctx), pl);
    if (cv.off > mem_bytes)
        return fail(ctx, SAM_ERR_ARG, "plan memory: %zu bytes given, %zu needed", mem_bytes, cv.off);

    if (n > 0) {
        std::vector<int> hnI(n);
        HIP_TRY(ctx, hipMemcpyAsync(pl->eoff, t.off, (size_t)(n + 1) * 8, hipMemcpyDeviceToDevice, s));
        HIP_TRY(ctx, samk::plan_positions(n, S_colptr, S_rowind, Ak->colptr, Ak->rowind, A0->colptr, A0->rowind,
                                          pl->eoff, pl->nI, pl->posA, pl->posB, longest, pl->max_len_A, s));
        HIP_TRY(ctx, hipMemcpyAsync(hnI.data(), pl->nI, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        for (int j = 0; j < n; ++j) {
            pl->max_rows = std::max(pl->max_rows, hnI[j]);
            const int cj = hcp[(size_t)j + 1] - hcp[(size_t)j];
            pl->max_cols = std::max(pl->max_cols, cj);
            const double r = hnI[j], c = cj;
            // Householder QR of the r x c block (2 r c^2 - 2/3 c^3), Q^T b
            // (4 r c) and three triangular solves (3 c^2: the solution and
            // the refinement's two)
            pl->fl_qr32 += 2.0 * r * c * c - 2.0 / 3.0 * c * c * c + 4.0 * r * c + 3.0 * c * c;
            pl->fl_ref64 += 6.0 * r * c + 2.0 * r;   // r = b - Am, A^T r, final residual
            // FP64 mode: QR, Q^T b, one triangular solve, explicit residual
            pl->fl_f64 += 2.0 * r * c * c - 2.0 / 3.0 * c * c * c + 4.0 * r * c + c * c + 2.0 * r * c + 2.0 * r;
            pl->m_rc2 += r * c * c;
            pl->m_c3 += c * c * c;
            pl->m_rc += r * c;
            pl->m_c2 += c * c;
            pl->m_r += r;
        }
        for (int p = 0; p < 2; ++p)
            for (int w = 0; w < 2; ++w)
                if ((st = plan_combo(pl, p, w, s))) return st;
    }
    return SAM_OK;
}

// Launch every non-empty bucket of a combination, then the column-residual sum.
sam_status run_numeric(sam_plan* pl, const double* Ak_val, const double* A0_val, const double* w, double mu, int prec,
                       int weighted, void* M_val, double* col_res2, double* res2, hipStream_t s) {
    sam_ctx* ctx = pl->ctx;
    Combo& cb = pl->combo[prec][weighted];
    if (!cb.ok) return fail(ctx, SAM_ERR_UNSUPPORTED, "%s", cb.why.c_str());
    NumericArgs a{};
    a.n = pl->n;
    a.nnzA = (uint32_t)pl->nnzA;
    a.nnzA0 = (uint32_t)pl->nnzA0;
    a.E = (uint32_t)pl->E;
    a.Ak_cp = pl->Ak_cp;
    a.Ak_v = Ak_val;
    a.A0_cp = pl->A0_cp;
    a.A0_v = A0_val;
    a.S_cp = pl->S_cp;
    a.S_ri = pl->S_ri;
    a.nI = pl->nI;
    a.eoff = pl->eoff;
    a.posA = pl->posA;
    a.posB = pl->posB;
    a.queue = cb.queue;
    a.bstart = cb.bstart;
    a.M = M_val;
    // the column residuals go to the caller's array when asked for; the
    // Frobenius sum comes from the blocks' partial sums
    a.col_res2 = col_res2;
    a.part = res2 ? pl->partbuf : nullptr;
    a.status = ctx->d_status;
    a.w = w;
    a.mu = mu;
    int parts = 0;
    for (size_t b = 0; b < cb.variants.size(); ++b) {
        // bucket sizes: exact (plan) or an upper bound (replanned sequence,
        // where the kernel reads the actual count from bstart on the device)
        const int cnt = cb.counts[b];
        if (cnt <= 0) continue;
        const NumericVariant* v = cb.variants[b];
        a.bucket = (int)b;
        int groups = (cnt + v->per_wave() - 1) / v->per_wave();
        // one round of resident blocks for the plain maps; the weighted
        // forms run faster over two rounds (as the adjoint's launch)
        const int per_cu = weighted ? std::min(16, 2 * resident_blocks(ctx, v)) : resident_blocks(ctx, v);
        int grid = std::min(groups, ctx->CUs * per_cu);
        if (grid >= 64) grid = grid / 8 * 8;
        if (res2 && parts + grid > pl->partcap)
            return fail(ctx, SAM_ERR_HIP, "partial-sum buffer too small (%d blocks)", parts + grid);
        a.part_base = parts;
        HIP_TRY(ctx, v->launch(a, grid, s));
        parts += grid;
    }
    if (res2 && parts > 0) HIP_TRY(ctx, samk::reduce_sum(pl->partbuf, parts, res2, pl->rtemp, s));
    if (res2 && parts == 0) HIP_TRY(ctx, samk::fill_i32((int*)res2, 2, 0, s));
    return SAM_OK;
}

}  // namespace samh

namespace {

// Residual scratch: the column residuals (n doubles) and the reduction
// temporary.
size_t residual_layout(Carve& cv, int n, int nnzA0, double** cols, void** rt) {
    double* c = cv.take<double>((size_t)std::max(n, 1));
    void* r = cv.take<char>(samk::reduce_temp_bytes(std::max<int64_t>(n, nnzA0)));
    if (cols) *cols = c;
    if (rt) *rt = r;
    return cv.off;
}

// Row-view scratch of sam_apply_prepare.
struct TransposeTemps {
    int* rowcount;
    int* cursor;
    int64_t* off;
    void* stemp;
};
size_t transpose_layout(Carve& cv, int n, TransposeTemps* t) {
    TransposeTemps x;
    x.rowcount = cv.take<int>((size_t)std::max(n, 1));
    x.cursor = cv.take<int>((size_t)std::max(n, 1));
    x.off = cv.take<int64_t>((size_t)n + 1);
    x.stemp = cv.take<char>(samk::scan_temp_bytes(n));
    if (t) *t = x;
    return cv.off;
}

}  // namespace

extern "C" {

const char* sam_version(void) { return "0.2.0"; }

const char* sam_status_string(sam_status s) {
    switch (s) {
        case SAM_OK: return "SAM_OK";
        case SAM_ERR_ARG: return "SAM_ERR_ARG";
        case SAM_ERR_SHAPE: return "SAM_ERR_SHAPE";
        case SAM_ERR_UNSORTED: return "SAM_ERR_UNSORTED";
        case SAM_ERR_OVERFLOW: return "SAM_ERR_OVERFLOW";
        case SAM_ERR_RANK: return "SAM_ERR_RANK";
        case SAM_ERR_NONFINITE: return "SAM_ERR_NONFINITE";
        case SAM_ERR_HIP: return "SAM_ERR_HIP";
        case SAM_ERR_UNSUPPORTED: return "SAM_ERR_UNSUPPORTED";
        case SAM_ERR_NOMEM: return "SAM_ERR_NOMEM";
    }
    return "SAM_ERR_UNKNOWN";
}

sam_status sam_create(sam_ctx** out, int device) {
    if (!out) return SAM_ERR_ARG;
    *out = nullptr;
    sam_ctx* ctx = new (std::nothrow) sam_ctx();
    if (!ctx) return SAM_ERR_NOMEM;
    ctx->device = device;
    if (device != SAM_NO_DEVICE) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
            delete ctx;
            return SAM_ERR_HIP;
        }
        if (hipSetDevice(device) != hipSuccess) {
            delete ctx;
            return SAM_ERR_HIP;
        }
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
            ctx->CUs = prop.multiProcessorCount;
        {
            int cnt = 0;
            const samk::NumericVariant* menu = samk::numeric_menu(&cnt);
            ctx->resident.assign(cnt, 0);
            for (int i = 0; i < cnt; ++i) ctx->resident[i] = menu[i].blocks_per_cu();
        }
        // the context's status block: the only device memory the library
        // allocates itself
        if (hipMalloc(&ctx->block, kCtxBlockBytes) != hipSuccess) {
            delete ctx;
            return SAM_ERR_NOMEM;
        }
        // sam_build_noalloc's fixed array: its address on this device (a
        // failure is kept and reported by that call, which alone needs it)
        (void)scratch_setup(device);
        ctx->d_status = (unsigned long long*)ctx->block;
        ctx->d_bad = (int*)((char*)ctx->block + 64);
        ctx->d_total = (unsigned long long*)((char*)ctx->block + 128);
        unsigned long long clear = kStatusClear;
        if (hipMemcpy(ctx->d_status, &clear, sizeof clear, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(ctx->block);
            delete ctx;
            return SAM_ERR_HIP;
        }
    }
    *out = ctx;
    return SAM_OK;
}

sam_status sam_destroy(sam_ctx* ctx) {
    if (!ctx) return SAM_OK;
    if (ctx->device != SAM_NO_DEVICE) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        if (ctx->block) (void)hipFree(ctx->block);
    }
    delete ctx;
    return SAM_OK;
}

const char* sam_last_error(const sam_ctx* ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

sam_status sam_sync_status(sam_ctx* ctx, sam_stream_t stream, int32_t* first_bad_col) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    if (first_bad_col) *first_bad_col = -1;
    sam_status st = need_device(ctx);
    if (st) return st;
    unsigned long long v = kStatusClear;
    HIP_TRY(ctx, hipStreamSynchronize(S(stream)));
    HIP_TRY(ctx, hipMemcpy(&v, ctx->d_status, sizeof v, hipMemcpyDeviceToHost));
    unsigned long long clear = kStatusClear;
    HIP_TRY(ctx, hipMemcpy(ctx->d_status, &clear, sizeof clear, hipMemcpyHostToDevice));
    if (v == kStatusClear) return SAM_OK;
    const int code = (int)(v & 0xff);
    const int col = (int)(v >> 8);
    if (first_bad_col) *first_bad_col = col;
    const char* what = code == SAM_ERR_RANK        ? "numerically rank deficient column block"
                       : code == SAM_ERR_NONFINITE ? "non-finite value"
                       : code == SAM_ERR_UNSORTED  ? "index outside [0, n) in the structure"
                                                   : "kernel failure";
    return fail(ctx, (sam_status)code, "%s at column %d", what, col);
}

sam_status sam_check_csc(sam_ctx* ctx, const sam_csc* A, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st = check_csc_args(ctx, A, "A", false);
    if (st) return st;
    if ((st = need_device(ctx))) return st;
    return validate_csc(ctx, A->n, A->nnz, A->colptr, A->rowind, "A", S(stream));
}

// ---------------------------------------------------------------- pattern

sam_status sam_pattern_workspace_size(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, size_t* bytes,
                                      sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", false))) return st;
    if ((st = check_spec(ctx, spec))) return st;
    if (!bytes) return fail(ctx, SAM_ERR_ARG, "bytes is NULL");
    if ((st = need_device(ctx))) return st;
    int longest = 0;
    if ((st = host_colptr(ctx, Ak->colptr, Ak->n, Ak->nnz, "Ak", &longest, S(stream)))) return st;
    Carve cv(nullptr);
    pattern_ws_layout(cv, Ak->n, Ak->nnz, longest, spec->power, nullptr);
    *bytes = cv.off;
    return SAM_OK;
}

sam_status sam_pattern_count(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, void* ws, size_t ws_bytes,
                             int64_t* nnz_S, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", spec && spec->kind != SAM_SPARSIFY_NONE))) return st;
    if ((st = check_spec(ctx, spec))) return st;
    if (!nnz_S) return fail(ctx, SAM_ERR_ARG, "nnz_S is NULL");
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    ctx->pat.valid = false;
    int longest = 0;
    if ((st = host_colptr(ctx, Ak->colptr, Ak->n, Ak->nnz, "Ak", &longest, s))) return st;
    Carve cv(ws);
    PatternWs w;
    pattern_ws_layout(cv, Ak->n, Ak->nnz, longest, spec->power, &w);
    if ((st = check_ws(ctx, ws, ws_bytes, cv.off, "pattern workspace"))) return st;
    if ((st = validate_csc(ctx, Ak->n, Ak->nnz, Ak->colptr, Ak->rowind, "Ak", s))) return st;
    PatternResult res;
    if ((st = compute_pattern(ctx, Ak, spec, w, &res, s))) return st;
    PatternState& ps = ctx->pat;
    ps.valid = true;
    ps.ws = ws;
    ps.n = Ak->n;
    ps.nnz_A = Ak->nnz;
    ps.cp = Ak->colptr;
    ps.ri = Ak->rowind;
    ps.val = Ak->val;
    ps.spec = *spec;
    ps.power = spec->power;
    ps.res = res;
    *nnz_S = res.nnz;
    return SAM_OK;
}

sam_status sam_pattern_fill(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, void* ws, size_t ws_bytes,
                            int32_t* S_colptr, int32_t* S_rowind, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", false))) return st;
    if ((st = check_spec(ctx, spec))) return st;
    const PatternState& ps = ctx->pat;
    if (!S_colptr || (!S_rowind && ps.valid && ps.res.nnz != 0)) return fail(ctx, SAM_ERR_ARG, "output array is NULL");
    if ((st = need_device(ctx))) return st;
    (void)ws_bytes;
    if (!ps.valid || ps.ws != ws || ps.n != Ak->n || ps.nnz_A != Ak->nnz || ps.cp != Ak->colptr ||
        ps.ri != Ak->rowind || ps.val != Ak->val || memcmp(&ps.spec, spec, sizeof *spec) != 0)
        return fail(ctx, SAM_ERR_ARG,
                    "sam_pattern_fill must follow sam_pattern_count with the same Ak, spec and workspace");
    return pattern_fill(ctx, Ak->n, ps.res, S_colptr, S_rowind, S(stream));
}

// ------------------------------------------------------------------ plan

sam_status sam_plan_size(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0, const int32_t* S_colptr,
                         const int32_t* S_rowind, int64_t nnz_S, size_t* bytes, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", false))) return st;
    if ((st = check_csc_args(ctx, A0, "A0", false))) return st;
    if (Ak->n != A0->n) return fail(ctx, SAM_ERR_SHAPE, "Ak is %d x %d but A0 is %d x %d", Ak->n, Ak->n, A0->n, A0->n);
    if (Ak->n > 0 && (Ak->nnz == 0 || A0->nnz == 0))
        return fail(ctx, SAM_ERR_ARG, "Ak and A0 must have stored entries (a nonsingular source has at least n)");
    if (nnz_S < 0) return fail(ctx, SAM_ERR_ARG, "nnz_S < 0");
    if (nnz_S > INT_MAX) return fail(ctx, SAM_ERR_OVERFLOW, "nnz_S = %lld does not fit in int32", (long long)nnz_S);
    if (!S_colptr || (nnz_S > 0 && !S_rowind)) return fail(ctx, SAM_ERR_ARG, "pattern array is NULL");
    if (!bytes) return fail(ctx, SAM_ERR_ARG, "bytes is NULL");
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    const int n = Ak->n;
    if ((st = validate_csc(ctx, n, Ak->nnz, Ak->colptr, Ak->rowind, "Ak", s))) return st;
    if ((st = validate_csc(ctx, n, nnz_S, S_colptr, S_rowind, "S", s))) return st;
    int64_t E = 0;
    if ((st = gathered_total(ctx, n, S_colptr, S_rowind, Ak->colptr, &E, s))) return st;
    *bytes = plan_bytes(n, E, A0->nnz, partial_capacity(ctx));
    return SAM_OK;
}

sam_status sam_plan_create(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0, const int32_t* S_colptr,
                           const int32_t* S_rowind, int64_t nnz_S, void* mem, size_t mem_bytes, sam_plan** plan,
                           sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if (!plan) return fail(ctx, SAM_ERR_ARG, "plan is NULL");
    *plan = nullptr;
    if ((st = check_csc_args(ctx, Ak, "Ak", false))) return st;
    if ((st = check_csc_args(ctx, A0, "A0", false))) return st;
    if (Ak->n != A0->n) return fail(ctx, SAM_ERR_SHAPE, "Ak is %d x %d but A0 is %d x %d", Ak->n, Ak->n, A0->n, A0->n);
    if (Ak->n > 0 && (Ak->nnz == 0 || A0->nnz == 0))
        return fail(ctx, SAM_ERR_ARG, "Ak and A0 must have stored entries (a nonsingular source has at least n)");
    if (nnz_S < 0) return fail(ctx, SAM_ERR_ARG, "nnz_S < 0");
    if (nnz_S > INT_MAX) return fail(ctx, SAM_ERR_OVERFLOW, "nnz_S = %lld does not fit in int32", (long long)nnz_S);
    if (!S_colptr || (nnz_S > 0 && !S_rowind)) return fail(ctx, SAM_ERR_ARG, "pattern array is NULL");
    if ((st = check_ws(ctx, mem, mem_bytes, 1, "plan memory"))) return st;
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    const int n = Ak->n;
    if ((st = validate_csc(ctx, n, Ak->nnz, Ak->colptr, Ak->rowind, "Ak", s))) return st;
    if ((st = validate_csc(ctx, n, A0->nnz, A0->colptr, A0->rowind, "A0", s))) return st;
    if ((st = validate_csc(ctx, n, nnz_S, S_colptr, S_rowind, "S", s))) return st;
    sam_plan* pl = new (std::nothrow) sam_plan();
    if (!pl) return fail(ctx, SAM_ERR_NOMEM, "host allocation failed");
    if ((st = plan_init(ctx, pl, Ak, A0, S_colptr, S_rowind, nnz_S, mem, mem_bytes, s))) {
        delete pl;
        return st;
    }
    *plan = pl;
    return SAM_OK;
}

sam_status sam_plan_destroy(sam_plan* plan) {
    if (!plan) return SAM_OK;
    if (plan->ctx && plan->ctx->device != SAM_NO_DEVICE) {
        (void)hipSetDevice(plan->ctx->device);
        (void)hipDeviceSynchronize();   // no launch on the plan's memory is still running
    }
    delete plan;
    return SAM_OK;
}

sam_status sam_plan_cost(const sam_plan* plan, int32_t prec, double* flops32, double* flops64,
                         double* bytes) {
    if (!plan || !prec_ok(prec)) return SAM_ERR_ARG;
    const bool f32 = prec == SAM_PREC_F32_REFINE;
    if (flops32) *flops32 = f32 ? plan->fl_qr32 : 0.0;
    if (flops64) *flops64 = f32 ? plan->fl_ref64 : plan->fl_f64;
    if (bytes) {
        const double vb = f32 ? 4.0 : 8.0;
        *bytes = 12.0 * plan->nnzA + 12.0 * plan->nnzA0 + 4.0 * (double)plan->nnzS + 12.0 * (plan->n + 1.0) +
                 vb * (double)plan->nnzS + 8.0 * plan->n;
    }
    return SAM_OK;
}

sam_status sam_plan_cost_weighted(const sam_plan* plan, int32_t prec, int32_t backward, double* flops32,
                                  double* flops64) {
    if (!plan || !prec_ok(prec) || (backward != 0 && backward != 1)) return SAM_ERR_ARG;
    const bool f32 = prec == SAM_PREC_F32_REFINE;
    const double nS = (double)plan->nnzS;
    // QR of the stacked (r + c) x c block and Q^T b, then one triangular
    // solve; FP32 + refinement adds one step of two solves (FP32) and of
    // r = b - A m, ||r||^2, A^T r and P m (FP64)
    const double qr = 2.0 * (plan->m_rc2 + plan->m_c3) - 2.0 / 3.0 * plan->m_c3 + 4.0 * (plan->m_rc + plan->m_c2);
    double q32 = f32 ? qr + 3.0 * plan->m_c2 : 0.0;
    double q64 = f32 ? 4.0 * plan->m_rc + 2.0 * plan->m_r + 2.0 * nS : qr + plan->m_c2;
    if (backward) {
        // lambda: two normal-equation solves (one refinement step), the
        // residual and A^T r, one scatter/gather pair, the final A lambda,
        // and five flops per gathered entry for the contributions
        const double s32 = 4.0 * plan->m_c2;
        const double s64 = 10.0 * plan->m_rc + 3.0 * nS + 5.0 * (double)plan->E;
        if (f32) {
            q32 += s32;
            q64 += s64;
        } else {
            q64 += s32 + s64;
        }
    }
    if (flops32) *flops32 = q32;
    if (flops64) *flops64 = q64;
    return SAM_OK;
}

sam_status sam_plan_info(const sam_plan* plan, int32_t* n, int32_t* max_rows, int32_t* max_cols, int64_t* gathered,
                         int32_t* nbuckets, int32_t* bucket_cols) {
    if (!plan) return SAM_ERR_ARG;
    if (n) *n = plan->n;
    if (max_rows) *max_rows = plan->max_rows;
    if (max_cols) *max_cols = plan->max_cols;
    if (gathered) *gathered = plan->E;
    const Combo& cb = plan->combo[1][0];
    if (nbuckets) *nbuckets = (int)cb.counts.size();
    if (bucket_cols)
        for (size_t b = 0; b < cb.counts.size() && b < 16; ++b) bucket_cols[b] = cb.counts[b];
    return SAM_OK;
}

// ------------------------------------------------------------------ build

sam_status sam_build_planned(sam_plan* plan, const double* Ak_val, const double* A0_val, int32_t prec,
                             void* M_val, double* col_res2, double* res2, sam_stream_t stream) {
    if (!plan || !plan->ctx) return SAM_ERR_ARG;
    sam_ctx* ctx = plan->ctx;
    check_ctx(ctx);
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if ((plan->nnzA > 0 && !Ak_val) || (plan->nnzA0 > 0 && !A0_val)) return fail(ctx, SAM_ERR_ARG, "value array is NULL");
    if (plan->nnzS > 0 && !M_val) return fail(ctx, SAM_ERR_ARG, "M_val is NULL");
    sam_status st = need_device(ctx);
    if (st) return st;
    return run_numeric(plan, Ak_val, A0_val, nullptr, 0.0, prec == SAM_PREC_F32_REFINE ? 1 : 0, 0, M_val, col_res2,
                       res2, S(stream));
}

sam_status sam_workspace_size(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0, const int32_t* S_colptr,
                              const int32_t* S_rowind, int64_t nnz_S, int32_t prec, size_t* bytes,
                              sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    return sam_plan_size(ctx, Ak, A0, S_colptr, S_rowind, nnz_S, bytes, stream);
}

sam_status sam_build(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0, const int32_t* S_colptr,
                     const int32_t* S_rowind, int64_t nnz_S, int32_t prec, void* M_val, double* col_res2,
                     double* res2, void* ws, size_t ws_bytes, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", true))) return st;
    if ((st = check_csc_args(ctx, A0, "A0", true))) return st;
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if (nnz_S > 0 && !M_val) return fail(ctx, SAM_ERR_ARG, "M_val is NULL");
    sam_plan* pl = nullptr;
    if ((st = sam_plan_create(ctx, Ak, A0, S_colptr, S_rowind, nnz_S, ws, ws_bytes, &pl, stream))) return st;
    st = sam_build_planned(pl, Ak->val, A0->val, prec, M_val, col_res2, res2, stream);
    delete pl;   // host record only: the launches hold their arguments by value
    return st;
}

// --------------------------------------------------------------- residual

sam_status sam_residual_workspace_size(int32_t n, int32_t nnz_A0, size_t* bytes) {
    if (n < 0 || nnz_A0 < 0 || !bytes) return SAM_ERR_ARG;
    Carve cv(nullptr);
    *bytes = residual_layout(cv, n, nnz_A0, nullptr, nullptr);
    return SAM_OK;
}

sam_status sam_residual(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0, const int32_t* M_colptr,
                        const int32_t* M_rowind, int64_t nnz_M, const void* M_val, int32_t prec, double* res2,
                        double* a02, void* ws, size_t ws_bytes, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", true))) return st;
    if ((st = check_csc_args(ctx, A0, "A0", true))) return st;
    if (Ak->n != A0->n) return fail(ctx, SAM_ERR_SHAPE, "Ak and A0 differ in order");
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if (!M_colptr || (nnz_M > 0 && (!M_rowind || !M_val)) || !res2) return fail(ctx, SAM_ERR_ARG, "NULL argument");
    if (nnz_M < 0 || nnz_M > INT_MAX) return fail(ctx, SAM_ERR_OVERFLOW, "nnz_M out of range");
    const int n = Ak->n;
    Carve cv(ws);
    double* cols = nullptr;
    void* rt = nullptr;
    if ((st = check_ws(ctx, ws, ws_bytes, residual_layout(cv, n, A0->nnz, &cols, &rt), "residual workspace")))
        return st;
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    if (n == 0) {
        HIP_TRY(ctx, samk::fill_i32((int*)res2, 2, 0, s));
        if (a02) HIP_TRY(ctx, samk::fill_i32((int*)a02, 2, 0, s));
        return SAM_OK;
    }
    HIP_TRY(ctx, samk::residual_columns(n, Ak->colptr, Ak->rowind, Ak->val, A0->colptr, A0->rowind, A0->val, M_colptr,
                                        M_rowind, M_val, prec == SAM_PREC_F32_REFINE, cols, ctx->d_status, s));
    HIP_TRY(ctx, samk::reduce_sum(cols, n, res2, rt, s));
    if (a02) HIP_TRY(ctx, samk::reduce_sumsq(A0->val, A0->nnz, a02, rt, s));
    return SAM_OK;
}

// ------------------------------------------------------------------ apply

sam_status sam_apply_workspace_size(int32_t n, size_t* bytes) {
    if (n < 0 || !bytes) return SAM_ERR_ARG;
    Carve cv(nullptr);
    *bytes = transpose_layout(cv, n, nullptr);
    return SAM_OK;
}

sam_status sam_apply_prepare(sam_ctx* ctx, int32_t n, const int32_t* M_colptr, const int32_t* M_rowind, int64_t nnz,
                             int32_t* T_rowptr, int32_t* T_colind, int32_t* T_perm, void* ws, size_t ws_bytes,
                             sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    if (n < 0 || nnz < 0) return fail(ctx, SAM_ERR_ARG, "negative size");
    if (nnz > INT_MAX) return fail(ctx, SAM_ERR_OVERFLOW, "nnz does not fit in int32");
    if (!M_colptr || !T_rowptr || (nnz > 0 && (!M_rowind || !T_colind || !T_perm)))
        return fail(ctx, SAM_ERR_ARG, "NULL argument");
    Carve cv(ws);
    TransposeTemps t;
    sam_status st;
    if ((st = check_ws(ctx, ws, ws_bytes, transpose_layout(cv, n, &t), "apply workspace"))) return st;
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    if ((st = validate_csc(ctx, n, nnz, M_colptr, M_rowind, "M", s))) return st;
    HIP_TRY(ctx, samk::fill_i32(t.rowcount, std::max(n, 1), 0, s));
    HIP_TRY(ctx, samk::fill_i32(t.cursor, std::max(n, 1), 0, s));
    HIP_TRY(ctx, samk::transpose_count(n, M_colptr, M_rowind, nnz, t.rowcount, s));
    HIP_TRY(ctx, samk::scan_counts(t.rowcount, n, t.off, T_rowptr, nullptr, t.stemp, s));
    HIP_TRY(ctx, samk::transpose_fill(n, M_colptr, M_rowind, T_rowptr, t.cursor, T_colind, T_perm, s));
    HIP_TRY(ctx, samk::transpose_sort_rows(n, T_rowptr, T_colind, T_perm, s));
    return SAM_OK;
}

sam_status sam_apply_permute(sam_ctx* ctx, int64_t nnz, const int32_t* T_perm, const void* M_val, int32_t prec,
                             void* T_val, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    if (nnz < 0) return fail(ctx, SAM_ERR_ARG, "negative size");
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if (nnz > 0 && (!T_perm || !M_val || !T_val)) return fail(ctx, SAM_ERR_ARG, "NULL argument");
    sam_status st = need_device(ctx);
    if (st) return st;
    HIP_TRY(ctx, samk::permute_vals(nnz, T_perm, M_val, prec == SAM_PREC_F32_REFINE, T_val, S(stream)));
    return SAM_OK;
}

sam_status sam_apply(sam_ctx* ctx, int32_t n, const int32_t* T_rowptr, const int32_t* T_colind, const int32_t* T_perm,
                     const void* M_val, int32_t prec, const double* x, double* y, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    if (n < 0) return fail(ctx, SAM_ERR_ARG, "negative size");
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if (n > 0 && (!T_rowptr || !T_colind || !M_val || !x || !y)) return fail(ctx, SAM_ERR_ARG, "NULL argument");
    sam_status st = need_device(ctx);
    if (st) return st;
    HIP_TRY(ctx, samk::spmv_rows(n, T_rowptr, T_colind, T_perm, M_val, prec == SAM_PREC_F32_REFINE, x, y, S(stream)));
    return SAM_OK;
}

sam_status sam_build_weighted(sam_plan* plan, const double* Ak_val, const double* A0_val, const double* w, double mu,
                              int32_t prec, void* M_val, double* col_res2, double* res2, sam_stream_t stream) {
    if (!plan || !plan->ctx) return SAM_ERR_ARG;
    sam_ctx* ctx = plan->ctx;
    check_ctx(ctx);
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if ((plan->nnzA > 0 && !Ak_val) || (plan->nnzA0 > 0 && !A0_val)) return fail(ctx, SAM_ERR_ARG, "value array is NULL");
    if (plan->nnzS > 0 && (!M_val || !w)) return fail(ctx, SAM_ERR_ARG, "M_val or w is NULL");
    if (!(mu >= 0.0)) return fail(ctx, SAM_ERR_ARG, "mu must be >= 0 (got %g)", mu);
    sam_status st = need_device(ctx);
    if (st) return st;
    return run_numeric(plan, Ak_val, A0_val, w, mu, prec == SAM_PREC_F32_REFINE ? 1 : 0, 1, M_val, col_res2, res2,
                       S(stream));
}

}  // extern "C"

// ------------------------------------------------------------- variants

namespace samh {

std::vector<const NumericVariant*> menu_subset(int prec, int weighted, const int32_t* order, int32_t count,
                                               bool* ok) {
    std::vector<const NumericVariant*> all, out;
    menu_table(prec, weighted, &all);
    *ok = count >= 1 && count <= samk::kMaxBuckets && order != nullptr;
    for (int32_t i = 0; *ok && i < count; ++i) {
        if (order[i] < 0 || order[i] >= (int32_t)all.size()) *ok = false;
        else out.push_back(all[order[i]]);
    }
    return out;
}

sam_status plan_select(sam_plan* pl, int prec, const std::vector<const NumericVariant*>& vars, hipStream_t s) {
    sam_ctx* ctx = pl->ctx;
    Combo& cb = pl->combo[prec][0];
    const std::vector<const NumericVariant*> previous = cb.variants;
    sam_status st = plan_combo_with(pl, prec, 0, vars, s);
    if (st) return st;
    if (!cb.ok) {
        const std::string why = cb.why;
        st = plan_combo_with(pl, prec, 0, previous, s);
        if (st) return st;
        return fail(ctx, SAM_ERR_UNSUPPORTED, "selection rejected: %s", why.c_str());
    }
    return SAM_OK;
}

}  // namespace samh

extern "C" {

sam_status sam_menu(int32_t prec, int32_t weighted, int32_t capacity, int32_t* count, int32_t* G, int32_t* R,
                    int32_t* NC, int32_t* TC) {
    if (!prec_ok(prec) || (weighted != 0 && weighted != 1) || !count || capacity < 0) return SAM_ERR_ARG;
    std::vector<const NumericVariant*> all;
    menu_table(prec == SAM_PREC_F32_REFINE ? 1 : 0, weighted, &all);
    *count = (int32_t)all.size();
    for (int32_t i = 0; i < capacity && i < (int32_t)all.size(); ++i) {
        if (G) G[i] = all[i]->G;
        if (R) R[i] = all[i]->R;
        if (NC) NC[i] = all[i]->NC;
        if (TC) TC[i] = all[i]->TC;
    }
    return SAM_OK;
}

sam_status sam_plan_select(sam_plan* plan, int32_t prec, const int32_t* order, int32_t count,
                           sam_stream_t stream) {
    if (!plan || !plan->ctx) return SAM_ERR_ARG;
    sam_ctx* ctx = plan->ctx;
    check_ctx(ctx);
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    const int pi = prec == SAM_PREC_F32_REFINE ? 1 : 0;
    bool ok = false;
    std::vector<const NumericVariant*> vars = menu_subset(pi, 0, order, count, &ok);
    if (!ok) return fail(ctx, SAM_ERR_ARG, "variant order must list 1..%d valid menu indices", samk::kMaxBuckets);
    sam_status st = need_device(ctx);
    if (st) return st;
    if (plan->n == 0) return SAM_OK;
    return plan_select(plan, pi, vars, S(stream));
}

}  // extern "C"
