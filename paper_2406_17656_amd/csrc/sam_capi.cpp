// sam_capi.cpp -- host implementation of the C ABI declared in include/sam.h:
// argument validation, context / pattern / plan objects, device memory
// management and the launch sequence of the gfx950 kernels.
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




hipError_t grow(DevBuf& b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = std::max<size_t>(align256(bytes), 256);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.bytes = want;
    return hipSuccess;
}

void release(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
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

samk::SparsifySpec to_sp(const sam_pattern_spec* spec) {
    samk::SparsifySpec sp;
    sp.kind = spec->kind;
    sp.thresh = spec->thresh;
    sp.global_scale = spec->global_scale;
    sp.tau = spec->tau;
    sp.lfil = spec->lfil;
    return sp;
}



// Pattern pipeline: B = sparsify(A_k) (diagonal added), then S = B, and
// p-1 times S <- expand(S, B).  Produces device arrays into out_cp/out_ri
// (grown as needed) and the host nnz.
sam_status compute_pattern(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, DevBuf& out_cp,
                           DevBuf& out_ri, int64_t* nnz_out, hipStream_t s, PatternLevels* levels) {
    const int n = Ak->n;
    const size_t cp_bytes = (size_t)(n + 1) * 4;
    DevBuf* levels_cp = levels ? levels->cp : nullptr;
    if (levels) {
        levels->nnz.clear();
        levels->maxcol.clear();
    }
    if (levels_cp) HIP_TRY(ctx, grow(*levels_cp, cp_bytes * (size_t)std::max(spec->power, 1)));
    auto keep_level = [&](int lev, const int* cp) {
        return levels_cp ? hipMemcpyAsync((char*)levels_cp->p + cp_bytes * lev, cp, cp_bytes,
                                          hipMemcpyDeviceToDevice, s)
                         : hipSuccess;
    };
    samk::SparsifySpec sp = to_sp(spec);
    // workspace: counts (n int), scan out (n+1 int64), scan temp, D (n double),
    // B_cp (n+1), B_ri (nnz+n), flags (overflow, bad column, longest column)
    const size_t nnzB_bound = (size_t)Ak->nnz + (size_t)n;
    size_t need = align256((size_t)n * 4) + align256((size_t)(n + 1) * 8) + align256(samk::scan_temp_bytes(n)) +
                  align256((size_t)n * 8) + align256((size_t)(n + 1) * 4) + align256(nnzB_bound * 4) + 512;
    HIP_TRY(ctx, grow(ctx->ws, need));
    Carve cv(ctx->ws.p);
    int* counts = cv.take<int>(n);
    int64_t* off = cv.take<int64_t>(n + 1);
    void* stemp = cv.take<char>(samk::scan_temp_bytes(n));
    double* D = cv.take<double>(n);
    int* B_cp = cv.take<int>(n + 1);
    int* B_ri = cv.take<int>(nnzB_bound);
    int* flags = cv.take<int>(3);  // [0] overflow, [1] bad column, [2] longest column of the last level
    const int init[3] = {0, n, 0};
    HIP_TRY(ctx, hipMemcpyAsync(flags, init, sizeof init, hipMemcpyHostToDevice, s));
    if (n == 0) {
        HIP_TRY(ctx, grow(out_cp, sizeof(int)));
        HIP_TRY(ctx, hipMemsetAsync(out_cp.p, 0, sizeof(int), s));
        *nnz_out = 0;
        HIP_TRY(ctx, hipStreamSynchronize(s));
        return SAM_OK;
    }
    // total and longest column of the level just counted
    auto level_facts = [&](int64_t* tot, int* maxc) {
        hipError_t e = hipMemcpyAsync(tot, off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(maxc, flags + 2, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    };
    HIP_TRY(ctx, samk::sparsify_count(n, Ak->colptr, Ak->rowind, Ak->val, sp, D, counts, s));
    HIP_TRY(ctx, samk::scan_counts(counts, n, off, B_cp, flags, stemp, s, flags + 2));
    HIP_TRY(ctx, samk::sparsify_fill(n, Ak->colptr, Ak->rowind, Ak->val, sp, D, B_cp, B_ri, s));
    HIP_TRY(ctx, keep_level(0, B_cp));
    int64_t nnzB = 0;
    int maxB = 0;
    HIP_TRY(ctx, level_facts(&nnzB, &maxB));
    if (levels) {
        levels->nnz.push_back(nnzB);
        levels->maxcol.push_back(maxB);
    }
    const int* cur_cp = B_cp;
    const int* cur_ri = B_ri;
    int64_t cur_nnz = nnzB;
    int cur_max = maxB;
    DevBuf level_cp, level_ri;  // alternating level buffers
    DevBuf level_cp2, level_ri2;
    for (int lev = 1; lev < spec->power; ++lev) {
        HIP_TRY(ctx, samk::expand_count(n, cur_cp, cur_ri, B_cp, B_ri, counts, flags + 1, cur_max, s));
        HIP_TRY(ctx, hipMemsetAsync(flags + 2, 0, sizeof(int), s));
        HIP_TRY(ctx, samk::scan_counts(counts, n, off, nullptr, flags, stemp, s, flags + 2));
        int64_t tot = 0;
        int tmax = 0;
        HIP_TRY(ctx, level_facts(&tot, &tmax));
        if (tot > INT_MAX) {
            release(level_cp); release(level_ri); release(level_cp2); release(level_ri2);
            return fail(ctx, SAM_ERR_OVERFLOW, "pattern level %d has %lld entries (>= 2^31)", lev + 1, (long long)tot);
        }
        DevBuf& ncp = (lev & 1) ? level_cp : level_cp2;
        DevBuf& nri = (lev & 1) ? level_ri : level_ri2;
        HIP_TRY(ctx, grow(ncp, (size_t)(n + 1) * 4));
        HIP_TRY(ctx, grow(nri, (size_t)std::max<int64_t>(tot, 1) * 4));
        HIP_TRY(ctx, samk::scan_counts(counts, n, off, (int*)ncp.p, flags, stemp, s));
        HIP_TRY(ctx, samk::expand_fill(n, cur_cp, cur_ri, B_cp, B_ri, (int*)ncp.p, (int*)nri.p, cur_max, maxB, s));
        HIP_TRY(ctx, keep_level(lev, (const int*)ncp.p));
        cur_cp = (int*)ncp.p;
        cur_ri = (int*)nri.p;
        cur_nnz = tot;
        cur_max = tmax;
        if (levels) {
            levels->nnz.push_back(tot);
            levels->maxcol.push_back(tmax);
        }
    }
    int hflags[2] = {0, n};
    HIP_TRY(ctx, hipMemcpyAsync(hflags, flags, sizeof hflags, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    sam_status st = SAM_OK;
    if (hflags[1] != n) st = fail(ctx, SAM_ERR_UNSORTED, "column %d references a column index outside [0, n)", hflags[1]);
    else if (hflags[0]) st = fail(ctx, SAM_ERR_OVERFLOW, "pattern size does not fit in int32");
    if (st == SAM_OK) {
        HIP_TRY(ctx, grow(out_cp, (size_t)(n + 1) * 4));
        HIP_TRY(ctx, grow(out_ri, (size_t)std::max<int64_t>(cur_nnz, 1) * 4));
        HIP_TRY(ctx, hipMemcpyAsync(out_cp.p, cur_cp, (size_t)(n + 1) * 4, hipMemcpyDeviceToDevice, s));
        if (cur_nnz > 0)
            HIP_TRY(ctx, hipMemcpyAsync(out_ri.p, cur_ri, (size_t)cur_nnz * 4, hipMemcpyDeviceToDevice, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        *nnz_out = cur_nnz;
    }
    release(level_cp); release(level_ri); release(level_cp2); release(level_ri2);
    return st;
}


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

sam_status plan_combo(sam_plan* pl, int prec, int weighted, void* temp, int* unfit_d, hipStream_t s) {
    std::vector<const NumericVariant*> vars;
    menu_table(prec, weighted, &vars);
    return plan_combo_with(pl, prec, weighted, vars, temp, unfit_d, s);
}

sam_status plan_combo_with(sam_plan* pl, int prec, int weighted, const std::vector<const NumericVariant*>& vars,
                           void* temp, int* unfit_d, hipStream_t s) {
    sam_ctx* ctx = pl->ctx;
    Combo& cb = pl->combo[prec][weighted];
    cb.variants = vars;
    if (cb.variants.size() > (size_t)samk::kMaxBuckets) cb.variants.resize(samk::kMaxBuckets);
    BucketTable tab = table_of(cb.variants, weighted);
    cb.tab = tab;
    HIP_TRY(ctx, hipMemsetAsync(unfit_d, 0, sizeof(int), s));
    HIP_TRY(ctx, samk::bucket_sort(pl->n, pl->S_cp, pl->nI, tab, cb.queue, cb.bstart, unfit_d, nullptr, temp, s));
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
        int grid = std::min(groups, ctx->CUs * resident_blocks(ctx, v));
        if (grid >= 64) grid = grid / 8 * 8;
        if (res2 && parts + grid > pl->partcap)
            return fail(ctx, SAM_ERR_HIP, "partial-sum buffer too small (%d blocks)", parts + grid);
        a.part_base = parts;
        HIP_TRY(ctx, v->launch(a, grid, s));
        parts += grid;
    }
    if (res2 && parts > 0) HIP_TRY(ctx, samk::reduce_sum(pl->partbuf, parts, res2, pl->rtemp, s));
    if (res2 && parts == 0) HIP_TRY(ctx, hipMemsetAsync(res2, 0, sizeof(double), s));
    return SAM_OK;
}

}  // namespace samh

extern "C" {

const char* sam_version(void) { return "0.1.0"; }

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
        if (hipMalloc(&ctx->d_status, sizeof(unsigned long long)) != hipSuccess) {
            delete ctx;
            return SAM_ERR_NOMEM;
        }
        unsigned long long clear = kStatusClear;
        if (hipMemcpy(ctx->d_status, &clear, sizeof clear, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(ctx->d_status);
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
        if (ctx->d_status) (void)hipFree(ctx->d_status);
        release(ctx->ws);
        release(ctx->S_cp);
        release(ctx->S_ri);
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
    hipStream_t s = S(stream);
    HIP_TRY(ctx, grow(ctx->ws, 256));
    int* bad = (int*)ctx->ws.p;
    int h = A->n;
    HIP_TRY(ctx, hipMemcpyAsync(bad, &h, sizeof h, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, samk::check_csc(A->n, A->nnz, A->colptr, A->rowind, bad, s));
    HIP_TRY(ctx, hipMemcpyAsync(&h, bad, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (h != A->n) return fail(ctx, SAM_ERR_UNSORTED, "invalid CSC structure at column %d", h);
    return SAM_OK;
}

sam_status sam_pattern_count(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, int64_t* nnz_S,
                             sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", spec && spec->kind != SAM_SPARSIFY_NONE))) return st;
    if ((st = check_spec(ctx, spec))) return st;
    if (!nnz_S) return fail(ctx, SAM_ERR_ARG, "nnz_S is NULL");
    if ((st = need_device(ctx))) return st;
    ctx->S_nnz = -1;
    int64_t nnz = 0;
    st = compute_pattern(ctx, Ak, spec, ctx->S_cp, ctx->S_ri, &nnz, S(stream));
    if (st) return st;
    ctx->S_nnz = nnz;
    ctx->S_n = Ak->n;
    ctx->key_cp = Ak->colptr;
    ctx->key_ri = Ak->rowind;
    ctx->key_val = Ak->val;
    ctx->key_spec = *spec;
    *nnz_S = nnz;
    return SAM_OK;
}

sam_status sam_pattern_fill(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, int32_t* S_colptr,
                            int32_t* S_rowind, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", false))) return st;
    if ((st = check_spec(ctx, spec))) return st;
    if (!S_colptr || (!S_rowind && ctx->S_nnz != 0)) return fail(ctx, SAM_ERR_ARG, "output array is NULL");
    if ((st = need_device(ctx))) return st;
    if (ctx->S_nnz < 0 || ctx->S_n != Ak->n || ctx->key_cp != Ak->colptr || ctx->key_ri != Ak->rowind ||
        ctx->key_val != Ak->val || memcmp(&ctx->key_spec, spec, sizeof *spec) != 0)
        return fail(ctx, SAM_ERR_ARG, "sam_pattern_fill must follow sam_pattern_count with the same Ak and spec");
    hipStream_t s = S(stream);
    HIP_TRY(ctx, hipMemcpyAsync(S_colptr, ctx->S_cp.p, (size_t)(Ak->n + 1) * 4, hipMemcpyDeviceToDevice, s));
    if (ctx->S_nnz > 0)
        HIP_TRY(ctx, hipMemcpyAsync(S_rowind, ctx->S_ri.p, (size_t)ctx->S_nnz * 4, hipMemcpyDeviceToDevice, s));
    return SAM_OK;
}

sam_status sam_plan_create(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0, const int32_t* S_colptr,
                           const int32_t* S_rowind, int64_t nnz_S, sam_plan** plan, sam_stream_t stream) {
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
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    const int n = Ak->n;

    sam_plan* pl = new (std::nothrow) sam_plan();
    if (!pl) return fail(ctx, SAM_ERR_NOMEM, "host allocation failed");
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
    auto bail = [&](sam_status code) {
        release(pl->mem);
        delete pl;
        return code;
    };

    // pass 1: gathered entries per column -> eoff (host needs E)
    size_t tmp_need = align256((size_t)n * 4) + align256((size_t)(n + 1) * 8) + align256(samk::scan_temp_bytes(n)) +
                      align256(samk::bucket_temp_bytes(n)) + 1024;
    hipError_t he = grow(ctx->ws, tmp_need);
    if (he != hipSuccess) return bail(fail(ctx, SAM_ERR_NOMEM, "workspace: %s", hipGetErrorString(he)));
    Carve tw(ctx->ws.p);
    int* counts = tw.take<int>(n);
    int64_t* off = tw.take<int64_t>(n + 1);
    void* stemp = tw.take<char>(samk::scan_temp_bytes(n));
    void* btemp = tw.take<char>(samk::bucket_temp_bytes(n));
    int* flags = tw.take<int>(4);

    // S's column pointers are checked on the host before any kernel reads S;
    // the longest column of A_k sizes the positions launch
    std::vector<int> hcp((size_t)n + 1, 0);
    int longest = 0;
    if (n > 0) {
        std::vector<int> hak((size_t)n + 1);
        if ((he = hipMemcpyAsync(hak.data(), Ak->colptr, hak.size() * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (he = hipStreamSynchronize(s)) != hipSuccess)
            return bail(fail(ctx, SAM_ERR_HIP, "reading Ak colptr: %s", hipGetErrorString(he)));
        for (int j = 0; j < n; ++j) pl->max_len_A = std::max(pl->max_len_A, hak[(size_t)j + 1] - hak[(size_t)j]);
        if ((he = hipMemcpyAsync(hcp.data(), S_colptr, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (he = hipStreamSynchronize(s)) != hipSuccess)
            return bail(fail(ctx, SAM_ERR_HIP, "reading S_colptr: %s", hipGetErrorString(he)));
        if (hcp[0] != 0 || hcp[n] != nnz_S)
            return bail(fail(ctx, SAM_ERR_SHAPE, "S_colptr[0] = %d, S_colptr[n] = %d but nnz_S = %lld", hcp[0], hcp[n],
                             (long long)nnz_S));
        for (int j = 0; j < n; ++j) {
            if (hcp[j + 1] < hcp[j])
                return bail(fail(ctx, SAM_ERR_UNSORTED, "S_colptr decreases at column %d", j));
            longest = std::max(longest, hcp[j + 1] - hcp[j]);
        }
    }
    int64_t E = 0;
    if (n > 0) {
        if ((he = samk::plan_gather_count(n, S_colptr, S_rowind, Ak->colptr, counts, s)) != hipSuccess ||
            (he = samk::scan_counts(counts, n, off, nullptr, nullptr, stemp, s)) != hipSuccess ||
            (he = read_back(off + n, &E, s)) != hipSuccess)
            return bail(fail(ctx, SAM_ERR_HIP, "plan count: %s", hipGetErrorString(he)));
    }
    pl->E = E;
    // the numeric kernels address A_k, A_0 and the gathered positions with
    // 32-bit byte offsets
    if ((int64_t)Ak->nnz * 8 > (int64_t)UINT32_MAX || (int64_t)A0->nnz * 8 > (int64_t)UINT32_MAX ||
        E > (int64_t)UINT32_MAX)
        return bail(fail(ctx, SAM_ERR_UNSUPPORTED,
                         "nnz(A_k) = %d, nnz(A_0) = %d, gathered entries = %lld: the numeric kernels need "
                         "nnz < 2^29 and fewer than 2^32 gathered entries (split the columns)",
                         Ak->nnz, A0->nnz, (long long)E));
    size_t mem = align256((size_t)n * 4) + align256((size_t)(n + 1) * 8) + align256((size_t)std::max<int64_t>(E, 1)) +
                 align256((size_t)std::max(A0->nnz, 1)) + 4 * (align256((size_t)n * 4) + align256(64 * 4)) +
                 align256((size_t)n * 8) + align256((size_t)partial_capacity(ctx) * 8) +
                 align256(samk::reduce_temp_bytes(std::max(n, partial_capacity(ctx)))) + 1024;
    if ((he = grow(pl->mem, mem)) != hipSuccess)
        return bail(fail(ctx, SAM_ERR_NOMEM, "plan memory (%zu bytes): %s", mem, hipGetErrorString(he)));
    Carve cv(pl->mem.p);
    pl->nI = cv.take<int>(n);
    pl->eoff = cv.take<int64_t>(n + 1);
    pl->posA = cv.take<unsigned char>((size_t)std::max<int64_t>(E, 1));
    pl->posB = cv.take<unsigned char>((size_t)std::max(A0->nnz, 1));
    for (int p = 0; p < 2; ++p)
        for (int w = 0; w < 2; ++w) {
            pl->combo[p][w].queue = cv.take<int>(n);
            pl->combo[p][w].bstart = cv.take<int>(64);
        }
    pl->colbuf = cv.take<double>(n);
    pl->partcap = partial_capacity(ctx);
    pl->partbuf = cv.take<double>((size_t)pl->partcap);
    pl->rtemp = cv.take<char>(samk::reduce_temp_bytes(std::max(n, pl->partcap)));

    if (n > 0) {
        std::vector<int> hnI(n);
        if ((he = hipMemcpyAsync(pl->eoff, off, (size_t)(n + 1) * 8, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
            (he = samk::plan_positions(n, S_colptr, S_rowind, Ak->colptr, Ak->rowind, A0->colptr, A0->rowind,
                                       pl->eoff, pl->nI, pl->posA, pl->posB, longest, pl->max_len_A, s)) !=
                hipSuccess)
            return bail(fail(ctx, SAM_ERR_HIP, "plan positions: %s", hipGetErrorString(he)));
        if ((he = hipMemcpyAsync(hnI.data(), pl->nI, (size_t)n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (he = hipStreamSynchronize(s)) != hipSuccess)
            return bail(fail(ctx, SAM_ERR_HIP, "plan stats: %s", hipGetErrorString(he)));
        for (int j = 0; j < n; ++j) {
            pl->max_rows = std::max(pl->max_rows, hnI[j]);
            pl->max_cols = std::max(pl->max_cols, hcp[j + 1] - hcp[j]);
            const double r = hnI[j], c = hcp[j + 1] - hcp[j];
            // Householder QR of the r x c block, Q^T b and back substitution
            const double qr = 2.0 * r * c * c - 2.0 / 3.0 * c * c * c + 4.0 * r * c - 2.0 * c * c + c * c;
            pl->fl_qr32 += qr + 2.0 * c * c;              // + two triangular solves of the refinement
            pl->fl_ref64 += 6.0 * r * c + 2.0 * r;         // r = b - Am, A^T r, final residual
            pl->fl_f64 += qr + 2.0 * r * c + 2.0 * r;      // FP64 mode: explicit residual
        }
        for (int p = 0; p < 2; ++p)
            for (int w = 0; w < 2; ++w)
                if ((st = plan_combo(pl, p, w, btemp, flags, s))) return bail(st);
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
    release(plan->mem);
    release(plan->bwd);
    delete plan;
    return SAM_OK;
}

sam_status sam_plan_cost(const sam_plan* plan, sam_precision prec, double* flops32, double* flops64,
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

}  // extern "C"


extern "C" {

sam_status sam_build_planned(sam_plan* plan, const double* Ak_val, const double* A0_val, sam_precision prec,
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

sam_status sam_build(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0, const int32_t* S_colptr,
                     const int32_t* S_rowind, int64_t nnz_S, sam_precision prec, void* M_val, double* col_res2,
                     double* res2, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", true))) return st;
    if ((st = check_csc_args(ctx, A0, "A0", true))) return st;
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if (nnz_S > 0 && !M_val) return fail(ctx, SAM_ERR_ARG, "M_val is NULL");
    sam_plan* pl = nullptr;
    if ((st = sam_plan_create(ctx, Ak, A0, S_colptr, S_rowind, nnz_S, &pl, stream))) return st;
    st = sam_build_planned(pl, Ak->val, A0->val, prec, M_val, col_res2, res2, stream);
    hipError_t e = hipStreamSynchronize(S(stream));
    sam_plan_destroy(pl);
    if (st) return st;
    if (e != hipSuccess) return fail(ctx, SAM_ERR_HIP, "sam_build: %s", hipGetErrorString(e));
    return SAM_OK;
}

sam_status sam_residual(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0, const int32_t* M_colptr,
                        const int32_t* M_rowind, int64_t nnz_M, const void* M_val, sam_precision prec, double* res2,
                        double* a02, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", true))) return st;
    if ((st = check_csc_args(ctx, A0, "A0", true))) return st;
    if (Ak->n != A0->n) return fail(ctx, SAM_ERR_SHAPE, "Ak and A0 differ in order");
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if (!M_colptr || (nnz_M > 0 && (!M_rowind || !M_val)) || !res2) return fail(ctx, SAM_ERR_ARG, "NULL argument");
    if (nnz_M < 0 || nnz_M > INT_MAX) return fail(ctx, SAM_ERR_OVERFLOW, "nnz_M out of range");
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    const int n = Ak->n;
    const size_t need = align256((size_t)std::max(n, 1) * 8) + align256(samk::reduce_temp_bytes(std::max<int64_t>(n, A0->nnz))) + 512;
    HIP_TRY(ctx, grow(ctx->ws, need));
    Carve cv(ctx->ws.p);
    double* cols = cv.take<double>(std::max(n, 1));
    void* rt = cv.take<char>(samk::reduce_temp_bytes(std::max<int64_t>(n, A0->nnz)));
    if (n == 0) {
        HIP_TRY(ctx, hipMemsetAsync(res2, 0, sizeof(double), s));
        if (a02) HIP_TRY(ctx, hipMemsetAsync(a02, 0, sizeof(double), s));
        return SAM_OK;
    }
    HIP_TRY(ctx, samk::residual_columns(n, Ak->colptr, Ak->rowind, Ak->val, A0->colptr, A0->rowind, A0->val, M_colptr,
                                        M_rowind, M_val, prec == SAM_PREC_F32_REFINE, cols, ctx->d_status, s));
    HIP_TRY(ctx, samk::reduce_sum(cols, n, res2, rt, s));
    if (a02) HIP_TRY(ctx, samk::reduce_sumsq(A0->val, A0->nnz, a02, rt, s));
    return SAM_OK;
}

sam_status sam_apply_prepare(sam_ctx* ctx, int32_t n, const int32_t* M_colptr, const int32_t* M_rowind, int64_t nnz,
                             int32_t* T_rowptr, int32_t* T_colind, int32_t* T_perm, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    if (n < 0 || nnz < 0) return fail(ctx, SAM_ERR_ARG, "negative size");
    if (nnz > INT_MAX) return fail(ctx, SAM_ERR_OVERFLOW, "nnz does not fit in int32");
    if (!M_colptr || !T_rowptr || (nnz > 0 && (!M_rowind || !T_colind || !T_perm)))
        return fail(ctx, SAM_ERR_ARG, "NULL argument");
    sam_status st = need_device(ctx);
    if (st) return st;
    hipStream_t s = S(stream);
    const size_t need = 2 * align256((size_t)std::max(n, 1) * 4) + align256((size_t)(n + 1) * 8) +
                        align256(samk::scan_temp_bytes(n)) + 512;
    HIP_TRY(ctx, grow(ctx->ws, need));
    Carve cv(ctx->ws.p);
    int* rowcount = cv.take<int>(std::max(n, 1));
    int* cursor = cv.take<int>(std::max(n, 1));
    int64_t* off = cv.take<int64_t>(n + 1);
    void* stemp = cv.take<char>(samk::scan_temp_bytes(n));
    HIP_TRY(ctx, hipMemsetAsync(rowcount, 0, (size_t)std::max(n, 1) * 4, s));
    HIP_TRY(ctx, hipMemsetAsync(cursor, 0, (size_t)std::max(n, 1) * 4, s));
    HIP_TRY(ctx, samk::transpose_count(n, M_colptr, M_rowind, nnz, rowcount, s));
    HIP_TRY(ctx, samk::scan_counts(rowcount, n, off, T_rowptr, nullptr, stemp, s));
    HIP_TRY(ctx, samk::transpose_fill(n, M_colptr, M_rowind, T_rowptr, cursor, T_colind, T_perm, s));
    HIP_TRY(ctx, samk::transpose_sort_rows(n, T_rowptr, T_colind, T_perm, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return SAM_OK;
}

sam_status sam_apply(sam_ctx* ctx, int32_t n, const int32_t* T_rowptr, const int32_t* T_colind, const int32_t* T_perm,
                     const void* M_val, sam_precision prec, const double* x, double* y, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    if (n < 0) return fail(ctx, SAM_ERR_ARG, "negative size");
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if (n > 0 && (!T_rowptr || !T_colind || !T_perm || !M_val || !x || !y)) return fail(ctx, SAM_ERR_ARG, "NULL argument");
    sam_status st = need_device(ctx);
    if (st) return st;
    HIP_TRY(ctx, samk::spmv_rows(n, T_rowptr, T_colind, T_perm, M_val, prec == SAM_PREC_F32_REFINE, x, y, S(stream)));
    return SAM_OK;
}

}  // extern "C"

extern "C" {

sam_status sam_build_weighted(sam_plan* plan, const double* Ak_val, const double* A0_val, const double* w, double mu,
                              sam_precision prec, void* M_val, double* col_res2, double* res2, sam_stream_t stream) {
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
    const int n = pl->n;
    const size_t need = align256(samk::bucket_temp_bytes(n)) + 512;
    HIP_TRY(ctx, grow(ctx->ws, need));
    Carve cv(ctx->ws.p);
    void* btemp = cv.take<char>(samk::bucket_temp_bytes(n));
    int* flag = cv.take<int>(4);
    Combo& cb = pl->combo[prec][0];
    const std::vector<const NumericVariant*> previous = cb.variants;
    sam_status st = plan_combo_with(pl, prec, 0, vars, btemp, flag, s);
    if (st) return st;
    if (!cb.ok) {
        const std::string why = cb.why;
        st = plan_combo_with(pl, prec, 0, previous, btemp, flag, s);
        if (st) return st;
        return fail(ctx, SAM_ERR_UNSUPPORTED, "selection rejected: %s", why.c_str());
    }
    return SAM_OK;
}

}  // namespace samh

extern "C" {

sam_status sam_menu(sam_precision prec, int32_t weighted, int32_t capacity, int32_t* count, int32_t* G, int32_t* R,
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

sam_status sam_plan_select(sam_plan* plan, sam_precision prec, const int32_t* order, int32_t count,
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
