// sam_adaptive_api.cpp -- C ABI of the adjoint-guided pattern adaptation:
// candidate weights over a higher-level pattern, the top-k selection by the
// weight gradient, and the penalty scale of the soft weights.
#include "sam_host.hpp"

#include <climits>
#include <vector>

using namespace samh;

namespace {

// Host check of a column-pointer array (synchronising): cp[0] = 0,
// non-decreasing, cp[n] = nnz.
sam_status check_colptr(sam_ctx* ctx, const int32_t* cp, int n, int64_t nnz, const char* name, hipStream_t s) {
    std::vector<int> h((size_t)n + 1);
    HIP_TRY(ctx, hipMemcpyAsync(h.data(), cp, h.size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (h[0] != 0 || h[(size_t)n] != nnz)
        return fail(ctx, SAM_ERR_SHAPE, "%s[0] = %d, %s[n] = %d but nnz = %lld", name, h[0], name, h[(size_t)n],
                    (long long)nnz);
    for (int j = 0; j < n; ++j)
        if (h[(size_t)j + 1] < h[(size_t)j]) return fail(ctx, SAM_ERR_UNSORTED, "%s decreases at column %d", name, j);
    return SAM_OK;
}

size_t topk_layout(Carve& cv, int n, int** counts, int64_t** off, void** stemp) {
    int* c = cv.take<int>((size_t)std::max(n, 1));
    int64_t* o = cv.take<int64_t>((size_t)n + 1);
    void* t = cv.take<char>(samk::scan_temp_bytes(n));
    if (counts) *counts = c;
    if (off) *off = o;
    if (stemp) *stemp = t;
    return cv.off;
}

size_t penalty_layout(Carve& cv, int nnz, double** out, void** rt) {
    double* o = cv.take<double>(1);
    void* r = cv.take<char>(samk::reduce_temp_bytes(std::max(nnz, 1)));
    if (out) *out = o;
    if (rt) *rt = r;
    return cv.off;
}

}  // namespace

extern "C" {

sam_status sam_topk_workspace_size(int32_t n, size_t* bytes) {
    if (n < 0 || !bytes) return SAM_ERR_ARG;
    Carve cv(nullptr);
    *bytes = topk_layout(cv, n, nullptr, nullptr, nullptr);
    return SAM_OK;
}

sam_status sam_penalty_workspace_size(int32_t nnz, size_t* bytes) {
    if (nnz < 0 || !bytes) return SAM_ERR_ARG;
    Carve cv(nullptr);
    *bytes = penalty_layout(cv, nnz, nullptr, nullptr);
    return SAM_OK;
}

sam_status sam_candidate_weights(sam_ctx* ctx, int32_t n, const int32_t* S_colptr, const int32_t* S_rowind,
                                 int64_t nnz_S, const int32_t* B_colptr, const int32_t* B_rowind, int64_t nnz_B,
                                 double w_base, double w_cand, double* w, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    if (n < 0 || nnz_S < 0 || nnz_B < 0) return fail(ctx, SAM_ERR_ARG, "negative size");
    if (nnz_S > INT_MAX || nnz_B > INT_MAX) return fail(ctx, SAM_ERR_OVERFLOW, "pattern size does not fit in int32");
    if (!S_colptr || !B_colptr || (nnz_S > 0 && (!S_rowind || !w)) || (nnz_B > 0 && !B_rowind))
        return fail(ctx, SAM_ERR_ARG, "NULL argument");
    sam_status st = need_device(ctx);
    if (st) return st;
    hipStream_t s = S(stream);
    if ((st = check_colptr(ctx, S_colptr, n, nnz_S, "S_colptr", s))) return st;
    if ((st = check_colptr(ctx, B_colptr, n, nnz_B, "B_colptr", s))) return st;
    HIP_TRY(ctx, samk::candidate_weights(n, S_colptr, S_rowind, B_colptr, B_rowind, w_base, w_cand, w, s));
    return SAM_OK;
}

sam_status sam_pattern_topk(sam_ctx* ctx, int32_t n, const int32_t* S_colptr, const int32_t* S_rowind,
                            int64_t nnz_S, const double* w, const double* grad, int32_t k, int32_t* out_colptr,
                            int32_t* out_rowind, int64_t* nnz_out, void* ws, size_t ws_bytes, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    if (n < 0 || nnz_S < 0 || k < 0) return fail(ctx, SAM_ERR_ARG, "negative size or k");
    if (nnz_S > INT_MAX) return fail(ctx, SAM_ERR_OVERFLOW, "nnz_S does not fit in int32");
    if (!S_colptr || !out_colptr || !nnz_out || (nnz_S > 0 && (!S_rowind || !w || !grad || !out_rowind)))
        return fail(ctx, SAM_ERR_ARG, "NULL argument");
    sam_status st = need_device(ctx);
    if (st) return st;
    hipStream_t s = S(stream);
    Carve cv(ws);
    int* counts = nullptr;
    int64_t* off = nullptr;
    void* stemp = nullptr;
    if ((st = check_ws(ctx, ws, ws_bytes, topk_layout(cv, n, &counts, &off, &stemp), "top-k workspace"))) return st;
    if ((st = check_colptr(ctx, S_colptr, n, nnz_S, "S_colptr", s))) return st;
    HIP_TRY(ctx, samk::topk_count(n, S_colptr, S_rowind, w, grad, k, counts, s));
    HIP_TRY(ctx, samk::scan_counts(counts, n, off, out_colptr, nullptr, stemp, s));
    int64_t tot = 0;
    HIP_TRY(ctx, read_back(off + n, &tot, s));
    HIP_TRY(ctx, samk::topk_fill(n, S_colptr, S_rowind, w, grad, k, out_colptr, out_rowind, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    *nnz_out = tot;
    return SAM_OK;
}

sam_status sam_penalty_scale(sam_ctx* ctx, const sam_csc* Ak, double* mu, void* ws, size_t ws_bytes,
                             sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", true))) return st;
    if (!mu) return fail(ctx, SAM_ERR_ARG, "mu is NULL");
    if (Ak->n == 0) return fail(ctx, SAM_ERR_ARG, "empty matrix (n = 0)");
    if ((st = need_device(ctx))) return st;
    hipStream_t s = S(stream);
    Carve cv(ws);
    double* out = nullptr;
    void* rt = nullptr;
    if ((st = check_ws(ctx, ws, ws_bytes, penalty_layout(cv, Ak->nnz, &out, &rt), "penalty workspace"))) return st;
    double ss = 0.0;
    if (Ak->nnz > 0) {
        HIP_TRY(ctx, samk::reduce_sumsq(Ak->val, Ak->nnz, out, rt, s));
        HIP_TRY(ctx, read_back(out, &ss, s));
    }
    *mu = ss / (double)Ak->n;
    return SAM_OK;
}

}  // extern "C"
