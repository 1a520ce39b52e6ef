// sam_noalloc.cpp -- sam_build_noalloc: the one-shot build with the plan of
// the column problems in a fixed device array of the library instead of a
// caller workspace, for callers that cannot allocate device memory.
#include "sam_host.hpp"

#include <climits>
#include <mutex>

using namespace samh;

namespace {

// Largest plan sam_build_noalloc accepts (the 512 x 512 level-2 map needs
// about 31 MiB).
constexpr size_t kScratchBytes = size_t(48) << 20;

// The plan memory of sam_build_noalloc.  Every GPU the library runs on holds
// its own copy until the process ends.  In host code this name stands for a
// host-side symbol, not a device address: the address each device uses is
// looked up once per device (scratch_setup) and only that address is handed
// to kernels and copies.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};
hipError_t g_setup_err[kMaxDevices] = {};

}  // namespace

namespace samh {

// Looks up the array's address on `device` (which must be current), once per
// device; called by sam_create.
hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_setup_err[device] = e;
    if (e == hipSuccess) g_scratch[device] = p;
    return e;
}

}  // namespace samh

extern "C" {

sam_status sam_build_noalloc(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0, const int32_t* S_colptr,
                             const int32_t* S_rowind, int64_t nnz_S, int32_t prec, void* M_val,
                             double* col_res2, double* res2, sam_stream_t stream) {
    if (check_ctx(ctx)) return SAM_ERR_ARG;
    sam_status st;
    if ((st = check_csc_args(ctx, Ak, "Ak", true))) return st;
    if ((st = check_csc_args(ctx, A0, "A0", true))) return st;
    if (!prec_ok(prec)) return fail(ctx, SAM_ERR_ARG, "unknown precision %d", (int)prec);
    if (nnz_S > 0 && !M_val) return fail(ctx, SAM_ERR_ARG, "M_val is NULL");
    if ((st = need_device(ctx))) return st;
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch[ctx->device];
        if (!base)
            return fail(ctx, SAM_ERR_HIP, "the fixed scratch array has no address on device %d: %s", ctx->device,
                        hipGetErrorString(ctx->device >= 0 && ctx->device < kMaxDevices ? g_setup_err[ctx->device]
                                                                                           : hipErrorInvalidDevice));
    }
    hipStream_t s = S(stream);
    // checks A_k and S and sizes the plan (the gathered entries are counted
    // in the context's status block)
    size_t need = 0;
    if ((st = sam_plan_size(ctx, Ak, A0, S_colptr, S_rowind, nnz_S, &need, stream))) return st;
    if (need > kScratchBytes)
        return fail(ctx, SAM_ERR_UNSUPPORTED,
                    "sam_build_noalloc: the plan of this problem needs %zu bytes, the fixed scratch holds %zu "
                    "(use sam_build with a workspace)", need, kScratchBytes);
    if ((st = validate_csc(ctx, A0->n, A0->nnz, A0->colptr, A0->rowind, "A0", s))) return st;
    sam_plan pl;
    if ((st = plan_init(ctx, &pl, Ak, A0, S_colptr, S_rowind, nnz_S, base, kScratchBytes, s))) return st;
    return run_numeric(&pl, Ak->val, A0->val, nullptr, 0.0, prec == SAM_PREC_F32_REFINE ? 1 : 0, 0, M_val, col_res2,
                       res2, s);
}

}  // extern "C"
