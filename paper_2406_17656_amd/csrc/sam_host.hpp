// sam_host.hpp -- host-side objects and helpers shared by the C ABI
// translation units (internal to the library).
#pragma once

#include "sam.h"
#include "sam_kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct sam_ctx {
    int device = SAM_NO_DEVICE;
    std::string err;
    unsigned long long* d_status = nullptr;
    DevBuf ws;  // scratch for synchronising calls
    // last pattern from sam_pattern_count
    DevBuf S_cp, S_ri;
    int64_t S_nnz = -1;
    int S_n = -1;
    const int32_t* key_cp = nullptr;
    const int32_t* key_ri = nullptr;
    const double* key_val = nullptr;
    sam_pattern_spec key_spec{};
    int CUs = 256;
    // resident blocks per CU of each numeric kernel variant (menu order),
    // queried once on the context's device
    std::vector<int> resident;
};

// One (precision, weighted) combination of a plan: the bucket order of the
// columns and the kernel variant per bucket.
struct Combo {
    bool ok = false;
    std::string why;
    std::vector<const samk::NumericVariant*> variants;
    samk::BucketTable tab{};
    int* queue = nullptr;   // device n
    int* bstart = nullptr;  // device nb+1
    std::vector<int> counts;
    // replanned sequences: one live bucket, so the queue is the identity and
    // bstart = {0, n}, written once instead of sorting every run
    bool identity = false;
};

struct sam_plan {
    sam_ctx* ctx = nullptr;
    int n = 0;
    int nnzA = 0, nnzA0 = 0;
    int64_t nnzS = 0;
    const int *Ak_cp = nullptr, *Ak_ri = nullptr, *A0_cp = nullptr, *A0_ri = nullptr;
    const int *S_cp = nullptr, *S_ri = nullptr;
    int max_len_A = 0;             // longest column of A_k
    DevBuf mem;          // nI, eoff, posA, posB, queues, colbuf, reduce temp
    int* nI = nullptr;
    int64_t* eoff = nullptr;
    unsigned char* posA = nullptr;
    unsigned char* posB = nullptr;
    double* colbuf = nullptr;
    void* rtemp = nullptr;  // reduction temp for max(n, partcap) values
    double* partbuf = nullptr;  // per-block partial sums of the column residuals
    int partcap = 0;
    int64_t E = 0;
    int max_rows = 0, max_cols = 0;
    // algorithmic flop counts of one build (dense column blocks)
    double fl_qr32 = 0.0, fl_ref64 = 0.0, fl_f64 = 0.0;
    Combo combo[2][2];  // [prec][weighted]
    // backward staging (allocated on the first sam_backward)
    DevBuf bwd;
    // device-resident counts: numeric launches size their grids from the
    // host copy in Combo::counts unless this is set (sequence replanning)
    bool device_counts = false;
};

namespace samh {

constexpr unsigned long long kStatusClear = 0x7fffffffffffffffull;

sam_status fail(sam_ctx* ctx, sam_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));

#define HIP_TRY(ctx, expr)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return samh::fail((ctx), e_ == hipErrorOutOfMemory ? SAM_ERR_NOMEM : SAM_ERR_HIP,    \
                              "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

inline hipStream_t S(sam_stream_t s) { return reinterpret_cast<hipStream_t>(s); }
inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

hipError_t grow(DevBuf& b, size_t bytes);
void release(DevBuf& b);

// bump allocator over a DevBuf
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* p) : base((char*)p) {}
    template <typename T>
    T* take(size_t count) {
        T* r = (T*)(base + off);
        off += align256(count * sizeof(T));
        return r;
    }
};

sam_status check_ctx(sam_ctx* ctx);
sam_status need_device(sam_ctx* ctx);
sam_status check_csc_args(sam_ctx* ctx, const sam_csc* A, const char* name, bool need_val);
sam_status check_spec(sam_ctx* ctx, const sam_pattern_spec* spec);
samk::SparsifySpec to_sp(const sam_pattern_spec* spec);
inline bool prec_ok(sam_precision p) { return p == SAM_PREC_F64 || p == SAM_PREC_F32_REFINE; }

template <typename T>
hipError_t read_back(const T* dptr, T* host, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(host, dptr, sizeof(T), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// Per-level facts of a pattern computation: the size and longest column of
// every level (level 0 is B, the last is S), and optionally (cp != null)
// every level's column pointers (p arrays of n+1 int32, level after level,
// grown as needed).
struct PatternLevels {
    std::vector<int64_t> nnz;
    std::vector<int> maxcol;
    DevBuf* cp = nullptr;
};

// Pattern S((I + B)^p) on the device.
sam_status compute_pattern(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, DevBuf& out_cp,
                           DevBuf& out_ri, int64_t* nnz_out, hipStream_t s, PatternLevels* levels = nullptr);
// The bucket table of one (precision, weighted) combination of the menu.
samk::BucketTable menu_table(int prec, int weighted, std::vector<const samk::NumericVariant*>* variants);
sam_status plan_combo(sam_plan* pl, int prec, int weighted, void* temp, int* unfit_d, hipStream_t s);
// Bucket the plan's columns over an explicit ordered list of variants.
sam_status plan_combo_with(sam_plan* pl, int prec, int weighted, const std::vector<const samk::NumericVariant*>& vars,
                           void* temp, int* unfit_d, hipStream_t s);
samk::BucketTable table_of(const std::vector<const samk::NumericVariant*>& vars, int weighted);
// Variants of sam_menu(prec, weighted) in the given order (nullptr entries when out of range).
std::vector<const samk::NumericVariant*> menu_subset(int prec, int weighted, const int32_t* order, int32_t count,
                                                     bool* ok);
// Re-bucket a plan's plain builds over a selected variant order (synchronising).
sam_status plan_select(sam_plan* pl, int prec, const std::vector<const samk::NumericVariant*>& vars, hipStream_t s);
// Capacity of a plan's partial-sum buffer: every bucket's launch at the
// largest resident grid of the menu.
int partial_capacity(const sam_ctx* ctx);
sam_status run_numeric(sam_plan* pl, const double* Ak_val, const double* A0_val, const double* w, double mu, int prec,
                       int weighted, void* M_val, double* col_res2, double* res2, hipStream_t s);

}  // namespace samh
