// sam_host.hpp -- host-side objects and helpers shared by the C ABI
// translation units (internal to the library).
//
// Device memory: a context holds one 256-byte status block (allocated by
// sam_create, released by sam_destroy).  Every other device buffer a call
// uses -- pattern workspaces, plan and sequence storage, the scratch of the
// residual, the row views, the adjoint's staging -- is caller memory, carved
// by the layout functions below; the same functions size it (Carve with a
// null base only adds up the pieces), so sizing and use cannot disagree.
#pragma once

#include "sam.h"
#include "sam_kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

namespace samh {

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Bump allocator over caller memory; with a null base it only measures (the
// pointers it returns are then null and must not be used).
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* p) : base((char*)p) {}
    template <typename T>
    T* take(size_t count) {
        T* r = base ? (T*)(base + off) : nullptr;
        off += align256(std::max<size_t>(count, 1) * sizeof(T));
        return r;
    }
};

// Pattern workspace of S((I + B)^p) for one source (sam_pattern_count /
// sam_pattern_fill, and the structural pattern of a sequence).  Sizes follow
// from n, nnz(A_k), its longest column and p: B holds at most nnz(A_k) + n
// entries; an intermediate level (powers 2 .. p-1) holds at most
// n min(n, (1 + longest)^power) entries, since a column of level q + 1 is the
// union of at most (1 + longest) columns of B per entry of level q.
struct PatternWs {
    int* counts = nullptr;    // n
    int64_t* off = nullptr;   // n + 1
    void* stemp = nullptr;    // scan temporary
    double* D = nullptr;      // n (global threshold scaling)
    int* B_cp = nullptr;      // n + 1
    int* B_ri = nullptr;      // nnz(A_k) + n
    int* flags = nullptr;     // [0] overflow, [1] bad column, [2] longest column of a level
    int* L_cp[2] = {nullptr, nullptr};  // intermediate levels, alternating
    int* L_ri[2] = {nullptr, nullptr};
    int64_t Lcap = 0;         // entries per intermediate buffer
    int* S_cp = nullptr;      // n + 1: column pointers of the final level (power >= 2)
};
int64_t level_bound(int n, int longest, int power);
void pattern_ws_layout(Carve& cv, int n, int nnzA, int longest, int power, PatternWs* w);

// Result of a pattern count, kept (host side) until the fill.
struct PatternResult {
    int64_t nnz = 0;
    const int* last_cp = nullptr;  // level p-1 (B when p = 2); null when p = 1
    const int* last_ri = nullptr;
    int last_max = 0;              // its longest column
    const int* B_cp = nullptr;
    const int* B_ri = nullptr;
    int maxB = 0;
    const int* S_cp = nullptr;     // final column pointers (B_cp when p = 1)
};

// Per-level facts of a pattern computation: the size and longest column of
// every level (level 0 is B, the last is S), and optionally (cp != null)
// every level's column pointers copied to cp + lev (n + 1).
struct PatternLevels {
    std::vector<int64_t> nnz;
    std::vector<int> maxcol;
    int* cp = nullptr;
};

// Host record of the last sam_pattern_count on a context: its levels stay in
// the caller's workspace until sam_pattern_fill.
struct PatternState {
    bool valid = false;
    const void* ws = nullptr;
    int n = -1, nnz_A = -1;
    const int32_t *cp = nullptr, *ri = nullptr;
    const double* val = nullptr;
    sam_pattern_spec spec{};
    int power = 1;
    PatternResult res;
};

}  // namespace samh

struct sam_ctx {
    int device = SAM_NO_DEVICE;
    std::string err;
    // 256-byte device status block: the status word (kernels' failures), the
    // bad-column flag of structure checks and a 64-bit accumulator
    void* block = nullptr;
    unsigned long long* d_status = nullptr;
    int* d_bad = nullptr;
    unsigned long long* d_total = nullptr;
    samh::PatternState pat;
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
    void* mem = nullptr;           // caller memory holding the arrays below
    size_t mem_bytes = 0;
    int* nI = nullptr;
    int64_t* eoff = nullptr;
    unsigned char* posA = nullptr;
    unsigned char* posB = nullptr;
    double* colbuf = nullptr;
    void* rtemp = nullptr;      // reduction temp for max(n, partcap) values
    double* partbuf = nullptr;  // per-block partial sums of the column residuals
    int partcap = 0;
    void* btemp = nullptr;      // bucket-sort temporary (selection)
    int* flags = nullptr;       // device ints for the bucket sort
    int64_t E = 0;
    int max_rows = 0, max_cols = 0;
    // algorithmic flop counts of one build (dense column blocks), and the
    // shape moments sum_j r c^2, c^3, r c, c^2, r (r = |I_j|, c = |J_j|) the
    // weighted and adjoint counts follow from
    double fl_qr32 = 0.0, fl_ref64 = 0.0, fl_f64 = 0.0;
    double m_rc2 = 0.0, m_c3 = 0.0, m_rc = 0.0, m_c2 = 0.0, m_r = 0.0;
    Combo combo[2][2];  // [prec][weighted]
    // the workspace sam_backward_prepare built the row view of S in
    const void* bwd_ws = nullptr;
    // device-resident counts: numeric launches size their grids from the
    // host copy in Combo::counts unless this is set (sequence replanning)
    bool device_counts = false;
};

namespace samh {

constexpr unsigned long long kStatusClear = 0x7fffffffffffffffull;
constexpr size_t kCtxBlockBytes = 256;

sam_status fail(sam_ctx* ctx, sam_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));

#define HIP_TRY(ctx, expr)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return samh::fail((ctx), e_ == hipErrorOutOfMemory ? SAM_ERR_NOMEM : SAM_ERR_HIP,    \
                              "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

inline hipStream_t S(sam_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

sam_status check_ctx(sam_ctx* ctx);
sam_status need_device(sam_ctx* ctx);
sam_status check_csc_args(sam_ctx* ctx, const sam_csc* A, const char* name, bool need_val);
sam_status check_spec(sam_ctx* ctx, const sam_pattern_spec* spec);
sam_status check_ws(sam_ctx* ctx, const void* ws, size_t ws_bytes, size_t need, const char* what);
samk::SparsifySpec to_sp(const sam_pattern_spec* spec);
// precision arguments are int32_t (one of sam_precision): any value a C
// caller passes is well defined and checked here
inline bool prec_ok(int32_t p) { return p == SAM_PREC_F64 || p == SAM_PREC_F32_REFINE; }

template <typename T>
hipError_t read_back(const T* dptr, T* host, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(host, dptr, sizeof(T), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// Column pointers read to the host (synchronising): checks colptr[0] = 0,
// monotone, colptr[n] = nnz; *longest receives the longest column.
sam_status host_colptr(sam_ctx* ctx, const int32_t* cp, int n, int64_t nnz, const char* name, int* longest,
                       hipStream_t s, std::vector<int>* keep = nullptr);
// Full structure check on the device before any other kernel reads the
// indices (synchronising): SAM_ERR_UNSORTED names the first bad column.
sam_status validate_csc(sam_ctx* ctx, int n, int64_t nnz, const int32_t* cp, const int32_t* ri, const char* name,
                        hipStream_t s);

// Pattern S((I + B)^p) counted in a pattern workspace: every level but the
// last is stored there, the last is counted (column pointers in w.S_cp);
// pattern_fill writes it to the caller's arrays.
sam_status compute_pattern(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, const PatternWs& w,
                           PatternResult* res, hipStream_t s, PatternLevels* levels = nullptr);
sam_status pattern_fill(sam_ctx* ctx, int n, const PatternResult& res, int* S_cp, int* S_ri, hipStream_t s);

// Plan memory: creation temporaries (sized by n), then the plan's arrays
// (sized by n, the gathered entries E, nnz(A_0) and the partial-sum
// capacity).
size_t plan_bytes(int n, int64_t E, int nnzA0, int partcap);
// A plan in caller memory `mem` (>= plan_bytes); structures validated by the
// caller.  E_known >= 0 skips nothing but is checked against the count.
sam_status plan_init(sam_ctx* ctx, sam_plan* pl, const sam_csc* Ak, const sam_csc* A0, const int32_t* S_colptr,
                     const int32_t* S_rowind, int64_t nnz_S, void* mem, size_t mem_bytes, hipStream_t s);
// sum_j sum_{l in S(:,j)} nnz(A_k(:,l)) (synchronising; S validated).
sam_status gathered_total(sam_ctx* ctx, int n, const int32_t* S_cp, const int32_t* S_ri, const int32_t* Ak_cp,
                          int64_t* E, hipStream_t s);

// The bucket table of one (precision, weighted) combination of the menu.
samk::BucketTable menu_table(int prec, int weighted, std::vector<const samk::NumericVariant*>* variants);
sam_status plan_combo(sam_plan* pl, int prec, int weighted, hipStream_t s);
// Bucket the plan's columns over an explicit ordered list of variants.
sam_status plan_combo_with(sam_plan* pl, int prec, int weighted, const std::vector<const samk::NumericVariant*>& vars,
                           hipStream_t s);
samk::BucketTable table_of(const std::vector<const samk::NumericVariant*>& vars, int weighted);
// Variants of sam_menu(prec, weighted) in the given order (nullptr entries when out of range).
std::vector<const samk::NumericVariant*> menu_subset(int prec, int weighted, const int32_t* order, int32_t count,
                                                     bool* ok);
// Re-bucket a plan's plain builds over a selected variant order (synchronising).
sam_status plan_select(sam_plan* pl, int prec, const std::vector<const samk::NumericVariant*>& vars, hipStream_t s);
// Capacity of a plan's partial-sum buffer: every bucket's launch at the
// largest resident grid of the menu.
int partial_capacity(const sam_ctx* ctx);
// Device address of sam_build_noalloc's fixed scratch array on `device`
// (current), looked up once per device; called by sam_create.
hipError_t scratch_setup(int device);
sam_status run_numeric(sam_plan* pl, const double* Ak_val, const double* A0_val, const double* w, double mu, int prec,
                       int weighted, void* M_val, double* col_res2, double* res2, hipStream_t s);

}  // namespace samh
