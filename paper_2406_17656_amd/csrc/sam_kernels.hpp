// sam_kernels.hpp -- host-side launchers of the gfx950 kernels (internal to
// the library; the public interface is include/sam.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sam_numeric_args.hpp"

namespace samk {

// ----------------------------------------------------------------- scans
// Exclusive prefix sum of n int32 counts into int64 offsets (n+1 entries,
// off[n] = total).  Optionally also writes the int32 copy (n+1), raises
// *overflow (device int) when the total does not fit in int32, and raises
// *maxcount (device int, preset by the caller) to the largest count.  Needs
// scan_temp_bytes(n) bytes of temporary device memory (any contents).  Two
// launches (tile sums, then the scan) up to 2^21 counts.
size_t scan_temp_bytes(int64_t n);
hipError_t scan_counts(const int* counts, int64_t n, int64_t* off, int* off32, int* overflow,
                       void* temp, hipStream_t s, int* maxcount = nullptr);

// ------------------------------------------------------------- structure
// Checks of a CSC structure; writes the earliest bad column to *bad
// (device int, must be preset to n by the caller; stays n when valid).
hipError_t check_csc(int n, int nnz, const int* cp, const int* ri, int* bad, hipStream_t s);

// ------------------------------------------------------------- patterns
struct SparsifySpec {
    int kind;
    double thresh;
    int global_scale;
    double tau;
    int lfil;
};
// B = S(A~) with the diagonal: count (counts[n]) then fill.
hipError_t sparsify_count(int n, const int* cp, const int* ri, const double* v,
                          SparsifySpec sp, double* dscratch, int* counts, hipStream_t s);
hipError_t sparsify_fill(int n, const int* cp, const int* ri, const double* v,
                         SparsifySpec sp, const double* dscratch, const int* out_cp,
                         int* out_ri, hipStream_t s);
// Slot form: B written at slot_cp[j] (a bound-sized layout, e.g. the
// structural B of the unsparsified matrix), counts[j] = its length.
hipError_t sparsify_slots(int n, const int* cp, const int* ri, const double* v, SparsifySpec sp,
                          double* dscratch, const int* slot_cp, int* slot_ri, int* counts, hipStream_t s);
// out(:,j) = union of rows(Q(:,l)) over l in P(:,j); count then fill.
// max_lists bounds the lists per column of P, max_len the entries per list
// of Q (<= 0: unknown); they only pick how much the kernel holds in
// registers.
hipError_t expand_count(int n, const int* P_cp, const int* P_ri, const int* Q_cp, const int* Q_ri,
                        int* counts, int* bad, int max_lists, hipStream_t s);
hipError_t expand_fill(int n, const int* P_cp, const int* P_ri, const int* Q_cp, const int* Q_ri,
                       const int* out_cp, int* out_ri, int max_lists, int max_len, hipStream_t s);
// Slot form: P and Q given as (cp, cnt, ri) with list l at cp[l], length
// cnt[l]; the union of column j goes to slot_ri[slot_cp[j]..], its length to
// counts[j].  The slots must be large enough (the structural bound).
hipError_t expand_slots(int n, const int* P_cp, const int* P_cnt, const int* P_ri, const int* Q_cp,
                        const int* Q_cnt, const int* Q_ri, const int* slot_cp, int* slot_ri, int* counts,
                        int max_lists, int max_len, hipStream_t s);

// ------------------------------------------------------------------ plan
// Per column j: E_j = sum_{l in J_j} nnz(A_k(:,l)).
hipError_t plan_gather_count(int n, const int* S_cp, const int* S_ri, const int* Ak_cp,
                             int* counts, hipStream_t s);
// *total (device, preset by the caller) += sum_j E_j.
hipError_t plan_gather_total(int n, const int* S_cp, const int* S_ri, const int* Ak_cp,
                             unsigned long long* total, hipStream_t s);
// Per column j: nI[j] = |I_j|, positions of the gathered A_k entries (posA,
// at eoff[j]) and of the A_0(:,j) entries (posB aligned with A_0's entries,
// 0xFF outside I_j).  Columns with |I_j| > 255 get nI = |I_j| and no
// positions (they are rejected by the bucket classifier).
hipError_t plan_positions(int n, const int* S_cp, const int* S_ri, const int* Ak_cp,
                          const int* Ak_ri, const int* A0_cp, const int* A0_ri,
                          const int64_t* eoff, int* nI, unsigned char* posA,
                          unsigned char* posB, int max_lists, int max_len, hipStream_t s);
// Same with S in slots (S_cnt lengths); also writes the compact copy of S
// (cS_ri at the offsets cS_cp) when cS_ri is given.  eoff may be any layout
// whose column ranges hold the gathered entries (e.g. the structural one).
hipError_t plan_positions_slots(int n, const int* S_cp, const int* S_cnt, const int* S_ri, const int* cS_cp,
                                int* cS_ri, const int* Ak_cp, const int* Ak_ri, const int* A0_cp,
                                const int* A0_ri, const int64_t* eoff, int* nI, unsigned char* posA,
                                unsigned char* posB, int max_lists, int max_len, hipStream_t s);

constexpr int kMaxBuckets = 16;
struct BucketTable {
    int nb;
    int penalty_rows;     // 1: a column needs max(|I_j|, 2|J_j|) rows (two-stage QR with penalty rows)
    int max_rows[kMaxBuckets];
    int max_cols[kMaxBuckets];
};
// Stable counting sort of the columns by bucket: queue[] lists the columns
// of bucket 0, then bucket 1, ...; bstart[b] (device, nb+1) are the bucket
// offsets.  Columns that fit no bucket are counted in *unfit (device int,
// may be null) and reported in the status word (may be null).
size_t bucket_temp_bytes(int n);
hipError_t bucket_sort(int n, const int* S_cp, const int* nI, BucketTable tab, int* queue,
                       int* bstart, int* unfit, unsigned long long* status, void* temp, hipStream_t s);

// --------------------------------------------------------------- numeric
// NumericArgs, NumericVariant and the menu: sam_numeric_args.hpp.

// Deterministic sums: out[0] = sum_i x[i] (fixed tree order).  Needs
// reduce_temp_bytes(n).
size_t reduce_temp_bytes(int64_t n);
hipError_t reduce_sum(const double* x, int64_t n, double* out, void* temp, hipStream_t s);
// out[0] = sum of squares of x (fixed order)
hipError_t reduce_sumsq(const double* x, int64_t n, double* out, void* temp, hipStream_t s);

// -------------------------------------------------------------- residual
// Per column: rho_j = ||A_k(:,J_j) m_j - A_0(:,j)||^2 computed explicitly.
hipError_t residual_columns(int n, const int* Ak_cp, const int* Ak_ri, const double* Ak_v,
                            const int* A0_cp, const int* A0_ri, const double* A0_v,
                            const int* M_cp, const int* M_ri, const void* M_v, int m_is_f32,
                            double* col_out, unsigned long long* status, hipStream_t s);

// ----------------------------------------------------------------- apply
// p[0 .. count) = v (a kernel, so that graph captures record no memset node)
hipError_t fill_i32(int* p, int64_t count, int v, hipStream_t s);
// queue = 0..n-1 and bstart = {0, n}: every column in bucket 0
hipError_t identity_queue(int n, int* queue, int* bstart, hipStream_t s);
hipError_t transpose_count(int n, const int* cp, const int* ri, int64_t nnz, int* rowcount,
                           hipStream_t s);
hipError_t transpose_fill(int n, const int* cp, const int* ri, const int* rowptr, int* cursor,
                          int* colind, int* perm, hipStream_t s);
hipError_t transpose_sort_rows(int n, const int* rowptr, int* colind, int* perm, hipStream_t s);
hipError_t spmv_rows(int n, const int* rowptr, const int* colind, const int* perm,
                     const void* val, int val_f32, const double* x, double* y, hipStream_t s);
hipError_t permute_vals(int64_t nnz, const int* perm, const void* val, int val_f32, void* out,
                        hipStream_t s);

// ---------------------------------------------------------------- adjoint
// gAk[f] = sum over the S entries (l, j) with l the column of entry f, in
// ascending j (row view of S: ST_rowptr / ST_perm), of the staged
// contribution of column j to entry f.
hipError_t backward_scatter(int n, const int* Ak_cp, const int* ST_rowptr, const int* ST_perm,
                            const int64_t* segoff, const double* contrib, double* gAk, hipStream_t s);

// ------------------------------------------------------ adaptive patterns
// w over S's entries: w_base where the entry is in B (same columns, rows
// ascending), w_cand elsewhere.
hipError_t candidate_weights(int n, const int* S_cp, const int* S_ri, const int* B_cp, const int* B_ri,
                             double w_base, double w_cand, double* w, hipStream_t s);
// Per column: the entries with w >= 1 and the k entries with w < 1 of
// smallest grad (NaN last, ties to the smaller row), in S's order.
hipError_t topk_count(int n, const int* S_cp, const int* S_ri, const double* w, const double* grad, int k,
                      int* counts, hipStream_t s);
hipError_t topk_fill(int n, const int* S_cp, const int* S_ri, const double* w, const double* grad, int k,
                     const int* out_cp, int* out_ri, hipStream_t s);

}  // namespace samk
