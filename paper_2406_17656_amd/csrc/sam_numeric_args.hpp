// sam_numeric_args.hpp -- the interface of the numeric least-squares kernels
// (internal to the library): their arguments, the kernel variants and the
// compiled menu.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace samk {

struct NumericArgs {
    int n;
    // extents of the arrays the kernels read through 32-bit buffer offsets
    // (the plan guarantees nnz(A_k) * 8, nnz(A_0) * 8 and E below 2^32)
    uint32_t nnzA, nnzA0, E;
    const int* Ak_cp;
    const double* Ak_v;
    const int* A0_cp;
    const double* A0_v;
    const int* S_cp;
    const int* S_ri;
    const int* nI;
    const int64_t* eoff;
    const unsigned char* posA;
    const unsigned char* posB;
    const int* queue;     // all buckets' columns
    const int* bstart;    // device, bucket offsets
    int bucket;           // which bucket this launch serves
    void* M;
    double* col_res2;     // n or nullptr
    // per-block partial sums of the column residuals (the launch's blocks
    // write part[part_base + block]); nullptr: none
    double* part;
    int part_base;
    unsigned long long* status;
    // soft weights (nullptr for the plain map)
    const double* w;
    double mu;
    // adjoint outputs (backward launches only)
    double dL;
    double* contrib;      // per gathered entry, at eoff[j] + offset in the block
    int64_t* segoff;      // per S entry: where its column's contributions start
    double* gA0;          // nnz(A_0)
    double* gw;           // nnz(S) or nullptr
};

// One kernel variant of the menu: solves every column of one bucket whose
// block fits max_rows x max_cols.
struct NumericVariant {
    int prec;        // 0 = FP64, 1 = FP32 + refinement
    int G;           // lanes per column problem
    int R;           // rows per lane
    int NC;          // max columns
    int weighted;    // 1: stacked penalty rows
    int TC;          // columns staged per LDS tile pass
    int LPL;         // entries per lane and column moved with static indices
    hipError_t (*launch)(const NumericArgs&, int grid, hipStream_t);
    hipError_t (*launch_backward)(const NumericArgs&, int grid, hipStream_t);  // weighted only
    int (*blocks_per_cu)();  // resident one-wave blocks per CU of the forward kernel (0: unknown)
    int max_rows() const { return G * R; }
    int per_wave() const { return 64 / G; }
};
// The compiled menu, ordered from the cheapest per column to the most
// general for each precision.
const NumericVariant* numeric_menu(int* count);

}  // namespace samk
