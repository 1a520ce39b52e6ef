// sam_adjoint.hip -- deterministic accumulation of the adjoint's A_k-value
// gradient.  Every column problem j contributes to each A_k entry of the
// columns J_j; the backward kernel stages those contributions per gathered
// entry, and this kernel sums, for each A_k entry, the contributions of all
// columns j in ascending order (no atomics: bitwise reproducible).
#include "sam_device.hpp"
#include "sam_kernels.hpp"

namespace samk {

namespace {

// One thread per column l of A_k: for every column j whose pattern holds l
// (the row view of S, ascending j) the staged contributions of j to the
// entries of A_k(:, l) are contiguous, so each j costs one offset lookup
// (prefetched one step ahead) and one contiguous read per entry, added into
// per-entry registers in ascending j.  Columns longer than kChunk entries
// take several passes.
constexpr int kChunk = 8;

__global__ void k_backward_scatter(int n, const int* Ak_cp, const int* ST_rowptr, const int* ST_perm,
                                   const int64_t* segoff, const double* contrib, double* gAk) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const int fa = Ak_cp[l], len = Ak_cp[l + 1] - fa;
    const int sa = ST_rowptr[l], sb = ST_rowptr[l + 1];
    for (int f0 = 0; f0 < len; f0 += kChunk) {
        double acc[kChunk];
#pragma unroll
        for (int i = 0; i < kChunk; ++i) acc[i] = 0.0;
        int64_t next = sa < sb ? segoff[ST_perm[sa]] : 0;
        for (int e = sa; e < sb; ++e) {
            const double* src = contrib + next + f0;
            if (e + 1 < sb) next = segoff[ST_perm[e + 1]];
#pragma unroll
            for (int i = 0; i < kChunk; ++i)
                if (f0 + i < len) acc[i] += src[i];
        }
#pragma unroll
        for (int i = 0; i < kChunk; ++i)
            if (f0 + i < len) gAk[fa + f0 + i] = acc[i];
    }
}

}  // namespace

hipError_t backward_scatter(int n, const int* Ak_cp, const int* ST_rowptr, const int* ST_perm,
                            const int64_t* segoff, const double* contrib, double* gAk, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_backward_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, Ak_cp,
                       ST_rowptr, ST_perm, segoff, contrib, gAk);
    return hipGetLastError();
}

}  // namespace samk
