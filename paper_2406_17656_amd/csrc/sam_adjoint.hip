// sam_adjoint.hip -- deterministic accumulation of the adjoint's A_k-value
// gradient.  Every column problem j contributes to each A_k entry of the
// columns J_j; the backward kernel stages those contributions per gathered
// entry, and this kernel sums, for each A_k entry, the contributions of all
// columns j in ascending order (no atomics: bitwise reproducible).
#include "sam_device.hpp"
#include "sam_kernels.hpp"

namespace samk {

namespace {

// kLanes threads per column l of A_k, thread i0 taking the entries i0,
// i0 + kLanes, ... of A_k(:, l): for every column j whose pattern holds l
// (the row view of S, ascending j) the staged contributions of j to the
// entries of A_k(:, l) are contiguous, so the threads of one column read one
// contiguous run per j.  Each entry's sum runs over j in ascending order;
// the index lookups and reads of kUnroll consecutive j are issued before
// their additions, which keep that order.
constexpr int kLanes = 8;
constexpr int kUnroll = 4;

__global__ void __launch_bounds__(256)
k_backward_scatter(int n, const int* Ak_cp, const int* ST_rowptr, const int* ST_perm, const int64_t* segoff,
                   const double* contrib, double* gAk) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int l = (int)(t / kLanes);
    const int i0 = (int)(t % kLanes);
    if (l >= n) return;
    const int fa = Ak_cp[l], len = Ak_cp[l + 1] - fa;
    const int sa = ST_rowptr[l], sb = ST_rowptr[l + 1];
    for (int i = i0; i < len; i += kLanes) {
        double acc = 0.0;
        int e = sa;
        for (; e + kUnroll <= sb; e += kUnroll) {
            int64_t off[kUnroll];
            double v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) off[u] = segoff[ST_perm[e + u]];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) v[u] = contrib[off[u] + i];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) acc += v[u];
        }
        for (; e < sb; ++e) acc += contrib[segoff[ST_perm[e]] + i];
        gAk[fa + i] = acc;
    }
}

}  // namespace

hipError_t backward_scatter(int n, const int* Ak_cp, const int* ST_rowptr, const int* ST_perm,
                            const int64_t* segoff, const double* contrib, double* gAk, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t threads = (int64_t)n * kLanes;
    hipLaunchKernelGGL(k_backward_scatter, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, n, Ak_cp,
                       ST_rowptr, ST_perm, segoff, contrib, gAk);
    return hipGetLastError();
}

}  // namespace samk
