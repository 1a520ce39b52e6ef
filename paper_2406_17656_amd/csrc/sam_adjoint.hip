// sam_adjoint.hip -- deterministic accumulation of the adjoint's A_k-value
// gradient.  Every column problem j contributes to each A_k entry of the
// columns J_j; the backward kernel stages those contributions per gathered
// entry, and this kernel sums, for each A_k entry, the contributions of all
// columns j in ascending order (no atomics: bitwise reproducible).
#include "sam_device.hpp"
#include "sam_kernels.hpp"

namespace samk {

namespace {

__global__ void k_backward_scatter(int n, const int* Ak_cp, const int* ST_rowptr, const int* ST_perm,
                                   const int64_t* segoff, const double* contrib, double* gAk) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const int fa = Ak_cp[l], fb = Ak_cp[l + 1];
    const int sa = ST_rowptr[l], sb = ST_rowptr[l + 1];
    for (int f = fa; f < fb; ++f) {
        double acc = 0.0;
        for (int e = sa; e < sb; ++e) acc += contrib[segoff[ST_perm[e]] + (f - fa)];
        gAk[f] = acc;
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
