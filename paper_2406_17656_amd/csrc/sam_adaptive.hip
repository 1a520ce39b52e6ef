// sam_adaptive.hip -- adjoint-guided pattern adaptation, the direction the
// paper leaves for future work (adaptive patterns in parallel environments,
// end of Section 2; more refined sparsification, Section 6): the entries
// of a candidate pattern S (a higher level) that are not in the base pattern
// B carry soft weights w < 1; the gradient of the loss with respect to w
// ranks them, and each column keeps its base entries plus the k candidates
// whose admission lowers the loss fastest (most negative dL/dw).
//
// One thread per column: columns hold tens of entries, so the rank of a
// candidate is counted directly over its column (no sort).
#include "sam_device.hpp"
#include "sam_kernels.hpp"

#include <cmath>

namespace samk {

namespace {

// w[e] = w_base where row S_ri[e] of column j is in B(:, j), else w_cand
// (both columns ascending: one merge).
__global__ void k_candidate_weights(int n, const int* S_cp, const int* S_ri, const int* B_cp, const int* B_ri,
                                    double w_base, double w_cand, double* w) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int f = B_cp[j];
    const int fb = B_cp[j + 1];
    for (int e = S_cp[j]; e < S_cp[j + 1]; ++e) {
        const int r = S_ri[e];
        while (f < fb && B_ri[f] < r) ++f;
        w[e] = (f < fb && B_ri[f] == r) ? w_base : w_cand;
    }
}

// Order of candidates: smaller gradient first (NaN counts as +inf), ties to
// the smaller row.
__device__ inline bool ahead(double ga, int ra, double gb, int rb) {
    ga = isnan(ga) ? INFINITY : ga;
    gb = isnan(gb) ? INFINITY : gb;
    return ga < gb || (ga == gb && ra < rb);
}

template <bool FILL>
__global__ void k_topk(int n, const int* S_cp, const int* S_ri, const double* w, const double* grad, int k,
                       int* counts, const int* out_cp, int* out_ri) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int a = S_cp[j], b = S_cp[j + 1];
    int o = FILL ? out_cp[j] : 0;
    int kept = 0;
    for (int e = a; e < b; ++e) {
        bool keep = w[e] >= 1.0;
        if (!keep) {
            int rank = 0;
            const double ge = grad[e];
            const int re = S_ri[e];
            for (int f = a; f < b && rank < k; ++f)
                if (f != e && w[f] < 1.0 && ahead(grad[f], S_ri[f], ge, re)) ++rank;
            keep = rank < k;
        }
        if (keep) {
            if (FILL) out_ri[o + kept] = S_ri[e];
            ++kept;
        }
    }
    if (!FILL) counts[j] = kept;
}

}  // namespace

hipError_t candidate_weights(int n, const int* S_cp, const int* S_ri, const int* B_cp, const int* B_ri,
                             double w_base, double w_cand, double* w, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_candidate_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, S_cp, S_ri,
                       B_cp, B_ri, w_base, w_cand, w);
    return hipGetLastError();
}

hipError_t topk_count(int n, const int* S_cp, const int* S_ri, const double* w, const double* grad, int k,
                      int* counts, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_topk<false>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, S_cp, S_ri, w, grad,
                       k, counts, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t topk_fill(int n, const int* S_cp, const int* S_ri, const double* w, const double* grad, int k,
                     const int* out_cp, int* out_ri, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_topk<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, S_cp, S_ri, w, grad,
                       k, nullptr, out_cp, out_ri);
    return hipGetLastError();
}

}  // namespace samk
