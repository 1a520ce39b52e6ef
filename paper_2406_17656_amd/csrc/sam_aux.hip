// sam_aux.hip -- gfx950 kernels for the explicit residual of a stored map
// (Section 2, eq. res: R = A_k M - A_0, recomputed column by column from M's
// values, independently of the build's own residuals) and for y = M x.
#include "sam_device.hpp"
#include "sam_kernels.hpp"

#include <algorithm>
#include <climits>

namespace samk {

namespace {

constexpr int kBmWords = 1024;
constexpr int kBmBits = kBmWords * 32;
constexpr int kAcc = 2048;  // residual entries held in LDS per pass

__device__ inline int wmin(int v) {
    for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d));
    return v;
}
__device__ inline int wmax(int v) {
    for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d));
    return v;
}
__device__ inline int wsum(int v) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}
__device__ inline int wscan_excl(int v) {
    const int lane = wave_lane();
    int x = v;
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    return x - v;
}

__device__ inline double mval(const void* M, int e, int f32) {
    return f32 ? (double)static_cast<const float*>(M)[e] : static_cast<const double*>(M)[e];
}

// One wave per column j.  The rows of column j of A_k M - A_0 are the union
// U of rows(A_k(:, l)) for l in M(:, j) and rows(A_0(:, j)); U is built as a
// bitmap over a window of rows, the rank of a row inside U indexes the LDS
// accumulator, and contributions are added column by column of M (rows are
// distinct inside one column, so no two lanes touch the same slot at once).
__global__ void __launch_bounds__(64)
k_residual_columns(int n, const int* Ak_cp, const int* Ak_ri, const double* Ak_v, const int* A0_cp,
                   const int* A0_ri, const double* A0_v, const int* M_cp, const int* M_ri,
                   const void* M_v, int f32, double* col_out, unsigned long long* status) {
    __shared__ unsigned bm[kBmWords];
    __shared__ int wpre[kBmWords];
    __shared__ double acc[kAcc];
    const int lane = wave_lane();
    for (int j = blockIdx.x; j < n; j += gridDim.x) {
        const int ma = M_cp[j], mb = M_cp[j + 1];
        // window of rows
        int mn = INT_MAX, mx = -1;
        for (int t = ma + lane; t < mb; t += 64) {
            const int l = M_ri[t];
            if (l < 0 || l >= n) {
                report(status, j, kStIndex);
                continue;
            }
            const int qa = Ak_cp[l], qb = Ak_cp[l + 1];
            if (qb > qa) {
                mn = min(mn, Ak_ri[qa]);
                mx = max(mx, Ak_ri[qb - 1]);
            }
        }
        if (A0_cp[j + 1] > A0_cp[j]) {
            mn = min(mn, A0_ri[A0_cp[j]]);
            mx = max(mx, A0_ri[A0_cp[j + 1] - 1]);
        }
        const int lo = wmin(mn), hi = wmax(mx);
        double colsum = 0.0;
        for (int base = lo; base <= hi; base += kBmBits) {
            const int nbits = min(kBmBits, hi - base + 1);
            const int nw = (nbits + 31) >> 5;
            for (int w = lane; w < nw; w += 64) bm[w] = 0u;
            wave_sync();
            for (int t = ma + lane; t < mb; t += 64) {
                const int l = M_ri[t];
                if (l < 0 || l >= n) continue;
                for (int f = Ak_cp[l]; f < Ak_cp[l + 1]; ++f) {
                    const int r = Ak_ri[f] - base;
                    if (r >= 0 && r < kBmBits) atomicOr(&bm[r >> 5], 1u << (r & 31));
                }
            }
            for (int e = A0_cp[j] + lane; e < A0_cp[j + 1]; e += 64) {
                const int r = A0_ri[e] - base;
                if (r >= 0 && r < kBmBits) atomicOr(&bm[r >> 5], 1u << (r & 31));
            }
            wave_sync();
            const int wpl = (nw + 63) >> 6;
            const int w0 = lane * wpl;
            int c = 0;
            for (int w = w0; w < min(nw, w0 + wpl); ++w) c += __popc(bm[w]);
            int run = wscan_excl(c);
            for (int w = w0; w < min(nw, w0 + wpl); ++w) {
                wpre[w] = run;
                run += __popc(bm[w]);
            }
            const int cnt = wsum(c);
            wave_sync();
            // accumulate in rank ranges of kAcc entries
            for (int r0 = 0; r0 < cnt; r0 += kAcc) {
                const int rn = min(kAcc, cnt - r0);
                for (int i = lane; i < rn; i += 64) acc[i] = 0.0;
                wave_sync();
                for (int t = ma; t < mb; ++t) {
                    const int l = M_ri[t];
                    if (l < 0 || l >= n) continue;
                    const double mlj = mval(M_v, t, f32);
                    for (int f = Ak_cp[l] + lane; f < Ak_cp[l + 1]; f += 64) {
                        const int r = Ak_ri[f] - base;
                        if (r >= 0 && r < kBmBits) {
                            const int w = r >> 5;
                            const int rank = wpre[w] + __popc(bm[w] & ((1u << (r & 31)) - 1u)) - r0;
                            if (rank >= 0 && rank < rn) acc[rank] += Ak_v[f] * mlj;
                        }
                    }
                    wave_sync();
                }
                for (int e = A0_cp[j] + lane; e < A0_cp[j + 1]; e += 64) {
                    const int r = A0_ri[e] - base;
                    if (r >= 0 && r < kBmBits) {
                        const int w = r >> 5;
                        const int rank = wpre[w] + __popc(bm[w] & ((1u << (r & 31)) - 1u)) - r0;
                        if (rank >= 0 && rank < rn) acc[rank] -= A0_v[e];
                    }
                }
                wave_sync();
                double s = 0.0;
                for (int i = lane; i < rn; i += 64) s += acc[i] * acc[i];
                for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
                colsum += s;
                wave_sync();
            }
        }
        if (lane == 0) col_out[j] = colsum;
    }
}

}  // namespace

hipError_t residual_columns(int n, const int* Ak_cp, const int* Ak_ri, const double* Ak_v,
                            const int* A0_cp, const int* A0_ri, const double* A0_v, const int* M_cp,
                            const int* M_ri, const void* M_v, int m_is_f32, double* col_out,
                            unsigned long long* status, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = std::min(n, 256 * 32);
    hipLaunchKernelGGL(k_residual_columns, dim3(grid), dim3(64), 0, s, n, Ak_cp, Ak_ri, Ak_v, A0_cp,
                       A0_ri, A0_v, M_cp, M_ri, M_v, m_is_f32, col_out, status);
    return hipGetLastError();
}

// ----------------------------------------------------------------- apply

namespace {

__global__ void k_tcount(int64_t nnz, const int* ri, int n, int* rowcount) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) {
        const int r = ri[e];
        if (r >= 0 && r < n) atomicAdd(&rowcount[r], 1);
    }
}

__global__ void k_tfill(int n, const int* cp, const int* ri, const int* rowptr, int* cursor, int* colind,
                        int* perm) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int e = cp[j]; e < cp[j + 1]; ++e) {
        const int r = ri[e];
        if (r < 0 || r >= n) continue;
        const int slot = rowptr[r] + atomicAdd(&cursor[r], 1);
        colind[slot] = j;
        perm[slot] = e;
    }
}

// insertion sort of each row's (col, perm) by column: makes the row view
// independent of the atomic slot order
__global__ void k_tsort(int n, const int* rowptr, int* colind, int* perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int a = rowptr[i], b = rowptr[i + 1];
    for (int x = a + 1; x < b; ++x) {
        const int c = colind[x], p = perm[x];
        int y = x - 1;
        while (y >= a && colind[y] > c) {
            colind[y + 1] = colind[y];
            perm[y + 1] = perm[y];
            --y;
        }
        colind[y + 1] = c;
        perm[y + 1] = p;
    }
}

// y = M x over the row view: kSpmvLanes lanes per row, so that the lanes of
// a wave read each row's column indices (and values) as one contiguous run
// instead of one entry of 64 different rows.  Lane g sums entries g, g + 4,
// ... of its row in ascending order; the four partials are added by the
// quad exchanges of group_sum (the same order on every call).  Each lane
// issues the loads of kSpmvUnroll of its entries (indices and values, then
// the x values they select) before it adds them, so a row of up to 16
// entries costs two dependent round trips instead of two per entry; slots
// past the row's end load a valid entry of the row with a zero value, which
// adds an exact zero.
// PERM: the values are read through the row view's permutation (else they
// are in the row view's order).
constexpr int kSpmvLanes = 4;
constexpr int kSpmvUnroll = 4;
template <bool F32, bool PERM>
__global__ void __launch_bounds__(256)
k_spmv_rows(int n, const int* rowptr, const int* colind, const int* perm, const void* val, const double* x,
            double* y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t / kSpmvLanes, g = t % kSpmvLanes;
    double s = 0.0;
    if (i < n) {
        const int b = rowptr[i + 1];
        for (int e = rowptr[i] + g; e < b; e += kSpmvLanes * kSpmvUnroll) {
            int c[kSpmvUnroll];
            double v[kSpmvUnroll], xv[kSpmvUnroll];
#pragma unroll
            for (int u = 0; u < kSpmvUnroll; ++u) {
                const int eu = e + u * kSpmvLanes < b ? e + u * kSpmvLanes : e;   // e < b: in the row
                c[u] = colind[eu];
                const int ev = PERM ? perm[eu] : eu;
                v[u] = F32 ? (double)static_cast<const float*>(val)[ev] : static_cast<const double*>(val)[ev];
            }
#pragma unroll
            for (int u = 0; u < kSpmvUnroll; ++u) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < kSpmvUnroll; ++u) s = fma(e + u * kSpmvLanes < b ? v[u] : 0.0, xv[u], s);
        }
    }
    s = group_sum<kSpmvLanes>(s);   // every lane takes part: rows past n add zeros
    if (i < n && g == 0) y[i] = s;
}

__global__ void k_permute_vals(int64_t nnz, const int* perm, const void* val, int f32, void* out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    if (f32) static_cast<float*>(out)[e] = static_cast<const float*>(val)[perm[e]];
    else static_cast<double*>(out)[e] = static_cast<const double*>(val)[perm[e]];
}

}  // namespace

__global__ void k_identity_queue(int n, int* queue, int* bstart) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) queue[i] = i;
    if (i == 0) {
        bstart[0] = 0;
        bstart[1] = n;
    }
}

hipError_t identity_queue(int n, int* queue, int* bstart, hipStream_t s) {
    hipLaunchKernelGGL(k_identity_queue, dim3((unsigned)((std::max(n, 1) + 255) / 256)), dim3(256), 0, s, n, queue,
                       bstart);
    return hipGetLastError();
}

__global__ void k_fill_i32(int* p, int64_t count, int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

hipError_t fill_i32(int* p, int64_t count, int v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t transpose_count(int n, const int* cp, const int* ri, int64_t nnz, int* rowcount,
                           hipStream_t s) {
    (void)cp;
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tcount, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, ri, n, rowcount);
    return hipGetLastError();
}

hipError_t transpose_fill(int n, const int* cp, const int* ri, const int* rowptr, int* cursor,
                          int* colind, int* perm, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tfill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, cp, ri, rowptr, cursor,
                       colind, perm);
    return hipGetLastError();
}

hipError_t transpose_sort_rows(int n, const int* rowptr, int* colind, int* perm, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tsort, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, rowptr, colind, perm);
    return hipGetLastError();
}

hipError_t spmv_rows(int n, const int* rowptr, const int* colind, const int* perm, const void* val,
                     int val_f32, const double* x, double* y, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t threads = (int64_t)n * kSpmvLanes;
    const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
    if (val_f32 && perm) hipLaunchKernelGGL((k_spmv_rows<true, true>), grid, block, 0, s, n, rowptr, colind, perm, val, x, y);
    else if (val_f32) hipLaunchKernelGGL((k_spmv_rows<true, false>), grid, block, 0, s, n, rowptr, colind, perm, val, x, y);
    else if (perm) hipLaunchKernelGGL((k_spmv_rows<false, true>), grid, block, 0, s, n, rowptr, colind, perm, val, x, y);
    else hipLaunchKernelGGL((k_spmv_rows<false, false>), grid, block, 0, s, n, rowptr, colind, perm, val, x, y);
    return hipGetLastError();
}

hipError_t permute_vals(int64_t nnz, const int* perm, const void* val, int val_f32, void* out, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_vals, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, nnz, perm, val,
                       val_f32, out);
    return hipGetLastError();
}

}  // namespace samk
