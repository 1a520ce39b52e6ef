// sam_symbolic.hip -- integer (symbolic) kernels of the SAM library for
// gfx950: prefix sums, CSC structure checks, the sparsification rules and
// level expansion that form the pattern S (Sections 3-4 of the paper), and
// the plan of the column problems (row sets, gather positions, buckets).
//
// Row-set construction uses a per-wave LDS bitmap over the window of
// candidate rows: every candidate sets its bit (ds_or), and the ascending
// union, its size and the rank of any row inside it follow from popcounts,
// with no sort.  Windows wider than the bitmap are processed in chunks.
#include "sam_device.hpp"
#include "sam_kernels.hpp"

#include <algorithm>
#include <climits>

namespace samk {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
    // Hillis-Steele over kScanThreads values in LDS
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        int64_t add = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t incl = sh[t];
    *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

// Scans in[0..N) where in[i] = i < n_in ? src[i] : 0 (the last virtual zero
// gives the total at off[n_in]).
template <typename Tin>
__global__ void __launch_bounds__(kScanThreads)
k_scan_local(const Tin* src, int64_t n_in, int64_t N, int64_t* out, int64_t* block_tot) {
    __shared__ int64_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        v[i] = (idx < n_in) ? (int64_t)src[idx] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t pre = block_exclusive_scan(s, sh, &tot);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < N) out[idx] = pre;
        pre += v[i];
    }
    if (threadIdx.x == 0) block_tot[blockIdx.x] = tot;
}

__global__ void k_scan_add(int64_t* out, int64_t N, const int64_t* block_off) {
    const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    const int64_t add = block_off[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = i + (int64_t)k * kScanThreads;
        if (idx < N) out[idx] += add;
    }
}

__global__ void k_to_i32(const int64_t* off, int64_t N, int* off32, int* overflow) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        int64_t v = off[i];
        if (off32) off32[i] = (int)v;
        if (v > INT_MAX && overflow) atomicOr(overflow, 1);
    }
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

size_t scan_temp_bytes(int64_t n) {
    int64_t N = n + 1;
    size_t bytes = 0;
    while (true) {
        int64_t nb = ceil_div(N, kScanTile);
        bytes += (size_t)(2 * nb + 1) * sizeof(int64_t);
        if (nb <= 1) break;
        N = nb;
    }
    return bytes + 256;
}

// Recursive three-phase scan.  Level buffers live in `temp`.
static hipError_t scan_i64_levels(int64_t* out, int64_t N, int64_t* temp, hipStream_t s);

template <typename Tin>
static hipError_t scan_any(const Tin* src, int64_t n_in, int64_t N, int64_t* out, int64_t* temp,
                           hipStream_t s) {
    const int64_t nb = ceil_div(N, kScanTile);
    int64_t* tot = temp;
    int64_t* totoff = temp + nb;
    hipLaunchKernelGGL(k_scan_local<Tin>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, src, n_in, N,
                       out, tot);
    if (nb > 1) {
        // exclusive scan of the block totals (nb values, one virtual zero not needed)
        hipError_t e = scan_any<int64_t>(tot, nb, nb, totoff, temp + 2 * nb + 1, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, out, N, totoff);
    }
    return hipGetLastError();
}

static hipError_t scan_i64_levels(int64_t* out, int64_t N, int64_t* temp, hipStream_t s) {
    return scan_any<int64_t>(out, N, N, out, temp, s);
}

hipError_t scan_counts(const int* counts, int64_t n, int64_t* off, int* off32, int* overflow,
                       void* temp, hipStream_t s) {
    const int64_t N = n + 1;
    hipError_t e = scan_any<int>(counts, n, N, off, (int64_t*)temp, s);
    if (e != hipSuccess) return e;
    if (off32 || overflow) {
        hipLaunchKernelGGL(k_to_i32, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, off, N, off32,
                           overflow);
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------- checks

__global__ void k_check_csc(int n, int nnz, const int* cp, const int* ri, int* bad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int a = cp[j], b = cp[j + 1];
    bool ok = a >= 0 && a <= b && b <= nnz;
    if (j == 0 && a != 0) ok = false;
    if (j == n - 1 && b != nnz) ok = false;
    if (ok) {
        int prev = -1;
        for (int e = a; e < b; ++e) {
            int r = ri[e];
            if (r <= prev || r >= n) { ok = false; break; }
            prev = r;
        }
    }
    if (!ok) atomicMin(bad, j);
}

hipError_t check_csc(int n, int nnz, const int* cp, const int* ri, int* bad, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_csc, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, nnz, cp, ri,
                       bad);
    return hipGetLastError();
}

// ------------------------------------------------------------ sparsify

// D_jj = |a_jj| if nonzero, else 1 (Section 4, definition of D).
__global__ void k_diag_scale(int n, const int* cp, const int* ri, const double* v, double* D) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double d = 0.0;
    for (int e = cp[j]; e < cp[j + 1]; ++e)
        if (ri[e] == j) d = fabs(v[e]);
    D[j] = d > 0.0 ? d : 1.0;
}

// Decision for entry e of column j (the diagonal is handled by the caller).
__device__ inline bool keep_entry(int j, int i, double a, const SparsifySpec& sp, const double* D,
                                  double colmax, int rank_lfil) {
    switch (sp.kind) {
        case 0:
            return true;
        case 1: {
            double s = sp.global_scale > 0 ? sqrt(D[i] * D[j]) : 1.0 / sqrt(D[i] * D[j]);
            return fabs(a) * s > sp.thresh;
        }
        case 2:
            return fabs(a) > (1.0 - sp.tau) * colmax;
        default:
            return rank_lfil < sp.lfil - 1;
    }
}

// rank of off-diagonal entry e among the column's off-diagonals by
// (magnitude descending, row ascending)
__device__ inline int lfil_rank(int j, int a, int b, int e, const int* ri, const double* v) {
    const double me = fabs(v[e]);
    const int re = ri[e];
    int rank = 0;
    for (int f = a; f < b; ++f) {
        int rf = ri[f];
        if (rf == j || f == e) continue;
        double mf = fabs(v[f]);
        if (mf > me || (mf == me && rf < re)) ++rank;
    }
    return rank;
}

template <bool FILL>
__global__ void k_sparsify(int n, const int* cp, const int* ri, const double* v, SparsifySpec sp,
                           const double* D, int* counts, const int* out_cp, int* out_ri) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int a = cp[j], b = cp[j + 1];
    double colmax = 0.0;
    if (sp.kind == 2)
        for (int e = a; e < b; ++e) colmax = fmax(colmax, fabs(v[e]));
    int cnt = 0;
    bool diag_done = false;
    int o = FILL ? out_cp[j] : 0;
    for (int e = a; e < b; ++e) {
        const int i = ri[e];
        bool keep;
        if (i == j) {
            keep = true;
        } else {
            int rk = sp.kind == 3 ? lfil_rank(j, a, b, e, ri, v) : 0;
            keep = keep_entry(j, i, v ? v[e] : 0.0, sp, D, colmax, rk);
        }
        if (!diag_done && i > j) {  // diagonal not stored: insert before
            if (FILL) out_ri[o + cnt] = j;
            ++cnt;
            diag_done = true;
        }
        if (i == j) diag_done = true;
        if (keep) {
            if (FILL) out_ri[o + cnt] = i;
            ++cnt;
        }
    }
    if (!diag_done) {
        if (FILL) out_ri[o + cnt] = j;
        ++cnt;
    }
    if (!FILL) counts[j] = cnt;
}

hipError_t sparsify_count(int n, const int* cp, const int* ri, const double* v, SparsifySpec sp,
                          double* dscratch, int* counts, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)ceil_div(n, 256);
    if (sp.kind == 1) hipLaunchKernelGGL(k_diag_scale, dim3(nb), dim3(256), 0, s, n, cp, ri, v, dscratch);
    hipLaunchKernelGGL(k_sparsify<false>, dim3(nb), dim3(256), 0, s, n, cp, ri, v, sp, dscratch, counts,
                       nullptr, nullptr);
    return hipGetLastError();
}

hipError_t sparsify_fill(int n, const int* cp, const int* ri, const double* v, SparsifySpec sp,
                         const double* dscratch, const int* out_cp, int* out_ri, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)ceil_div(n, 256);
    hipLaunchKernelGGL(k_sparsify<true>, dim3(nb), dim3(256), 0, s, n, cp, ri, v, sp, dscratch, nullptr,
                       out_cp, out_ri);
    return hipGetLastError();
}

// ------------------------------------------------------- row-set bitmaps
//
// One 16-lane DPP row per column (four columns per wave).  The candidates of
// column j are the rows of Q(:, l) for l in P(:, j); lane g of the group owns
// the lists l = P(:, j)[g], P(:, j)[g+16], ...  The window of candidate rows
// is swept in chunks of kChunk rows: each chunk gets an LDS bitmap (four
// 32-bit words per lane), set with ds_or, counted with popcount and a row
// prefix scan.  After a chunk the sweep jumps to the smallest candidate
// beyond it, so only occupied chunks cost anything, whatever the bandwidth.

constexpr int kGS = 16;                   // lanes per column
constexpr int kChunkWords = 64;           // 4 words per lane
constexpr int kChunk = kChunkWords * 32;  // 2048 rows
constexpr int kSymThreads = 256;
constexpr int kGroupsPerBlock = kSymThreads / kGS;

template <int CTRL>
__device__ inline int dppi(int v) { return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false); }

// sums / minima over the 16 lanes of a row (all lanes get the result)
__device__ inline int row_sum_i(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true);
    return v;
}
__device__ inline int row_min_i(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true));
    return v;
}
// exclusive prefix sum inside the row (Kogge-Stone with row_shr; lanes whose
// source lies before the row start add 0)
__device__ inline int row_excl_scan_i(int v) {
    int x = v;
    x += dppi<0x111>(x);
    x += dppi<0x112>(x);
    x += dppi<0x114>(x);
    x += dppi<0x118>(x);
    return x - v;
}

enum { kModeCount = 0, kModeFill = 1, kModePositions = 2 };

constexpr int kListRounds = 2;   // lists per lane held in registers (32 per column)
constexpr int kListLen = 8;      // entries per list held in registers

__device__ inline int row_max_i(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true));
    return v;
}

// Rank of row d (relative to the chunk base) inside the chunk's bitmap.
__device__ inline int chunk_rank(const unsigned* bm, const int* wpre, int d) {
    const int w = d >> 5;
    return wpre[w] + __popc(bm[w] & ((1u << (d & 31)) - 1u));
}

template <int MODE>
__global__ void __launch_bounds__(kSymThreads)
k_union(int n, const int* P_cp, const int* P_ri, const int* Q_cp, const int* Q_ri, int* counts,
        const int* out_cp, int* out_ri, const int64_t* eoff, unsigned char* posA, const int* A0_cp,
        const int* A0_ri, unsigned char* posB, int* bad) {
    __shared__ unsigned bm_all[kGroupsPerBlock][kChunkWords];
    __shared__ int pre_all[kGroupsPerBlock][kChunkWords];
    const int grp = threadIdx.x / kGS;
    const int g = threadIdx.x % kGS;
    unsigned* bm = bm_all[grp];
    int* wpre = pre_all[grp];
    const int stride = gridDim.x * kGroupsPerBlock;
    for (int j = blockIdx.x * kGroupsPerBlock + grp; j < n; j += stride) {
        const int pa = P_cp[j], pb = P_cp[j + 1];
        // Lists t = pa + g + 16 u of this lane, first kListLen rows of each in
        // registers (all loads independent); `big` marks columns that need the
        // memory loops (more than 32 lists, or a list longer than kListLen).
        int qa[kListRounds], len[kListRounds], lofs[kListRounds];
        int rows[kListRounds][kListLen];
        int big = (pb - pa > kGS * kListRounds) ? 1 : 0;
        int lo = INT_MAX, carry = 0;
#pragma unroll
        for (int u = 0; u < kListRounds; ++u) {
            const int t = pa + g + u * kGS;
            int l = -1;
            if (t < pb) {
                l = P_ri[t];
                if (l < 0 || l >= n) {
                    if (bad) atomicMin(bad, j);
                    l = -1;
                }
            }
            qa[u] = l >= 0 ? Q_cp[l] : 0;
            len[u] = l >= 0 ? Q_cp[l + 1] - qa[u] : 0;
            big |= len[u] > kListLen ? 1 : 0;
            // flat offset of this list among the column's gathered entries
            lofs[u] = carry + row_excl_scan_i(len[u]);
            carry += row_sum_i(len[u]);
            if (len[u] > 0) {
#pragma unroll
                for (int e = 0; e < kListLen; ++e) {
                    const bool ok = e < len[u];
                    const int r = Q_ri[qa[u] + (ok ? e : 0)];  // clamped: always in bounds
                    rows[u][e] = ok ? r : INT_MAX;
                }
            } else {
#pragma unroll
                for (int e = 0; e < kListLen; ++e) rows[u][e] = INT_MAX;
            }
            lo = min(lo, rows[u][0]);
        }
        big = row_max_i(big);
        if (big) {  // heads of every list, from memory
            lo = INT_MAX;
            for (int t = pa + g; t < pb; t += kGS) {
                const int l = P_ri[t];
                if (l >= 0 && l < n && Q_cp[l + 1] > Q_cp[l]) lo = min(lo, Q_ri[Q_cp[l]]);
            }
        }
        lo = row_min_i(lo);
        if (MODE == kModePositions)
            for (int e = A0_cp[j] + g; e < A0_cp[j + 1]; e += kGS) posB[e] = 0xFF;
        int running = 0;
        int base = lo;
        while (base != INT_MAX) {
#pragma unroll
            for (int w = 0; w < 4; ++w) bm[g * 4 + w] = 0u;
            wave_sync();
            int next = INT_MAX;
            if (!big) {
#pragma unroll
                for (int u = 0; u < kListRounds; ++u)
#pragma unroll
                    for (int e = 0; e < kListLen; ++e) {
                        const int r = rows[u][e];
                        const int d = r - base;  // r = INT_MAX for empty slots: d >= kChunk
                        if (d >= 0 && d < kChunk) atomicOr(&bm[d >> 5], 1u << (d & 31));
                        if (d >= kChunk) next = min(next, r);
                    }
            } else {
                for (int t = pa + g; t < pb; t += kGS) {
                    const int l = P_ri[t];
                    if (l < 0 || l >= n) continue;
                    for (int f = Q_cp[l]; f < Q_cp[l + 1]; ++f) {
                        const int r = Q_ri[f];
                        const int d = r - base;
                        if (d >= 0 && d < kChunk) atomicOr(&bm[d >> 5], 1u << (d & 31));
                        if (d >= kChunk) next = min(next, r);
                    }
                }
            }
            wave_sync();
            int c = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) c += __popc(bm[g * 4 + w]);
            const int pre = row_excl_scan_i(c);
            const int tot = row_sum_i(c);
            if (MODE != kModeCount) {
                int run = running + pre;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    wpre[g * 4 + w] = run;
                    run += __popc(bm[g * 4 + w]);
                }
            }
            wave_sync();
            if (MODE == kModeFill) {
                int o = out_cp[j] + running + pre;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    unsigned x = bm[g * 4 + w];
                    while (x) {
                        const int b = __ffs(x) - 1;
                        x &= x - 1;
                        out_ri[o++] = base + ((g * 4 + w) << 5) + b;
                    }
                }
            }
            if (MODE == kModePositions) {
                // ranks of the gathered A_k entries, in the order of the lists
                unsigned char* pj = posA + eoff[j];
                if (!big) {
#pragma unroll
                    for (int u = 0; u < kListRounds; ++u)
#pragma unroll
                        for (int e = 0; e < kListLen; ++e) {
                            const int d = rows[u][e] - base;
                            if (d >= 0 && d < kChunk) pj[lofs[u] + e] = (unsigned char)min(chunk_rank(bm, wpre, d), 255);
                        }
                } else {
                    int cy = 0;
                    for (int t0 = pa; t0 < pb; t0 += kGS) {
                        const int t = t0 + g;
                        int l = -1, ln = 0;
                        if (t < pb) {
                            l = P_ri[t];
                            if (l >= 0 && l < n) ln = Q_cp[l + 1] - Q_cp[l];
                        }
                        const int off = cy + row_excl_scan_i(ln);
                        for (int f = 0; f < ln; ++f) {
                            const int d = Q_ri[Q_cp[l] + f] - base;
                            if (d >= 0 && d < kChunk) pj[off + f] = (unsigned char)min(chunk_rank(bm, wpre, d), 255);
                        }
                        cy += row_sum_i(ln);
                    }
                }
                for (int e = A0_cp[j] + g; e < A0_cp[j + 1]; e += kGS) {
                    const int d = A0_ri[e] - base;
                    if (d >= 0 && d < kChunk && ((bm[d >> 5] >> (d & 31)) & 1u))
                        posB[e] = (unsigned char)min(chunk_rank(bm, wpre, d), 254);
                }
            }
            running += tot;
            base = row_min_i(next);
            wave_sync();
        }
        if (g == 0 && MODE != kModeFill) counts[j] = running;  // |union| (= |I_j| for positions)
    }
}

static unsigned union_grid(int n) {
    int64_t blocks = ceil_div(n, kGroupsPerBlock);
    return (unsigned)std::min<int64_t>(blocks, 256 * 32);
}

hipError_t expand_count(int n, const int* P_cp, const int* P_ri, const int* Q_cp, const int* Q_ri,
                        int* counts, int* bad, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_union<kModeCount>, dim3(union_grid(n)), dim3(kSymThreads), 0, s, n, P_cp, P_ri, Q_cp,
                       Q_ri, counts, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, bad);
    return hipGetLastError();
}

hipError_t expand_fill(int n, const int* P_cp, const int* P_ri, const int* Q_cp, const int* Q_ri,
                       const int* out_cp, int* out_ri, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_union<kModeFill>, dim3(union_grid(n)), dim3(kSymThreads), 0, s, n, P_cp, P_ri, Q_cp,
                       Q_ri, nullptr, out_cp, out_ri, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ plan

__global__ void k_gather_count(int n, const int* S_cp, const int* S_ri, const int* Ak_cp, int* counts) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int s = 0;
    for (int e = S_cp[j]; e < S_cp[j + 1]; ++e) {
        int l = S_ri[e];
        if (l >= 0 && l < n) s += Ak_cp[l + 1] - Ak_cp[l];
    }
    counts[j] = s;
}

hipError_t plan_gather_count(int n, const int* S_cp, const int* S_ri, const int* Ak_cp, int* counts,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_count, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, S_cp, S_ri,
                       Ak_cp, counts);
    return hipGetLastError();
}

// Row set I_j of every column as a bitmap sweep; every gathered A_k entry (in
// the order: entries of A_k(:, J_j[0]), then of A_k(:, J_j[1]), ...) gets its
// rank inside I_j, and so does every entry of A_0(:, j) (0xFF when its row is
// not in I_j).  nI[j] = |I_j|.
hipError_t plan_positions(int n, const int* S_cp, const int* S_ri, const int* Ak_cp, const int* Ak_ri,
                          const int* A0_cp, const int* A0_ri, const int64_t* eoff, int* nI,
                          unsigned char* posA, unsigned char* posB, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_union<kModePositions>, dim3(union_grid(n)), dim3(kSymThreads), 0, s, n, S_cp, S_ri,
                       Ak_cp, Ak_ri, nI, nullptr, nullptr, eoff, posA, A0_cp, A0_ri, posB, nullptr);
    return hipGetLastError();
}

// --------------------------------------------------------------- buckets

constexpr int kBucketThreads = 256;

__device__ inline int bucket_of(int nI, int nJ, const BucketTable& tab) {
    const int rows = tab.rows_plus_cols ? nI + nJ : nI;
    for (int b = 0; b < tab.nb; ++b)
        if (rows <= tab.max_rows[b] && nJ <= tab.max_cols[b]) return b;
    return -1;
}

// hist is bucket-major: hist[b * nblocks + block]
__global__ void __launch_bounds__(kBucketThreads)
k_bucket_hist(int n, const int* S_cp, const int* nI, BucketTable tab, int* hist, int* unfit,
              unsigned long long* status) {
    __shared__ int h[kMaxBuckets];
    if (threadIdx.x < kMaxBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    const int j = blockIdx.x * kBucketThreads + threadIdx.x;
    if (j < n) {
        int b = bucket_of(nI[j], S_cp[j + 1] - S_cp[j], tab);
        if (b >= 0) {
            atomicAdd(&h[b], 1);
        } else {
            if (unfit) atomicAdd(unfit, 1);
            if (status) report(status, j, kStUnsupported);
        }
    }
    __syncthreads();
    if (threadIdx.x < tab.nb) hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kBucketThreads)
k_bucket_scatter(int n, const int* S_cp, const int* nI, BucketTable tab, const int64_t* off,
                 int* queue) {
    __shared__ int wcount[kBucketThreads / 64][kMaxBuckets];
    const int j = blockIdx.x * kBucketThreads + threadIdx.x;
    const int wv = threadIdx.x >> 6;
    const int lane = wave_lane();
    int b = -1;
    if (j < n) b = bucket_of(nI[j], S_cp[j + 1] - S_cp[j], tab);
    int my_rank = 0;
    for (int k = 0; k < tab.nb; ++k) {
        unsigned long long m = __ballot(b == k);
        if (b == k) my_rank = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[wv][k] = __popcll(m);
    }
    __syncthreads();
    if (b >= 0) {
        int r = my_rank;
        for (int w = 0; w < wv; ++w) r += wcount[w][b];
        queue[off[(int64_t)b * gridDim.x + blockIdx.x] + r] = j;
    }
}

__global__ void k_bucket_starts(int nb, int nblocks, const int64_t* off, int* bstart) {
    const int b = threadIdx.x;
    if (b <= nb) bstart[b] = (int)off[(int64_t)b * nblocks];
}

size_t bucket_temp_bytes(int n) {
    int64_t nblocks = ceil_div(std::max(n, 1), kBucketThreads);
    int64_t cells = nblocks * kMaxBuckets;
    return (size_t)cells * sizeof(int) + (size_t)(cells + 1) * sizeof(int64_t) + scan_temp_bytes(cells) + 512;
}

hipError_t bucket_sort(int n, const int* S_cp, const int* nI, BucketTable tab, int* queue, int* bstart,
                       int* unfit, unsigned long long* status, void* temp, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nblocks = (int)ceil_div(n, kBucketThreads);
    const int64_t cells = (int64_t)nblocks * tab.nb;
    char* p = (char*)temp;
    int* hist = (int*)p;
    p += (((size_t)nblocks * kMaxBuckets * sizeof(int)) + 255) / 256 * 256;
    int64_t* off = (int64_t*)p;
    p += (((size_t)(nblocks * kMaxBuckets + 1) * sizeof(int64_t)) + 255) / 256 * 256;
    hipLaunchKernelGGL(k_bucket_hist, dim3(nblocks), dim3(kBucketThreads), 0, s, n, S_cp, nI, tab, hist,
                       unfit, status);
    hipError_t e = scan_counts(hist, cells, off, nullptr, nullptr, p, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bucket_scatter, dim3(nblocks), dim3(kBucketThreads), 0, s, n, S_cp, nI, tab, off,
                       queue);
    hipLaunchKernelGGL(k_bucket_starts, dim3(1), dim3(kMaxBuckets + 1), 0, s, tab.nb, nblocks, off, bstart);
    return hipGetLastError();
}

}  // namespace samk
