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
constexpr int kScanTile = kScanThreads * kScanItems;   // 1024 values per tile

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Inclusive scan of one int64 per lane over the wave (shuffles through
// ds_bpermute; lanes below the distance add nothing).
__device__ inline int64_t wave_incl_scan(int64_t v) {
    const int lane = wave_lane();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

__device__ inline int64_t block_sum_i64(int64_t v, int64_t* sh) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (wave_lane() == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// Pass 1: the sum of every tile of kScanTile inputs (and the largest input,
// when asked).
template <typename Tin>
__global__ void __launch_bounds__(kScanThreads)
k_scan_tiles(const Tin* src, int64_t n_in, int64_t* tile_sum, int* maxval) {
    __shared__ int64_t sh[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0, mx = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        const int64_t x = idx < n_in ? (int64_t)src[idx] : 0;
        s += x;
        mx = x > mx ? x : mx;
    }
    const int64_t t = block_sum_i64(s, sh);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = t;
    if (maxval) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const int64_t o = __shfl_xor(mx, d, 64);
            mx = o > mx ? o : mx;
        }
        if (wave_lane() == 0 && mx > 0) atomicMax(maxval, (int)(mx < INT_MAX ? mx : INT_MAX));
    }
}

// Pass 2: every tile adds the sums of the tiles before it (read directly
// when tile_off is null, else taken from tile_off) and scans its own inputs.
template <typename Tin>
__global__ void __launch_bounds__(kScanThreads)
k_scan_apply(const Tin* src, int64_t n_in, int64_t N, const int64_t* tile_sum, const int64_t* tile_off,
             int64_t* out, int* out32, int* overflow) {
    __shared__ int64_t sh[kScanThreads / 64];
    __shared__ int64_t wsum[kScanThreads / 64];
    const int lane = wave_lane();
    const int wv = threadIdx.x >> 6;
    const int tile = blockIdx.x;
    int64_t before_tile;
    if (tile_off) {
        before_tile = tile_off[tile];
    } else {
        int64_t acc = 0;
        for (int t = threadIdx.x; t < tile; t += kScanThreads) acc += tile_sum[t];
        before_tile = block_sum_i64(acc, sh);
    }
    const int64_t base = (int64_t)tile * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < n_in ? (int64_t)src[idx] : 0;
        s += v[i];
    }
    const int64_t wincl = wave_incl_scan(s);
    if (lane == 63) wsum[wv] = wincl;
    __syncthreads();
    int64_t run = before_tile + wincl - s;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) run += w < wv ? wsum[w] : 0;
    bool big = false;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        if (idx < N) {
            out[idx] = run;
            if (out32) out32[idx] = (int)run;
            big |= run > INT_MAX;
        }
        run += v[i];
    }
    if (overflow && big) atomicOr(overflow, 1);
}

constexpr int64_t kDirectTiles = 2048;   // tiles summed directly by pass 2

int64_t scan_tiles(int64_t N) { return std::max<int64_t>(ceil_div(N, kScanTile), 1); }

size_t scan_temp_rec(int64_t N) {
    const int64_t nt = scan_tiles(N);
    size_t b = (size_t)((nt * 8 + 255) / 256) * 256;
    if (nt > kDirectTiles) b += (size_t)(((nt + 1) * 8 + 255) / 256) * 256 + scan_temp_rec(nt);
    return b;
}

}  // namespace

size_t scan_temp_bytes(int64_t n) { return scan_temp_rec(n + 1) + 256; }

// Reduce-then-scan: two launches while the tile count allows the direct
// sum (2^21 values), recursing on the tile sums beyond that.  No state
// survives between calls, so the temporary memory may hold anything.
template <typename Tin>
static hipError_t scan_any(const Tin* src, int64_t n_in, int64_t N, int64_t* out, int* out32, int* overflow,
                           int* maxval, void* temp, hipStream_t s) {
    const int64_t nt = scan_tiles(N);
    char* p = (char*)temp;
    int64_t* tile_sum = (int64_t*)p;
    p += ((nt * 8 + 255) / 256) * 256;
    int64_t* tile_off = nullptr;
    hipLaunchKernelGGL(k_scan_tiles<Tin>, dim3((unsigned)nt), dim3(kScanThreads), 0, s, src, n_in, tile_sum, maxval);
    if (nt > kDirectTiles) {
        tile_off = (int64_t*)p;
        p += (((nt + 1) * 8 + 255) / 256) * 256;
        hipError_t e = scan_any<int64_t>(tile_sum, nt, nt, tile_off, nullptr, nullptr, nullptr, p, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scan_apply<Tin>, dim3((unsigned)nt), dim3(kScanThreads), 0, s, src, n_in, N, tile_sum,
                       tile_off, out, out32, overflow);
    return hipGetLastError();
}

hipError_t scan_counts(const int* counts, int64_t n, int64_t* off, int* off32, int* overflow,
                       void* temp, hipStream_t s, int* maxcount) {
    return scan_any<int>(counts, n, n + 1, off, off32, overflow, maxcount, temp, s);
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

// The first kSpReg entries of a column are loaded before anything is
// stored: a store through out_ri may alias ri, so a load issued after it
// would wait for the store before it, one memory round trip per entry.
constexpr int kSpReg = 8;

template <bool FILL>
__global__ void k_sparsify(int n, const int* cp, const int* ri, const double* v, SparsifySpec sp,
                           const double* D, int* counts, const int* out_cp, int* out_ri) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int a = cp[j], b = cp[j + 1];
    const int o = FILL ? out_cp[j] : 0;
    int rr[kSpReg];
    double vr[kSpReg];
#pragma unroll
    for (int u = 0; u < kSpReg; ++u) {
        const bool ok = a + u < b;
        rr[u] = ok ? ri[a + u] : 0;
        vr[u] = (ok && v) ? v[a + u] : 0.0;
    }
    double colmax = 0.0;
    if (sp.kind == 2) {
#pragma unroll
        for (int u = 0; u < kSpReg; ++u)
            if (a + u < b) colmax = fmax(colmax, fabs(vr[u]));
        for (int e = a + kSpReg; e < b; ++e) colmax = fmax(colmax, fabs(v[e]));
    }
    int cnt = 0;
    bool diag_done = false;
    auto visit = [&](int e, int i, double x) {
        bool keep;
        if (i == j) {
            keep = true;
        } else {
            int rk = sp.kind == 3 ? lfil_rank(j, a, b, e, ri, v) : 0;
            keep = keep_entry(j, i, x, sp, D, colmax, rk);
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
    };
#pragma unroll
    for (int u = 0; u < kSpReg; ++u)
        if (a + u < b) visit(a + u, rr[u], vr[u]);
    for (int e = a + kSpReg; e < b; ++e) visit(e, ri[e], v ? v[e] : 0.0);
    if (!diag_done) {
        if (FILL) out_ri[o + cnt] = j;
        ++cnt;
    }
    if (counts) counts[j] = cnt;   // the count pass, or a fill into bound-sized slots
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

hipError_t sparsify_slots(int n, const int* cp, const int* ri, const double* v, SparsifySpec sp,
                          double* dscratch, const int* slot_cp, int* slot_ri, int* counts, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)ceil_div(n, 256);
    if (sp.kind == 1) hipLaunchKernelGGL(k_diag_scale, dim3(nb), dim3(256), 0, s, n, cp, ri, v, dscratch);
    hipLaunchKernelGGL(k_sparsify<true>, dim3(nb), dim3(256), 0, s, n, cp, ri, v, sp, dscratch, counts,
                       slot_cp, slot_ri);
    return hipGetLastError();
}

// ------------------------------------------------------- row-set bitmaps
//
// A group of GS lanes (8 or 16: eight or four columns per wave) per column.  The
// candidates of column j are the rows of Q(:, l) for l in P(:, j); lane g of
// the group owns the lists l = P(:, j)[g], P(:, j)[g + GS], ...  The window
// of candidate rows is swept in chunks of kChunk rows: each chunk gets an
// LDS bitmap (128 or 256 words per column), set with ds_or, counted with popcount
// and a prefix scan over the group.  After a chunk the sweep jumps to the
// smallest candidate beyond it, so only occupied chunks cost anything,
// whatever the bandwidth.

// Chunk of the sweep: 4096 rows for eight lanes per column, 8192 for
// sixteen (the 9-point and 3D stencils, whose level-2 row sets span six grid
// lines or planes: at 4096 rows a 1024^2 9-point column took two chunks).
template <int GS>
constexpr int chunk_words() { return GS == 16 ? 256 : 128; }
constexpr int kSymThreads = 256;

template <int CTRL>
__device__ inline int dppi(int v) { return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false); }
template <int CTRL>
__device__ inline int dppb(int v) { return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true); }

// sums / minima / maxima over the GS lanes of a group (all lanes get the
// result): quad exchanges, then the half-row mirror, then (GS = 16) the row
// mirror
template <int GS>
__device__ inline int grp_sum(int v) {
    v += dppb<0xB1>(v);
    v += dppb<0x4E>(v);
    v += dppb<0x141>(v);
    if (GS == 16) v += dppb<0x140>(v);
    return v;
}
template <int GS>
__device__ inline int grp_min(int v) {
    v = min(v, dppb<0xB1>(v));
    v = min(v, dppb<0x4E>(v));
    v = min(v, dppb<0x141>(v));
    if (GS == 16) v = min(v, dppb<0x140>(v));
    return v;
}
template <int GS>
__device__ inline int grp_max(int v) {
    v = max(v, dppb<0xB1>(v));
    v = max(v, dppb<0x4E>(v));
    v = max(v, dppb<0x141>(v));
    if (GS == 16) v = max(v, dppb<0x140>(v));
    return v;
}
// exclusive prefix sum inside the group (Kogge-Stone with row_shr; a lane
// whose source lies before its group's first lane adds 0)
template <int GS>
__device__ inline int grp_excl_scan(int v) {
    const int p = (int)(threadIdx.x & (GS - 1));
    int x = v, y;
    y = dppi<0x111>(x);
    x += (GS == 16 || p >= 1) ? y : 0;
    y = dppi<0x112>(x);
    x += (GS == 16 || p >= 2) ? y : 0;
    y = dppi<0x114>(x);
    x += (GS == 16 || p >= 4) ? y : 0;
    if (GS == 16) x += dppi<0x118>(x);
    return x - v;
}

enum { kModeCount = 0, kModeFill = 1, kModePositions = 2 };

// Bitmap word wi (rows 32 wi .. 32 wi + 31 of the chunk) belongs to lane
// wi / WPL of the group (the lanes own consecutive row ranges, so ranks
// follow a prefix over the lanes).  The block's bitmaps are interleaved: word
// w of a lane sits at w * kSymThreads + the lane's thread index, so that in
// the passes where every lane touches its own words a wave reads or writes 64
// consecutive words, the groups need no padding between them, and each of a
// lane's words is a constant offset from one base address.  Relative to the
// group's base (its first thread), word wi is at the slot below.
template <int GS, int WPL>
__device__ inline int word_slot(int wi) {
    return (wi & (WPL - 1)) * kSymThreads + wi / WPL;
}

// Rank of row d (relative to the chunk base) inside the chunk's bitmap.  The
// word prefixes are kept as bytes saturated at 255: every rank is stored
// clamped to 255 (254 for A_0's entries), and min(min(p, 255) + c, 255) =
// min(p + c, 255), so the clamp is exact while the column's LDS shrinks from
// eight bytes per word to five.
template <int GS, int WPL>
__device__ inline int chunk_rank(const unsigned* bm, const unsigned char* wpre, int d) {
    const int p = word_slot<GS, WPL>(d >> 5);
    return wpre[p] + __popc(bm[p] & ((1u << (d & 31)) - 1u));
}

// Operands of the union kernel.  A list set X is (X_cp, X_cnt, X_ri): list l
// holds X_ri[X_cp[l] .. X_cp[l] + len), len = X_cnt[l] when X_cnt is given
// (lists in bound-sized slots), X_cp[l+1] - X_cp[l] otherwise.
struct UnionArgs {
    int n;
    const int *P_cp, *P_cnt, *P_ri;       // the lists of column j: P(:, j)
    const int *Q_cp, *Q_cnt, *Q_ri;       // the candidates of list l: Q(:, l)
    int* counts;                          // |union| per column (may be null in fill mode)
    const int* out_cp;                    // fill: where column j's union goes
    int* out_ri;
    const int64_t* eoff;                  // positions: start of column j's gathered entries
    unsigned char* posA;
    const int *A0_cp, *A0_ri;
    unsigned char* posB;
    const int* cP_cp;                     // positions: compact copy of P (may be null)
    int* cP_ri;
    int* bad;                             // count mode: earliest column with a bad index
};

// ROUNDS lists per lane (GS * ROUNDS per column) and their first kListLen
// rows live in registers; longer columns or lists take the memory loops.
template <int MODE, int GS, int ROUNDS, int kListLen>
__global__ void __launch_bounds__(kSymThreads)
k_union(UnionArgs a) {
    constexpr int kGroups = kSymThreads / GS;
    constexpr int kChunkWords = chunk_words<GS>();
    constexpr int kChunk = kChunkWords * 32;
    constexpr int kWPL = kChunkWords / GS;   // bitmap words per lane
    // the block's bitmaps and word prefixes, interleaved (see word_slot)
    __shared__ unsigned bm_all[kChunkWords * kGroups];
    __shared__ unsigned char pre_all[kChunkWords * kGroups];
    const int n = a.n;
    const int grp = threadIdx.x / GS;
    const int g = threadIdx.x % GS;
    unsigned* bm = bm_all + grp * GS;
    unsigned char* wpre = pre_all + grp * GS;
    auto slot = [](int wi) { return word_slot<GS, kWPL>(wi); };
    const int stride = gridDim.x * kGroups;
    auto q_len = [&](int l) { return a.Q_cnt ? a.Q_cnt[l] : a.Q_cp[l + 1] - a.Q_cp[l]; };
    for (int j = blockIdx.x * kGroups + grp; j < n; j += stride) {
        const int pa = a.P_cp[j];
        const int pb = a.P_cnt ? pa + a.P_cnt[j] : a.P_cp[j + 1];
        // The column's output operands are loaded here, beside the list
        // loads: a store through a byte or int pointer may alias them, so a
        // load issued after the first store would wait for every store before
        // it, one more memory round trip per column.  a0r: the A_0 entry
        // a0a + g, the first this lane handles.
        int a0a = 0, a0b = 0, a0r = 0, oc = 0, ob = 0;
        int64_t eo = 0;
        if (MODE == kModePositions) {
            a0a = a.A0_cp[j];
            a0b = a.A0_cp[j + 1];
            eo = a.eoff[j];
            if (a.cP_ri) oc = a.cP_cp[j] - pa;
            if (a0a + g < a0b) a0r = a.A0_ri[a0a + g];
        }
        if (MODE == kModeFill) ob = a.out_cp[j];
        // lists t = pa + g + GS u of this lane (all loads independent); `big`
        // marks columns that need the memory loops
        int qa[ROUNDS], len[ROUNDS], lofs[ROUNDS], lraw[ROUNDS];
        int rows[ROUNDS][kListLen];
        int big = (pb - pa > GS * ROUNDS) ? 1 : 0;
        int lo = INT_MAX, carry = 0;
#pragma unroll
        for (int u = 0; u < ROUNDS; ++u) {
            const int t = pa + g + u * GS;
            int l = -1;
            lraw[u] = 0;
            if (t < pb) {
                l = lraw[u] = a.P_ri[t];
                if (l < 0 || l >= n) {
                    if (a.bad) atomicMin(a.bad, j);
                    l = -1;
                }
            }
            qa[u] = l >= 0 ? a.Q_cp[l] : 0;
            len[u] = l >= 0 ? q_len(l) : 0;
            big |= len[u] > kListLen ? 1 : 0;
            // flat offset of this list among the column's gathered entries
            lofs[u] = carry + grp_excl_scan<GS>(len[u]);
            carry += grp_sum<GS>(len[u]);
            if (len[u] > 0) {
#pragma unroll
                for (int e = 0; e < kListLen; ++e) {
                    const bool ok = e < len[u];
                    const int r = a.Q_ri[qa[u] + (ok ? e : 0)];  // clamped: always in bounds
                    rows[u][e] = ok ? r : INT_MAX;
                }
            } else {
#pragma unroll
                for (int e = 0; e < kListLen; ++e) rows[u][e] = INT_MAX;
            }
            lo = min(lo, rows[u][0]);
        }
        big = grp_max<GS>(big);
        if (big) {  // heads of every list, from memory
            lo = INT_MAX;
            for (int t = pa + g; t < pb; t += GS) {
                const int l = a.P_ri[t];
                if (l >= 0 && l < n && q_len(l) > 0) lo = min(lo, a.Q_ri[a.Q_cp[l]]);
            }
        }
        lo = grp_min<GS>(lo);
        if (MODE == kModePositions) {
            for (int e = a0a + g; e < a0b; e += GS) a.posB[e] = 0xFF;
            if (a.cP_ri) {
#pragma unroll
                for (int u = 0; u < ROUNDS; ++u)
                    if (pa + g + u * GS < pb) a.cP_ri[oc + pa + g + u * GS] = lraw[u];
                for (int t = pa + g + ROUNDS * GS; t < pb; t += GS) a.cP_ri[oc + t] = a.P_ri[t];
            }
        }
        int running = 0;
        int base = lo;
        while (base != INT_MAX) {
#pragma unroll
            for (int w = 0; w < kWPL; ++w) bm[w * kSymThreads + g] = 0u;
            wave_sync();
            int next = INT_MAX;
            if (!big) {
#pragma unroll
                for (int u = 0; u < ROUNDS; ++u)
#pragma unroll
                    for (int e = 0; e < kListLen; ++e) {
                        const int r = rows[u][e];
                        const int d = r - base;  // r = INT_MAX for empty slots: d >= kChunk
                        if (d >= 0 && d < kChunk) atomicOr(&bm[slot(d >> 5)], 1u << (d & 31));
                        if (d >= kChunk) next = min(next, r);
                    }
            } else {
                for (int t = pa + g; t < pb; t += GS) {
                    const int l = a.P_ri[t];
                    if (l < 0 || l >= n) continue;
                    const int f0 = a.Q_cp[l], f1 = f0 + q_len(l);
                    for (int f = f0; f < f1; ++f) {
                        const int r = a.Q_ri[f];
                        const int d = r - base;
                        if (d >= 0 && d < kChunk) atomicOr(&bm[slot(d >> 5)], 1u << (d & 31));
                        if (d >= kChunk) next = min(next, r);
                    }
                }
            }
            wave_sync();
            unsigned wd[kWPL];
            int c = 0;
#pragma unroll
            for (int w = 0; w < kWPL; ++w) {
                wd[w] = bm[w * kSymThreads + g];
                c += __popc(wd[w]);
            }
            const int pre = grp_excl_scan<GS>(c);
            const int tot = grp_sum<GS>(c);
            if (MODE == kModePositions) {
                int run = running + pre;
#pragma unroll
                for (int w = 0; w < kWPL; ++w) {
                    wpre[w * kSymThreads + g] = (unsigned char)min(run, 255);
                    run += __popc(wd[w]);
                }
            }
            if (MODE == kModeFill) {
                int o = ob + running + pre;
#pragma unroll
                for (int w = 0; w < kWPL; ++w) {
                    unsigned x = wd[w];
                    while (x) {
                        const int b = __ffs(x) - 1;
                        x &= x - 1;
                        a.out_ri[o++] = base + ((g * kWPL + w) << 5) + b;
                    }
                }
            }
            if (MODE == kModePositions) {
                wave_sync();
                // ranks of the gathered A_k entries, in the order of the lists
                unsigned char* pj = a.posA + eo;
                if (!big) {
#pragma unroll
                    for (int u = 0; u < ROUNDS; ++u)
#pragma unroll
                        for (int e = 0; e < kListLen; ++e) {
                            const int d = rows[u][e] - base;
                            if (d >= 0 && d < kChunk)
                                pj[lofs[u] + e] = (unsigned char)min(chunk_rank<GS, kWPL>(bm, wpre, d), 255);
                        }
                } else {
                    int cy = 0;
                    for (int t0 = pa; t0 < pb; t0 += GS) {
                        const int t = t0 + g;
                        int l = -1, ln = 0;
                        if (t < pb) {
                            l = a.P_ri[t];
                            if (l >= 0 && l < n) ln = q_len(l);
                        }
                        const int off = cy + grp_excl_scan<GS>(ln);
                        for (int f = 0; f < ln; ++f) {
                            const int d = a.Q_ri[a.Q_cp[l] + f] - base;
                            if (d >= 0 && d < kChunk)
                                pj[off + f] = (unsigned char)min(chunk_rank<GS, kWPL>(bm, wpre, d), 255);
                        }
                        cy += grp_sum<GS>(ln);
                    }
                }
                for (int e = a0a + g; e < a0b; e += GS) {
                    const int d = (e == a0a + g ? a0r : a.A0_ri[e]) - base;
                    if (d >= 0 && d < kChunk && ((bm[slot(d >> 5)] >> (d & 31)) & 1u))
                        a.posB[e] = (unsigned char)min(chunk_rank<GS, kWPL>(bm, wpre, d), 254);
                }
            }
            running += tot;
            base = grp_min<GS>(next);
            wave_sync();
        }
        if (g == 0 && a.counts) a.counts[j] = running;  // |union| (= |I_j| for positions)
    }
}

// Eight lanes per column: one list per lane up to 8 lists, two up to 16 (eight
// columns per wave either way; at 640 bytes of LDS per column of the positions
// pass, eight such waves per SIMD fill a CU's LDS); then 16
// lanes with two lists each (32 lists in registers); beyond that the memory
// loops.  The rows held per list follow the longest list
// (5, 8, 9 or 12; longer lists take the memory loops).  Bounds <= 0: unknown.
template <int MODE, int LEN>
static hipError_t launch_union_len(const UnionArgs& a, int max_lists, hipStream_t s) {
    auto grid = [&](int gs) {
        return dim3((unsigned)std::min<int64_t>(ceil_div(a.n, kSymThreads / gs), 256 * 32));
    };
    const dim3 block(kSymThreads);
    if (max_lists > 0 && max_lists <= 8)
        hipLaunchKernelGGL((k_union<MODE, 8, 1, LEN>), grid(8), block, 0, s, a);
    else if (max_lists > 0 && max_lists <= 16)
        hipLaunchKernelGGL((k_union<MODE, 8, 2, LEN>), grid(8), block, 0, s, a);
    else
        hipLaunchKernelGGL((k_union<MODE, 16, 2, LEN>), grid(16), block, 0, s, a);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_union(const UnionArgs& a, int max_lists, int max_len, hipStream_t s) {
    if constexpr (MODE != kModeCount) {   // the count pass (one-shot patterns) keeps 8 rows
        if (max_len > 0 && max_len <= 5) return launch_union_len<MODE, 5>(a, max_lists, s);
        if (max_len == 9) return launch_union_len<MODE, 9>(a, max_lists, s);   // 9-point stencils
        if (max_len > 8) return launch_union_len<MODE, 12>(a, max_lists, s);
    }
    return launch_union_len<MODE, 8>(a, max_lists, s);
}

static UnionArgs union_args(int n) {
    UnionArgs a{};
    a.n = n;
    return a;
}

hipError_t expand_count(int n, const int* P_cp, const int* P_ri, const int* Q_cp, const int* Q_ri,
                        int* counts, int* bad, int max_lists, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    UnionArgs a = union_args(n);
    a.P_cp = P_cp; a.P_ri = P_ri; a.Q_cp = Q_cp; a.Q_ri = Q_ri;
    a.counts = counts; a.bad = bad;
    return launch_union<kModeCount>(a, max_lists, 0, s);
}

hipError_t expand_fill(int n, const int* P_cp, const int* P_ri, const int* Q_cp, const int* Q_ri,
                       const int* out_cp, int* out_ri, int max_lists, int max_len, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    UnionArgs a = union_args(n);
    a.P_cp = P_cp; a.P_ri = P_ri; a.Q_cp = Q_cp; a.Q_ri = Q_ri;
    a.out_cp = out_cp; a.out_ri = out_ri;
    return launch_union<kModeFill>(a, max_lists, max_len, s);
}

hipError_t expand_slots(int n, const int* P_cp, const int* P_cnt, const int* P_ri, const int* Q_cp,
                        const int* Q_cnt, const int* Q_ri, const int* slot_cp, int* slot_ri, int* counts,
                        int max_lists, int max_len, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    UnionArgs a = union_args(n);
    a.P_cp = P_cp; a.P_cnt = P_cnt; a.P_ri = P_ri;
    a.Q_cp = Q_cp; a.Q_cnt = Q_cnt; a.Q_ri = Q_ri;
    a.out_cp = slot_cp; a.out_ri = slot_ri; a.counts = counts;
    return launch_union<kModeFill>(a, max_lists, max_len, s);
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

// *total += sum_j sum_{l in S(:,j)} nnz(A_k(:,l)): a column per thread, the
// wave's sum added once (integer, so the order does not matter).
__global__ void k_gather_total(int n, const int* S_cp, const int* S_ri, const int* Ak_cp,
                               unsigned long long* total) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    long long s = 0;
    if (j < n) {
        for (int e = S_cp[j]; e < S_cp[j + 1]; ++e) {
            const int l = S_ri[e];
            if (l >= 0 && l < n) s += Ak_cp[l + 1] - Ak_cp[l];
        }
    }
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if ((threadIdx.x & 63) == 0 && s != 0) atomicAdd(total, (unsigned long long)s);
}

hipError_t plan_gather_total(int n, const int* S_cp, const int* S_ri, const int* Ak_cp, unsigned long long* total,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_total, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, S_cp, S_ri, Ak_cp,
                       total);
    return hipGetLastError();
}

// Row set I_j of every column as a bitmap sweep; every gathered A_k entry (in
// the order: entries of A_k(:, J_j[0]), then of A_k(:, J_j[1]), ...) gets its
// rank inside I_j, and so does every entry of A_0(:, j) (0xFF when its row is
// not in I_j).  nI[j] = |I_j|.
hipError_t plan_positions(int n, const int* S_cp, const int* S_ri, const int* Ak_cp, const int* Ak_ri,
                          const int* A0_cp, const int* A0_ri, const int64_t* eoff, int* nI,
                          unsigned char* posA, unsigned char* posB, int max_lists, int max_len, hipStream_t s) {
    return plan_positions_slots(n, S_cp, nullptr, S_ri, nullptr, nullptr, Ak_cp, Ak_ri, A0_cp, A0_ri, eoff, nI,
                                posA, posB, max_lists, max_len, s);
}

hipError_t plan_positions_slots(int n, const int* S_cp, const int* S_cnt, const int* S_ri, const int* cS_cp,
                                int* cS_ri, const int* Ak_cp, const int* Ak_ri, const int* A0_cp,
                                const int* A0_ri, const int64_t* eoff, int* nI, unsigned char* posA,
                                unsigned char* posB, int max_lists, int max_len, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    UnionArgs a = union_args(n);
    a.P_cp = S_cp; a.P_cnt = S_cnt; a.P_ri = S_ri;
    a.Q_cp = Ak_cp; a.Q_ri = Ak_ri;
    a.counts = nI; a.eoff = eoff; a.posA = posA; a.A0_cp = A0_cp; a.A0_ri = A0_ri; a.posB = posB;
    a.cP_cp = cS_cp; a.cP_ri = cS_ri;
    return launch_union<kModePositions>(a, max_lists, max_len, s);
}

// --------------------------------------------------------------- buckets

constexpr int kBucketThreads = 256;

__device__ inline int bucket_of(int nI, int nJ, const BucketTable& tab) {
    const int rows = tab.penalty_rows ? max(nI, 2 * nJ) : nI;
    for (int b = 0; b < tab.nb; ++b)
        if (rows <= tab.max_rows[b] && nJ <= tab.max_cols[b]) return b;
    return -1;
}

// The columns are cut into at most kBucketBlocks contiguous ranges of `len`
// columns (a multiple of 256); pass 1 counts every range's columns per
// bucket (hist is bucket-major: hist[b * nblk + blk]), pass 2 lets every
// range sum the counts before it (all ranges of earlier buckets, earlier
// ranges of its own bucket) and scatter its columns in column order.  With
// one or two buckets the ranges are single chunks of 256 columns (many
// blocks, cheap prefix sums); with more, at least 2048 columns.
constexpr int kBucketBlocks = 1024;

static int64_t range_len(int n, int nb) {
    const int64_t per = ((int64_t)n + kBucketBlocks * kBucketThreads - 1) / ((int64_t)kBucketBlocks * kBucketThreads);
    const int64_t lo = nb <= 2 ? 1 : 8;
    return (per > lo ? per : lo) * kBucketThreads;
}

__global__ void __launch_bounds__(kBucketThreads)
k_bucket_hist(int n, int64_t len, const int* S_cp, const int* nI, BucketTable tab, int* hist, int* unfit,
              unsigned long long* status) {
    __shared__ int h[kMaxBuckets];
    if (threadIdx.x < kMaxBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t j0 = (int64_t)blockIdx.x * len;
    const int64_t j1 = std::min<int64_t>(j0 + len, n);
    for (int64_t c0 = j0; c0 < j1; c0 += kBucketThreads) {   // uniform trip count across the block
        const int64_t jj = c0 + threadIdx.x;
        int b = -2;
        if (jj < j1) {
            const int j = (int)jj;
            b = bucket_of(nI[j], S_cp[j + 1] - S_cp[j], tab);
            if (b < 0) {
                if (unfit) atomicAdd(unfit, 1);
                if (status) report(status, j, kStUnsupported);
            }
        }
        // per-wave counts (one LDS atomic per wave and bucket, not per column)
        for (int k = 0; k < tab.nb; ++k) {
            const int c = __popcll(__ballot(b == k));
            if (wave_lane() == 0 && c) atomicAdd(&h[k], c);
        }
    }
    __syncthreads();
    if (threadIdx.x < tab.nb) hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kBucketThreads)
k_bucket_scatter(int n, int64_t len, const int* S_cp, const int* nI, BucketTable tab, const int* hist,
                 int* queue, int* bstart) {
    __shared__ int tot[kMaxBuckets], pre[kMaxBuckets], base[kMaxBuckets + 1];
    __shared__ int wcount[kBucketThreads / 64][kMaxBuckets];
    const int nblk = gridDim.x;
    const int me = blockIdx.x;
    if (threadIdx.x < kMaxBuckets) tot[threadIdx.x] = pre[threadIdx.x] = 0;
    __syncthreads();
    for (int b = 0; b < tab.nb; ++b) {   // every thread strides over the ranges of bucket b
        int t = 0, p = 0;
#pragma unroll 4
        for (int blk = threadIdx.x; blk < nblk; blk += kBucketThreads) {
            const int c = hist[b * nblk + blk];
            t += c;
            p += blk < me ? c : 0;
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            t += __shfl_xor(t, d, 64);
            p += __shfl_xor(p, d, 64);
        }
        if (wave_lane() == 0) {   // one LDS atomic per wave
            if (t) atomicAdd(&tot[b], t);
            if (p) atomicAdd(&pre[b], p);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int b = 0; b < tab.nb; ++b) {
            if (me == 0) bstart[b] = run;
            base[b] = run + pre[b];
            run += tot[b];
        }
        if (me == 0) bstart[tab.nb] = run;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6;
    const int lane = wave_lane();
    const int64_t j0 = (int64_t)me * len;
    const int64_t j1 = std::min<int64_t>(j0 + len, n);
    for (int64_t c0 = j0; c0 < j1; c0 += kBucketThreads) {
        const int64_t jj = c0 + threadIdx.x;
        int b = -1;
        if (jj < j1) b = bucket_of(nI[jj], S_cp[jj + 1] - S_cp[jj], tab);
        int my_rank = 0;
        for (int k = 0; k < tab.nb; ++k) {
            const unsigned long long m = __ballot(b == k);
            if (b == k) my_rank = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) wcount[wv][k] = __popcll(m);
        }
        __syncthreads();
        if (b >= 0) {
            int r = base[b] + my_rank;
            for (int w = 0; w < wv; ++w) r += wcount[w][b];
            queue[r] = (int)jj;
        }
        __syncthreads();
        if (threadIdx.x < tab.nb) {
            int c = 0;
            for (int w = 0; w < kBucketThreads / 64; ++w) c += wcount[w][threadIdx.x];
            base[threadIdx.x] += c;
        }
        __syncthreads();
    }
}


size_t bucket_temp_bytes(int n) {
    return (size_t)kBucketBlocks * kMaxBuckets * sizeof(int) + 512;
}

hipError_t bucket_sort(int n, const int* S_cp, const int* nI, BucketTable tab, int* queue, int* bstart,
                       int* unfit, unsigned long long* status, void* temp, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t len = range_len(n, tab.nb);
    const int nblk = (int)ceil_div(n, len);
    int* hist = (int*)temp;
    hipLaunchKernelGGL(k_bucket_hist, dim3(nblk), dim3(kBucketThreads), 0, s, n, len, S_cp, nI, tab, hist, unfit,
                       status);
    hipLaunchKernelGGL(k_bucket_scatter, dim3(nblk), dim3(kBucketThreads), 0, s, n, len, S_cp, nI, tab, hist,
                       queue, bstart);
    return hipGetLastError();
}

}  // namespace samk
