// sam_numeric.hip -- batched column least-squares solves of the SAM on
// gfx950 (Section 2 of the paper: N_k = argmin ||A_k N - A_0||_F over the
// pattern S splits into the n problems min ||A_k(I_j,J_j) m - A_0(I_j,j)||).
//
// Layout.  A group of G consecutive lanes of a wave64 owns one column
// problem; a wave holds 64/G problems of the same size class (bucket).  The
// |I_j| x |J_j| block lives in registers distributed by rows: lane g of the
// group holds rows g, g+G, g+2G, ... (R rows, NC columns, zero padded).  The
// Householder QR then needs one G-lane reduction per column and step, done
// with DPP quad/mirror exchanges (no LDS), and every other operation is a
// lane-local FMA on registers with static indices.
//
// Gather.  The plan stores, for every A_k entry of A_k(:,J_j), its row's
// rank inside I_j (one byte), so the block is staged column-chunk by
// column-chunk through an LDS tile without searching, then read row-wise into
// registers.  A_0(:,j) goes to an LDS vector the same way; its entries whose
// rows lie outside I_j only add out_j = sum a_0(i,j)^2 to the residual.
//
// Precision.  TQ = double: QR and solve in FP64.  TQ = float: QR and solves
// in FP32, then one seminormal refinement step
//     r = b - A m (FP64),  g = A^T r (FP64),  m += R^{-1} R^{-T} g,
// with r and g accumulated in FP64 straight from the FP64 values (sparse
// passes over the block's entries, through the LDS residual vector).  The
// reported column residual is always recomputed in FP64 from the final m.
//
// Soft weights (WEIGHTED): the block is extended by the rows diag(sqrt(p_l)),
// p_l = mu (1/w_l - 1), which the QR sees as extra rows |I_j| .. |I_j|+|J_j|-1
// (so a variant must have G*R >= |I_j| + |J_j|); the residual excludes them.
#include "sam_device.hpp"
#include "sam_kernels.hpp"

#include <algorithm>
#include <type_traits>

namespace samk {

namespace {

template <typename T>
__device__ inline T sgn_copy(T mag, T s) { return copysign(mag, s); }

// XCD-aware block order: consecutive logical blocks run on the same XCD so
// that neighbouring columns (which share most of their A_k columns) hit the
// same L2.
__device__ inline int logical_block() {
    const int b = blockIdx.x, nb = gridDim.x;
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

template <typename TQ, int G, int R, int NC, int TC, bool WEIGHTED>
__global__ void __launch_bounds__(64)
k_numeric(NumericArgs a) {
    constexpr int P = 64 / G;        // problems per wave
    constexpr int RM = G * R;        // rows per problem (padded)
    constexpr bool REFINE = std::is_same<TQ, float>::value;
    static_assert(TC >= 1, "tile chunk");
    __shared__ double tile[P * RM * TC];  // gather staging, reused for r
    __shared__ double bsh[P * RM];        // b = A_0(I_j, j)
    __shared__ int cst[P][NC + 1];        // entry offset of column c in the block
    __shared__ int vbs[P][NC];            // start of A_k(:, J_j[c]) in the value array

    const int lane = threadIdx.x;
    const int g = lane % G;
    const int q = lane / G;
    const int b0 = a.bstart[a.bucket];
    const int count = a.bstart[a.bucket + 1] - b0;
    const int ngroups = (count + P - 1) / P;
    const int per_block = (ngroups + gridDim.x - 1) / gridDim.x;
    const int lb = logical_block();
    const int grp_lo = lb * per_block;
    const int grp_hi = min(ngroups, grp_lo + per_block);

    for (int grp = grp_lo; grp < grp_hi; ++grp) {
        const int slot = grp * P + q;
        const bool valid = slot < count;
        const int j = valid ? a.queue[b0 + slot] : 0;
        int nJ = 0, nIj = 0, scol = 0;
        int64_t eo = 0;
        if (valid) {
            scol = a.S_cp[j];
            nJ = a.S_cp[j + 1] - scol;
            nIj = a.nI[j];
            eo = a.eoff[j];
        }
        // rows the QR sees: I_j, plus the penalty rows in the weighted form
        const int nrows = WEIGHTED ? nIj + nJ : nIj;
        const int ncw = __builtin_amdgcn_readfirstlane((int)group_max<64>((float)nJ));

        // ---- column metadata
        if (g == 0) {
            int acc = 0;
            for (int c = 0; c < NC; ++c) {
                int vb = 0, len = 0;
                if (c < nJ) {
                    const int l = a.S_ri[scol + c];
                    vb = a.Ak_cp[l];
                    len = a.Ak_cp[l + 1] - vb;
                }
                cst[q][c] = acc;
                vbs[q][c] = vb;
                acc += len;
            }
            cst[q][NC] = acc;
        }
        // ---- b = A_0(I_j, j), out_j
#pragma unroll
        for (int t = 0; t < R; ++t) bsh[q * RM + t * G + g] = 0.0;
        wave_sync();
        double outj = 0.0;
        if (valid) {
            for (int e = a.A0_cp[j] + g; e < a.A0_cp[j + 1]; e += G) {
                const int p = a.posB[e];
                const double v = a.A0_v[e];
                if (p != 0xFF) bsh[q * RM + p] = v;
                else outj += v * v;
            }
        }
        outj = group_sum<G>(outj);
        wave_sync();

        // ---- gather the block, TC columns at a time
        TQ A[R][NC];
#pragma unroll
        for (int c0 = 0; c0 < NC; c0 += TC) {
            if (c0 < ncw) {
#pragma unroll
                for (int t = 0; t < R; ++t)
#pragma unroll
                    for (int cc = 0; cc < TC; ++cc) tile[(q * RM + t * G + g) * TC + cc] = 0.0;
                wave_sync();
#pragma unroll
                for (int cc = 0; cc < TC; ++cc) {
                    const int c = c0 + cc;
                    if (c < NC && c < nJ) {
                        const int e0 = cst[q][c], e1 = cst[q][c + 1];
                        const int vb = vbs[q][c];
                        for (int e = g; e < e1 - e0; e += G) {
                            const int p = a.posA[eo + e0 + e];
                            tile[(q * RM + p) * TC + cc] = a.Ak_v[vb + e];
                        }
                    }
                }
                wave_sync();
#pragma unroll
                for (int t = 0; t < R; ++t)
#pragma unroll
                    for (int cc = 0; cc < TC; ++cc)
                        if (c0 + cc < NC) A[t][c0 + cc] = (TQ)tile[(q * RM + t * G + g) * TC + cc];
                wave_sync();
            } else {
#pragma unroll
                for (int t = 0; t < R; ++t)
#pragma unroll
                    for (int cc = 0; cc < TC; ++cc)
                        if (c0 + cc < NC) A[t][c0 + cc] = (TQ)0;
            }
        }
        // penalty rows: row nIj + c holds sqrt(p_c) in column c
        if constexpr (WEIGHTED) {
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int row = t * G + g;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    if (valid && c < nJ && row == nIj + c) {
                        const double wl = a.w[scol + c];
                        A[t][c] = (TQ)sqrt(a.mu * (1.0 / wl - 1.0));
                    }
                }
            }
        }
        TQ bq[R];
#pragma unroll
        for (int t = 0; t < R; ++t) bq[t] = (TQ)bsh[q * RM + t * G + g];

        // ---- Householder QR (dgeqr2 conventions), applied to b as well
        TQ rdiag[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            rdiag[k] = (TQ)0;
            if (k < ncw) {
                constexpr int dummy = 0;
                (void)dummy;
                const int tk = k / G, gk = k % G;
                TQ sig = 0, alp = 0;
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    if (t < tk) continue;
                    const TQ x = A[t][k];
                    const bool below = (t > tk) || (g > gk);
                    sig += below ? x * x : (TQ)0;
                    if (t == tk) alp = (g == gk) ? x : (TQ)0;
                }
                sig = group_sum<G>(sig);
                alp = group_sum<G>(alp);
                const bool zero = !(sig > (TQ)0);
                const TQ nrm = sqrt(alp * alp + sig);
                const TQ beta = zero ? alp : -sgn_copy(nrm, alp);
                const TQ tau = zero ? (TQ)0 : (beta - alp) / beta;
                const TQ scal = zero ? (TQ)0 : (TQ)1 / (alp - beta);
                rdiag[k] = beta;
                TQ v[R];
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    if (t < tk) { v[t] = 0; continue; }
                    const bool below = (t > tk) || (g > gk);
                    const bool diag = (t == tk) && (g == gk);
                    v[t] = below ? A[t][k] * scal : (diag ? (TQ)1 : (TQ)0);
                    if (below) A[t][k] = v[t];
                    if (diag) A[t][k] = beta;
                }
                TQ w[NC];
#pragma unroll
                for (int c = k + 1; c < NC; ++c) {
                    TQ s = 0;
#pragma unroll
                    for (int t = tk; t < R; ++t) s += v[t] * A[t][c];
                    w[c] = s;
                }
                TQ wb = 0;
#pragma unroll
                for (int t = tk; t < R; ++t) wb += v[t] * bq[t];
#pragma unroll
                for (int c = k + 1; c < NC; ++c)
                    if (c < ncw) w[c] = group_sum<G>(w[c]) * tau;
                wb = group_sum<G>(wb) * tau;
#pragma unroll
                for (int c = k + 1; c < NC; ++c)
                    if (c < ncw)
#pragma unroll
                        for (int t = tk; t < R; ++t) A[t][c] -= w[c] * v[t];
#pragma unroll
                for (int t = tk; t < R; ++t) bq[t] -= wb * v[t];
            }
        }

        // ---- rank test: |R_kk| <= 10 * rows * eps * max |R_ii|
        bool bad_rank = false;
        {
            TQ mx = 0;
#pragma unroll
            for (int k = 0; k < NC; ++k)
                if (k < nJ) mx = fmax(mx, fabs(rdiag[k]));
            const TQ eps = std::is_same<TQ, float>::value ? (TQ)1.1920928955078125e-07
                                                          : (TQ)2.220446049250313e-16;
            const TQ tol = (TQ)10 * (TQ)nrows * eps * mx;
            if (nJ > 0 && !(mx > (TQ)0)) bad_rank = true;
#pragma unroll
            for (int k = 0; k < NC; ++k)
                if (k < nJ && !(fabs(rdiag[k]) > tol)) bad_rank = true;
        }

        // ---- back substitution R m = c1 (owner lane of row k computes,
        //      then broadcasts inside the group)
        TQ m[NC];
#pragma unroll
        for (int k = NC - 1; k >= 0; --k) {
            m[k] = 0;
            if (k < ncw) {
                const int tk = k / G, gk = k % G;
                TQ s = bq[tk];
#pragma unroll
                for (int c = k + 1; c < NC; ++c) s -= A[tk][c] * m[c];
                TQ mk = s / rdiag[k];
                mk = group_bcast<G>(mk, g, gk);
                m[k] = (k < nJ) ? mk : (TQ)0;
            }
        }

        double* rsh = tile + q * RM;  // residual vector (tile is free now)
        // r = b - A mm over the gathered entries, in FP64; rows beyond nIj
        // (penalty rows) are not part of the residual.
        auto residual_pass = [&](const double (&mm)[NC]) {
#pragma unroll
            for (int t = 0; t < R; ++t) rsh[t * G + g] = bsh[q * RM + t * G + g];
            wave_sync();
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (c < ncw) {
                    if (c < nJ) {
                        const int e0 = cst[q][c], e1 = cst[q][c + 1];
                        const int vb = vbs[q][c];
                        const double mc = mm[c];
                        for (int e = g; e < e1 - e0; e += G) {
                            const int p = a.posA[eo + e0 + e];
                            rsh[p] -= a.Ak_v[vb + e] * mc;
                        }
                    }
                    wave_sync();
                }
            }
        };

        double mfin[NC];
        if constexpr (REFINE) {
            double m64[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) m64[c] = (double)m[c];
#pragma unroll
            for (int it = 0; it < (WEIGHTED ? 2 : 1); ++it) {
                residual_pass(m64);
                // g = A^T r (FP64) minus the penalty term p .* m
                double gc[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    double s = 0.0;
                    if (c < ncw && c < nJ) {
                        const int e0 = cst[q][c], e1 = cst[q][c + 1];
                        const int vb = vbs[q][c];
                        for (int e = g; e < e1 - e0; e += G) {
                            const int p = a.posA[eo + e0 + e];
                            s += a.Ak_v[vb + e] * rsh[p];
                        }
                    }
                    gc[c] = s;
                }
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    if (c < ncw) gc[c] = group_sum<G>(gc[c]);
                if constexpr (WEIGHTED) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        if (valid && c < nJ) gc[c] -= a.mu * (1.0 / a.w[scol + c] - 1.0) * m64[c];
                }
                // y = R^{-T} g (FP32): y_c = (g_c - sum_{k<c} R_kc y_k) / R_cc
                TQ ydist[R];
                TQ yrep[NC];
#pragma unroll
                for (int t = 0; t < R; ++t) ydist[t] = 0;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    yrep[c] = 0;
                    if (c < ncw) {
                        TQ part = 0;
#pragma unroll
                        for (int t = 0; t < R; ++t) {
                            const int row = t * G + g;
                            if (t * G < c) part += (row < c) ? A[t][c] * ydist[t] : (TQ)0;
                        }
                        part = group_sum<G>(part);
                        TQ yc = ((TQ)gc[c] - part) / rdiag[c];
                        yc = (c < nJ) ? yc : (TQ)0;
                        yrep[c] = yc;
                        if (g == c % G) ydist[c / G] = yc;
                    }
                }
                // delta = R^{-1} y
                TQ dl[NC];
#pragma unroll
                for (int k = NC - 1; k >= 0; --k) {
                    dl[k] = 0;
                    if (k < ncw) {
                        const int tk = k / G, gk = k % G;
                        TQ s = yrep[k];
#pragma unroll
                        for (int c = k + 1; c < NC; ++c) s -= A[tk][c] * dl[c];
                        TQ dk = s / rdiag[k];
                        dk = group_bcast<G>(dk, g, gk);
                        dl[k] = (k < nJ) ? dk : (TQ)0;
                    }
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) m64[c] += (double)dl[c];
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) mfin[c] = m64[c];
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) mfin[c] = (double)m[c];
        }

        // ---- column residual rho_j = ||b - A m||^2 + out_j (FP64)
        residual_pass(mfin);
        double rr = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const double x = rsh[t * G + g];
            rr += (t * G + g < nIj) ? x * x : 0.0;
        }
        rr = group_sum<G>(rr) + outj;
        wave_sync();

        // ---- outputs
        bool nonfinite = !isfinite(rr);
#pragma unroll
        for (int c = 0; c < NC; ++c) nonfinite |= (c < nJ) && !isfinite(mfin[c]);
        if (valid) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (c < nJ && (c % G) == g) {
                    if constexpr (REFINE) static_cast<float*>(a.M)[scol + c] = (float)mfin[c];
                    else static_cast<double*>(a.M)[scol + c] = mfin[c];
                }
            }
            if (g == 0) {
                if (a.col_res2) a.col_res2[j] = rr;
                if (bad_rank) report(a.status, j, kStRank);
                else if (nonfinite) report(a.status, j, kStNonfinite);
            }
        }
    }
}

template <typename TQ, int G, int R, int NC, int TC, bool W>
hipError_t launch_numeric(const NumericArgs& args, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_numeric<TQ, G, R, NC, TC, W>), dim3(grid), dim3(64), 0, s, args);
    return hipGetLastError();
}

#define SAM_VARIANT(TQ, PREC, G, R, NC, TC, W) \
    NumericVariant{PREC, G, R, NC, W, &launch_numeric<TQ, G, R, NC, TC, W>}

// Menu per precision, cheapest first.  Shapes of the workloads: 2D 5-point
// level 1 (13 x 5), level 2 (25 x 13); 3D 7-point level 2 (63 x 25); 2D
// 9-point level 2 with thresholds (<= 49 x 24); weighted 3D (88 x 25).
const NumericVariant kMenu[] = {
    // FP32 + refinement
    SAM_VARIANT(float, 1, 2, 8, 8, 4, false),
    SAM_VARIANT(float, 1, 4, 7, 13, 2, false),
    SAM_VARIANT(float, 1, 4, 8, 16, 2, false),
    SAM_VARIANT(float, 1, 16, 4, 25, 1, false),
    SAM_VARIANT(float, 1, 16, 4, 32, 1, false),
    SAM_VARIANT(float, 1, 32, 4, 32, 1, false),
    // FP64
    SAM_VARIANT(double, 0, 2, 8, 8, 4, false),
    SAM_VARIANT(double, 0, 4, 7, 13, 2, false),
    SAM_VARIANT(double, 0, 8, 4, 16, 2, false),
    SAM_VARIANT(double, 0, 32, 2, 25, 1, false),
    SAM_VARIANT(double, 0, 32, 2, 32, 1, false),
    SAM_VARIANT(double, 0, 64, 2, 32, 1, false),
    // soft-weighted (stacked penalty rows)
    SAM_VARIANT(float, 1, 4, 8, 13, 2, true),
    SAM_VARIANT(float, 1, 32, 3, 25, 1, true),
    SAM_VARIANT(float, 1, 64, 2, 32, 1, true),
    SAM_VARIANT(double, 0, 4, 8, 13, 2, true),
    SAM_VARIANT(double, 0, 64, 2, 25, 1, true),
    SAM_VARIANT(double, 0, 64, 2, 32, 1, true),
};

}  // namespace

const NumericVariant* numeric_menu(int* count) {
    *count = (int)(sizeof(kMenu) / sizeof(kMenu[0]));
    return kMenu;
}

// ------------------------------------------------ deterministic reductions

namespace {
constexpr int kRedThreads = 256;
constexpr int kRedItems = 8;

template <bool SQ>
__global__ void __launch_bounds__(kRedThreads)
k_reduce(const double* x, int64_t n, double* out) {
    __shared__ double sh[kRedThreads];
    const int64_t base = (int64_t)blockIdx.x * kRedThreads * kRedItems;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kRedItems; ++i) {
        int64_t idx = base + (int64_t)i * kRedThreads + threadIdx.x;
        if (idx < n) {
            double v = x[idx];
            s += SQ ? v * v : v;
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int d = kRedThreads / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}
}  // namespace

size_t reduce_temp_bytes(int64_t n) {
    size_t bytes = 0;
    int64_t m = n;
    while (m > 1) {
        m = (m + kRedThreads * kRedItems - 1) / (kRedThreads * kRedItems);
        bytes += (size_t)m * sizeof(double) + 256;
    }
    return bytes + 512;
}

static hipError_t reduce_impl(const double* x, int64_t n, double* out, double* temp, bool sq,
                              hipStream_t s) {
    const int64_t tile = kRedThreads * kRedItems;
    int64_t m = (n + tile - 1) / tile;
    if (m <= 1) {
        if (sq) hipLaunchKernelGGL(k_reduce<true>, dim3(1), dim3(kRedThreads), 0, s, x, n, out);
        else hipLaunchKernelGGL(k_reduce<false>, dim3(1), dim3(kRedThreads), 0, s, x, n, out);
        return hipGetLastError();
    }
    if (sq) hipLaunchKernelGGL(k_reduce<true>, dim3((unsigned)m), dim3(kRedThreads), 0, s, x, n, temp);
    else hipLaunchKernelGGL(k_reduce<false>, dim3((unsigned)m), dim3(kRedThreads), 0, s, x, n, temp);
    double* next = temp + ((m * sizeof(double) + 255) / 256) * 256 / sizeof(double);
    return reduce_impl(temp, m, out, next, false, s);
}

hipError_t reduce_sum(const double* x, int64_t n, double* out, void* temp, hipStream_t s) {
    return reduce_impl(x, n, out, (double*)temp, false, s);
}

hipError_t reduce_sumsq(const double* x, int64_t n, double* out, void* temp, hipStream_t s) {
    return reduce_impl(x, n, out, (double*)temp, true, s);
}

}  // namespace samk
