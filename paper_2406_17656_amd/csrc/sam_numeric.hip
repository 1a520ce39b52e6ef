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
// column residual is then ||r||^2 (FP64) less the update's second-order
// term; in FP64 mode it is ||c_2||^2 of Q^T b.
//
// Soft weights (WEIGHTED): the block is extended by the rows diag(sqrt(p_l)),
// p_l = mu (1/w_l - 1); the QR of the stacked matrix is taken in two stages
// (A, then R_1 with the penalty of column c on row NC + c), so a variant
// must have G*R >= max(|I_j|, 2 NC); the residual excludes the penalty.
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

// Raw buffer resources over the arrays the gather reads: 32-bit byte offsets
// (no 64-bit address arithmetic per load, constant parts folded into the
// instruction's offset field) and loads past the extent return 0.
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ inline double ld_f64(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ inline int ld_u8(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return (int)__builtin_amdgcn_raw_buffer_load_b8(r, (int)off, 0, 0);
}

// vec[p] += x as an LDS atomic without return (ds_add_f64): no read-modify-
// write round trip per entry.  The lanes of one instruction always target
// distinct slots and a wave's LDS operations complete in issue order, so each
// slot's sum is formed in program order, as with plain loads and stores.
__device__ inline void lds_add(double* p, double x) {
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

template <typename T>
__device__ inline T recip(T x);
template <>
__device__ inline float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ inline double recip<double>(double x) { return 1.0 / x; }

template <typename T>
__device__ inline T root(T x);
template <>
__device__ inline float root<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <>
__device__ inline double root<double>(double x) { return sqrt(x); }

// One kernel variant serves one bucket: every column problem with
// |I_j| (+ |J_j| when weighted) <= G*R rows and |J_j| <= NC columns.  The
// code is straight-line in NC and R (no runtime column guards): columns past
// |J_j| are zero and pass through the Householder steps as identities.
// MODE 0: plain least squares; 1: soft-weighted (stacked penalty rows);
// 2: adjoint of the soft-weighted map (forward recomputed, then lambda and
// the gradient contributions).
// The 64-row FP32 class of the plain map (63 x 25 blocks of 3D seven-point
// level-2 patterns) is held to three waves per SIMD (168 VGPRs; it would
// take 175 and fit two): the compiler then keeps a few loop-invariant values
// in scratch (28 bytes per lane, reloaded a handful of times per group), and
// the launch is about 8% faster.
constexpr int numeric_min_waves(bool f32, int G, int R, int NC, int MODE) {
    return (f32 && MODE == 0 && G == 16 && R == 4 && NC == 25) ? 3 : 1;
}

template <typename TQ, int G, int R, int NC, int TC, int LPL, int MODE>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(numeric_min_waves(std::is_same<TQ, float>::value, G, R, NC, MODE))))
k_numeric(NumericArgs a) {
    constexpr bool WEIGHTED = MODE >= 1;
    constexpr bool BACKWARD = MODE == 2;
    constexpr int P = 64 / G;        // problems per wave
    constexpr int RM = G * R;        // rows per problem (padded)
    constexpr int RX = RM + G;       // plus one scratch row per lane
    // LDS stride between the problems of a wave: RS = G (mod 16) rows, so
    // that rows t*G + g of the P problems spread over all the banks (a
    // stride of 32 rows would put all 16 problems of a G = 4 wave on one)
    constexpr int RS = RX + (((G - RX) % 16) + 16) % 16;
    constexpr bool REFINE = std::is_same<TQ, float>::value;
    static_assert(TC >= 1, "tile chunk");
    static_assert(!WEIGHTED || 2 * NC <= RM, "penalty rows NC .. 2 NC - 1");
    // Per-group metadata is software-pipelined for blocks of 8 to 13 columns
    // of the plain map (see the stages below); only they double-buffer the
    // column extents.
    constexpr bool PIPE = NC >= 8 && NC <= 13 && MODE == 0;
    // FP64-residual refinement steps of the weighted forms (m, and the
    // adjoint's lambda)
    constexpr int kWSteps = 1;
    // gather staging in the QR's precision; afterwards the weighted and
    // adjoint forms reuse the same memory for the FP64 residual vector
    // (P * RS doubles; the plain map forms its residual over b instead)
    constexpr int kTileD = (P * RS * TC * (int)sizeof(TQ) + 7) / 8;
    constexpr int kResD = (WEIGHTED || BACKWARD) ? P * RS : 1;
    __shared__ double lds_tile[kTileD > kResD ? kTileD : kResD];
    TQ* tile = reinterpret_cast<TQ*>(lds_tile);
    __shared__ double bsh[P * RS];        // b = A_0(I_j, j)
    __shared__ int cst[P][NC];            // entry offset of column c in the block
    __shared__ int vbs2[PIPE ? 2 : 1][P][NC];  // start of A_k(:, J_j[c]) in the value array
    __shared__ int cln2[PIPE ? 2 : 1][P][NC];  // nnz of A_k(:, J_j[c])
    __shared__ int mta[P][9];             // next group: valid, j, scol, nJ, nIj, eo (2), a0, a1
    __shared__ double alsh[BACKWARD ? P * RS : 1];  // A lambda (adjoint)
    __shared__ double racc;               // the block's running sum of column residuals
    __shared__ double pen_sh[WEIGHTED ? P * NC : 1];  // penalties p_c of the group's problems
    // The weighted and adjoint forms keep their length-NC FP64 vectors (m,
    // A^T r, the corrections, lambda and its right side) in LDS: one slot per
    // problem and column, which every lane of the group reads at once (a
    // broadcast), instead of a copy in every lane's registers.
    constexpr int kNV = BACKWARD ? 5 : (WEIGHTED ? 4 : 1);
    __shared__ double vsh[WEIGHTED ? P * kNV * NC : 1];
    __shared__ TQ rinv_sh[WEIGHTED ? P * NC : 1];  // weighted forms: 1 / R_kk

    const int lane = threadIdx.x;
    const int g = lane % G;
    const int q = lane / G;
    const int trash = RM + g;             // this lane's scratch row: absorbs masked writes
    const int b0 = a.bstart[a.bucket];
    const int count = a.bstart[a.bucket + 1] - b0;
    const int ngroups = (count + P - 1) / P;
    // groups split evenly over the blocks (the launch sizes the grid to the
    // blocks the GPU holds at once, so every block runs in one round)
    const int lb = logical_block();
    const int grp_lo = (int)((int64_t)lb * ngroups / gridDim.x);
    const int grp_hi = (int)((int64_t)(lb + 1) * ngroups / gridDim.x);
    const __amdgpu_buffer_rsrc_t rAv = buf_rsrc(a.Ak_v, a.nnzA * 8u);
    const __amdgpu_buffer_rsrc_t rA0 = buf_rsrc(a.A0_v, a.nnzA0 * 8u);
    const __amdgpu_buffer_rsrc_t rPA = buf_rsrc(a.posA, a.E);
    const __amdgpu_buffer_rsrc_t rPB = buf_rsrc(a.posB, a.nnzA0);

    // Per-group metadata pipelining: the dependent loads that
    // locate group grp + 1 (its queue entry; its pattern and row-set data;
    // its pattern columns; their extents in A_k) are issued in stages while
    // group grp is solved and land in LDS (the column extents in the other
    // half of a double buffer), so a group starts with only its value loads
    // outstanding.  Lane g resolves columns g, g+G, ... of J_j.
    // Blocks of 8 to 13 columns of the plain map prefetch; wider blocks and
    // the weighted forms have no registers to spare (and the narrowest lose
    // a wave slot per SIMD, or gain nothing): they run the same stages for
    // their own group at its top.
    constexpr int NCG = (NC + G - 1) / G;
    bool n_valid = false;
    int n_j = 0, n_cp0 = 0, n_cp1 = 0, n_nI = 0, n_a0 = 0, n_a1 = 0;
    int64_t n_eo = 0;
    int n_l[NCG], n_v0[NCG], n_v1[NCG];
    // A bucket that holds all n columns lists them in column order (the
    // bucket sort is stable, and a single class gets the identity queue), so
    // its queue entry is the slot itself: one dependent load less per group.
    const bool ident = b0 == 0 && count == a.n;
    auto stage1 = [&](int gr) {  // queue entry
        const int slot = gr * P + q;
        n_valid = gr < grp_hi && slot < count;
        n_j = n_valid ? (ident ? slot : a.queue[b0 + slot]) : 0;
    };
    auto stage2 = [&]() {  // pattern and row-set data of column j
        n_cp0 = n_cp1 = n_nI = n_a0 = n_a1 = 0;
        n_eo = 0;
        if (n_valid) {
            n_cp0 = a.S_cp[n_j];
            n_cp1 = a.S_cp[n_j + 1];
            n_nI = a.nI[n_j];
            n_eo = a.eoff[n_j];
            n_a0 = a.A0_cp[n_j];
            n_a1 = a.A0_cp[n_j + 1];
        }
    };
    auto stage3 = [&]() {  // to LDS; then the pattern's columns
        const int nj = n_cp1 - n_cp0;
        mta[q][0] = n_valid;
        mta[q][1] = n_j;
        mta[q][2] = n_cp0;
        mta[q][3] = nj;
        mta[q][4] = n_nI;
        mta[q][5] = (int)(uint32_t)(uint64_t)n_eo;
        mta[q][6] = (int)((uint64_t)n_eo >> 32);
        mta[q][7] = n_a0;
        mta[q][8] = n_a1;
#pragma unroll
        for (int i = 0; i < NCG; ++i) {
            const int c = g + i * G;
            n_l[i] = c < nj ? a.S_ri[n_cp0 + c] : -1;
        }
    };
    auto stage4 = [&]() {  // extents of the pattern's columns in A_k
#pragma unroll
        for (int i = 0; i < NCG; ++i) {
            n_v0[i] = n_v1[i] = 0;
            if (n_l[i] >= 0) {
                n_v0[i] = a.Ak_cp[n_l[i]];
                n_v1[i] = a.Ak_cp[n_l[i] + 1];
            }
        }
    };
    auto stage5 = [&](int nb) {  // to the other LDS buffer
#pragma unroll
        for (int i = 0; i < NCG; ++i) {
            const int c = g + i * G;
            if (c < NC) {
                vbs2[nb][q][c] = n_v0[i];
                cln2[nb][q][c] = n_v1[i] - n_v0[i];
            }
        }
    };
    if (lane == 0) racc = 0.0;  // this block's sum of column residuals, group by group
    if constexpr (PIPE) {
        stage1(grp_lo);
        stage2();
        stage3();
        stage4();
        stage5(0);
        wave_sync();
    }

    for (int grp = grp_lo; grp < grp_hi; ++grp) {
        const int bi = PIPE ? (grp - grp_lo) & 1 : 0;
        if constexpr (!PIPE) {
            stage1(grp);
            stage2();
            stage3();
            stage4();
            stage5(0);
            wave_sync();
        }
        int (&vbs)[P][NC] = vbs2[bi];
        int (&cln)[P][NC] = cln2[bi];
        const bool valid = mta[q][0] != 0;
        const int j = mta[q][1];
        const int scol = mta[q][2];
        const int nJ = mta[q][3];
        const int nIj = mta[q][4];
        const int64_t eo = (int64_t)(((uint64_t)(uint32_t)mta[q][6] << 32) | (uint32_t)mta[q][5]);
        const int a0 = mta[q][7];
        const int a1 = mta[q][8];
        const int nrows = WEIGHTED ? nIj + nJ : nIj;

        // ---- longc (wave-uniform): some column needs the memory loops
        bool mylong = false;
#pragma unroll
        for (int i = 0; i < NCG; ++i) {
            const int c = g + i * G;
            if (c < NC) mylong |= cln[q][c] > LPL * G;
        }
        const bool longc = __ballot(mylong) != 0ull;
        // ---- b = A_0(I_j, j) and out_j (rows outside I_j)
#pragma unroll
        for (int t = 0; t < R; ++t) bsh[q * RS + t * G + g] = 0.0;
        bsh[q * RS + trash] = 0.0;
        int bp[LPL];
        double bv[LPL];
#pragma unroll
        for (int s = 0; s < LPL; ++s) {
            const bool ok = a0 + g + s * G < a1;
            const uint32_t e = (uint32_t)(a0 + g) + (uint32_t)(s * G);
            const int p = ld_u8(rPB, e);
            const double v = ld_f64(rA0, e * 8u);
            bp[s] = ok ? p : -1;
            bv[s] = ok ? v : 0.0;
        }
        wave_sync();
        if (g == 0) {
            int acc = 0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                cst[q][c] = acc;
                acc += cln[q][c];
            }
        }
        double outj = 0.0;
#pragma unroll
        for (int s = 0; s < LPL; ++s) {
            outj += bp[s] == 0xFF ? bv[s] * bv[s] : 0.0;
            bsh[q * RS + ((bp[s] >= 0 && bp[s] != 0xFF) ? bp[s] : trash)] = bv[s];
        }
        for (int e = a0 + g + LPL * G; e < a1; e += G) {  // long columns
            const int p = a.posB[e];
            const double v = a.A0_v[e];
            if (p != 0xFF) bsh[q * RS + p] = v;
            else outj += v * v;
        }
        outj = group_sum<G>(outj);
        wave_sync();

        // ---- gather: every A_k value this lane moves is loaded first (static
        //      indices), then staged TC columns at a time through the LDS
        //      tile and read back row-wise; masked entries go to the lane's
        //      scratch row.
        double pv[NC][LPL];
        int pp[NC][LPL];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int len = cln[q][c];
            const uint32_t po = (uint32_t)eo + (uint32_t)(cst[q][c] + g);
            const uint32_t vo = (uint32_t)(vbs[q][c] + g) * 8u;
#pragma unroll
            for (int s = 0; s < LPL; ++s) {
                const bool ok = g + s * G < len;
                const int p = ld_u8(rPA, po + s * G);
                const double v = ld_f64(rAv, vo + s * G * 8);
                pp[c][s] = ok ? p : trash;   // masked slots: zero into the lane's scratch row
                pv[c][s] = ok ? v : 0.0;
            }
        }
        if constexpr (PIPE) {
            __builtin_amdgcn_sched_barrier(0);
            stage1(grp + 1);
            __builtin_amdgcn_sched_barrier(0);
        }
        TQ A[R][NC];
#pragma unroll
        for (int c0 = 0; c0 < NC; c0 += TC) {
#pragma unroll
            for (int t = 0; t <= R; ++t) {
                const int row = t < R ? t * G + g : trash;
#pragma unroll
                for (int cc = 0; cc < TC; ++cc) tile[(q * RS + row) * TC + cc] = (TQ)0;
            }
            wave_sync();
#pragma unroll
            for (int cc = 0; cc < TC; ++cc) {
                const int c = c0 + cc;
                if (c < NC) {
#pragma unroll
                    for (int s = 0; s < LPL; ++s) tile[(q * RS + pp[c][s]) * TC + cc] = (TQ)pv[c][s];
                    const int len = longc ? cln[q][c] : 0;
                    if (len > LPL * G) {  // long columns: the rest straight from memory
                        const int e0 = cst[q][c], vb = vbs[q][c];
                        for (int e = g + LPL * G; e < len; e += G)
                            tile[(q * RS + a.posA[eo + e0 + e]) * TC + cc] = (TQ)a.Ak_v[vb + e];
                    }
                }
            }
            wave_sync();
#pragma unroll
            for (int t = 0; t < R; ++t)
#pragma unroll
                for (int cc = 0; cc < TC; ++cc)
                    if (c0 + cc < NC) A[t][c0 + cc] = tile[(q * RS + t * G + g) * TC + cc];
            wave_sync();
        }
        TQ bq[R];
#pragma unroll
        for (int t = 0; t < R; ++t) bq[t] = (TQ)bsh[q * RS + t * G + g];
        if constexpr (PIPE) {
            __builtin_amdgcn_sched_barrier(0);
            stage2();
            __builtin_amdgcn_sched_barrier(0);
        }

        // ---- Householder QR (dgeqr2's sign convention, beta = -sign(alpha) ||x||),
        //      applied to b as well
        // 1 / R_kk: in registers for the plain map, in LDS for the weighted
        // forms (whose solves run beside the adjoint's FP64 passes)
        TQ rinv[WEIGHTED ? 1 : NC];
        auto RINV = [&](int k) -> TQ {
            if constexpr (WEIGHTED) return rinv_sh[q * NC + k];
            else return rinv[k];
        };
        // |R_kk| over the live columns, for the rank test: largest, smallest,
        // and whether one is NaN (of the last stage when there are two)
        TQ dmax = 0, dmin = (TQ)INFINITY;
        bool dnan = false;
        // Soft weights: the penalised problem min ||A m - b||^2 + m^T P m is
        // the least-squares problem of the stacked [A; diag(sqrt p)].  Its QR
        // is taken in two stages: the QR of A, then the QR of
        // [R_1; diag(sqrt p)] (rows 0..|J_j|-1: R_1, zero below its diagonal;
        // rows NC..NC+|J_j|-1: the penalty rows; zero rows between them change
        // no reflector), so a block needs max(|I_j|, 2 NC) rows, not
        // |I_j| + |J_j|.  The right
        // side keeps c_1 and drops c_2, whose norm is the first stage's share
        // of the penalised residual.
        double c2s1 = 0.0;
#pragma unroll 1
        for (int stage = 0; stage < (WEIGHTED ? 2 : 1); ++stage) {
            if (stage == 1) {
                double r2 = 0.0;
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    const int row = t * G + g;
                    const double x = (double)bq[t];
                    r2 += row >= nJ ? x * x : 0.0;
                    if (row >= nJ) bq[t] = (TQ)0;
                }
                c2s1 = group_sum<G>(r2);
                // p_c into the group's LDS slots and sqrt(p_c) through the (now
                // free) LDS tile: lane g computes the columns g, g+G, ...
                TQ* sp = tile + q * RS * TC;
                double* pen0 = pen_sh + q * NC;
#pragma unroll
                for (int c = g; c < NC; c += G) {
                    const double p = (valid && c < nJ) ? a.mu * (1.0 / a.w[scol + c] - 1.0) : 0.0;
                    pen0[c] = p;
                    sp[c] = (TQ)sqrt(p);
                }
                wave_sync();
                // The first stage left R_1 in rows 0..|J_j|-1 and zeros below
                // (its reflectors clear the entries under the diagonal), so only
                // the penalty entries go in: sqrt(p_c) at row NC + c, a row fixed
                // at compile time (rows |J_j|..NC-1 stay zero, which changes no
                // reflector), held by one lane of the group.
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const int rc = NC + c;
                    const TQ s = sp[c];
                    A[rc / G][c] = (g == rc % G) ? s : A[rc / G][c];
                }
                wave_sync();
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                if (PIPE && (k == NC / 3 || k == (2 * NC) / 3)) {
                    __builtin_amdgcn_sched_barrier(0);
                    if (k == NC / 3) stage3();
                    else stage4();
                    __builtin_amdgcn_sched_barrier(0);
                }
                const int tk = k / G, gk = k % G;
                TQ sig = 0;
#pragma unroll
                for (int t = tk; t < R; ++t) {
                    const TQ x = A[t][k];
                    const bool below = (t > tk) || (g > gk);
                    sig += below ? x * x : (TQ)0;
                }
                sig = group_sum<G>(sig);
                // the diagonal entry, from the lane that holds row k (one
                // quad-permute move for groups of up to four lanes)
                const TQ alp = group_bcast<G>(A[tk][k], g, gk);
                const bool zero = !(sig > (TQ)0);
                const TQ nrm = root<TQ>(alp * alp + sig);
                const TQ beta = zero ? alp : -copysign(nrm, alp);
                const TQ ib = recip<TQ>(beta);
                // H = I - sigma u u^T with the unnormalised vector u = x - beta e_k
                // (u_k = alpha - beta, x below the diagonal): the reflector of the
                // normalised form (v_k = 1, tau = (beta - alpha) / beta) without the
                // scaling of v; sigma = 1 / (beta (beta - alpha)), 0 when x is
                // already a multiple of e_k.  Entries below the diagonal are not
                // read again.
                const TQ sigma = zero ? (TQ)0 : recip<TQ>(beta * (beta - alp));
                if (stage == (WEIGHTED ? 1 : 0)) {
                    // columns past |J_j| are zero, so their beta is an exact 0:
                    // it leaves the largest and the NaN flag as they are, and only
                    // the smallest needs the live columns' mask
                    const TQ ab = fabs(beta);
                    dmax = fmax(dmax, ab);
                    dmin = k < nJ ? fmin(dmin, ab) : dmin;
                    dnan |= !(ab == ab);
                }
                if constexpr (WEIGHTED) {
                    if (g == 0) rinv_sh[q * NC + k] = ib;
                } else {
                    rinv[k] = ib;
                }
                TQ v[R];
#pragma unroll
                for (int t = tk; t < R; ++t) {
                    const bool below = (t > tk) || (g > gk);
                    const bool diag = (t == tk) && (g == gk);
                    v[t] = below ? A[t][k] : (diag ? alp - beta : (TQ)0);
                    if (diag) A[t][k] = beta;
                    // weighted forms: exact zeros under the diagonal (what the
                    // second stage needs below R_1; nothing else reads them)
                    if (WEIGHTED && below) A[t][k] = (TQ)0;
                }
                TQ w[NC + 1];
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
                // sigma scales whichever is shorter: the reduced dot products
                // (one per trailing column and b) or this lane's rows of v.
                // FP64 blocks, and FP32 blocks of more than 100 entries per
                // lane, keep the per-column scaling: scaling v changes their
                // schedule and costs them a wave slot or scratch.
                const bool scale_v = REFINE && R * NC <= 100 && (NC - k) > (R - tk);
#pragma unroll
                for (int c = k + 1; c < NC; ++c) {
                    TQ wc;
                    if constexpr (REFINE && MODE == 1) wc = group_sum_x<G>(w[c]);
                    else wc = group_sum<G>(w[c]);
                    w[c] = scale_v ? wc : wc * sigma;
                }
                wb = scale_v ? group_sum<G>(wb) : group_sum<G>(wb) * sigma;
                if (scale_v) {
#pragma unroll
                    for (int t = tk; t < R; ++t) v[t] *= sigma;
                }
#pragma unroll
                for (int c = k + 1; c < NC; ++c)
#pragma unroll
                    for (int t = tk; t < R; ++t) A[t][c] -= w[c] * v[t];
#pragma unroll
                for (int t = tk; t < R; ++t) bq[t] -= wb * v[t];
            }
        }

        if constexpr (PIPE) {
            __builtin_amdgcn_sched_barrier(0);
            stage5(bi ^ 1);
            __builtin_amdgcn_sched_barrier(0);
        }

        // ---- rank test: |R_kk| <= 10 * rows * eps * max |R_ii|
        bool bad_rank = false;
        {
            const TQ eps = std::is_same<TQ, float>::value ? (TQ)1.1920928955078125e-07
                                                          : (TQ)2.220446049250313e-16;
            const TQ tol = (TQ)10 * (TQ)nrows * eps * dmax;
            // some live |R_kk| <= tol (or NaN), or all of them zero
            if (nJ > 0) bad_rank = dnan || !(dmax > (TQ)0) || !(dmin > tol);
        }

        // ||c2||^2 = rows nJ.. of Q^T b, before the back substitution consumes b
        double c2sq = 0.0;
        if constexpr (!REFINE) {
            double r2 = 0.0;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const double x = (double)bq[t];
                r2 += (t * G + g >= nJ) ? x * x : 0.0;
            }
            c2sq = group_sum<G>(r2) + c2s1;
        }

        // Back substitution x = R^{-1} z, column by column: z holds the right
        // side distributed like the rows (z[t]: row t*G + g) and is consumed.
        // x_k comes from the lane owning row k and is broadcast; then every
        // lane takes x_k times column k off its rows in blocks t <= k / G.
        // Rows at or below k are done by then, so the entries below the
        // diagonal (Householder vectors) only touch finished rows.
        auto back_solve = [&](TQ (&z)[R], TQ (&x)[NC]) {
#pragma unroll
            for (int k = NC - 1; k >= 0; --k) {
                const int tk = k / G, gk = k % G;
                const TQ xk = group_bcast<G>(z[tk] * RINV(k), g, gk);
                x[k] = (k < nJ) ? xk : (TQ)0;
#pragma unroll
                for (int t = 0; t <= tk; ++t) z[t] -= A[t][k] * x[k];
            }
        };
        // x = R^{-1} z into an LDS vector (the weighted forms): as back_solve,
        // with x_k stored by one lane of the group
        auto back_solve_v = [&](TQ (&z)[R], double* x_sh) {
#pragma unroll
            for (int k = NC - 1; k >= 0; --k) {
                const int tk = k / G, gk = k % G;
                TQ xk = group_bcast<G>(z[tk] * RINV(k), g, gk);
                xk = (k < nJ) ? xk : (TQ)0;
                if (g == 0) x_sh[k] = (double)xk;
#pragma unroll
                for (int t = 0; t <= tk; ++t) z[t] -= A[t][k] * xk;
            }
            wave_sync();
        };
        // ---- R m = c1 (the weighted forms solve it into their LDS slot below)
        TQ m[WEIGHTED ? 1 : NC];
        if constexpr (!WEIGHTED) back_solve(bq, m);

        double* rsh = lds_tile + q * RS;  // residual vector (the tile is free now)

        // Sparse FP64 passes over the gathered entries of the block.  Rows are
        // distinct inside one column, so the lanes of a group never update
        // one LDS slot in the same instruction, and the wave's LDS operations
        // complete in program order from column to column.  The values are
        // reloaded (L2-resident) with all loads issued first.  A slot past
        // the column's length loads its value from the first offset past the
        // value array, which reads 0, and its row is clamped into the
        // problem's own LDS rows: it adds exactly zero wherever it lands.
        const uint32_t v_end = a.nnzA * 8u;
        auto load_entries = [&]() {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int len = cln[q][c];
                const uint32_t po = (uint32_t)eo + (uint32_t)(cst[q][c] + g);
                const uint32_t vo = (uint32_t)(vbs[q][c] + g) * 8u;
#pragma unroll
                for (int u = 0; u < LPL; ++u) {
                    const bool ok = g + u * G < len;
                    const int p = ld_u8(rPA, po + u * G);
                    pv[c][u] = ld_f64(rAv, ok ? vo + u * G * 8 : v_end);
                    pp[c][u] = min(p, trash);
                }
            }
        };
        // vec += sgn * A x, x an LDS vector.  Entries past the register
        // cache of a long column are taken in one loop over the columns
        // (not unrolled: one copy of the memory path).
        auto scatter_v = [&](double* vec, const double* x_sh, double sgn) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double xc = sgn * x_sh[c];
#pragma unroll
                for (int u = 0; u < LPL; ++u) lds_add(&vec[pp[c][u]], pv[c][u] * xc);
            }
            if (longc) {
#pragma unroll 1
                for (int c = 0; c < NC; ++c) {
                    const int len = cln[q][c];
                    const double xc = sgn * x_sh[c];
                    const int e0 = cst[q][c], vb = vbs[q][c];
                    for (int e = g + LPL * G; e < len; e += G) lds_add(&vec[a.posA[eo + e0 + e]], a.Ak_v[vb + e] * xc);
                }
            }
            wave_sync();
        };
        // out = A^T vec (summed over the group) into an LDS vector; a long
        // column's remaining entries are added in a second, rolled loop
        auto gather_v = [&](const double* vec, double* out_sh) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double sacc = 0.0;
#pragma unroll
                for (int u = 0; u < LPL; ++u) sacc += pv[c][u] * vec[pp[c][u]];
                sacc = group_sum<G>(sacc);
                if (g == 0) out_sh[c] = sacc;
            }
            if (longc) {
                wave_sync();
#pragma unroll 1
                for (int c = 0; c < NC; ++c) {
                    const int len = cln[q][c];
                    const int e0 = cst[q][c], vb = vbs[q][c];
                    double sacc = 0.0;
                    for (int e = g + LPL * G; e < len; e += G) sacc += a.Ak_v[vb + e] * vec[a.posA[eo + e0 + e]];
                    sacc = group_sum<G>(sacc);
                    if (g == 0) out_sh[c] += sacc;
                }
            }
            wave_sync();
        };
        // x = R^{-1} R^{-T} rhs in the QR's precision (R^T R = A^T A + P), rhs
        // and x LDS vectors; returns ||y||^2 for y = R^{-T} rhs
        auto solve_normal_v = [&](const double* rhs_sh, double* x_sh) {
            TQ ydist[R];
#pragma unroll
            for (int t = 0; t < R; ++t) ydist[t] = 0;
            double yy = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                TQ part = 0;
#pragma unroll
                // rows at or past c hold ydist = 0 (not solved yet), so they
                // add nothing and need no mask
                for (int t = 0; t < R; ++t)
                    if (t * G < c) part += A[t][c] * ydist[t];
                part = group_sum<G>(part);
                TQ yc = ((TQ)rhs_sh[c] - part) * RINV(c);
                yc = (c < nJ) ? yc : (TQ)0;
                yy += (double)yc * (double)yc;
                if (g == c % G) ydist[c / G] = yc;
            }
            back_solve_v(ydist, x_sh);
            return yy;
        };
        auto reset = [&](double* vec, bool from_b) {
#pragma unroll
            for (int t = 0; t < R; ++t) vec[t * G + g] = from_b ? bsh[q * RS + t * G + g] : 0.0;
            vec[trash] = 0.0;
        };

        // penalties p_c = mu (1/w_c - 1) in LDS, written before the second
        // QR stage (read by every lane of the group, so they hold no
        // registers across the refinement and the adjoint)
        double* pen = pen_sh + q * NC;

        double mfin[WEIGHTED ? 1 : NC];
        double rr;
        double* msh = vsh + q * kNV * NC;      // weighted forms: m
        if constexpr (REFINE && MODE == 0) {
            // One seminormal refinement step, residual in FP64, taken in
            // column chunks so that one chunk of entries at a time is held in
            // registers:  r = b - A m (in place over b);  R^T y = A^T r, with
            // each column's partial of A^T r folded into the forward solve's
            // own FP64 group reduction;  R d = y;  m += d.  The new residual
            // ||b - A(m + d)||^2 = ||r||^2 - 2 d^T A^T r + ||A d||^2, where
            // d^T A^T r and ||A d||^2 both equal ||y||^2 up to rounding.
            // Blocks of up to 13 columns keep the entries the gather loaded
            // (held through the QR) for both passes; wider ones reload them
            // three columns at a time (a whole block's entries would hold
            // 3 * NC * LPL registers and cost a wave slot per SIMD).
            constexpr int CH = NC <= 13 ? NC : 3;
            constexpr bool ONE = CH >= NC;
            double* rv = bsh + q * RS;
            rv[trash] = 0.0;
            auto load_chunk = [&](int c0, double (&cv)[CH][LPL], int (&cp)[CH][LPL]) {
#pragma unroll
                for (int cc = 0; cc < CH; ++cc) {
                    const int c = c0 + cc;
                    if (c < NC) {
                        const int len = cln[q][c];
                        const uint32_t po = (uint32_t)eo + (uint32_t)(cst[q][c] + g);
                        const uint32_t vo = (uint32_t)(vbs[q][c] + g) * 8u;
#pragma unroll
                        for (int u = 0; u < LPL; ++u) {
                            const bool ok = g + u * G < len;
                            const int p = ld_u8(rPA, po + u * G);
                            cv[cc][u] = ld_f64(rAv, ok ? vo + u * G * 8 : v_end);
                            cp[cc][u] = min(p, trash);
                        }
                    }
                }
            };
            double cv[CH][LPL];
            int cp[CH][LPL];
            if constexpr (ONE) {
#pragma unroll
                for (int c = 0; c < CH; ++c)
#pragma unroll
                    for (int u = 0; u < LPL; ++u) {
                        cv[c][u] = pv[c][u];
                        cp[c][u] = pp[c][u];
                    }
            }
#pragma unroll
            for (int c0 = 0; c0 < NC; c0 += CH) {
                if constexpr (!ONE) load_chunk(c0, cv, cp);
#pragma unroll
                for (int cc = 0; cc < CH; ++cc) {
                    const int c = c0 + cc;
                    if (c < NC) {
                        const double xc = -(double)m[c];
#pragma unroll
                        for (int u = 0; u < LPL; ++u) lds_add(&rv[cp[cc][u]], cv[cc][u] * xc);
                        const int len = longc ? cln[q][c] : 0;
                        if (len > LPL * G) {  // long columns: the rest straight from memory
                            const int e0 = cst[q][c], vb = vbs[q][c];
                            for (int e = g + LPL * G; e < len; e += G)
                                lds_add(&rv[a.posA[eo + e0 + e]], a.Ak_v[vb + e] * xc);
                        }
                    }
                }
            }
            wave_sync();
            double r2 = 0.0;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const double x = rv[t * G + g];  // rows past |I_j| hold zeros
                r2 += x * x;
            }
            const double rr0 = group_sum<G>(r2);
            TQ ydist[R];
            TQ yrep[NC];
#pragma unroll
            for (int t = 0; t < R; ++t) ydist[t] = 0;
#pragma unroll
            for (int c0 = 0; c0 < NC; c0 += CH) {
                if constexpr (!ONE) load_chunk(c0, cv, cp);
#pragma unroll
                for (int cc = 0; cc < CH; ++cc) {
                    const int c = c0 + cc;
                    if (c < NC) {
                        double gp = 0.0;
#pragma unroll
                        for (int u = 0; u < LPL; ++u) gp += cv[cc][u] * rv[cp[cc][u]];
                        const int len = longc ? cln[q][c] : 0;
                        if (len > LPL * G) {
                            const int e0 = cst[q][c], vb = vbs[q][c];
                            for (int e = g + LPL * G; e < len; e += G) gp += a.Ak_v[vb + e] * rv[a.posA[eo + e0 + e]];
                        }
                        TQ part = 0;
#pragma unroll
                        for (int t = 0; t < R; ++t)  // rows >= c: ydist = 0
                            if (t * G < c) part += A[t][c] * ydist[t];
                        const double sc = group_sum<G>(gp - (double)part);
                        TQ yc = (TQ)sc * RINV(c);
                        yc = (c < nJ) ? yc : (TQ)0;
                        yrep[c] = yc;
                        if (g == c % G) ydist[c / G] = yc;
                    }
                }
            }
            TQ dl[NC];
            back_solve(ydist, dl);
            // ||y||^2 is the step's decrease of the residual, (u kappa)^2 of
            // it at most: the QR's precision is ample.  The map is stored in
            // FP32, so m + d is formed there too (the correctly rounded sum
            // of the two floats).
            TQ yy = 0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                yy += yrep[c] * yrep[c];
                mfin[c] = (double)(m[c] + dl[c]);
            }
            rr = rr0 - (double)yy + outj;
        } else if constexpr (!WEIGHTED) {
#pragma unroll
            for (int c = 0; c < NC; ++c) mfin[c] = (double)m[c];
            rr = c2sq + outj;   // ||c2||^2
        } else {
            // soft-weighted forms: m, A^T r, the correction and A^T r - P m
            // in the problem's LDS slots
            double* gsh = msh + NC;
            double* dsh = msh + 2 * NC;
            double* csh = msh + 3 * NC;
            back_solve_v(bq, msh);          // R m = c1
            if constexpr (REFINE) {
                // refinement steps on the normal equations
                // (A^T A + P) m = A^T b with the residual in FP64:
                // r = b - A m,  m += R^{-1} R^{-T} (A^T r - P m)
                double rr_it = 0.0;
#pragma unroll
                for (int it = 0; it < kWSteps; ++it) {
                    reset(rsh, true);
                    load_entries();
                    wave_sync();
                    scatter_v(rsh, msh, -1.0);
                    double r2 = 0.0;
#pragma unroll
                    for (int t = 0; t < R; ++t) {
                        const double x = rsh[t * G + g];
                        r2 += (t * G + g < nIj) ? x * x : 0.0;
                    }
                    rr_it = group_sum<G>(r2);
                    gather_v(rsh, gsh);
                    for (int c = g; c < NC; c += G) csh[c] = gsh[c] - pen[c] * msh[c];
                    wave_sync();
                    const double yy = solve_normal_v(csh, dsh);
                    // ||b - A(m + d)||^2 = ||r||^2 - 2 d^T A^T r + ||A d||^2, and
                    // ||A d||^2 = ||R d||^2 - d^T P d with R d = y (second order in d)
                    double dg = 0.0, pdd = 0.0;
                    for (int c = g; c < NC; c += G) {
                        const double d = dsh[c];
                        dg += d * gsh[c];
                        pdd += pen[c] * d * d;
                        msh[c] += d;
                    }
                    dg = group_sum<G>(dg);
                    pdd = group_sum<G>(pdd);
                    wave_sync();
                    rr_it = rr_it - 2.0 * dg + (yy - pdd);
                }
                rr = rr_it + outj;
            } else {
                // ||c2||^2 of the stacked form less m^T P m
                double pm = 0.0;
                for (int c = g; c < NC; c += G) pm += pen[c] * msh[c] * msh[c];
                rr = c2sq - group_sum<G>(pm) + outj;
            }
        }

        if constexpr (BACKWARD) {
            __builtin_amdgcn_sched_barrier(0);
            // r = A m - b is held as rsh = b - A m = -r
            double* hsh = msh + NC;         // h = 2 A^T r
            double* dsh = msh + 2 * NC;     // correction of lambda
            double* tsh = msh + 3 * NC;     // its right side
            double* lsh = msh + 4 * NC;     // lambda
            double* al = alsh + q * RS;
            reset(rsh, true);
            load_entries();
            wave_sync();
            scatter_v(rsh, msh, -1.0);
            // h = 2 A^T r,  lambda = (A^T A + P)^{-1} h
            gather_v(rsh, hsh);
            for (int c = g; c < NC; c += G) hsh[c] *= -2.0;
            wave_sync();
            solve_normal_v(hsh, lsh);
            if constexpr (REFINE) {
#pragma unroll
                for (int it = 0; it < kWSteps; ++it) {  // FP64-residual refinement of lambda
                    reset(al, false);
                    load_entries();   // reloaded per pass: no entries held across the solves
                    wave_sync();
                    scatter_v(al, lsh, 1.0);
                    gather_v(al, tsh);
                    for (int c = g; c < NC; c += G) tsh[c] = hsh[c] - tsh[c] - pen[c] * lsh[c];
                    wave_sync();
                    solve_normal_v(tsh, dsh);
                    for (int c = g; c < NC; c += G) lsh[c] += dsh[c];
                    wave_sync();
                }
            }
            reset(al, false);
            load_entries();
            wave_sync();
            scatter_v(al, lsh, 1.0);
            // dL/dA at the gathered entries: 2 r m^T - r lambda^T - (A lambda) m^T
            const double dL = a.dL;
            double* cj = a.contrib + eo;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int e0 = cst[q][c];
                const int clen = cln[q][c];
                const double mc = msh[c], lc = lsh[c];
#pragma unroll
                for (int u = 0; u < LPL; ++u) {
                    const int p = pp[c][u];
                    if (g + u * G < clen) cj[e0 + g + u * G] = dL * (-2.0 * rsh[p] * mc + rsh[p] * lc - al[p] * mc);
                }
            }
            if (longc) {
#pragma unroll 1
                for (int c = 0; c < NC; ++c) {
                    const int e0 = cst[q][c];
                    const int len = cln[q][c];
                    const double mc = msh[c], lc = lsh[c];
                    for (int e = g + LPL * G; e < len; e += G) {
                        const int p = a.posA[eo + e0 + e];
                        cj[e0 + e] = dL * (-2.0 * rsh[p] * mc + rsh[p] * lc - al[p] * mc);
                    }
                }
            }
            // dL/dA_0(:, j): -2 r + A lambda inside I_j, 2 a_0 outside
            for (int e = a0 + g; e < a1; e += G) {
                const int p = a.posB[e];
                a.gA0[e] = p != 0xFF ? dL * (2.0 * rsh[p] + al[p]) : dL * 2.0 * a.A0_v[e];
            }
            if (valid) {
                for (int c = g; c < NC; c += G) {
                    if (c < nJ) {
                        a.segoff[scol + c] = eo + cst[q][c];
                        if (a.gw) {
                            const double wl = a.w[scol + c];
                            a.gw[scol + c] = dL * a.mu * lsh[c] * msh[c] / (wl * wl);
                        }
                    }
                }
            }
            wave_sync();
        }

        // ---- outputs
        bool nonfinite = !isfinite(rr);
        if constexpr (WEIGHTED) {
            float bad = 0.f;
            for (int c = g; c < NC; c += G) bad = (c < nJ && !isfinite(msh[c])) ? 1.f : bad;
            nonfinite |= group_max<G>(bad) > 0.f;
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) nonfinite |= (c < nJ) && !isfinite(mfin[c]);
        }
        if (valid) {
            if (a.M) {
                if constexpr (WEIGHTED) {
                    for (int c = g; c < nJ; c += G) {
                        if constexpr (REFINE) static_cast<float*>(a.M)[scol + c] = (float)msh[c];
                        else static_cast<double*>(a.M)[scol + c] = msh[c];
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        if (c < nJ && (c % G) == g) {
                            if constexpr (REFINE) static_cast<float*>(a.M)[scol + c] = (float)mfin[c];
                            else static_cast<double*>(a.M)[scol + c] = mfin[c];
                        }
                    }
                }
            }
            if (g == 0) {
                if (a.col_res2) a.col_res2[j] = rr;
                if (bad_rank) report(a.status, j, kStRank);
                else if (nonfinite) report(a.status, j, kStNonfinite);
            }
        }
        if (a.part) {  // the group's residuals, summed by a fixed wave-wide tree
            const double gs = group_sum<64>((g == 0 && valid) ? rr : 0.0);
            if (lane == 0) racc += gs;
        }
        wave_sync();  // the next group's metadata is in LDS
    }
    if (a.part && lane == 0) a.part[a.part_base + (int)blockIdx.x] = racc;
}

template <typename TQ, int G, int R, int NC, int TC, int LPL, int MODE>
hipError_t launch_numeric(const NumericArgs& args, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_numeric<TQ, G, R, NC, TC, LPL, MODE>), dim3(grid), dim3(64), 0, s, args);
    return hipGetLastError();
}

template <typename TQ, int G, int R, int NC, int TC, int LPL, int MODE>
int numeric_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_numeric<TQ, G, R, NC, TC, LPL, MODE>, 64, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

// LPL: entries of one A_k column a lane moves with static indices (longer
// columns fall back to a loop over memory), sized for 5- to 9-point stencils.
using LaunchFn = hipError_t (*)(const NumericArgs&, int, hipStream_t);

// the adjoint exists for the weighted variants only
template <typename TQ, int G, int R, int NC, int TC, int LPL, bool W>
constexpr LaunchFn backward_launcher() {
    if constexpr (W) return &launch_numeric<TQ, G, R, NC, TC, LPL, 2>;
    else return nullptr;
}

#define SAM_VARIANT(TQ, PREC, G, R, NC, TC, LPL, W)                                                \
    NumericVariant{PREC, G, R, NC, W, TC, LPL, &launch_numeric<TQ, G, R, NC, TC, LPL, W ? 1 : 0>, \
                   backward_launcher<TQ, G, R, NC, TC, LPL, W>(),                             \
                   &numeric_blocks_per_cu<TQ, G, R, NC, TC, LPL, W ? 1 : 0>}

// Menu per precision, cheapest first.  Shapes of the workloads: 2D 5-point
// level 1 (13 x 5), level 2 (25 x 13); 3D 7-point level 2 (63 x 25); 2D
// 9-point level 2 with thresholds (ragged, mostly 20..45 x 5..20, at most
// 49 x 24); weighted 3D (63 x 25 with 25 penalty rows: 64 rows in two stages).  The first fitting entry of a (precision,
// weighting) group serves a column by default; later entries of the same
// shape class are alternatives the autotuner can put in front
// (sam_plan_select).  The FP32 classes between 36 x 10 and 48 x 24 follow the
// ragged 9-point distribution: each halves the padded work of the columns
// it takes from the next wider class.
const NumericVariant kMenu[] = {
    // FP32 + refinement
    SAM_VARIANT(float, 1, 2, 8, 5, 4, 3, false),
    SAM_VARIANT(float, 1, 2, 8, 8, 4, 3, false),
    SAM_VARIANT(float, 1, 4, 9, 10, 1, 2, false),   // ragged 9-point / thresholded blocks
    SAM_VARIANT(float, 1, 4, 9, 12, 1, 2, false),
    SAM_VARIANT(float, 1, 4, 7, 13, 1, 2, false),
    SAM_VARIANT(float, 1, 4, 8, 16, 2, 2, false),
    SAM_VARIANT(float, 1, 8, 5, 14, 1, 2, false),
    SAM_VARIANT(float, 1, 8, 6, 16, 1, 2, false),
    SAM_VARIANT(float, 1, 8, 5, 20, 1, 2, false),
    SAM_VARIANT(float, 1, 8, 6, 24, 1, 2, false),
    SAM_VARIANT(float, 1, 16, 4, 25, 1, 1, false),
    SAM_VARIANT(float, 1, 32, 4, 32, 1, 1, false),
    SAM_VARIANT(float, 1, 1, 13, 5, 1, 5, false),   // one problem per lane, no reductions
    SAM_VARIANT(float, 1, 8, 4, 13, 2, 1, false),
    SAM_VARIANT(float, 1, 32, 2, 25, 1, 1, false),
    // FP64
    SAM_VARIANT(double, 0, 2, 8, 5, 4, 3, false),
    SAM_VARIANT(double, 0, 2, 8, 8, 4, 3, false),
    SAM_VARIANT(double, 0, 4, 7, 13, 2, 2, false),
    SAM_VARIANT(double, 0, 8, 4, 16, 2, 1, false),
    SAM_VARIANT(double, 0, 32, 2, 25, 1, 1, false),
    SAM_VARIANT(double, 0, 64, 2, 32, 1, 1, false),
    SAM_VARIANT(double, 0, 1, 13, 5, 1, 5, false),
    SAM_VARIANT(double, 0, 8, 4, 13, 2, 1, false),
    // soft-weighted (stacked penalty rows)
    SAM_VARIANT(float, 1, 4, 7, 13, 2, 2, true),
    SAM_VARIANT(float, 1, 16, 4, 25, 1, 1, true),
    SAM_VARIANT(float, 1, 32, 3, 25, 1, 1, true),
    SAM_VARIANT(float, 1, 64, 2, 32, 1, 1, true),
    SAM_VARIANT(double, 0, 4, 8, 13, 2, 2, true),
    SAM_VARIANT(double, 0, 64, 2, 25, 1, 1, true),
    SAM_VARIANT(double, 0, 64, 2, 32, 1, 1, true),
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
