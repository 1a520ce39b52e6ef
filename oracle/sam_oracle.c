/*
 * sam_oracle.c -- plain, slow, FP64 CPU reference for the sparse approximate
 * map (SAM) construction of Islam, Carr and Jacobs, "Optimization of
 * Approximate Maps for Linear Systems Arising in Discretized PDEs".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU path is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header or table with the
 * GPU library, and the GPU library never calls it.
 *
 * What it computes (paper notation):
 *   - Section 2, eq. (approx_map): N_k = argmin ||A_k N - A_0||_F over N with
 *     pattern S, split by columns into n independent least-squares problems
 *     min_m ||A_k(:,J_j) m - A_0(:,j)||_2 (the column split is stated at the
 *     end of Section 2).  Rows outside I_j = rows(A_k(:,J_j)) are zero in the
 *     submatrix, so the problem is solved on A_k(I_j, J_j); the A_0 entries of
 *     column j outside I_j only add the constant out_j to the residual.
 *     The minimiser is unique when A_k is nonsingular; it is computed here by
 *     Householder QR (LAPACK dgeqr2 conventions) followed by back substitution.
 *   - Section 2, eq. (res): R_k = A_k N_k - A_0 and its Frobenius norm, the
 *     quality measure of Section 5.
 *   - Section 3: level neighbours of the adjacency graph, i.e. the pattern of
 *     (I + B)^p column by column.
 *   - Section 4: the three sparsification rules (global threshold on the
 *     diagonally scaled matrix, column threshold tau, fixed count lfil).
 *   - A soft-weighted variant (penalty p = mu (1/w - 1) on pattern entries)
 *     and the exact gradient of sum_j ||A m_j - b_j||^2 with respect to the
 *     values of A_k, A_0 and the weights w.  This variant is not in the paper;
 *     it is the differentiable extension used to rank candidate entries.
 *
 * Conventions: CSC with int32 indices, rows sorted ascending in each column,
 * no duplicates; values FP64.  Status codes: 0 ok, 1 bad argument,
 * 5 rank deficient block, 6 non-finite value.
 */
#include <math.h>
#include <float.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_RANK 5
#define OR_ERR_NONFINITE 6

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

static int cmp_int(const void* a, const void* b) {
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* Section 4: sparsification of A into the boolean pattern B = S(A~).        */
/* kind 0: none (stored entries), 1: global threshold, 2: column tau,        */
/* 3: lfil.  The diagonal is always part of B (each rule keeps i == j).      */
/* Writes out_cp (n+1) and, if out_ri != NULL, the rows (capacity nnz + n).  */
/* ------------------------------------------------------------------------ */
typedef struct { double mag; int row; } magrow;

static int cmp_magrow(const void* a, const void* b) {
    const magrow* x = (const magrow*)a;
    const magrow* y = (const magrow*)b;
    if (x->mag > y->mag) return -1;      /* larger magnitude first */
    if (x->mag < y->mag) return 1;
    return (x->row > y->row) - (x->row < y->row); /* ties: smaller row first */
}

int or_sparsify(int n, const int* cp, const int* ri, const double* v,
                int kind, double thresh, int global_scale, double tau, int lfil,
                int* out_cp, int* out_ri) {
    if (n < 0 || kind < 0 || kind > 3) return OR_ERR_ARG;
    if (kind == 2 && (tau < 0.0 || tau > 1.0)) return OR_ERR_ARG;
    double* D = NULL;
    if (kind == 1) {
        /* D_ii = |A_ii| if nonzero, else 1 */
        D = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        for (int j = 0; j < n; ++j) {
            D[j] = 0.0;
            for (int e = cp[j]; e < cp[j + 1]; ++e)
                if (ri[e] == j) D[j] = fabs(v[e]);
            if (!(D[j] > 0.0)) D[j] = 1.0;
        }
    }
    int* keep = (int*)malloc(sizeof(int) * 64);
    int cap = 64;
    magrow* mr = (magrow*)malloc(sizeof(magrow) * 64);
    out_cp[0] = 0;
    for (int j = 0; j < n; ++j) {
        int len = cp[j + 1] - cp[j];
        if (len + 1 > cap) {
            cap = 2 * (len + 1);
            keep = (int*)realloc(keep, sizeof(int) * (size_t)cap);
            mr = (magrow*)realloc(mr, sizeof(magrow) * (size_t)cap);
        }
        int nk = 0, has_diag = 0;
        if (kind == 0) {
            for (int e = cp[j]; e < cp[j + 1]; ++e) keep[nk++] = ri[e];
        } else if (kind == 1) {
            for (int e = cp[j]; e < cp[j + 1]; ++e) {
                int i = ri[e];
                double s = global_scale > 0 ? sqrt(D[i] * D[j]) : 1.0 / sqrt(D[i] * D[j]);
                if (i == j || fabs(v[e]) * s > thresh) keep[nk++] = i;
            }
        } else if (kind == 2) {
            double mx = 0.0;
            for (int e = cp[j]; e < cp[j + 1]; ++e) if (fabs(v[e]) > mx) mx = fabs(v[e]);
            for (int e = cp[j]; e < cp[j + 1]; ++e) {
                int i = ri[e];
                if (i == j || fabs(v[e]) > (1.0 - tau) * mx) keep[nk++] = i;
            }
        } else {
            /* diagonal plus the (lfil - 1) largest off-diagonal magnitudes */
            int m = 0;
            for (int e = cp[j]; e < cp[j + 1]; ++e)
                if (ri[e] != j) { mr[m].mag = fabs(v[e]); mr[m].row = ri[e]; ++m; }
            qsort(mr, (size_t)m, sizeof(magrow), cmp_magrow);
            int take = lfil - 1;
            if (take < 0) take = 0;
            if (take > m) take = m;
            for (int t = 0; t < take; ++t) keep[nk++] = mr[t].row;
        }
        for (int t = 0; t < nk; ++t) if (keep[t] == j) has_diag = 1;
        if (!has_diag) keep[nk++] = j;
        qsort(keep, (size_t)nk, sizeof(int), cmp_int);
        if (out_ri) memcpy(out_ri + out_cp[j], keep, sizeof(int) * (size_t)nk);
        out_cp[j + 1] = out_cp[j] + nk;
    }
    free(keep); free(mr); free(D);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Section 3: column j of the product pattern S(Q P):                       */
/*   out(:,j) = union over l in P(:,j) of rows(Q(:,l)), sorted.             */
/* With P = Q = B (diagonal included) this climbs one neighbour level.      */
/* Two calls: out_ri == NULL fills only out_cp.                             */
/* ------------------------------------------------------------------------ */
int or_expand(int n, const int* P_cp, const int* P_ri,
              const int* Q_cp, const int* Q_ri, int* out_cp, int* out_ri) {
    if (n < 0) return OR_ERR_ARG;
    int* mark = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) mark[i] = -1;
    int cap = 256;
    int* list = (int*)malloc(sizeof(int) * (size_t)cap);
    out_cp[0] = 0;
    for (int j = 0; j < n; ++j) {
        int cnt = 0;
        for (int e = P_cp[j]; e < P_cp[j + 1]; ++e) {
            int l = P_ri[e];
            for (int f = Q_cp[l]; f < Q_cp[l + 1]; ++f) {
                int i = Q_ri[f];
                if (mark[i] != j) {
                    mark[i] = j;
                    if (cnt == cap) { cap *= 2; list = (int*)realloc(list, sizeof(int) * (size_t)cap); }
                    list[cnt++] = i;
                }
            }
        }
        if (out_ri) {
            qsort(list, (size_t)cnt, sizeof(int), cmp_int);
            memcpy(out_ri + out_cp[j], list, sizeof(int) * (size_t)cnt);
        }
        out_cp[j + 1] = out_cp[j] + cnt;
    }
    free(mark); free(list);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Per-column dense block assembly                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    int* mark;      /* n, stamp: column id that touched row i */
    int* pos;       /* n, position of row i inside I_j */
    int* I;         /* row set */
    int capI;
    double* A;      /* nI x nJ column major, overwritten by QR */
    double* A0;     /* copy of the gathered block */
    double* b;
    double* b0;
    double* tau;
    double* m;
    double* r;
    double* y;
    double* lam;
    double* Alam;
    int capA, capJ;
} colws;

static void ws_init(colws* w, int n) {
    memset(w, 0, sizeof(*w));
    w->n = n;
    w->mark = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    w->pos = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) w->mark[i] = -1;
}

static void ws_free(colws* w) {
    free(w->mark); free(w->pos); free(w->I); free(w->A); free(w->A0);
    free(w->b); free(w->b0); free(w->tau); free(w->m); free(w->r);
    free(w->y); free(w->lam); free(w->Alam);
}

static void ws_reserve(colws* w, int nI, int nJ) {
    if (nI > w->capI) {
        w->capI = 2 * nI;
        w->I = (int*)realloc(w->I, sizeof(int) * (size_t)w->capI);
        w->b = (double*)realloc(w->b, sizeof(double) * (size_t)w->capI);
        w->b0 = (double*)realloc(w->b0, sizeof(double) * (size_t)w->capI);
        w->r = (double*)realloc(w->r, sizeof(double) * (size_t)w->capI);
        w->Alam = (double*)realloc(w->Alam, sizeof(double) * (size_t)w->capI);
    }
    if ((size_t)nI * nJ > (size_t)w->capA) {
        w->capA = 2 * nI * nJ;
        w->A = (double*)realloc(w->A, sizeof(double) * (size_t)w->capA);
        w->A0 = (double*)realloc(w->A0, sizeof(double) * (size_t)w->capA);
    }
    if (nJ > w->capJ) {
        w->capJ = 2 * nJ;
        w->tau = (double*)realloc(w->tau, sizeof(double) * (size_t)w->capJ);
        w->m = (double*)realloc(w->m, sizeof(double) * (size_t)w->capJ);
        w->y = (double*)realloc(w->y, sizeof(double) * (size_t)w->capJ);
        w->lam = (double*)realloc(w->lam, sizeof(double) * (size_t)w->capJ);
    }
}

/* I_j = sorted union of rows(Ak(:,l)) for l in J; pos[] maps row -> index. */
static int build_rowset(colws* w, int j, const int* J, int nJ,
                        const int* Ak_cp, const int* Ak_ri) {
    int cnt = 0;
    for (int c = 0; c < nJ; ++c) {
        int l = J[c];
        for (int e = Ak_cp[l]; e < Ak_cp[l + 1]; ++e) {
            int i = Ak_ri[e];
            if (w->mark[i] != j) {
                w->mark[i] = j;
                ws_reserve(w, cnt + 1, 1);
                w->I[cnt++] = i;
            }
        }
    }
    qsort(w->I, (size_t)cnt, sizeof(int), cmp_int);
    for (int p = 0; p < cnt; ++p) w->pos[w->I[p]] = p;
    return cnt;
}

/* Dense A = Ak(I,J) (plus optional sqrt(p) rows below), b = A0(I,j); returns
 * out_j = sum of A0(i,j)^2 over rows i not in I.  The block has `ld` rows. */
static double gather_block(colws* w, int j, const int* J, int nJ, int nI, int ld,
                           const int* Ak_cp, const int* Ak_ri, const double* Ak_v,
                           const int* A0_cp, const int* A0_ri, const double* A0_v) {
    memset(w->A, 0, sizeof(double) * (size_t)ld * nJ);
    memset(w->b, 0, sizeof(double) * (size_t)ld);
    for (int c = 0; c < nJ; ++c) {
        int l = J[c];
        for (int e = Ak_cp[l]; e < Ak_cp[l + 1]; ++e)
            w->A[(size_t)c * ld + w->pos[Ak_ri[e]]] = Ak_v[e];
    }
    double out = 0.0;
    for (int e = A0_cp[j]; e < A0_cp[j + 1]; ++e) {
        int i = A0_ri[e];
        if (w->mark[i] == j) w->b[w->pos[i]] = A0_v[e];
        else out += A0_v[e] * A0_v[e];
    }
    return out;
}

/* Householder QR of the ld x nJ column-major block (dgeqr2 conventions:
 * v_k = 1, beta = -sign(alpha) ||x||, sign(0) = +1, tau = 0 when the part of
 * the column below the diagonal is zero), applied to the right-hand side. */
static void householder_qr(double* A, int ld, int nJ, double* b, double* tau) {
    for (int k = 0; k < nJ; ++k) {
        double* ak = A + (size_t)k * ld;
        double alpha = ak[k];
        double sigma = 0.0;
        for (int i = k + 1; i < ld; ++i) sigma += ak[i] * ak[i];
        if (sigma == 0.0) {
            tau[k] = 0.0;
            continue;
        }
        double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
        tau[k] = (beta - alpha) / beta;
        double scal = 1.0 / (alpha - beta);
        for (int i = k + 1; i < ld; ++i) ak[i] *= scal;
        ak[k] = beta;
        for (int c = k + 1; c < nJ; ++c) {
            double* ac = A + (size_t)c * ld;
            double s = ac[k];
            for (int i = k + 1; i < ld; ++i) s += ak[i] * ac[i];
            s *= tau[k];
            ac[k] -= s;
            for (int i = k + 1; i < ld; ++i) ac[i] -= s * ak[i];
        }
        if (b) {
            double s = b[k];
            for (int i = k + 1; i < ld; ++i) s += ak[i] * b[i];
            s *= tau[k];
            b[k] -= s;
            for (int i = k + 1; i < ld; ++i) b[i] -= s * ak[i];
        }
    }
}

/* Rank test on the triangular factor: |R_kk| <= 10 * rows * eps * max|R_ii|. */
static int rank_ok(const double* A, int ld, int nJ, int rows) {
    double mx = 0.0;
    for (int k = 0; k < nJ; ++k) {
        double d = fabs(A[(size_t)k * ld + k]);
        if (!isfinite(d)) return OR_ERR_NONFINITE;
        if (d > mx) mx = d;
    }
    if (nJ > 0 && !(mx > 0.0)) return OR_ERR_RANK;
    for (int k = 0; k < nJ; ++k)
        if (fabs(A[(size_t)k * ld + k]) <= 10.0 * rows * DBL_EPSILON * mx) return OR_ERR_RANK;
    return OR_OK;
}

/* R x = rhs (upper triangular, leading nJ x nJ part of the block). */
static void back_solve(const double* A, int ld, int nJ, const double* rhs, double* x) {
    for (int k = nJ - 1; k >= 0; --k) {
        double s = rhs[k];
        for (int c = k + 1; c < nJ; ++c) s -= A[(size_t)c * ld + k] * x[c];
        x[k] = s / A[(size_t)k * ld + k];
    }
}

/* R^T x = rhs (forward substitution with the transpose). */
static void forward_solve_t(const double* A, int ld, int nJ, const double* rhs, double* x) {
    for (int k = 0; k < nJ; ++k) {
        double s = rhs[k];
        for (int c = 0; c < k; ++c) s -= A[(size_t)k * ld + c] * x[c];
        x[k] = s / A[(size_t)k * ld + k];
    }
}

/* Solve one column problem.  weights == NULL: plain least squares; else the
 * penalised problem min ||A m - b||^2 + sum_l p_l m_l^2 with
 * p_l = mu (1/w_l - 1), solved as the stacked problem [A; diag(sqrt p)].
 * On return w->m holds m, w->r holds r = b - A m (FP64, explicit), rho the
 * squared residual norm plus out_j.  Leaves the QR factor in w->A. */
static int solve_column(colws* w, int j, const int* J, int nJ,
                        const int* Ak_cp, const int* Ak_ri, const double* Ak_v,
                        const int* A0_cp, const int* A0_ri, const double* A0_v,
                        const double* weights, double mu,
                        int* nI_out, double* rho, double* out_j) {
    int nI = build_rowset(w, j, J, nJ, Ak_cp, Ak_ri);
    int ld = weights ? nI + nJ : nI;
    ws_reserve(w, ld, nJ);
    double out = gather_block(w, j, J, nJ, nI, ld, Ak_cp, Ak_ri, Ak_v, A0_cp, A0_ri, A0_v);
    if (weights) {
        for (int c = 0; c < nJ; ++c) {
            double wl = weights[c];
            if (!(wl > 0.0) || wl > 1.0) return OR_ERR_ARG;
            w->A[(size_t)c * ld + nI + c] = sqrt(mu * (1.0 / wl - 1.0));
        }
    }
    memcpy(w->A0, w->A, sizeof(double) * (size_t)ld * nJ);
    memcpy(w->b0, w->b, sizeof(double) * (size_t)ld);
    householder_qr(w->A, ld, nJ, w->b, w->tau);
    int st = rank_ok(w->A, ld, nJ, ld);
    if (st != OR_OK) return st;
    back_solve(w->A, ld, nJ, w->b, w->m);
    double s = 0.0;
    for (int i = 0; i < nI; ++i) {
        double ri = w->b0[i];
        for (int c = 0; c < nJ; ++c) ri -= w->A0[(size_t)c * ld + i] * w->m[c];
        w->r[i] = ri;
        s += ri * ri;
    }
    for (int c = 0; c < nJ; ++c) if (!isfinite(w->m[c])) return OR_ERR_NONFINITE;
    *nI_out = nI;
    *rho = s + out;
    if (out_j) *out_j = out;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* SAM build (Section 2): M values on the pattern S, per-column squared      */
/* residuals.  cols == NULL means all columns; otherwise only the listed     */
/* columns are solved (M entries of other columns are left untouched).      */
/* On failure *bad_col receives the smallest failing column.                 */
/* ------------------------------------------------------------------------ */
int or_sam_build(int n,
                 const int* Ak_cp, const int* Ak_ri, const double* Ak_v,
                 const int* A0_cp, const int* A0_ri, const double* A0_v,
                 const int* S_cp, const int* S_ri,
                 const double* w_S, double mu,
                 const int* cols, int ncols,
                 double* M_v, double* rho, int* bad_col) {
    if (n < 0) return OR_ERR_ARG;
    int total = cols ? ncols : n;
    int status = OR_OK;
    int first_bad = n;
#pragma omp parallel
    {
        colws w;
        ws_init(&w, n);
        int my_status = OR_OK, my_bad = n;
#pragma omp for schedule(dynamic, 64)
        for (int t = 0; t < total; ++t) {
            int j = cols ? cols[t] : t;
            const int* J = S_ri + S_cp[j];
            int nJ = S_cp[j + 1] - S_cp[j];
            int nI = 0;
            double r2 = 0.0;
            int st = solve_column(&w, j, J, nJ, Ak_cp, Ak_ri, Ak_v, A0_cp, A0_ri, A0_v,
                                  w_S ? w_S + S_cp[j] : NULL, mu, &nI, &r2, NULL);
            if (st != OR_OK) {
                if (j < my_bad) { my_bad = j; my_status = st; }
                continue;
            }
            for (int c = 0; c < nJ; ++c) M_v[S_cp[j] + c] = w.m[c];
            if (rho) rho[j] = r2;
        }
#pragma omp critical
        {
            if (my_bad < first_bad) { first_bad = my_bad; status = my_status; }
        }
        ws_free(&w);
    }
    if (bad_col) *bad_col = status == OR_OK ? -1 : first_bad;
    return status;
}

/* ------------------------------------------------------------------------ */
/* Row sets I_j (for inspection and tests): out(:,j) = rows of Ak(:,J_j).    */
/* ------------------------------------------------------------------------ */
int or_row_sets(int n, const int* S_cp, const int* S_ri, const int* Ak_cp, const int* Ak_ri,
                int* out_cp, int* out_ri) {
    return or_expand(n, S_cp, S_ri, Ak_cp, Ak_ri, out_cp, out_ri);
}

/* ------------------------------------------------------------------------ */
/* Explicit residual (Section 2, eq. res): ||Ak M - A0||_F^2 and ||A0||_F^2 */
/* computed straight from the definition with a dense work column.          */
/* ------------------------------------------------------------------------ */
int or_residual(int n,
                const int* Ak_cp, const int* Ak_ri, const double* Ak_v,
                const int* A0_cp, const int* A0_ri, const double* A0_v,
                const int* M_cp, const int* M_ri, const double* M_v,
                double* res2, double* a02) {
    double* col = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    int* touched = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int* mark = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) mark[i] = -1;
    double s = 0.0, a = 0.0;
    for (int j = 0; j < n; ++j) {
        int nt = 0;
        for (int e = M_cp[j]; e < M_cp[j + 1]; ++e) {
            int l = M_ri[e];
            double mlj = M_v[e];
            for (int f = Ak_cp[l]; f < Ak_cp[l + 1]; ++f) {
                int i = Ak_ri[f];
                if (mark[i] != j) { mark[i] = j; touched[nt++] = i; col[i] = 0.0; }
                col[i] += Ak_v[f] * mlj;
            }
        }
        for (int e = A0_cp[j]; e < A0_cp[j + 1]; ++e) {
            int i = A0_ri[e];
            if (mark[i] != j) { mark[i] = j; touched[nt++] = i; col[i] = 0.0; }
            col[i] -= A0_v[e];
            a += A0_v[e] * A0_v[e];
        }
        for (int t = 0; t < nt; ++t) { s += col[touched[t]] * col[touched[t]]; }
    }
    free(col); free(touched); free(mark);
    *res2 = s;
    if (a02) *a02 = a;
    return OR_OK;
}

/* y = M x for M in CSC (definition of the matrix-vector product). */
int or_apply(int n, const int* M_cp, const int* M_ri, const double* M_v,
             const double* x, double* y) {
    for (int i = 0; i < n; ++i) y[i] = 0.0;
    for (int j = 0; j < n; ++j)
        for (int e = M_cp[j]; e < M_cp[j + 1]; ++e) y[M_ri[e]] += M_v[e] * x[j];
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Gradient of L = sum_j ( ||A_j m_j - b_j||^2 + out_j ), scaled by dL, for  */
/* the soft-weighted map (w_S == NULL or all ones gives the plain map).      */
/* With K = A^T A + P and r = A m - b:                                       */
/*   lambda = K^{-1} (2 A^T r)                                               */
/*   dL/dA  = 2 r m^T - r lambda^T - (A lambda) m^T   (stored entries only)  */
/*   dL/db  = -2 r + A lambda,  dL/dA0 outside I_j = 2 A0(i,j)               */
/*   dL/dw_l = mu lambda_l m_l / w_l^2        (p_l = mu (1/w_l - 1))         */
/* Derivation: differentiate the normal equations K m = A^T b.               */
/* Outputs are overwritten; gw may be NULL.                                  */
/* ------------------------------------------------------------------------ */
int or_backward(int n,
                const int* Ak_cp, const int* Ak_ri, const double* Ak_v,
                const int* A0_cp, const int* A0_ri, const double* A0_v,
                const int* S_cp, const int* S_ri,
                const double* w_S, double mu, double dL,
                double* gAk, double* gA0, double* gw, double* loss, int* bad_col) {
    int nnzA = Ak_cp[n];
    /* per-column contribution slots to the Ak values: for column j, the
     * entries of Ak(:, l) for l in J_j, in that order */
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    off[0] = 0;
    for (int j = 0; j < n; ++j) {
        int64_t s = 0;
        for (int e = S_cp[j]; e < S_cp[j + 1]; ++e) s += Ak_cp[S_ri[e] + 1] - Ak_cp[S_ri[e]];
        off[j + 1] = off[j] + s;
    }
    double* contrib = (double*)malloc(sizeof(double) * (size_t)(off[n] > 0 ? off[n] : 1));
    double* rho = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int status = OR_OK, first_bad = n;
#pragma omp parallel
    {
        colws w;
        ws_init(&w, n);
        int my_status = OR_OK, my_bad = n;
#pragma omp for schedule(dynamic, 64)
        for (int j = 0; j < n; ++j) {
            const int* J = S_ri + S_cp[j];
            int nJ = S_cp[j + 1] - S_cp[j];
            int nI = 0;
            double r2 = 0.0;
            const double* wj = w_S ? w_S + S_cp[j] : NULL;
            int st = solve_column(&w, j, J, nJ, Ak_cp, Ak_ri, Ak_v, A0_cp, A0_ri, A0_v,
                                  wj, mu, &nI, &r2, NULL);
            if (st != OR_OK) {
                if (j < my_bad) { my_bad = j; my_status = st; }
                continue;
            }
            rho[j] = r2;
            int ld = wj ? nI + nJ : nI;
            /* solve_column leaves r = b - A m; the formulas use r = A m - b */
            for (int i = 0; i < nI; ++i) w.r[i] = -w.r[i];
            /* g = 2 A^T r, lambda = R^{-1} R^{-T} g with R^T R = K */
            for (int c = 0; c < nJ; ++c) {
                double s = 0.0;
                for (int i = 0; i < nI; ++i) s += w.A0[(size_t)c * ld + i] * w.r[i];
                w.y[c] = 2.0 * s;
            }
            forward_solve_t(w.A, ld, nJ, w.y, w.lam);
            memcpy(w.y, w.lam, sizeof(double) * (size_t)nJ);
            back_solve(w.A, ld, nJ, w.y, w.lam);
            for (int i = 0; i < nI; ++i) {
                double s = 0.0;
                for (int c = 0; c < nJ; ++c) s += w.A0[(size_t)c * ld + i] * w.lam[c];
                w.Alam[i] = s;
            }
            int64_t o = off[j];
            for (int c = 0; c < nJ; ++c) {
                int l = J[c];
                for (int e = Ak_cp[l]; e < Ak_cp[l + 1]; ++e) {
                    int p = w.pos[Ak_ri[e]];
                    contrib[o++] = dL * (2.0 * w.r[p] * w.m[c] - w.r[p] * w.lam[c]
                                         - w.Alam[p] * w.m[c]);
                }
            }
            for (int e = A0_cp[j]; e < A0_cp[j + 1]; ++e) {
                int i = A0_ri[e];
                if (w.mark[i] == j) {
                    int p = w.pos[i];
                    gA0[e] = dL * (-2.0 * w.r[p] + w.Alam[p]);
                } else {
                    gA0[e] = dL * 2.0 * A0_v[e];
                }
            }
            if (gw) {
                for (int c = 0; c < nJ; ++c) {
                    double wl = wj ? wj[c] : 1.0;
                    gw[S_cp[j] + c] = dL * mu * w.lam[c] * w.m[c] / (wl * wl);
                }
            }
        }
#pragma omp critical
        {
            if (my_bad < first_bad) { first_bad = my_bad; status = my_status; }
        }
        ws_free(&w);
    }
    if (status == OR_OK) {
        /* deterministic accumulation in column order */
        for (int e = 0; e < nnzA; ++e) gAk[e] = 0.0;
        for (int j = 0; j < n; ++j) {
            int64_t o = off[j];
            for (int e = S_cp[j]; e < S_cp[j + 1]; ++e) {
                int l = S_ri[e];
                for (int f = Ak_cp[l]; f < Ak_cp[l + 1]; ++f) gAk[f] += contrib[o++];
            }
        }
        if (loss) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += rho[j];
            *loss = s;
        }
    }
    if (bad_col) *bad_col = status == OR_OK ? -1 : first_bad;
    free(off); free(contrib); free(rho);
    return status;
}
