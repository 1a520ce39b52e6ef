"""FP64 CPU oracle for the sparse approximate map (SAM) construction.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library never calls it and shares no code with it; the two meet only through
the seeded inputs of ``pde_inputs``.

Thin ctypes marshalling over ``sam_oracle.c`` (plain C, FP64, OpenMP over
columns).  Each wrapper names the passage of the paper it follows:

* ``sparsify``   -- Section 4, the global / column / lfil rules.
* ``pattern``    -- Section 3, level neighbours: S((I + B)^p) with B = S(A~).
* ``row_sets``   -- Section 2, the rows touched by the columns J_j.
* ``sam_build``  -- Section 2, eq. (approx_map) split into column problems.
* ``residual``   -- Section 2, eq. (res), Frobenius norm used in Section 5.
* ``frobenius_sq`` -- Section 2, eq. (res): ||R||_F^2 as the sum of the
                    column residuals, correctly rounded (math.fsum).
* ``apply``      -- y = M x (definition).
* ``backward``   -- exact gradient of ||A_k M - A_0||_F^2 (not in the paper;
                    derived from the normal equations, see sam_oracle.c).
* ``candidate_weights``, ``select_topk`` -- the adaptive-pattern step the
                    paper leaves as future work (end of Section 2): weights
                    over a candidate pattern, and per column the base entries
                    plus the k candidates of smallest gradient (definitions).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sam_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KIND = {"none": 0, "global": 1, "column": 2, "lfil": 3}
STATUS = {0: "ok", 1: "bad argument", 5: "rank deficient", 6: "non-finite"}


_LIB_ASAN = os.path.join(_HERE, "liboracle_asan.so")


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile sam_oracle.c with gcc into liboracle.so (in place); with
    sanitize=True into liboracle_asan.so with AddressSanitizer and
    UndefinedBehaviorSanitizer (any report aborts)."""
    out = _LIB_ASAN if sanitize else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
        subprocess.check_call(["gcc"] + flags + ["-std=c11", "-fopenmp", "-fPIC", "-shared",
                                                 "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        # SAM_ORACLE_LIB: another build of the same source (the sanitizer test)
        _lib = ctypes.CDLL(os.environ.get("SAM_ORACLE_LIB") or build())
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        _lib.or_sparsify.argtypes = [I, P, P, P, I, D, I, D, I, P, P]
        _lib.or_expand.argtypes = [I, P, P, P, P, P, P]
        _lib.or_row_sets.argtypes = [I, P, P, P, P, P, P]
        _lib.or_sam_build.argtypes = [I, P, P, P, P, P, P, P, P, P, D, P, I, P, P, P]
        _lib.or_residual.argtypes = [I, P, P, P, P, P, P, P, P, P, P, P]
        _lib.or_apply.argtypes = [I, P, P, P, P, P]
        _lib.or_backward.argtypes = [I, P, P, P, P, P, P, P, P, P, D, D, P, P, P, P, P]
        _lib.or_set_num_threads.argtypes = [I]
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(t: int) -> None:
    lib().or_set_num_threads(int(t))


@dataclass
class Pattern:
    n: int
    colptr: np.ndarray
    rowind: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])


class OracleError(RuntimeError):
    def __init__(self, status, col):
        super().__init__(f"oracle: {STATUS.get(status, status)} at column {col}")
        self.status = status
        self.col = col


def sparsify(A, kind="none", thresh=0.0, global_scale=-1, tau=0.0, lfil=0) -> Pattern:
    """Section 4: B = S(A~) with the diagonal always kept."""
    cp, ri, v = _i32(A.colptr), _i32(A.rowind), _f64(A.val)
    out_cp = np.zeros(A.n + 1, dtype=np.int32)
    out_ri = np.zeros(A.nnz + A.n, dtype=np.int32)
    st = lib().or_sparsify(A.n, _p(cp), _p(ri), _p(v), KIND[kind], float(thresh),
                           int(global_scale), float(tau), int(lfil), _p(out_cp), _p(out_ri))
    if st:
        raise OracleError(st, -1)
    return Pattern(A.n, out_cp, out_ri[:out_cp[-1]].copy())


def expand(P: Pattern, Q) -> Pattern:
    """Column j of S(Q P): union over l in P(:,j) of rows(Q(:,l))."""
    pcp, pri = _i32(P.colptr), _i32(P.rowind)
    qcp, qri = _i32(Q.colptr), _i32(Q.rowind)
    out_cp = np.zeros(P.n + 1, dtype=np.int32)
    lib().or_expand(P.n, _p(pcp), _p(pri), _p(qcp), _p(qri), _p(out_cp), None)
    out_ri = np.zeros(max(int(out_cp[-1]), 1), dtype=np.int32)
    lib().or_expand(P.n, _p(pcp), _p(pri), _p(qcp), _p(qri), _p(out_cp), _p(out_ri))
    return Pattern(P.n, out_cp, out_ri[:out_cp[-1]].copy())


def pattern(A, power=1, kind="none", **kw) -> Pattern:
    """Section 3/4: S((I + B)^power), B = S(A~) including the diagonal."""
    if power < 1:
        raise ValueError("power must be >= 1")
    B = sparsify(A, kind, **kw)
    S = B
    for _ in range(power - 1):
        S = expand(S, B)
    return S


def row_sets(S: Pattern, A) -> Pattern:
    """I_j = sorted union of rows(A(:, l)) over l in S(:, j)."""
    return expand(S, A)


def sam_build(Ak, A0, S: Pattern, cols=None, weights=None, mu=0.0, raise_on_error=True):
    """Section 2: M values on S (FP64) and per-column squared residuals.

    Returns (M_val, rho, status, bad_col).  With ``cols`` only those columns
    are solved and the rest of M_val / rho stay NaN."""
    n = Ak.n
    M = np.full(S.nnz, np.nan)
    rho = np.full(n, np.nan)
    bad = np.array([-1], dtype=np.int32)
    cl = None if cols is None else _i32(cols)
    w = None if weights is None else _f64(weights)
    st = lib().or_sam_build(n, _p(_i32(Ak.colptr)), _p(_i32(Ak.rowind)), _p(_f64(Ak.val)),
                            _p(_i32(A0.colptr)), _p(_i32(A0.rowind)), _p(_f64(A0.val)),
                            _p(_i32(S.colptr)), _p(_i32(S.rowind)), _p(w), float(mu),
                            _p(cl), 0 if cl is None else int(cl.size), _p(M), _p(rho), _p(bad))
    if st and raise_on_error:
        raise OracleError(st, int(bad[0]))
    return M, rho, int(st), int(bad[0])


def frobenius_sq(rho) -> float:
    """||R||_F^2 = sum_j rho_j (Section 2, eq. res: the squared Frobenius
    norm is the sum of the squared column norms).  math.fsum returns the
    correctly rounded sum, so no summation order is implied."""
    return math.fsum(float(x) for x in np.asarray(rho, dtype=np.float64))


def residual(Ak, A0, S: Pattern, M_val):
    """Section 2 eq. (res): returns (||A_k M - A_0||_F^2, ||A_0||_F^2)."""
    r2 = np.zeros(1)
    a2 = np.zeros(1)
    lib().or_residual(Ak.n, _p(_i32(Ak.colptr)), _p(_i32(Ak.rowind)), _p(_f64(Ak.val)),
                      _p(_i32(A0.colptr)), _p(_i32(A0.rowind)), _p(_f64(A0.val)),
                      _p(_i32(S.colptr)), _p(_i32(S.rowind)), _p(_f64(M_val)), _p(r2), _p(a2))
    return float(r2[0]), float(a2[0])


def apply(S: Pattern, M_val, x):
    """y = M x."""
    y = np.zeros(S.n)
    lib().or_apply(S.n, _p(_i32(S.colptr)), _p(_i32(S.rowind)), _p(_f64(M_val)),
                   _p(_f64(x)), _p(y))
    return y


def backward(Ak, A0, S: Pattern, weights=None, mu=0.0, dL=1.0):
    """Gradient of L = ||A_k M - A_0||_F^2 (M the soft-weighted map) with
    respect to the stored values of A_k and A_0 and the weights on S.
    Returns (gAk, gA0, gw, L)."""
    gAk = np.zeros(Ak.nnz)
    gA0 = np.zeros(A0.nnz)
    gw = np.zeros(S.nnz)
    loss = np.zeros(1)
    bad = np.array([-1], dtype=np.int32)
    w = None if weights is None else _f64(weights)
    st = lib().or_backward(Ak.n, _p(_i32(Ak.colptr)), _p(_i32(Ak.rowind)), _p(_f64(Ak.val)),
                           _p(_i32(A0.colptr)), _p(_i32(A0.rowind)), _p(_f64(A0.val)),
                           _p(_i32(S.colptr)), _p(_i32(S.rowind)), _p(w), float(mu), float(dL),
                           _p(gAk), _p(gA0), _p(gw), _p(loss), _p(bad))
    if st:
        raise OracleError(st, int(bad[0]))
    return gAk, gA0, gw, float(loss[0])


def candidate_weights(S: Pattern, B: Pattern, w_base=1.0, w_cand=0.1) -> np.ndarray:
    """w[e] = w_base when entry e of S (row, column) is also an entry of B,
    w_cand otherwise (plain set membership per column)."""
    w = np.full(S.nnz, float(w_cand))
    for j in range(S.n):
        base = set(int(r) for r in B.rowind[B.colptr[j]:B.colptr[j + 1]])
        for e in range(S.colptr[j], S.colptr[j + 1]):
            if int(S.rowind[e]) in base:
                w[e] = float(w_base)
    return w


def select_topk(S: Pattern, w, grad, k: int) -> Pattern:
    """Per column j: the entries of S(:, j) with w >= 1, and the k entries
    with w < 1 ordered first by (grad ascending, NaN as +inf; row ascending);
    kept in S's row order.  Vectorised: candidates sorted by (column, grad,
    row); the rank of a candidate is its position within its column."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    g = np.where(np.isnan(g), np.inf, g)
    col = np.repeat(np.arange(S.n), np.diff(S.colptr))
    row = np.asarray(S.rowind, dtype=np.int64)
    keep = w >= 1.0
    cand = np.flatnonzero(~keep)
    order = cand[np.lexsort((row[cand], g[cand], col[cand]))]
    ccol = col[order]
    first = np.searchsorted(ccol, ccol, side="left")
    rank = np.arange(order.size) - first
    keep[order[rank < k]] = True
    counts = np.bincount(col[keep], minlength=S.n)
    colptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    return Pattern(S.n, colptr, np.asarray(S.rowind)[keep].astype(np.int32))
