"""Seeded synthetic PDE matrix sequences in CSC form.

These generators stand in for the paper's application matrices (the CD2D
Newton-Jacobian sequence of Section 5.1 and the NWP sequence of Section 5.2
are not available): 2D/3D finite-difference stencils with variable
coefficients, a nonsymmetric upwind convection-diffusion operator and a
ragged 9-point stencil with dropped couplings.  Every matrix is square,
FP64, int32-indexed, with row indices sorted ascending inside each column
and no duplicates.

This module holds no part of the sparse-approximate-map arithmetic: it only
builds inputs.  It is the one module that both the CPU oracle's tests and
the GPU path's tests/bench import.

Grid convention: m nodes per axis, x_i = (i+1) h, h = 1/(m+1), homogeneous
Dirichlet boundary; node index p = ix + m*iy (+ m*m*iz); the common 1/h^2
factor is dropped (the map and the relative residual are invariant under a
common scalar).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSC", "coo_to_csc", "diffusion_2d", "diffusion_3d", "convdiff_3d",
    "laplacian_2d", "config1", "config2", "config3", "config4", "config5",
    "candidate_weights", "splitmix_uniform", "random_on_pattern", "penalty_scale",
]


@dataclass
class CSC:
    """Square sparse matrix in compressed-sparse-column form."""
    n: int
    colptr: np.ndarray  # int32, n+1
    rowind: np.ndarray  # int32, nnz, ascending within each column
    val: np.ndarray     # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        cols = np.repeat(np.arange(self.n), np.diff(self.colptr))
        d[self.rowind, cols] = self.val
        return d

    def with_values(self, val: np.ndarray) -> "CSC":
        return CSC(self.n, self.colptr, self.rowind, np.ascontiguousarray(val, dtype=np.float64))


def coo_to_csc(n: int, rows, cols, vals) -> CSC:
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((rows, cols))
    rows, cols, vals = rows[order], cols[order], vals[order]
    key = cols * n + rows
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate entries")
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr)
    return CSC(n, colptr.astype(np.int32), rows.astype(np.int32), vals)


def dense_to_csc(d: np.ndarray) -> CSC:
    d = np.asarray(d, dtype=np.float64)
    r, c = np.nonzero(d)
    return coo_to_csc(d.shape[0], r, c, d[r, c])


# ---------------------------------------------------------------------------
# stencil assembly
# ---------------------------------------------------------------------------

def _axis_faces(coef: np.ndarray, axis: int):
    """Interior face coefficients (mean of the two node values) along `axis`
    and the two boundary-face coefficient arrays (node value)."""
    sl_lo = [slice(None)] * coef.ndim
    sl_hi = [slice(None)] * coef.ndim
    sl_lo[axis] = slice(0, -1)
    sl_hi[axis] = slice(1, None)
    interior = 0.5 * (coef[tuple(sl_lo)] + coef[tuple(sl_hi)])
    return interior


def _diffusion(coef: np.ndarray) -> tuple[list, list, list, np.ndarray]:
    """-div(coef grad u) on an m^d node grid with face coefficient = mean of
    node values and boundary faces = node value.  Arrays are indexed
    [iz, iy, ix] (C order) so that the flat index is ix + m*iy + m*m*iz."""
    shape = coef.shape
    n = coef.size
    idx = np.arange(n).reshape(shape)
    diag = np.zeros(shape)
    rows, cols, vals = [], [], []
    for axis in range(coef.ndim):
        f = _axis_faces(coef, axis)
        sl_lo = [slice(None)] * coef.ndim
        sl_hi = [slice(None)] * coef.ndim
        sl_lo[axis] = slice(0, -1)
        sl_hi[axis] = slice(1, None)
        lo = idx[tuple(sl_lo)].ravel()
        hi = idx[tuple(sl_hi)].ravel()
        fv = f.ravel()
        rows += [lo, hi]
        cols += [hi, lo]
        vals += [-fv, -fv]
        diag[tuple(sl_lo)] += f
        diag[tuple(sl_hi)] += f
        # boundary faces at both ends of this axis
        first = [slice(None)] * coef.ndim
        last = [slice(None)] * coef.ndim
        first[axis] = 0
        last[axis] = shape[axis] - 1
        diag[tuple(first)] += coef[tuple(first)]
        diag[tuple(last)] += coef[tuple(last)]
    return rows, cols, vals, diag


def diffusion_2d(a: np.ndarray) -> CSC:
    """5-point -div(a grad u) for node coefficients a[iy, ix]."""
    rows, cols, vals, diag = _diffusion(np.asarray(a, dtype=np.float64))
    n = a.size
    rows.append(np.arange(n)); cols.append(np.arange(n)); vals.append(diag.ravel())
    return coo_to_csc(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def diffusion_3d(k: np.ndarray) -> CSC:
    """7-point -div(k grad u) for node coefficients k[iz, iy, ix]."""
    return diffusion_2d(k)  # the assembly is dimension-generic


def convdiff_3d(D: np.ndarray, vel, h: float) -> CSC:
    """7-point -div(D grad u) + v.grad u with first-order upwinding
    (v components >= 0), scaled by h^2, on D[iz, iy, ix]."""
    D = np.asarray(D, dtype=np.float64)
    rows, cols, vals, diag = _diffusion(D)
    shape = D.shape
    n = D.size
    idx = np.arange(n).reshape(shape)
    # axis order in the array is (z, y, x); vel is (vx, vy, vz)
    v_axis = {2: vel[0], 1: vel[1], 0: vel[2]}
    for axis, v in v_axis.items():
        if v < 0:
            raise ValueError("upwind assembly expects non-negative velocity")
        diag += h * v
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[axis] = slice(0, -1)
        sl_hi[axis] = slice(1, None)
        lo = idx[tuple(sl_lo)].ravel()   # upstream neighbour
        hi = idx[tuple(sl_hi)].ravel()   # node whose equation uses it
        rows.append(hi); cols.append(lo); vals.append(np.full(lo.size, -h * v))
    rows.append(np.arange(n)); cols.append(np.arange(n)); vals.append(diag.ravel())
    r = np.concatenate(rows); c = np.concatenate(cols); v = np.concatenate(vals)
    # merge the diffusion and convection contributions to the same entry
    key = c.astype(np.int64) * n + r
    uk, inv = np.unique(key, return_inverse=True)
    vs = np.zeros(uk.size)
    np.add.at(vs, inv, v)
    return coo_to_csc(n, uk % n, uk // n, vs)


def laplacian_2d(m: int) -> CSC:
    """Constant-coefficient 5-point Laplacian (4 on the diagonal, -1 off)."""
    return diffusion_2d(np.ones((m, m)))


def _grid_xy(m: int):
    h = 1.0 / (m + 1)
    x = (np.arange(m) + 1) * h
    X, Y = np.meshgrid(x, x, indexing="xy")  # X[iy, ix] = x_ix
    return X, Y, h


# ---------------------------------------------------------------------------
# workload configurations
# ---------------------------------------------------------------------------

def config1():
    """2D 5-point variable-coefficient diffusion, 32x32 (n=1024).
    A_0 from a0 = 1 + 0.5 sin(2 pi x) sin(2 pi y); A_1 from a0 * (1 + 0.1 N(0,1))
    per node (seed 1).  Returns (A0, [A1])."""
    m = 32
    X, Y, _ = _grid_xy(m)
    a0 = 1.0 + 0.5 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    rng = np.random.default_rng(1)
    a1 = a0 * (1.0 + 0.1 * rng.standard_normal((m, m)))
    return diffusion_2d(a0), [diffusion_2d(a1)]


def config2(m: int = 512, nmat: int = 8):
    """2D 5-point diffusion sequence, m x m grid, matrices k=0..nmat-1 with
    a_k = 1 + 0.5 sin(2 pi x + t_k) cos(2 pi y) + 0.05 N(0,1), t_k = 0.1 k,
    fresh noise per k from seed 2+k.  Returns (A0, [A1..A_{nmat-1}])."""
    X, Y, _ = _grid_xy(m)
    mats = []
    for k in range(nmat):
        rng = np.random.default_rng(2 + k)
        a = 1.0 + 0.5 * np.sin(2 * np.pi * X + 0.1 * k) * np.cos(2 * np.pi * Y) \
            + 0.05 * rng.standard_normal((m, m))
        mats.append(diffusion_2d(a))
    return mats[0], mats[1:]


def config3(m: int = 64, pe=(1, 1, 10, 10, 100, 100)):
    """3D 7-point upwind convection-diffusion, m^3 grid, v = (1, .5, .25) Pe_k.
    D = 1 for even k, D = 1 + 0.05 N(0,1) per node for odd k (seed 3).
    Returns (A0, [A1..])."""
    h = 1.0 / (m + 1)
    rng = np.random.default_rng(3)
    mats = []
    for k, p in enumerate(pe):
        if k % 2 == 0:
            D = np.ones((m, m, m))
        else:
            D = 1.0 + 0.05 * rng.standard_normal((m, m, m))
        mats.append(convdiff_3d(D, (1.0 * p, 0.5 * p, 0.25 * p), h))
    return mats[0], mats[1:]


def _ninept_edges(m: int):
    idx = np.arange(m * m).reshape(m, m)  # [iy, ix]
    e = [
        (idx[:, :-1].ravel(), idx[:, 1:].ravel()),        # east
        (idx[:-1, :].ravel(), idx[1:, :].ravel()),        # north
        (idx[:-1, :-1].ravel(), idx[1:, 1:].ravel()),     # north-east
        (idx[:-1, 1:].ravel(), idx[1:, :-1].ravel()),     # north-west
    ]
    u = np.concatenate([a for a, _ in e])
    v = np.concatenate([b for _, b in e])
    return u, v


def config4(m: int = 1024, nmat: int = 16, drop: float = 0.15):
    """2D 9-point stencil on an m x m grid with lognormal(0,1) undirected
    couplings c, each dropped with probability `drop` (at least two kept per
    node), a_ij = -c, a_ii = 1.01 (sum of kept incident c + boundary c).
    Values evolve by c <- c (1 + 0.01 N(0,1)) per step (seed 4).
    Returns (A0, [A1..A_{nmat-1}])."""
    n = m * m
    rng = np.random.default_rng(4)
    u, v = _ninept_edges(m)
    ne = u.size
    c = rng.lognormal(0.0, 1.0, ne)
    keep = rng.random(ne) >= drop
    # outside-the-grid couplings: 8 neighbour slots per node
    iy, ix = np.divmod(np.arange(n), m)
    outside = np.zeros(n)
    bc = rng.lognormal(0.0, 1.0, (n, 8))
    offs = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)]
    out_mask = np.zeros((n, 8), dtype=bool)
    for s, (dx, dy) in enumerate(offs):
        jx, jy = ix + dx, iy + dy
        out_mask[:, s] = (jx < 0) | (jx >= m) | (jy < 0) | (jy >= m)
    # at least two kept couplings per node: restore dropped incident edges
    for _ in range(16):
        deg = np.bincount(u[keep], minlength=n) + np.bincount(v[keep], minlength=n)
        bad = np.nonzero(deg < 2)[0]
        if bad.size == 0:
            break
        badset = np.zeros(n, dtype=bool)
        badset[bad] = True
        cand = np.nonzero(~keep & (badset[u] | badset[v]))[0]
        # restore the first dropped incident edge of every deficient node
        first = {}
        for e in cand:
            for node in (u[e], v[e]):
                if badset[node] and node not in first:
                    first[node] = e
        keep[list(set(first.values()))] = True
    ku, kv = u[keep], v[keep]
    kc = c[keep]
    bvals = np.where(out_mask, bc, 0.0)

    def assemble(kc, bvals):
        diag = np.bincount(ku, weights=kc, minlength=n) + np.bincount(kv, weights=kc, minlength=n)
        diag = 1.01 * (diag + bvals.sum(axis=1))
        rows = np.concatenate([ku, kv, np.arange(n)])
        cols = np.concatenate([kv, ku, np.arange(n)])
        vals = np.concatenate([-kc, -kc, diag])
        return coo_to_csc(n, rows, cols, vals)

    mats = [assemble(kc, bvals)]
    for _ in range(1, nmat):
        kc = kc * (1.0 + 0.01 * rng.standard_normal(kc.size))
        bvals = bvals * (1.0 + 0.01 * rng.standard_normal(bvals.shape))
        mats.append(assemble(kc, bvals))
    return mats[0], mats[1:]


def config5(m: int = 48):
    """3D 7-point diffusion, m^3 grid, node coefficient kappa0 ~ lognormal(0, .5)
    (seed 5); A_1 from kappa0 * exp(0.1 N(0,1)).  Returns (A0, A1)."""
    rng = np.random.default_rng(5)
    k0 = rng.lognormal(0.0, 0.5, (m, m, m))
    k1 = k0 * np.exp(0.1 * rng.standard_normal((m, m, m)))
    return diffusion_3d(k0), diffusion_3d(k1)


# ---------------------------------------------------------------------------
# counter-based random values (order independent)
# ---------------------------------------------------------------------------

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix_uniform(seed: int, key: np.ndarray) -> np.ndarray:
    """Uniform [0,1) doubles from the SplitMix64 finaliser (Steele, Lea and
    Flood, OOPSLA 2014) applied to seed*golden + key; depends only on the key,
    so any side can regenerate the value of one entry on its own."""
    with np.errstate(over="ignore"):
        z = (np.uint64(seed) * np.uint64(0x9E3779B97F4A7C15)
             + np.asarray(key, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def candidate_weights(n: int, S_colptr, S_rowind, A: CSC, seed: int = 5,
                      lo: float = 0.1, hi: float = 0.99) -> np.ndarray:
    """Soft weights aligned with the entries of a pattern S: 1.0 where (i, j)
    is a stored entry of A or on the diagonal, U(lo, hi) elsewhere, drawn from
    the counter-based generator keyed by i*n + j."""
    S_colptr = np.asarray(S_colptr, dtype=np.int64)
    S_rowind = np.asarray(S_rowind, dtype=np.int64)
    scol = np.repeat(np.arange(n, dtype=np.int64), np.diff(S_colptr))
    key = S_rowind * n + scol
    acol = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.colptr.astype(np.int64)))
    akey = np.sort(A.rowind.astype(np.int64) * n + acol)
    pos = np.searchsorted(akey, key)
    pos = np.minimum(pos, akey.size - 1)
    fixed = (akey[pos] == key) | (S_rowind == scol)
    u = splitmix_uniform(seed, key)
    w = lo + (hi - lo) * u
    w[fixed] = 1.0
    return w


def random_on_pattern(pattern: CSC, rng: np.random.Generator, diag_shift: float = 0.0) -> CSC:
    """Same structure, values N(0,1), plus diag_shift on stored diagonal entries."""
    val = rng.standard_normal(pattern.nnz)
    if diag_shift:
        cols = np.repeat(np.arange(pattern.n), np.diff(pattern.colptr))
        val = val + diag_shift * (pattern.rowind == cols)
    return pattern.with_values(val)


def penalty_scale(A: CSC) -> float:
    """Mean squared column norm of A: the fixed scale mu of the soft-weight
    penalty, computed once from the inputs and passed to both sides."""
    cols = np.repeat(np.arange(A.n), np.diff(A.colptr))
    return float(np.bincount(cols, weights=np.asarray(A.val) ** 2, minlength=A.n).mean())
