"""The map as a preconditioner update inside GMRES: the use the SAM is built
for (Section 1; the paper defers the iteration counts to earlier work and
expects smaller ||R_k||_F to mean fewer iterations, Section 5).

For the system A_k x = b and a preconditioner P_0 of the target A_0 (here
Jacobi, P_0 = diag(A_0)^-1), the updated right preconditioner is N_k P_0:
A_k N_k P_0 ~ A_0 P_0.  ``gmres`` is restarted GMRES(m) with modified
Gram-Schmidt and Givens rotations, right-preconditioned.  The sparse products
(A_k x and N_k y) are library calls (``sam_apply`` on row views built by
``sam_apply_prepare``); the vector arithmetic of the Krylov driver (dot
products, updates, the small Hessenberg system) uses torch and the host.
"""
from __future__ import annotations

import math

import torch

from .sam import Context, DeviceCSC


class SparseOp:
    """y = A x for a CSC matrix held on the device (values double or float);
    the values are put in the row view's order once (sam_apply_permute)."""

    def __init__(self, ctx: Context, n: int, colptr, rowind, val, prec="f64"):
        self.ctx, self.prec = ctx, prec
        self.T = ctx.apply_prepare(n, colptr, rowind)
        self.val = ctx.apply_permute(self.T, val, prec)

    def __call__(self, x):
        return self.ctx.apply(self.T, self.val, x, self.prec, permuted=True)


def jacobi_diag(A: DeviceCSC) -> torch.Tensor:
    """diag(A) from the CSC arrays (entries with row == column)."""
    n = A.n
    cols = torch.repeat_interleave(torch.arange(n, device=A.colptr.device),
                                   (A.colptr[1:] - A.colptr[:-1]).long())
    d = torch.zeros(n, dtype=torch.float64, device=A.colptr.device)
    on = A.rowind.long() == cols
    d[cols[on]] = A.val[on]
    return d


def gmres(apply_A, apply_M, b, tol=1e-8, restart=50, maxiter=2000):
    """Right-preconditioned restarted GMRES: solve A M u = b, x = M u.
    Returns (x, iterations, relative residual history)."""
    n = b.numel()
    x = torch.zeros_like(b)
    bnorm = float(torch.linalg.vector_norm(b))
    hist = []
    its = 0
    while its < maxiter:
        r = b - apply_A(x)
        beta = float(torch.linalg.vector_norm(r))
        hist.append(beta / bnorm)
        if beta <= tol * bnorm:
            break
        V = [r / beta]
        Z = []
        H = [[0.0] * restart for _ in range(restart + 1)]
        cs, sn = [0.0] * restart, [0.0] * restart
        g = [beta] + [0.0] * restart
        k_used = 0
        for k in range(restart):
            z = apply_M(V[k])
            Z.append(z)
            w = apply_A(z)
            for i in range(k + 1):                       # modified Gram-Schmidt
                H[i][k] = float(torch.dot(w, V[i]))
                w = w - H[i][k] * V[i]
            hnorm = float(torch.linalg.vector_norm(w))
            H[k + 1][k] = hnorm
            for i in range(k):                           # earlier rotations
                t = cs[i] * H[i][k] + sn[i] * H[i + 1][k]
                H[i + 1][k] = -sn[i] * H[i][k] + cs[i] * H[i + 1][k]
                H[i][k] = t
            den = math.hypot(H[k][k], H[k + 1][k])
            cs[k], sn[k] = (1.0, 0.0) if den == 0.0 else (H[k][k] / den, H[k + 1][k] / den)
            H[k][k] = cs[k] * H[k][k] + sn[k] * H[k + 1][k]
            H[k + 1][k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            its += 1
            k_used = k + 1
            hist.append(abs(g[k + 1]) / bnorm)
            if abs(g[k + 1]) <= tol * bnorm or its >= maxiter or hnorm == 0.0:
                break
            V.append(w / hnorm)
        # y = H^{-1} g (upper triangular k_used x k_used)
        y = [0.0] * k_used
        for i in range(k_used - 1, -1, -1):
            s = g[i] - sum(H[i][j] * y[j] for j in range(i + 1, k_used))
            y[i] = s / H[i][i]
        for i in range(k_used):
            x = x + y[i] * Z[i]
        if abs(g[k_used]) <= tol * bnorm:
            r = b - apply_A(x)
            hist.append(float(torch.linalg.vector_norm(r)) / bnorm)
            break
    return x, its, hist


def solve_with_map(ctx: Context, Ak: DeviceCSC, A0: DeviceCSC, M_colptr, M_rowind, M_val, b,
                   prec="f32", tol=1e-8, restart=50, maxiter=2000):
    """GMRES on A_k x = b with the right preconditioner N_k diag(A_0)^-1
    (M_val None: the frozen preconditioner diag(A_0)^-1 alone)."""
    A = SparseOp(ctx, Ak.n, Ak.colptr, Ak.rowind, Ak.val, "f64")
    dinv = 1.0 / jacobi_diag(A0)
    if M_val is None:
        apply_M = lambda v: dinv * v                       # noqa: E731
    else:
        N = SparseOp(ctx, Ak.n, M_colptr, M_rowind, M_val, prec)
        apply_M = lambda v: N(dinv * v)                    # noqa: E731
    return gmres(A, apply_M, b, tol, restart, maxiter)


def main():
    """GMRES iterations per map of a sequence for several maps.

        python -m paper_2406_17656_amd.krylov --grid 128 --maps 8
    """
    import argparse
    import numpy as np
    import pde_inputs as P
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--maps", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-8)
    args = ap.parse_args()
    A0h, Ash = P.config2(m=args.grid, nmat=args.maps)
    ctx = Context(0)
    A0 = DeviceCSC.from_host(A0h)
    b = torch.as_tensor(np.random.default_rng(0).standard_normal(A0h.n)).cuda()
    print("| Map | frozen P_0 its | S(A_0) its (rel. res.) | level 1 its (rel. res.) | level 2 its (rel. res.) |")
    print("|---|---|---|---|---|")
    S0 = ctx.pattern(A0, 1)
    for k, Ah in enumerate(Ash):
        Ak = DeviceCSC.from_host(Ah)
        cells = []
        _, its, _ = solve_with_map(ctx, Ak, A0, None, None, None, b, tol=args.tol, restart=50, maxiter=5000)
        cells.append(str(its))
        for cp, ri in (S0, ctx.pattern(Ak, 1), ctx.pattern(Ak, 2)):
            M, _, _ = ctx.build(Ak, A0, cp, ri, "f32", want_cols=False)
            r2, a02 = ctx.residual(Ak, A0, cp, ri, M, "f32")
            _, its, _ = solve_with_map(ctx, Ak, A0, cp, ri, M, b, "f32", args.tol, 50, 5000)
            cells.append(f"{its} ({math.sqrt(float(r2.cpu()[0]) / float(a02.cpu()[0])):.2e})")
        print(f"| N_{k + 1} | " + " | ".join(cells) + " |")
    ctx.close()


if __name__ == "__main__":
    main()
