"""Adjoint-guided adaptive patterns: the paper's future-work direction
(adaptive sparsity patterns computed in parallel, end of Section 2; more
refined sparsification, Section 6), built from the soft-weighted map and its
adjoint.

For a source A_k and the target A_0:

1. base pattern B = S(A_k) (level 1, Section 3) and candidates S = S(A_k^2);
2. weights w = 1 on B's entries and w_cand < 1 on the other candidates
   (``sam_candidate_weights``), penalty scale mu = ||A_k||_F^2 / n
   (``sam_penalty_scale``);
3. the soft-weighted map on S and dL/dw from its adjoint (``sam_backward``);
4. per column, B's entries plus the k candidates with the most negative
   dL/dw (``sam_pattern_topk``);
5. the plain SAM on that pattern (``sam_plan_create`` + ``sam_build_planned``).

Every step is a library call; this module only sequences them.
"""
from __future__ import annotations

from .sam import Context, DeviceCSC


def adaptive_pattern(ctx: Context, Ak: DeviceCSC, A0: DeviceCSC, k: int, w_cand: float = 0.1,
                     prec: str = "f32"):
    """Returns (colptr, rowind, info): the adapted pattern and the
    intermediate quantities (B, S, w, mu, dL/dw, weighted loss)."""
    B_cp, B_ri = ctx.pattern(Ak, 1)
    S_cp, S_ri = ctx.pattern(Ak, 2)
    w = ctx.candidate_weights(S_cp, S_ri, B_cp, B_ri, 1.0, w_cand)
    mu = ctx.penalty_scale(Ak)
    plan = ctx.plan(Ak, A0, S_cp, S_ri)
    try:
        _, _, gw, loss = plan.backward(Ak.val, A0.val, w, mu, dL=1.0, prec=prec)
    finally:
        plan.close()
    cp, ri = ctx.pattern_topk(S_cp, S_ri, w, gw, k)
    info = {"B": (B_cp, B_ri), "S": (S_cp, S_ri), "w": w, "mu": mu, "gw": gw, "loss_weighted": loss}
    return cp, ri, info


def adaptive_map(ctx: Context, Ak: DeviceCSC, A0: DeviceCSC, k: int, w_cand: float = 0.1, prec: str = "f32"):
    """The SAM on the adapted pattern: (colptr, rowind, M, ||A_k M - A_0||_F^2, info)."""
    cp, ri, info = adaptive_pattern(ctx, Ak, A0, k, w_cand, prec)
    plan = ctx.plan(Ak, A0, cp, ri)
    try:
        M, _, res2 = plan.build(Ak.val, A0.val, prec)
    finally:
        plan.close()
    return cp, ri, M, res2, info
