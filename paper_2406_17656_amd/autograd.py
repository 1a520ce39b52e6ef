"""torch.autograd.Function over the soft-weighted SAM and its adjoint.

``SamResidualLoss.apply(plan, Ak_val, A0_val, w, mu, prec)`` returns
L = ||A_k M - A_0||_F^2 where M is the soft-weighted map (column problems
min ||A m - b||^2 + sum_l mu (1/w_l - 1) m_l^2 on the plan's pattern); its
backward calls sam_backward, which recomputes each column's QR and returns
dL/dA_k (stored values), dL/dA_0 (stored values) and dL/dw.  mu is a fixed
scale (not differentiated).
"""
import torch


class SamResidualLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, Ak_val, A0_val, w, mu, prec="f32"):
        _, _, res2 = plan.build_weighted(Ak_val, A0_val, w, mu, prec)
        ctx.plan = plan
        ctx.mu = float(mu)
        ctx.prec = prec
        ctx.save_for_backward(Ak_val, A0_val, w)
        return res2.reshape(())

    @staticmethod
    def backward(ctx, dL):
        Ak_val, A0_val, w = ctx.saved_tensors
        gAk, gA0, gw, _ = ctx.plan.backward(Ak_val, A0_val, w, ctx.mu, dL=float(dL), prec=ctx.prec)
        return None, gAk, gA0, gw, None, None
