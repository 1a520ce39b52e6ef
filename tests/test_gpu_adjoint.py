"""GPU tests of the soft-weighted map and its adjoint (sam_build_weighted,
sam_backward, SamResidualLoss) against the oracle's weighted map and FP64
reference gradient, and against central finite differences of the GPU's own
FP64 forward."""
import numpy as np
import pytest
import torch

import oracle as O
import pde_inputs as P
from parity_util import TOL, colmax_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_17656_amd import Context
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(A):
    from paper_2406_17656_amd import DeviceCSC
    return DeviceCSC.from_host(A)


def problem(m=8, seed=0):
    rng = np.random.default_rng(seed)
    k0 = rng.lognormal(0.0, 0.5, (m, m, m))
    k1 = k0 * np.exp(0.1 * rng.standard_normal((m, m, m)))
    A0, A1 = P.diffusion_3d(k0), P.diffusion_3d(k1)
    S = O.pattern(A1, 2)
    w = P.candidate_weights(A1.n, S.colptr, S.rowind, A1, seed=seed + 5)
    return A0, A1, S, w, P.penalty_scale(A1)


def setup(ctx, A0, A1, S):
    dA0, dA1 = dev(A0), dev(A1)
    Scp = torch.as_tensor(S.colptr).cuda()
    Sri = torch.as_tensor(S.rowind).cuda()
    return dA0, dA1, ctx.plan(dA1, dA0, Scp, Sri)


def rel_err(g, gref):
    return float(np.abs(g - gref).max() / np.abs(gref).max())


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_weighted_forward(ctx, prec):
    A0, A1, S, w, mu = problem()
    dA0, dA1, plan = setup(ctx, A0, A1, S)
    wt = torch.as_tensor(w).cuda()
    M, _, res2 = plan.build_weighted(dA1.val, dA0.val, wt, mu, prec)
    ctx.sync_status()
    Mo, rho, _, _ = O.sam_build(A1, A0, S, weights=w, mu=mu)
    wc, we = colmax_rel(M.cpu().numpy().astype(np.float64), Mo, S.colptr)
    assert wc <= TOL[prec], (wc, we)
    assert np.isclose(float(res2.cpu()[0]), rho.sum(), rtol=1e-9)
    plan.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("f32", 1e-6)])
def test_backward_vs_oracle(ctx, prec, tol):
    A0, A1, S, w, mu = problem(seed=1)
    dA0, dA1, plan = setup(ctx, A0, A1, S)
    wt = torch.as_tensor(w).cuda()
    gAk, gA0, gw, loss = plan.backward(dA1.val, dA0.val, wt, mu, dL=1.0, prec=prec)
    ctx.sync_status()
    rAk, rA0, rw, L = O.backward(A1, A0, S, w, mu)
    assert rel_err(gAk.cpu().numpy(), rAk) <= tol
    assert rel_err(gA0.cpu().numpy(), rA0) <= tol
    assert rel_err(gw.cpu().numpy(), rw) <= tol
    assert np.isclose(float(loss.cpu()[0]), L, rtol=1e-9)
    # deterministic accumulation: a second call is bitwise identical
    gAk2, gA02, gw2, _ = plan.backward(dA1.val, dA0.val, wt, mu, dL=1.0, prec=prec)
    assert torch.equal(gAk, gAk2) and torch.equal(gA0, gA02) and torch.equal(gw, gw2)
    plan.close()


def test_backward_vs_central_fd(ctx):
    """Central differences (h = 1e-6 relative) of the GPU FP64 forward loss."""
    A0, A1, S, w, mu = problem(m=6, seed=2)
    dA0, dA1, plan = setup(ctx, A0, A1, S)
    wt = torch.as_tensor(w).cuda()
    gAk, gA0, gw, _ = plan.backward(dA1.val, dA0.val, wt, mu, prec="f64")

    def L(ak, a0, ww):
        return float(plan.build_weighted(ak, a0, ww, mu, "f64")[2].cpu()[0])

    rng = np.random.default_rng(3)
    for name, base, grad in (("Ak", dA1.val, gAk), ("A0", dA0.val, gA0), ("w", wt, gw)):
        g = grad.cpu().numpy()
        idx = rng.choice(base.numel(), 8, replace=False)
        if name == "w":
            idx = rng.choice(np.nonzero(w < 1.0)[0], 8, replace=False)
        for e in idx:
            h = 1e-6 * max(1.0, abs(float(base[e])))
            xp, xm = base.clone(), base.clone()
            xp[e] += h
            xm[e] -= h
            args_p = {"Ak": (xp, dA0.val, wt), "A0": (dA1.val, xp, wt), "w": (dA1.val, dA0.val, xp)}[name]
            args_m = {"Ak": (xm, dA0.val, wt), "A0": (dA1.val, xm, wt), "w": (dA1.val, dA0.val, xm)}[name]
            fd = (L(*args_p) - L(*args_m)) / (2 * h)
            assert abs(fd - g[e]) <= 1e-6 * np.abs(g).max(), (name, e, fd, g[e])
    plan.close()


def test_autograd_function(ctx):
    from paper_2406_17656_amd.autograd import SamResidualLoss
    A0, A1, S, w, mu = problem(m=6, seed=4)
    dA0, dA1, plan = setup(ctx, A0, A1, S)
    ak = dA1.val.clone().requires_grad_(True)
    a0 = dA0.val.clone().requires_grad_(True)
    wt = torch.as_tensor(w).cuda().requires_grad_(True)
    loss = SamResidualLoss.apply(plan, ak, a0, wt, mu, "f32")
    (3.0 * loss).backward()
    rAk, rA0, rw, L = O.backward(A1, A0, S, w, mu, dL=3.0)
    assert np.isclose(float(loss.detach().cpu()), L, rtol=1e-9)
    assert rel_err(ak.grad.cpu().numpy(), rAk) <= 1e-6
    assert rel_err(a0.grad.cpu().numpy(), rA0) <= 1e-6
    assert rel_err(wt.grad.cpu().numpy(), rw) <= 1e-6
    plan.close()


def test_unit_weights_reduce_to_plain_map(ctx):
    """w = 1: no penalty; the weighted map equals the plain map and the
    adjoint's lambda vanishes (dL/dw ~ 0 relative to dL/dA)."""
    A0, A1, S, w, mu = problem(m=6, seed=5)
    dA0, dA1, plan = setup(ctx, A0, A1, S)
    ones = torch.ones(S.nnz, dtype=torch.float64, device="cuda")
    Mw, _, rw = plan.build_weighted(dA1.val, dA0.val, ones, mu, "f64")
    Mp, _, rp = plan.build(dA1.val, dA0.val, "f64")
    assert torch.allclose(Mw, Mp, rtol=1e-12, atol=1e-14)
    gAk, gA0, gw, _ = plan.backward(dA1.val, dA0.val, ones, mu, prec="f64")
    assert float(gw.abs().max()) <= 1e-9 * float(gAk.abs().max())
    plan.close()


def test_full_size_config5_adjoint(ctx):
    """48^3 diffusion (n = 110592), lognormal(0, 0.5) coefficients, soft
    weights on the level-2 candidates: FP32 adjoint against the oracle's FP64
    reference gradient on every entry."""
    A0, A1 = P.config5()
    S = O.pattern(A1, 2)
    w = P.candidate_weights(A1.n, S.colptr, S.rowind, A1, seed=5)
    mu = P.penalty_scale(A1)
    dA0, dA1, plan = setup(ctx, A0, A1, S)
    wt = torch.as_tensor(w).cuda()
    gAk, gA0, gw, loss = plan.backward(dA1.val, dA0.val, wt, mu, prec="f32")
    ctx.sync_status()
    rAk, rA0, rw, L = O.backward(A1, A0, S, w, mu)
    errs = (rel_err(gAk.cpu().numpy(), rAk), rel_err(gA0.cpu().numpy(), rA0), rel_err(gw.cpu().numpy(), rw))
    print("cfg5 adjoint relative errors (Ak, A0, w):", errs)
    assert max(errs) <= 1e-6
    assert np.isclose(float(loss.cpu()[0]), L, rtol=1e-9)
    plan.close()
