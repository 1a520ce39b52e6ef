"""Full-size GPU parity of the timed paths against the FP64 oracle.

Each workload runs exactly as bench.py times it: the variant order tuned on
the first source's plan and then on whole runs of the sequence, then the
replanned sequence (every source's pattern,
plan, buckets, build and residual inside one HIP graph), captured on the
first run and replayed on the second.  For every source:
- the pattern S_k is compared with the oracle's, bit for bit;
- every column of M_k is compared with the oracle's map (per column
  ||m - m*||_inf <= tol ||m*||_inf, and in FP32 + refinement also entrywise);
- ||A_k M_k - A_0||_F^2 is compared with the oracle's sum of column residuals.
Workloads: the 512^2 diffusion sequence with level 2 (the benchmark step, 7
sources), the 64^3 upwind convection-diffusion sequence (5 sources) with
level 2 and with the column threshold, and the 1024^2 ragged 9-point
sequence (15 sources) with the global threshold then level 2.  Lines
starting with PARITY report the measured errors."""
import numpy as np
import pytest
import torch

import bench
import oracle as O
import pde_inputs as P
from parity_util import ENTRY_FLOOR, TOL, colmax_rel, entrywise_rel

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


def run_step(ctx, name, A0, As, prec="f32", power=2):
    """bench.py's step for workload `name`: the order tuned on the first
    source's plan and then on whole runs of the replanned sequence, one run
    and one replay."""
    spec = bench.WORKLOADS[name]["spec"]
    dA0 = dev(A0)
    dAs = [dev(A) for A in As]
    vals = [d.val for d in dAs]
    order = bench.tune_order(ctx, dAs[0], dA0, prec, power, spec)["order"]
    seq = bench.step_sequence(ctx, dA0, dAs[0], len(As), prec, power, spec, order, vals=vals)
    order = seq.tuned["order"]
    Ms = seq.alloc_maps()
    res2 = torch.zeros(len(As), dtype=torch.float64, device="cuda")
    seq.run(vals, Ms, res2)            # captured (the tuner's final selection)
    ctx.sync_status()
    first = [M.clone() for M in Ms]
    seq.run(vals, Ms, res2)            # replayed
    ctx.sync_status()
    for M, F in zip(Ms, first):   # bit for bit (the unused tail too: it may hold NaN patterns)
        iv = torch.int32 if M.dtype == torch.float32 else torch.int64
        assert torch.equal(M.view(iv), F.view(iv))
    return seq, spec, order, Ms, res2


def check_sources(ctx, name, seq, spec, A0, As, Ms, res2, prec, power=2):
    worst = (0.0, 0.0, 0.0, 0.0)
    for k, Ak in enumerate(As):
        Sp = O.pattern(Ak, power, **spec)
        cp, ri = seq.pattern(k)
        assert np.array_equal(cp.cpu().numpy(), Sp.colptr), k
        assert np.array_equal(ri.cpu().numpy(), Sp.rowind), k
        Mo, rho, _, _ = O.sam_build(Ak, A0, Sp)
        Mg = Ms[k][:Sp.nnz].cpu().numpy().astype(np.float64)
        wc, we = colmax_rel(Mg, Mo, Sp.colptr)
        wf = entrywise_rel(Mg, Mo, Sp.colptr, ENTRY_FLOOR)
        assert wc <= TOL[prec], (k, wc, we)
        if prec == "f32":
            assert wf <= TOL[prec], (k, wc, wf)
        ref = O.frobenius_sq(rho)
        rr = abs(float(res2[k].cpu()) - ref) / ref
        assert rr <= 1e-9, (k, rr)
        worst = tuple(max(x, y) for x, y in zip(worst, (wc, wf, we, rr)))
    print(f"PARITY {name} {prec} level {power}: {len(As)} sources, every column: colmax {worst[0]:.2e} "
          f"entrywise (>= {ENTRY_FLOOR:g} of column max) {worst[1]:.2e}, all entries {worst[2]:.2e}, "
          f"frobenius rel {worst[3]:.2e}")


@pytest.fixture(scope="module")
def cfg2():
    return P.config2()


@pytest.fixture(scope="module")
def cfg3():
    return P.config3()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_bench_step_512_level2(ctx, cfg2, prec):
    """The benchmark step itself: 512^2, 7 sources, replanned, tuned order
    (the FP64 leg of the same step as well)."""
    A0, As = cfg2
    seq, spec, order, Ms, res2 = run_step(ctx, "diffusion2d", A0, As, prec)
    check_sources(ctx, "diffusion2d-512", seq, spec, A0, As, Ms, res2, prec)
    seq.close()


@pytest.mark.parametrize("name", ["convdiff3d", "convdiff3d_tau"])
def test_convdiff3d_sequence(ctx, cfg3, name):
    A0, As = cfg3
    seq, spec, order, Ms, res2 = run_step(ctx, name, A0, As)
    check_sources(ctx, name + "-64", seq, spec, A0, As, Ms, res2, "f32")
    seq.close()


def test_convdiff3d_level2_f64(ctx, cfg3):
    A0, As = cfg3
    seq, spec, order, Ms, res2 = run_step(ctx, "convdiff3d", A0, As[-2:], "f64")
    check_sources(ctx, "convdiff3d-64", seq, spec, A0, As[-2:], Ms, res2, "f64")
    seq.close()


def test_ninepoint_sequence_16(ctx):
    """The 1024^2 ragged 9-point sequence of 16 matrices (15 sources), global
    threshold 0.1 then level 2, as bench.py --workload ninepoint2d runs it."""
    A0, As = P.config4()
    assert len(As) == 15
    seq, spec, order, Ms, res2 = run_step(ctx, "ninepoint2d", A0, As)
    check_sources(ctx, "ninepoint2d-1024", seq, spec, A0, As, Ms, res2, "f32")
    seq.close()


def test_ninepoint_level2_f64(ctx):
    A0, As = P.config4(nmat=3)
    seq, spec, order, Ms, res2 = run_step(ctx, "ninepoint2d", A0, As, "f64")
    check_sources(ctx, "ninepoint2d-1024", seq, spec, A0, As, Ms, res2, "f64")
    seq.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_config1_every_column(ctx, prec):
    """32^2 diffusion, S(A_1), one-shot build: every column and the
    Frobenius residual."""
    A0, (A1,) = P.config1()
    Sp = O.pattern(A1, 1)
    Scp, Sri = ctx.pattern(dev(A1), 1)
    assert np.array_equal(Scp.cpu().numpy(), Sp.colptr) and np.array_equal(Sri.cpu().numpy(), Sp.rowind)
    M, col, res2 = ctx.build(dev(A1), dev(A0), Scp, Sri, prec)
    ctx.sync_status()
    Mo, rho, _, _ = O.sam_build(A1, A0, Sp)
    Mg = M.cpu().numpy().astype(np.float64)
    wc, we = colmax_rel(Mg, Mo, Sp.colptr)
    wf = entrywise_rel(Mg, Mo, Sp.colptr, ENTRY_FLOOR)
    assert wc <= TOL[prec], (wc, we)
    if prec == "f32":
        assert wf <= TOL[prec], (wc, wf)
    rr = abs(float(res2.cpu()[0]) - O.frobenius_sq(rho)) / O.frobenius_sq(rho)
    assert rr <= 1e-9
    print(f"PARITY config1-32 {prec} level 1: every column: colmax {wc:.2e} entrywise (>= {ENTRY_FLOOR:g} "
          f"of column max) {wf:.2e}, all entries {we:.2e}, frobenius rel {rr:.2e}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_config5_weighted_forward_every_column(ctx, prec):
    """48^3 diffusion with soft weights on the level-2 candidates: the
    weighted map on every column against the oracle's stacked solve."""
    A0, A1 = P.config5()
    S = O.pattern(A1, 2)
    w = P.candidate_weights(A1.n, S.colptr, S.rowind, A1, seed=5)
    mu = P.penalty_scale(A1)
    dA0, dA1 = dev(A0), dev(A1)
    plan = ctx.plan(dA1, dA0, torch.as_tensor(S.colptr).cuda(), torch.as_tensor(S.rowind).cuda())
    M, _, res2 = plan.build_weighted(dA1.val, dA0.val, torch.as_tensor(w).cuda(), mu, prec)
    ctx.sync_status()
    Mo, rho, _, _ = O.sam_build(A1, A0, S, weights=w, mu=mu)
    Mg = M.cpu().numpy().astype(np.float64)
    wc, we = colmax_rel(Mg, Mo, S.colptr)
    wf = entrywise_rel(Mg, Mo, S.colptr, ENTRY_FLOOR)
    assert wc <= TOL[prec], (wc, we)
    if prec == "f32":
        assert wf <= TOL[prec], (wc, wf)
    rr = abs(float(res2.cpu()[0]) - O.frobenius_sq(rho)) / O.frobenius_sq(rho)
    assert rr <= 1e-9
    print(f"PARITY config5-48 weighted {prec}: every column: colmax {wc:.2e} entrywise (>= {ENTRY_FLOOR:g} "
          f"of column max) {wf:.2e}, all entries {we:.2e}, frobenius rel {rr:.2e}")
    plan.close()
