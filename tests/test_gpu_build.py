"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI:
patterns (bit-exact), the batched least-squares map in FP64 and FP32 +
refinement (per-column max-relative tolerance 1e-10 / 1e-6), per-column and
Frobenius residuals, the explicit residual and y = M x."""
import numpy as np
import pytest
import torch

import oracle as O
import pde_inputs as P
from parity_util import TOL, colmax_rel, sample_columns

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_17656_amd import Context
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(A):
    from paper_2406_17656_amd import DeviceCSC
    return DeviceCSC.from_host(A)


def host(t):
    return t.detach().cpu().numpy()


def gpu_pattern(ctx, A, power, kind="none", **kw):
    cp, ri = ctx.pattern(dev(A), power, kind, **kw)
    return host(cp), host(ri)


def small_cases():
    A0, (A1,) = P.config1()
    yield "cfg1", A0, A1
    A0, As = P.config2(m=40, nmat=3)
    yield "cfg2-40", A0, As[1]
    A0, As = P.config3(m=10)
    yield "cfg3-10", A0, As[-1]
    A0, As = P.config4(m=48, nmat=3)
    yield "cfg4-48", A0, As[1]


CASES = list(small_cases())


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("spec", [
    dict(power=1), dict(power=2), dict(power=3),
    dict(power=2, kind="column", tau=0.6), dict(power=2, kind="column", tau=0.85),
    dict(power=2, kind="lfil", lfil=3), dict(power=2, kind="global", thresh=0.1),
    dict(power=1, kind="global", thresh=0.05, global_scale=1),
], ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
def test_pattern_bitexact(ctx, case, spec):
    _, A0, Ak = case
    want = O.pattern(Ak, **spec)
    cp, ri = gpu_pattern(ctx, Ak, **spec)
    assert np.array_equal(cp, want.colptr)
    assert np.array_equal(ri, want.rowind)


def test_table_counts_on_gpu(ctx):
    L = P.laplacian_2d(64)
    assert gpu_pattern(ctx, L, 1)[0][-1] == 20224
    assert gpu_pattern(ctx, L, 2)[0][-1] == 51972
    assert gpu_pattern(ctx, L, 3)[0][-1] == 98836
    assert gpu_pattern(ctx, L, 2, "column", tau=0.7)[0][-1] == 4096


def check_build(ctx, A0, Ak, power, prec, kind="none", cols=None, **kw):
    Sp = O.pattern(Ak, power, kind, **kw)
    dAk, dA0 = dev(Ak), dev(A0)
    Scp, Sri = ctx.pattern(dAk, power, kind, **kw)
    assert np.array_equal(host(Scp), Sp.colptr) and np.array_equal(host(Sri), Sp.rowind)
    M, col, res2 = ctx.build(dAk, dA0, Scp, Sri, prec)
    ctx.sync_status()
    Mo, rho, _, _ = O.sam_build(Ak, A0, Sp, cols=cols)
    Mg, colg = host(M).astype(np.float64), host(col)
    wc, we = colmax_rel(Mg, Mo, Sp.colptr, cols)
    assert wc <= TOL[prec], (wc, we)
    js = np.arange(Ak.n) if cols is None else cols
    assert np.allclose(colg[js], rho[js], rtol=1e-9, atol=1e-13 * max(rho[js].max(), 1e-300))
    # Frobenius residual: fixed-order device sum of the column residuals
    assert np.isclose(float(host(res2)[0]), colg.sum(), rtol=1e-12)
    if cols is None:
        assert np.isclose(float(host(res2)[0]), rho.sum(), rtol=1e-9)
    return Sp, M, wc, we


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("power", [1, 2])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_build_small(ctx, case, power, prec):
    _, A0, Ak = case
    _, _, wc, we = check_build(ctx, A0, Ak, power, prec)
    print(f"{case[0]} p={power} {prec}: colmax {wc:.2e} entrywise {we:.2e}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_build_thresholded_ragged(ctx, prec):
    _, A0, Ak = CASES[3]
    check_build(ctx, A0, Ak, 2, prec, kind="global", thresh=0.1)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_identity_when_source_equals_target(ctx, prec):
    A0, _ = P.config1()
    S = O.pattern(A0, 2)
    dA = dev(A0)
    Scp, Sri = ctx.pattern(dA, 2)
    M, col, res2 = ctx.build(dA, dA, Scp, Sri, prec)
    ctx.sync_status()
    cols = np.repeat(np.arange(S.n), np.diff(S.colptr))
    tol = 1e-13 if prec == "f64" else 1e-7
    assert np.abs(host(M) - (S.rowind == cols)).max() < tol
    assert float(host(res2)[0]) < 1e-20 * (A0.val ** 2).sum()


def test_rank_deficient_reported(ctx):
    from paper_2406_17656_amd import SamError
    n = 5
    Ad = np.eye(n) * 2.0
    Ad[:, 3] = Ad[:, 2]
    Ad[4, 2] = Ad[4, 3] = 1.0
    Ak = P.dense_to_csc(Ad)
    Scp = torch.tensor([0, 1, 2, 4, 5, 6], dtype=torch.int32, device="cuda")
    Sri = torch.tensor([0, 1, 2, 3, 3, 4], dtype=torch.int32, device="cuda")
    for prec in ("f64", "f32"):
        dAk = dev(Ak)
        M, col, res2 = ctx.build(dAk, dAk, Scp, Sri, prec)
        with pytest.raises(SamError) as ei:
            ctx.sync_status()
        assert ei.value.name == "SAM_ERR_RANK" and ei.value.column == 2
    ctx.sync_status()  # cleared


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_residual_explicit(ctx, prec):
    _, A0, Ak = CASES[2]
    Sp = O.pattern(Ak, 2)
    dAk, dA0 = dev(Ak), dev(A0)
    Scp, Sri = ctx.pattern(dAk, 2)
    M, col, res2 = ctx.build(dAk, dA0, Scp, Sri, prec)
    r2, a2 = ctx.residual(dAk, dA0, Scp, Sri, M, prec)
    ctx.sync_status()
    Mo = host(M).astype(np.float64)
    r2o, a2o = O.residual(Ak, A0, Sp, Mo)
    assert np.isclose(float(host(r2)[0]), r2o, rtol=1e-12)
    assert np.isclose(float(host(a2)[0]), a2o, rtol=1e-14)
    assert np.isclose(float(host(r2)[0]), float(host(res2)[0]), rtol=1e-9)


def test_residual_arbitrary_map(ctx):
    """The explicit residual of any M on any pattern (not a minimiser)."""
    _, A0, Ak = CASES[3]
    Sp = O.pattern(Ak, 2)
    M = np.random.default_rng(3).standard_normal(Sp.nnz)
    r2, a2 = ctx.residual(dev(Ak), dev(A0), torch.as_tensor(Sp.colptr).cuda(),
                          torch.as_tensor(Sp.rowind).cuda(), torch.as_tensor(M).cuda(), "f64")
    ctx.sync_status()
    r2o, _ = O.residual(Ak, A0, Sp, M)
    assert np.isclose(float(host(r2)[0]), r2o, rtol=1e-12)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("power", [2, 3])   # rows of about 13 and 25 entries: one and two unrolled chunks
def test_apply(ctx, prec, power):
    _, A0, Ak = CASES[1]
    Sp = O.pattern(Ak, power)
    Scp, Sri = torch.as_tensor(Sp.colptr).cuda(), torch.as_tensor(Sp.rowind).cuda()
    M = np.random.default_rng(1).standard_normal(Sp.nnz)
    Mt = torch.as_tensor(M.astype(np.float32 if prec == "f32" else np.float64)).cuda()
    x = np.random.default_rng(2).standard_normal(Ak.n)
    T = ctx.apply_prepare(Ak.n, Scp, Sri)
    xt = torch.as_tensor(x).cuda()
    y = ctx.apply(T, Mt, xt, prec)
    Mref = host(Mt).astype(np.float64)
    yref = O.apply(Sp, Mref, x)
    assert np.allclose(host(y), yref, rtol=1e-13, atol=1e-13)
    # values in the row view's order: the same sums, bit for bit
    Tv = ctx.apply_permute(T, Mt, prec)
    assert np.array_equal(host(Tv), host(Mt)[host(T[2])])
    y2 = ctx.apply(T, Tv, xt, prec, permuted=True)
    assert np.array_equal(host(y2), host(y))
    assert np.array_equal(host(ctx.apply(T, Mt, xt, prec)), host(y))   # reproducible
    # the row view is a permutation of the entries, columns ascending per row
    rp, ci, pm = (host(t) for t in T)
    assert np.array_equal(np.sort(pm), np.arange(Sp.nnz))
    for i in range(0, Ak.n, 97):
        assert np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("power", [1, 2])
def test_full_size_config2_sampled(ctx, prec, power):
    """512 x 512 diffusion (n = 262144), the benchmark's sizes and launch
    configuration: sampled columns against the oracle, plus the whole
    Frobenius residual against the oracle's per-column sum."""
    A0, As = P.config2()
    Ak = As[-1]
    Sp = O.pattern(Ak, power)
    cols = sample_columns(Ak.n, Sp.colptr, k=3000, seed=power)
    _, _, wc, we = check_build(ctx, A0, Ak, power, prec, cols=cols)
    print(f"cfg2 full p={power} {prec}: colmax {wc:.2e} entrywise {we:.2e}")


def random_wide(n=240, per_col=11, seed=12):
    """Unstructured sparse matrix with long columns: level-2 columns have
    more than 32 lists and lists longer than 8 (the kernels' memory path)."""
    rng = np.random.default_rng(seed)
    d = np.zeros((n, n))
    for j in range(n):
        rows = rng.choice(n, size=per_col, replace=False)
        d[rows, j] = rng.uniform(-1, 1, per_col)
    d += np.diag(np.abs(d).sum(axis=0) + 1.0)
    return P.dense_to_csc(d)


@pytest.mark.parametrize("power", [1, 2, 3])
def test_pattern_long_lists(ctx, power):
    A = random_wide()
    want = O.pattern(A, power)
    cp, ri = gpu_pattern(ctx, A, power)
    assert np.array_equal(cp, want.colptr) and np.array_equal(ri, want.rowind)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_build_long_lists(ctx, prec):
    """|J_j| = 12, |I_j| up to ~120: the widest buckets and the memory path
    of the gather for columns longer than the register cache."""
    A0 = random_wide(seed=13)
    Ak = A0.with_values(A0.val * (1 + 0.05 * np.random.default_rng(1).standard_normal(A0.nnz)))
    check_build(ctx, A0, Ak, 1, prec)
