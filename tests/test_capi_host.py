"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/sam.h declares, and validates arguments before it
touches a device."""
import ctypes

import pytest

from paper_2406_17656_amd import _capi as C


def test_exports_every_declared_symbol():
    lib = C.load()
    names = C.header_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(C.SIGNATURES), set(names) ^ set(C.SIGNATURES)


def test_status_strings_and_version():
    lib = C.load()
    for code, name in C.STATUS_NAMES.items():
        assert lib.sam_status_string(code).decode() == name
    assert lib.sam_version().decode().count(".") == 2


@pytest.fixture
def hctx():
    lib = C.load()
    h = ctypes.c_void_p()
    assert lib.sam_create(ctypes.byref(h), C.SAM_NO_DEVICE) == C.SAM_OK
    yield lib, h
    lib.sam_destroy(h)


def csc(n=4, nnz=4, ptr=1):
    return C.sam_csc(n, nnz, ptr, ptr, ptr)


def spec(**kw):
    d = dict(kind=0, power=1, thresh=0.0, global_scale=-1, tau=0.0, lfil=1)
    d.update(kw)
    return C.sam_pattern_spec(d["kind"], d["power"], d["thresh"], d["global_scale"], d["tau"], d["lfil"])


WS = 256          # a stand-in device address with the required alignment (never dereferenced)


def test_null_context_rejected():
    lib = C.load()
    nnz = ctypes.c_int64()
    a = csc()
    sp = spec()
    assert lib.sam_pattern_count(None, ctypes.byref(a), ctypes.byref(sp), WS, 1 << 20, ctypes.byref(nnz), None) == 1
    assert lib.sam_create(None, 0) == 1


@pytest.mark.parametrize("bad,code", [
    (dict(power=0), 1), (dict(kind=7), 1), (dict(kind=2, tau=1.5), 1), (dict(kind=2, tau=-0.1), 1),
    (dict(kind=3, lfil=0), 1), (dict(kind=1, global_scale=0), 1),
])
def test_pattern_spec_validation(hctx, bad, code):
    lib, h = hctx
    nnz = ctypes.c_int64()
    a = csc()
    sp = spec(**bad)
    assert lib.sam_pattern_count(h, ctypes.byref(a), ctypes.byref(sp), WS, 1 << 20, ctypes.byref(nnz), None) == code
    assert lib.sam_last_error(h).decode()
    nb = ctypes.c_size_t()
    assert lib.sam_pattern_workspace_size(h, ctypes.byref(a), ctypes.byref(sp), ctypes.byref(nb), None) == code


def test_valid_arguments_reach_the_device_check(hctx):
    lib, h = hctx
    nnz = ctypes.c_int64()
    a = csc()
    sp = spec(power=2)
    assert lib.sam_pattern_count(h, ctypes.byref(a), ctypes.byref(sp), WS, 1 << 20, ctypes.byref(nnz), None) == 8
    assert "no device" in lib.sam_last_error(h).decode()


def test_plan_shape_and_overflow_checks(hctx):
    lib, h = hctx
    pl = ctypes.c_void_p()
    nb = ctypes.c_size_t()
    M = 1 << 20

    def create(a, b, nnz, mem=WS):
        return lib.sam_plan_create(h, ctypes.byref(a), ctypes.byref(b), 1, 1, nnz, mem, M, ctypes.byref(pl), None)

    def size(a, b, nnz):
        return lib.sam_plan_size(h, ctypes.byref(a), ctypes.byref(b), 1, 1, nnz, ctypes.byref(nb), None)

    a, b = csc(n=4), csc(n=5)
    assert create(a, b, 4) == 2 and size(a, b, 4) == 2
    b = csc(n=4)
    assert create(a, b, 2 ** 31) == 4 and size(a, b, 2 ** 31) == 4
    assert create(a, b, -1) == 1 and size(a, b, -1) == 1
    neg = csc(n=-1)
    assert create(neg, b, 4) == 1
    nullrows = C.sam_csc(4, 4, 1, None, 1)
    assert create(nullrows, b, 4) == 1
    # plan memory: NULL or unaligned is an argument error before any device work
    assert create(a, b, 4, mem=None) == 1
    assert create(a, b, 4, mem=WS + 8) == 1 and "aligned" in lib.sam_last_error(h).decode()
    assert create(a, b, 4) == C.SAM_ERR_UNSUPPORTED and size(a, b, 4) == C.SAM_ERR_UNSUPPORTED


def test_build_and_residual_argument_checks(hctx):
    lib, h = hctx
    a, b = csc(n=4), csc(n=4)
    M = 1 << 20
    nb = ctypes.c_size_t()
    # unknown precision
    assert lib.sam_build(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, 7, 1, None, None, WS, M, None) == 1
    assert lib.sam_workspace_size(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, 7, ctypes.byref(nb), None) == 1
    # missing M
    assert lib.sam_build(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, 0, None, None, None, WS, M, None) == 1
    # valid arguments on a host-only context
    assert lib.sam_build(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, 0, 1, None, None, WS, M, None) == 8
    # residual: order mismatch, nnz overflow, null res2, workspace too small
    c = csc(n=3)
    assert lib.sam_residual(h, ctypes.byref(a), ctypes.byref(c), 1, 1, 4, 1, 0, 1, None, WS, M, None) == 2
    assert lib.sam_residual(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 2 ** 31, 1, 0, 1, None, WS, M, None) == 4
    assert lib.sam_residual(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, 1, 0, None, None, WS, M, None) == 1
    assert lib.sam_residual(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, 1, 0, 1, None, WS, 8, None) == 1
    assert "workspace" in lib.sam_last_error(h).decode()
    assert lib.sam_residual(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, 1, 0, 1, None, WS, M, None) == 8
    # apply
    assert lib.sam_apply_prepare(h, 4, 1, 1, 2 ** 31, 1, 1, 1, WS, M, None) == 4
    assert lib.sam_apply_prepare(h, 4, 1, 1, 4, 1, 1, 1, WS, 8, None) == 1
    assert lib.sam_apply(h, 4, 1, 1, 1, 1, 9, 1, 1, None) == 1


def test_workspace_sizes_without_device():
    """The n-sized workspaces are sized on the host, grow with n, and reject
    negative sizes."""
    lib = C.load()
    def size(fn, *a):
        nb = ctypes.c_size_t()
        assert fn(*a, ctypes.byref(nb)) == 0
        return nb.value
    for fn, small, big in ((lib.sam_residual_workspace_size, (100, 500), (10 ** 6, 5 * 10 ** 6)),
                           (lib.sam_apply_workspace_size, (100,), (10 ** 6,)),
                           (lib.sam_topk_workspace_size, (100,), (10 ** 6,)),
                           (lib.sam_penalty_workspace_size, (100,), (10 ** 8,))):
        s0, s1 = size(fn, *small), size(fn, *big)
        assert 0 < s0 < s1 and s0 % 256 == 0
    nb = ctypes.c_size_t()
    assert lib.sam_residual_workspace_size(-1, 4, ctypes.byref(nb)) == 1
    assert lib.sam_apply_workspace_size(4, None) == 1
    assert lib.sam_residual_workspace_size(10 ** 6, 0, ctypes.byref(nb)) == 0 and nb.value >= 8 * 10 ** 6


def test_empty_matrices_rejected(hctx):
    lib, h = hctx
    pl = ctypes.c_void_p()
    a, b = csc(n=4, nnz=0), csc(n=4)
    assert lib.sam_plan_create(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, WS, 1 << 20, ctypes.byref(pl), None) == 1
    assert "stored entries" in lib.sam_last_error(h).decode()


def test_empty_sequence_rejected(hctx):
    lib, h = hctx
    sq = ctypes.c_void_p()
    a = csc(n=0, nnz=0)
    spec = C.sam_pattern_spec(0, 2, 0.0, -1, 0.0, 1)
    assert lib.sam_sequence_create(h, ctypes.byref(a), ctypes.byref(a), ctypes.byref(spec), 2, 1, 1,
                                   WS, 1 << 20, ctypes.byref(sq), None) == 1
    assert "empty" in lib.sam_last_error(h).decode()
    nb = ctypes.c_size_t()
    assert lib.sam_sequence_size(h, ctypes.byref(a), ctypes.byref(a), ctypes.byref(spec), 2, 1, 1,
                                 WS, 1 << 20, ctypes.byref(nb), None) == 1
    b = csc(n=4)
    assert lib.sam_sequence_create(h, ctypes.byref(b), ctypes.byref(b), ctypes.byref(spec), 0, 1, 1,
                                   WS, 1 << 20, ctypes.byref(sq), None) == 1
    assert lib.sam_sequence_create(h, ctypes.byref(b), ctypes.byref(b), ctypes.byref(spec), 2, 1, 1,
                                   None, 1 << 20, ctypes.byref(sq), None) == 1


def test_menu_without_device():
    from paper_2406_17656_amd import autotune
    for prec in ("f32", "f64"):
        m = autotune.menu(prec)
        assert len(m) >= 6 and all(v["max_rows"] >= 13 and v["NC"] >= 5 for v in m)
        assert autotune.menu(prec, weighted=1)
    orders = autotune.candidate_orders(5)
    assert orders[0] == [0, 1, 2, 3, 4] and [3, 0, 1, 2, 4] in orders
    lib = C.load()
    cnt = ctypes.c_int32()
    assert lib.sam_menu(7, 0, 0, ctypes.byref(cnt), None, None, None, None) == 1


def test_plan_select_validation(hctx):
    lib, h = hctx
    # no plan: argument error before anything else
    arr = (ctypes.c_int32 * 1)(0)
    assert lib.sam_plan_select(None, 1, arr, 1, None) == 1


def test_adaptive_calls_validate_arguments(hctx):
    """Argument checks of the adaptive-pattern calls come before any device
    work: NULLs, negative sizes and k < 0 are SAM_ERR_ARG, oversized patterns
    SAM_ERR_OVERFLOW; valid arguments on a context without a device reach
    SAM_ERR_UNSUPPORTED."""
    lib, h = hctx
    out = ctypes.c_int64()
    w = ctypes.c_double()
    # sam_candidate_weights(ctx, n, S_cp, S_ri, nnz_S, B_cp, B_ri, nnz_B, w_base, w_cand, w, stream)
    assert lib.sam_candidate_weights(h, -1, 1, 1, 4, 1, 1, 4, 1.0, 0.1, 1, None) == C.SAM_ERR_ARG
    assert lib.sam_candidate_weights(h, 4, None, 1, 4, 1, 1, 4, 1.0, 0.1, 1, None) == C.SAM_ERR_ARG
    assert lib.sam_candidate_weights(h, 4, 1, 1, 4, 1, 1, 4, 1.0, 0.1, None, None) == C.SAM_ERR_ARG
    assert lib.sam_candidate_weights(h, 4, 1, 1, 2 ** 31, 1, 1, 4, 1.0, 0.1, 1, None) == C.SAM_ERR_OVERFLOW
    assert lib.sam_candidate_weights(h, 4, 1, 1, 4, 1, 1, 4, 1.0, 0.1, 1, None) == C.SAM_ERR_UNSUPPORTED
    # sam_pattern_topk(ctx, n, S_cp, S_ri, nnz_S, w, grad, k, out_cp, out_ri, nnz_out, ws, ws_bytes, stream)
    M = 1 << 20
    assert lib.sam_pattern_topk(h, 4, 1, 1, 4, 1, 1, -1, 1, 1, ctypes.byref(out), WS, M, None) == C.SAM_ERR_ARG
    assert lib.sam_pattern_topk(h, 4, 1, 1, 4, None, 1, 2, 1, 1, ctypes.byref(out), WS, M, None) == C.SAM_ERR_ARG
    assert lib.sam_pattern_topk(h, 4, 1, 1, 4, 1, 1, 2, 1, 1, None, WS, M, None) == C.SAM_ERR_ARG
    assert lib.sam_pattern_topk(h, 4, 1, 1, 4, 1, 1, 2, 1, 1, ctypes.byref(out), WS, M,
                                None) == C.SAM_ERR_UNSUPPORTED
    # sam_penalty_scale(ctx, Ak, mu, ws, ws_bytes, stream)
    a = csc()
    assert lib.sam_penalty_scale(h, ctypes.byref(a), None, WS, M, None) == C.SAM_ERR_ARG
    e = csc(n=0, nnz=0)
    assert lib.sam_penalty_scale(h, ctypes.byref(e), ctypes.byref(w), WS, M, None) == C.SAM_ERR_ARG
    nv = C.sam_csc(4, 4, 1, 1, None)
    assert lib.sam_penalty_scale(h, ctypes.byref(nv), ctypes.byref(w), WS, M, None) == C.SAM_ERR_ARG
    assert lib.sam_penalty_scale(h, ctypes.byref(a), ctypes.byref(w), WS, M, None) == C.SAM_ERR_UNSUPPORTED


def test_library_allocates_only_the_context_block():
    """Source check: the only device allocation in the library is the
    context's status block in sam_create."""
    import glob
    import os
    import re
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2406_17656_amd", "csrc")
    hits = []
    for f in sorted(glob.glob(os.path.join(root, "*"))):
        for i, line in enumerate(open(f), 1):
            if re.search(r"\bhip(Malloc|MallocAsync|ExtMallocWithFlags|MallocManaged|MallocPitch|HostMalloc)\b", line):
                hits.append((os.path.basename(f), line.strip()))
    assert hits == [("sam_capi.cpp", "if (hipMalloc(&ctx->block, kCtxBlockBytes) != hipSuccess) {")], hits
