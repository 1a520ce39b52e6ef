"""Autotuner of the numeric kernel's size classes.

The library compiles a menu of kernel variants per precision (lanes per
column problem G, rows per lane R, columns NC, LDS tile chunk TC; see
sam_menu).  A plan buckets each column into the first variant of an ordered
list that its block fits.  ``tune`` times candidate orders on the plan's own
shape histogram -- the default order and, for every variant, the order that
puts it first -- then refines the class boundaries of the fastest by leaving
classes out and swapping neighbours, keeps the fastest (sam_plan_select) and
caches the choice per device, precision and shape signature in a JSON file
($SAM_TUNE_CACHE, default ~/.cache/sam_mi355x_tune.json).
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os

import torch

from . import _capi as C
from .sam import PREC, SamError, _prec

CACHE = os.environ.get("SAM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                      "sam_mi355x_tune.json"))


def menu(prec="f32", weighted=0) -> list[dict]:
    lib = C.load()
    cap = 64
    cnt = ctypes.c_int32()
    arrs = [(ctypes.c_int32 * cap)() for _ in range(4)]
    st = lib.sam_menu(_prec(prec), int(weighted), cap, ctypes.byref(cnt), *arrs)
    if st != C.SAM_OK:
        raise SamError(st, "sam_menu")
    return [{"index": i, "G": arrs[0][i], "R": arrs[1][i], "NC": arrs[2][i], "TC": arrs[3][i],
             "max_rows": arrs[0][i] * arrs[1][i]} for i in range(min(cnt.value, cap))]


def candidate_orders(n_variants: int) -> list[list[int]]:
    default = list(range(n_variants))
    out = [default]
    for i in range(n_variants):
        o = [i] + [k for k in default if k != i]
        if o not in out:
            out.append(o)
    return [o[:16] for o in out]


def complete(order, prec="f32") -> list[int]:
    """The order with the menu's other variants appended (at most 16): the
    listed classes keep every column they fit, and a wider pattern (e.g. the
    unsparsified bound of a replanned sequence) still finds a class."""
    rest = [i for i in range(len(menu(prec))) if i not in order]
    return (list(order) + rest)[:16]


def signature(plan, prec) -> str:
    info = plan.info()
    dev = torch.cuda.get_device_name(plan.ctx.device)
    # selection-invariant shape data (the bucket split depends on the selection)
    key = json.dumps([dev, prec, info["n"], info["max_rows"], info["max_cols"], info["gathered"],
                      plan.nnz_S])
    return hashlib.sha256(key.encode()).hexdigest()[:24]


def _time(plan, Ak_val, A0_val, prec, reps):
    M = torch.empty(max(plan.nnz_S, 1), dtype=torch.float32 if PREC[prec] == 1 else torch.float64,
                    device=Ak_val.device)
    r = torch.empty(1, dtype=torch.float64, device=Ak_val.device)
    plan.build(Ak_val, A0_val, prec, M=M, res2=r)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.build(Ak_val, A0_val, prec, M=M, res2=r)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e3  # microseconds


def _load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(d: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def tune(plan, Ak_val, A0_val, prec="f32", reps=10, use_cache=True, refine=True) -> dict:
    """Pick the fastest variant order for this plan; returns
    {"order", "us", "timings", "cached"} and leaves the plan selected."""
    sig = signature(plan, prec)
    cache = _load_cache() if use_cache else {}
    if sig in cache:
        order = cache[sig]["order"]
        plan.select(order, prec)
        return {"order": order, "us": cache[sig]["us"], "timings": cache[sig].get("timings", {}),
                "cached": True}
    n_var = len(menu(prec))
    timings = {}

    def trial(order):
        try:
            plan.select(order, prec)
        except SamError:
            return None  # some column fits none of the listed variants
        us = _time(plan, Ak_val, A0_val, prec, reps)
        timings[",".join(map(str, order[:4])) + ("" if len(order) == n_var else f"/{len(order)}")] = us
        return us

    best = None
    for order in candidate_orders(n_var):
        us = trial(order)
        if us is not None and (best is None or us < best[1]):
            best = (order, us)
    if refine and best is not None:
        # Class boundaries: a column goes to the first listed class it fits,
        # so leaving a class out hands its columns to the next wider one and
        # swapping two neighbours moves the boundary between them.  Greedy
        # passes keep a change that is faster by more than 2 %.
        for _ in range(2):
            changed = False
            for v in list(best[0][1:]):
                cand = [x for x in best[0] if x != v]
                us = trial(cand)
                if us is not None and us < 0.98 * best[1]:
                    best, changed = (cand, us), True
            for i in range(1, len(best[0]) - 1):
                cand = list(best[0])
                cand[i], cand[i + 1] = cand[i + 1], cand[i]
                us = trial(cand)
                if us is not None and us < 0.98 * best[1]:
                    best, changed = (cand, us), True
            if not changed:
                break
    plan.select(best[0], prec)
    if use_cache:
        cache[sig] = {"order": best[0], "us": best[1], "timings": timings}
        _store_cache(cache)
    return {"order": best[0], "us": best[1], "timings": timings, "cached": False}


def tune_sequence(seq, vals, order, prec="f32", reps=3, refine=True) -> dict:
    """Pick the variant order of a replanned sequence by timing whole runs.

    ``tune`` times orders on one source's plan; the sources of a sequence can
    differ in shape (a threshold drops more couplings from some sources than
    from others), and which classes pay off depends on all of them.  The
    candidates are ``order`` and the orders that put each variant first (the
    menu's other variants appended, see ``complete``); the fastest is refined
    as in ``tune`` (a class moved to the end, neighbours swapped, kept when 2 %
    faster).  Leaves the sequence selected; returns {"order", "ms",
    "timings"}."""
    import time

    Ms = seq.alloc_maps()
    res2 = torch.zeros(seq.n_src, dtype=torch.float64, device=vals[0].device)
    n_var = len(menu(prec))
    timings = {}

    def trial(o):
        o = complete(o, prec)
        key = ",".join(map(str, o))
        if key in timings:
            return o, timings[key]
        try:
            seq.select(o)
        except SamError:
            return o, None
        seq.run(vals, Ms, res2)          # captures the graph for this order
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            seq.run(vals, Ms, res2)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        timings[key] = ms
        return o, ms

    best = None
    for cand in [list(order)] + candidate_orders(n_var):
        o, ms = trial(cand)
        if ms is not None and (best is None or ms < best[1]):
            best = (o, ms)
    if refine and best is not None:
        for _ in range(2):
            changed = False
            for v in list(best[0][1:]):
                o, ms = trial([x for x in best[0] if x != v])
                if ms is not None and ms < 0.98 * best[1]:
                    best, changed = (o, ms), True
            for i in range(1, len(best[0]) - 1):
                cand = list(best[0])
                cand[i], cand[i + 1] = cand[i + 1], cand[i]
                o, ms = trial(cand)
                if ms is not None and ms < 0.98 * best[1]:
                    best, changed = (o, ms), True
            if not changed:
                break
    if best is None:
        raise SamError(C.SAM_ERR_UNSUPPORTED, "no variant order fits every column of the sequence")
    seq.select(best[0])
    return {"order": best[0], "ms": best[1], "timings": timings}
