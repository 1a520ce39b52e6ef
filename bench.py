#!/usr/bin/env python
"""Benchmark of the SAM construction on one MI355X.

Workload (one step): the 2D variable-coefficient diffusion sequence on a
512 x 512 grid (n = 262144), target A_0 and sources A_1..A_7 with
a_k = 1 + 0.5 sin(2 pi x + 0.1 k) cos(2 pi y) + 0.05 N(0,1).  For every
source the whole path runs inside one HIP graph: the level-2 pattern
S(A_k^2) (Sections 3-4), the plan of the column problems (row sets, gather
positions, size buckets), the batched least-squares build in FP32 with one
FP64 refinement step, and the Frobenius residual ||A_k M_k - A_0||_F
(Section 2).  Inputs are resident in HBM before the timed region.  Prints
one JSON line; progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --copy-calibration   # plain copy of known size, for PMC scaling
    python bench.py --roofline-only      # only the dominant kernel's timed launches
    python bench.py --adjoint-only       # only the 48^3 weighted forward and adjoint
    python bench.py --level1-cold        # level-1 builds over separate copies of 7 maps (HBM, not MALL)

The roofline object describes the dominant kernel: the numeric variant that
serves the most columns, launched alone over every column of one map (all of
them fit it) with the Frobenius sum left out, timed with HIP events on the
stream it runs on.  Its HBM traffic comes from the committed rocprofv3 PMC
summary (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by what the same
counters read for a copy of known size) and is reported only while the
kernel's sources still hash to the value recorded there.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "fp32_TFs": 157.3, "fp64_TFs": 78.6}
KERNEL_SOURCES = ["sam_numeric.hip", "sam_device.hpp", "sam_numeric_args.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_numeric_cfg2_512_level2.txt")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2406_17656_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(variant: str):
    """Bytes per launch from the committed PMC summary, or None when the
    summary is missing or was taken on other kernel sources or variant."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if "=" in line and not line.lstrip().startswith("#"):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != kernel_source_hash():
            return None
        return float(kv[f"variant.{variant}.fetch_kib"]) * 1024 * float(kv["fetch_factor"]) + \
            float(kv[f"variant.{variant}.write_kib"]) * 1024 * float(kv["write_factor"])
    except (OSError, KeyError, ValueError):
        return None


# Workloads: the default is the benchmark's; the others are the 3D upwind
# convection-diffusion sequence and the ragged 9-point sequence with the
# global threshold, timed the same way (one replanned HIP-graph step).
WORKLOADS = {
    "diffusion2d": dict(desc="2D var-coeff diffusion {m}x{m} (n={n}), {k} sources mapped to A_0, pattern S(A_k^2) "
                             "recomputed per source, FP32 QR + FP64 refinement, one HIP graph",
                        spec={}, pattern="S(A_k^2)"),
    "convdiff3d": dict(desc="3D upwind convection-diffusion 64^3 (n={n}), Pe 1..100, {k} sources mapped to A_0, "
                            "pattern S(A_k^2) recomputed per source, FP32 QR + FP64 refinement, one HIP graph",
                       spec={}, pattern="S(A_k^2)"),
    "convdiff3d_tau": dict(desc="3D upwind convection-diffusion 64^3 (n={n}), {k} sources, column threshold "
                                "tau=0.85 then S(A~_k^2) recomputed per source, FP32 QR + FP64 refinement, one HIP graph",
                           spec={"kind": "column", "tau": 0.85}, pattern="S(A~_k^2), column tau 0.85"),
    "ninepoint2d": dict(desc="2D 9-point lognormal couplings 1024x1024 (n={n}), {k} sources, global threshold 0.1 "
                             "then S(A~_k^2) recomputed per source, FP32 QR + FP64 refinement, one HIP graph",
                        spec={"kind": "global", "thresh": 0.1}, pattern="S(A~_k^2), global threshold 0.1"),
}


def make_inputs(P, name, grid=512):
    if name == "diffusion2d":
        return P.config2(m=grid, nmat=8)
    if name.startswith("convdiff3d"):
        return P.config3()
    return P.config4()


def tune_order(ctx, dAk0, dA0, prec, power, spec, reps=5):
    """The autotuner's variant order for a (precision, pattern) pair, timed
    on the first source's plan on this GPU (not cached)."""
    from paper_2406_17656_amd import autotune
    cp, ri = ctx.pattern(dAk0, power, **spec)
    pl = ctx.plan(dAk0, dA0, cp, ri)
    res = autotune.tune(pl, dAk0.val, dA0.val, prec, reps=reps, use_cache=False)
    pl.close()
    return res


def step_sequence(ctx, dA0, dAk0, nmaps, prec, power, spec, order, replan=True, vals=None):
    """The timed step: every source's pattern, plan, build and residual in
    one graph-captured sequence, with the given variant order, or (sources'
    values given, replanned) the order the sequence-level autotuner picks
    starting from it."""
    from paper_2406_17656_amd import autotune
    seq = ctx.sequence(dA0, dAk0, nmaps, prec=prec, power=power, replan_each_run=replan, **spec)
    seq.select(autotune.complete(order, prec))
    if vals is not None and replan:
        seq.tuned = autotune.tune_sequence(seq, vals, order, prec)
    return seq


def adjoint_variant(ctx, P, torch, log, reps=10):
    """The 48^3 adjoint workload: 7-point diffusion with lognormal(0, 0.5)
    coefficients, soft weights on the level-2 candidates (1 on S(A) and the
    diagonal); the weighted forward and the backward timed with HIP events on
    the library's stream, with their algorithmic flops."""
    from paper_2406_17656_amd import DeviceCSC
    log("timing: adjoint, 48^3 diffusion, weighted forward and backward")
    A0c, A1c = P.config5()
    dA0c, dA1c = DeviceCSC.from_host(A0c), DeviceCSC.from_host(A1c)
    cp5, ri5 = ctx.pattern(dA1c, 2)
    w5 = torch.as_tensor(P.candidate_weights(A1c.n, cp5.cpu().numpy(), ri5.cpu().numpy(), A1c),
                         dtype=torch.float64, device="cuda")
    mu5 = P.penalty_scale(A1c)
    pl5 = ctx.plan(dA1c, dA0c, cp5, ri5)
    timing = {}
    for name, call in (("forward", lambda: pl5.build_weighted(dA1c.val, dA0c.val, w5, mu5, "f32")),
                       ("backward", lambda: pl5.backward(dA1c.val, dA0c.val, w5, mu5, 1.0, "f32"))):
        call()
        ctx.sync_status()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)   # the library runs on torch's current stream
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        timing[name] = e0.elapsed_time(e1) / reps * 1e-3
    ctx.sync_status()
    adj = {"n": A1c.n, "nnz_S": int(ri5.numel())}
    for name, bwd in (("forward", False), ("backward", True)):
        c = pl5.cost_weighted("f32", backward=bwd)
        fl = c["flops32"] + c["flops64"]
        tf = fl / timing[name] / 1e12
        adj[f"{name}_ms"] = timing[name] * 1e3
        adj[f"{name}_cols_per_s"] = A1c.n / timing[name]
        adj[f"{name}_algorithmic_flops"] = fl
        adj[f"{name}_TFLOPs"] = tf
        adj[f"{name}_frac_fp32_peak"] = tf / PEAK["fp32_TFs"]
    adj["backward_over_forward"] = timing["backward"] / timing["forward"]
    pl5.close()
    return adj


def workload_variant(ctx, P, torch, log, name, steps=5, warmup=2):
    """Another replanned workload, timed like the step: the 1024^2 9-point
    sequence of 16 matrices (15 sources, global threshold 0.1 then level 2,
    ragged classes) or the 64^3 upwind convection-diffusion sequence (5
    sources, level 2, with or without the column threshold 0.85), with the
    autotuned classes, in one HIP graph."""
    from paper_2406_17656_amd import DeviceCSC
    spec = WORKLOADS[name]["spec"]
    A0h, Ash = make_inputs(P, name)
    dA0 = DeviceCSC.from_host(A0h)
    dAk = [DeviceCSC.from_host(A) for A in Ash]
    vals = [d.val for d in dAk]
    res = tune_order(ctx, dAk[0], dA0, "f32", 2, spec)
    seq = step_sequence(ctx, dA0, dAk[0], len(Ash), "f32", 2, spec, res["order"], vals=vals)
    Ms = seq.alloc_maps()
    res2 = torch.zeros(len(Ash), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        seq.run(vals, Ms, res2)
    ctx.sync_status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        seq.run(vals, Ms, res2)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ctx.sync_status()
    seq_order = seq.tuned["order"]
    seq.close()
    cols = A0h.n * len(Ash)
    log(f"{name}: {wall * 1e3:.2f} ms per step, {cols / wall / 1e6:.1f} M columns/s")
    return {"n": A0h.n, "maps": len(Ash), "cols_per_s": cols / wall, "ms_per_step": wall * 1e3,
            "order": seq_order[:4]}


def apply_variant(ctx, plan, dA0, dAk0, Scp, Sri, torch, reps=50):
    """y = M x for the first source's FP32 level-2 map (the product of a
    Krylov iteration), timed with HIP events: with M's values read through
    the row view's permutation, and with them put in row order once
    (sam_apply_permute).  Bytes: row pointers, column indices, values
    (and the permutation), x and y, each read or written once."""
    n = dA0.n
    M = torch.empty(max(Sri.numel(), 1), dtype=torch.float32, device="cuda")
    plan.build(dAk0.val, dA0.val, "f32", M=M, fro=False)
    T = ctx.apply_prepare(n, Scp, Sri)
    Tv = ctx.apply_permute(T, M, "f32")
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    nnz = int(Sri.numel())
    out = {"n": n, "nnz": nnz}
    for name, vals, permuted in (("perm", M, False), ("row_order", Tv, True)):
        ctx.apply(T, vals, x, "f32", y=y, permuted=permuted)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ctx.apply(T, vals, x, "f32", y=y, permuted=permuted)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        by = 4 * (n + 1) + 4 * nnz + 4 * nnz + (0 if permuted else 4 * nnz) + 8 * n + 8 * n
        out[f"{name}_us"] = us
        out[f"{name}_algorithmic_bytes"] = by
        out[f"{name}_hbm_frac"] = by / us / 1e3 / PEAK["hbm_GBs"]
    ctx.sync_status()
    return out


def level1_cold(ctx, P, torch, log, copies=7, rounds=6):
    """The level-1 (13 x 5 blocks) numeric build, the HBM-class case, on a
    working set larger than the 256 MB last-level cache: `copies` maps of the
    512 x 512 sequence, each with its own structure arrays, pattern, plan and
    output (about 47 MB of compulsory bytes each), built round-robin, so every
    launch finds its data evicted by the launches in between."""
    from paper_2406_17656_amd import DeviceCSC
    A0h, Ash = P.config2(m=512, nmat=copies + 1)
    maps = []
    for A in Ash[:copies]:
        dA, dA0 = DeviceCSC.from_host(A), DeviceCSC.from_host(A0h)   # separate copies of every array
        cp, ri = ctx.pattern(dA, 1)
        pl = ctx.plan(dA, dA0, cp, ri)
        maps.append((dA, dA0, cp, ri, pl))
    # the one-problem-per-lane class first (the autotuner's choice for level 1,
    # fixed here so that profiler runs, whose timings are perturbed, time the
    # same kernel)
    from paper_2406_17656_amd import autotune
    lane = next(v["index"] for v in autotune.menu("f32") if v["G"] == 1)
    order = autotune.complete([lane], "f32")
    outs = []
    for dA, dA0, cp, ri, pl in maps:
        pl.select(order, "f32")
        outs.append(torch.empty(max(ri.numel(), 1), dtype=torch.float32, device="cuda"))
    for (dA, dA0, cp, ri, pl), M in zip(maps, outs):
        pl.build(dA.val, dA0.val, "f32", M=M, fro=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(rounds):
        for (dA, dA0, cp, ri, pl), M in zip(maps, outs):
            pl.build(dA.val, dA0.val, "f32", M=M, fro=False)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / (rounds * copies) * 1e3
    by = maps[0][4].cost("f32")["bytes"]
    out = {"maps": copies, "launches": rounds * copies, "us_per_build": us, "algorithmic_bytes": by,
           "hbm_GBs": by / us / 1e3, "hbm_frac": by / us / 1e3 / PEAK["hbm_GBs"], "order": order[:3]}
    for m in maps:
        m[4].close()
    log(f"level-1 cold: {us:.1f} us per build, {out['hbm_GBs']:.0f} GB/s")
    return out


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def copy_calibration():
    """One device-to-device copy of 1 GiB (read 1 GiB, write 1 GiB): the
    reference the FETCH_SIZE / WRITE_SIZE counters are scaled by."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--roofline-only", action="store_true")
    ap.add_argument("--adjoint-only", action="store_true")
    ap.add_argument("--level1-cold", action="store_true")
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="diffusion2d")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): sharding the column "
              "problems across GPUs (contiguous column ranges, one halo exchange of A_k columns) "
              "is not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import numpy as np
    import torch

    import pde_inputs as P
    from paper_2406_17656_amd import Context, DeviceCSC

    if args.adjoint_only or args.level1_cold:
        ctx = Context(0)
        if args.adjoint_only:
            print(json.dumps({"adjoint_48cubed": adjoint_variant(ctx, P, torch, log)}), flush=True)
        else:
            print(json.dumps({"f32_level1_cold": level1_cold(ctx, P, torch, log)}), flush=True)
        torch.cuda.synchronize()
        ctx.close()
        return

    m = args.grid
    wl = WORKLOADS[args.workload]
    spec = wl["spec"]
    A0h, Ash = make_inputs(P, args.workload, m)
    n = A0h.n
    nmaps = len(Ash)
    cols = n * nmaps
    log(f"inputs ({args.workload}): n={n}, {nmaps} sources, nnz(A)={A0h.nnz}")
    if args.workload != "diffusion2d":
        args.no_variants = True
    ctx = Context(0)
    dA0 = DeviceCSC.from_host(A0h)
    dAk = [DeviceCSC.from_host(A) for A in Ash]
    vals = [d.val for d in dAk]
    torch.cuda.synchronize()
    a02 = float((A0h.val ** 2).sum())

    from paper_2406_17656_amd import autotune

    # autotuner: pick the kernel-variant order for each (precision, pattern)
    # on the first source's plan (timed on this GPU, not cached)
    tuned = {}

    def tuned_order(prec, power):
        if (prec, power) not in tuned:
            res = tune_order(ctx, dAk[0], dA0, prec, power, spec)
            tuned[(prec, power)] = res
            log(f"autotune {prec} level {power}: order {res['order'][:3]}..., {res['us']:.1f} us/map")
        return tuned[(prec, power)]["order"]

    seq_tuned = {}

    def time_sequence(prec, power, replan, steps, warmup):
        order = tuned_order(prec, power)
        seq = step_sequence(ctx, dA0, dAk[0], nmaps, prec, power, spec, order, replan, vals=vals)
        if replan:
            seq_tuned[(prec, power)] = seq.tuned["order"]
            log(f"sequence autotune {prec} level {power}: order {seq.tuned['order'][:3]}..., "
                f"{seq.tuned['ms']:.3f} ms per run")
        Ms = seq.alloc_maps()
        res2 = torch.zeros(nmaps, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            seq.run(vals, Ms, res2)
        ctx.sync_status()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            seq.run(vals, Ms, res2)
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        ev = e0.elapsed_time(e1) / steps * 1e-3
        ctx.sync_status()
        r2 = res2.cpu().numpy().copy()
        seq.close()
        return wall, ev, r2

    value = wall = None
    r2_f32 = None
    if not args.roofline_only:
        log("timing: replanned sequence, FP32+refine, S(A_k^2) (the step)")
        wall, ev, r2_f32 = time_sequence("f32", 2, True, args.steps, args.warmup)
        value = cols / wall
        log(f"step {wall * 1e3:.3f} ms (events {ev * 1e3:.3f} ms), {value / 1e6:.1f} M columns/s")

    # dominant kernel: the variant that serves most columns under the tuned
    # order, selected alone so that one launch covers every column of the map
    Scp, Sri = ctx.pattern(dAk[0], 2, **spec)
    plan = ctx.plan(dAk[0], dA0, Scp, Sri)
    # (the order of the timed step when it was tuned on the whole sequence)
    order32 = seq_tuned.get(("f32", 2)) or tuned_order("f32", 2)
    plan.select(order32, "f32")
    bcols = plan.info()["bucket_cols"]
    dom_idx = order32[max(range(len(bcols)), key=lambda b: bcols[b])]
    dom = autotune.menu("f32")[dom_idx]
    from paper_2406_17656_amd import SamError
    try:
        plan.select([dom_idx], "f32")
        single = True
    except SamError:   # some column needs a wider variant: the dominant one first, then the rest
        plan.select([dom_idx] + [v for v in order32 if v != dom_idx], "f32")
        single = False
    cost = plan.cost("f32")
    info = plan.info()
    variant = f"float,{dom['G']},{dom['R']},{dom['NC']},{dom['TC']}"
    kname = f"k_numeric<float, {dom['G']}, {dom['R']}, {dom['NC']}, {dom['TC']}, ...>"

    def time_build(prec, reps=20, fro=True):
        M = torch.empty(max(Sri.numel(), 1), dtype=torch.float32 if prec == "f32" else torch.float64,
                        device="cuda")
        c = torch.empty(n, dtype=torch.float64, device="cuda")
        r = torch.empty(1, dtype=torch.float64, device="cuda") if fro else None
        for _ in range(3):
            plan.build(dAk[0].val, dA0.val, prec, M=M, col_res2=c, res2=r, fro=fro)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)   # the library runs on torch's current stream
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.build(dAk[0].val, dA0.val, prec, M=M, col_res2=c, res2=r, fro=fro)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    kern_ms = time_build("f32", fro=False)
    flops = cost["flops32"] + cost["flops64"]
    achieved_tf = flops / (kern_ms * 1e-3) / 1e12
    achieved_gbs = cost["bytes"] / (kern_ms * 1e-3) / 1e9
    traffic = measured_traffic(variant)
    log(f"dominant kernel {kname}: {kern_ms * 1e3:.1f} us/launch, {achieved_tf:.2f} TFLOP/s, "
        f"{achieved_gbs:.0f} GB/s, traffic {traffic}")
    roofline = {"bound": "alu", "achieved": achieved_tf, "peak": PEAK["fp32_TFs"], "unit": "TFLOP/s",
                "frac": achieved_tf / PEAK["fp32_TFs"], "traffic": traffic,
                "kernel": kname + (" (one launch over all columns of one map)" if single else
                                   " first, with the other buckets' launches (no single-variant fit)"),
                "kernel_us": kern_ms * 1e3, "algorithmic_flops": flops,
                "algorithmic_bytes": cost["bytes"], "hbm_GBs": achieved_gbs,
                "hbm_frac": achieved_gbs / PEAK["hbm_GBs"],
                "traffic_hbm_GBs": None if traffic is None else traffic / (kern_ms * 1e-3) / 1e9}
    if args.roofline_only:
        print(json.dumps({"roofline": roofline, "variant": variant}), flush=True)
        plan.close()
        torch.cuda.synchronize()
        ctx.close()
        return
    plan.select(order32, "f32")
    build_ms = time_build("f32")

    variants = {"f32_level2_replanned": {"cols_per_s": value, "ms_per_step": wall * 1e3},
                "f32_level2_numeric_build_us": build_ms * 1e3}
    eq = None
    level_r2 = {}
    if not args.no_variants:
        plan.select(tuned_order("f64", 2), "f64")
        b64 = time_build("f64")
        variants["f64_level2_numeric_build_us"] = b64 * 1e3
        plan.select(order32, "f32")
        log("timing: y = M x on the first map (sam_apply)")
        variants["f32_level2_apply"] = apply_variant(ctx, plan, dA0, dAk[0], Scp, Sri, torch)
        plan.close()
        for prec in ("f32", "f64"):
            for power in (1, 2):
                log(f"timing: static sequence {prec} level {power}")
                w, e, r2 = time_sequence(prec, power, False, max(5, args.steps // 2), 2)
                variants[f"{prec}_level{power}_static"] = {"cols_per_s": cols / w, "ms_per_step": w * 1e3}
                if prec == "f32":
                    level_r2[power] = r2
                if prec == "f64" and power == 2:
                    r2_f64 = r2
        w, e, _ = time_sequence("f64", 2, True, max(5, args.steps // 2), 2)
        variants["f64_level2_replanned"] = {"cols_per_s": cols / w, "ms_per_step": w * 1e3}
        # level 1 (13 x 5 blocks) is the case that HBM could bound: the
        # numeric launches of one map alone (no Frobenius sum), tuned order
        log("timing: level-1 numeric build alone")
        cp1, ri1 = ctx.pattern(dAk[0], 1, **spec)
        pl1 = ctx.plan(dAk[0], dA0, cp1, ri1)
        pl1.select(tuned_order("f32", 1), "f32")
        M1 = torch.empty(max(ri1.numel(), 1), dtype=torch.float32, device="cuda")
        for _ in range(3):
            pl1.build(dAk[0].val, dA0.val, "f32", M=M1, fro=False)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            pl1.build(dAk[0].val, dA0.val, "f32", M=M1, fro=False)
        e1.record()
        torch.cuda.synchronize()
        us1 = e0.elapsed_time(e1) / 20 * 1e3
        # The map's 47 MB fit in the 256 MB last-level cache (MALL), so the
        # repeated launches above read much of it from there.  Cold: a 1 GiB
        # write before each launch evicts L2 and the MALL, and each launch is
        # timed alone, so its bytes come from HBM.
        # The same one-launch bracket without the flush gives the bracket's own
        # overhead (warm_single_us against us); cold_kernel_us takes it off.
        flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        cold = warm1 = 0.0
        for flushed in (True, False):
            for _ in range(10):
                if flushed:
                    flush.fill_(1.0)
                e0.record()
                pl1.build(dAk[0].val, dA0.val, "f32", M=M1, fro=False)
                e1.record()
                torch.cuda.synchronize()
                if flushed:
                    cold += e0.elapsed_time(e1)
                else:
                    warm1 += e0.elapsed_time(e1)
        del flush
        us1c = cold / 10 * 1e3
        us1k = us1c - (warm1 / 10 * 1e3 - us1)
        by1 = pl1.cost("f32")["bytes"]
        variants["f32_level1_numeric_build"] = {"us": us1, "algorithmic_bytes": by1,
                                                "hbm_GBs": by1 / us1 / 1e3,
                                                "hbm_frac": by1 / us1 / 1e3 / PEAK["hbm_GBs"],
                                                "cold_us": us1c,
                                                "warm_single_us": warm1 / 10 * 1e3,
                                                "cold_kernel_us": us1k,
                                                "cold_hbm_GBs": by1 / us1k / 1e3,
                                                "cold_hbm_frac": by1 / us1k / 1e3 / PEAK["hbm_GBs"]}
        pl1.close()
        eq = float(max(abs(a - b) / b for a, b in zip(r2_f32, r2_f64)))
        # the one-shot API (pattern, plan with host syncs and allocation, build) per map
        # the plain GPU build: per map the pattern, the plan (host
        # synchronisation, default variant order) and the build, one launch
        # after the other with no graph, in FP64 and in FP32 + refinement
        for prec in ("f64", "f32"):
            log(f"timing: plain per-map build ({prec})")
            for rep in range(2):       # the first pass warms the allocator
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for k, A in enumerate(dAk):
                    cp, ri = ctx.pattern(A, 2)
                    pl = ctx.plan(A, dA0, cp, ri)
                    pl.build(A.val, dA0.val, prec)
                    pl.close()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            variants[f"{prec}_level2_plain_per_map"] = {"cols_per_s": cols / dt, "ms_per_step": dt * 1e3}
        f64_plain = variants["f64_level2_plain_per_map"]["cols_per_s"]
        variants["ratios"] = {
            "f32_replanned_graph_vs_f64_plain_per_map": value / f64_plain,
            "f32_vs_f64_replanned_graph_same_batching": value / variants["f64_level2_replanned"]["cols_per_s"],
            "f32_vs_f64_numeric_build_same_batching": variants["f64_level2_numeric_build_us"] / (build_ms * 1e3),
            "f32_vs_f64_static_same_batching": variants["f32_level2_static"]["cols_per_s"] /
            variants["f64_level2_static"]["cols_per_s"],
        }
        # adaptive patterns on the first source: level 1 plus, per column, the
        # k level-2 candidates with the most negative dL/dw (weights 0.1)
        from paper_2406_17656_amd.adaptive import adaptive_map
        log("adaptive patterns: level 1 + top-k level-2 candidates by the adjoint")
        ad = {"level1": {"nnz": None, "rel_res": float(np.sqrt(level_r2[1][0] / a02))},
              "level2": {"nnz": None, "rel_res": float(np.sqrt(level_r2[2][0] / a02))}}
        for p_, key in ((1, "level1"), (2, "level2")):
            ad[key]["nnz"] = int(ctx.pattern(dAk[0], p_)[1].numel())
        for kk in (1, 2, 4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cp, ri, M, r2a, _ = adaptive_map(ctx, dAk[0], dA0, kk, w_cand=0.1, prec="f32")
            ctx.sync_status()
            dt = time.perf_counter() - t0
            ad[f"level1_plus_top{kk}"] = {"nnz": int(ri.numel()), "rel_res": float(np.sqrt(float(r2a.cpu()[0]) / a02)),
                                          "ms_whole_pipeline": dt * 1e3}
        variants["adaptive_map0"] = ad
        variants["adjoint_48cubed"] = adjoint_variant(ctx, P, torch, log)
        log("timing: 1024^2 9-point sequence, global threshold 0.1 then level 2 (ragged classes)")
        variants["f32_ninepoint_1024_replanned"] = workload_variant(ctx, P, torch, log, "ninepoint2d")
        log("timing: 64^3 upwind convection-diffusion sequence, level 2, without and with tau = 0.85")
        variants["f32_convdiff3d_64_replanned"] = workload_variant(ctx, P, torch, log, "convdiff3d")
        variants["f32_convdiff3d_tau_64_replanned"] = workload_variant(ctx, P, torch, log, "convdiff3d_tau")
    else:
        plan.close()
    rel_res = [float(np.sqrt(r / a02)) for r in r2_f32]

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O

        def oracle_rate(seconds):
            t0 = time.perf_counter()
            done = 0
            while time.perf_counter() - t0 < seconds:
                for A in Ash:
                    S = O.pattern(A, 2, **spec)
                    O.sam_build(A, A0h, S)
                    done += n
                    if time.perf_counter() - t0 > seconds:
                        break
            tc = time.perf_counter() - t0
            return done / tc, done // n, tc

        nthreads = O.num_threads()
        log(f"cpu baseline: oracle on the same sequence, {nthreads} threads")
        v_all, maps_all, t_all = oracle_rate(10.0)
        log("cpu baseline: oracle, 1 thread")
        O.set_num_threads(1)
        v_one, maps_one, t_one = oracle_rate(8.0)
        O.set_num_threads(nthreads)
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
        except OSError:
            pass
        cpu = {"value": v_all, "unit": "columns/s", "cores": nthreads, "kind": "oracle",
               "sample": f"{maps_all} maps of the same sequence ({nmaps} sources, cycled): pattern + FP64 "
                         f"Householder build of every column, {t_all:.1f} s",
               "value_1thread": v_one,
               "sample_1thread": f"{maps_one} maps, {t_one:.1f} s, 1 thread",
               "host": {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}}

    out = {
        "metric": "SAM columns/sec (whole path per map: level-2 pattern, plan, FP32+FP64-refine build, residual)",
        "value": value,
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64refine",
        "data": "synthetic",
        "config": {"workload": wl["desc"].format(m=m, n=n, k=nmaps),
                   "n": n, "maps": nmaps, "pattern": wl["pattern"],
                   "max_rows": info["max_rows"], "max_cols": info["max_cols"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
        "autotuned_variant_order": {f"{p}_level{l}": v["order"][:4] for (p, l), v in tuned.items()},
        "sequence_tuned_variant_order": {f"{p}_level{l}": v[:4] for (p, l), v in seq_tuned.items()},
        "equal_residual_max_rel_diff_f32_vs_f64": eq,
        "relative_residual_per_map": rel_res,
    }
    print(json.dumps(out), flush=True)
    torch.cuda.synchronize()
    ctx.close()


if __name__ == "__main__":
    main()
