"""The paper's experimental protocol (Section 5) as a sweep over a matrix
sequence: for every sparsification strategy and level, the pattern of every
map N_k, its number of entries (Tables 1-3) and the relative residual
||A_k N_k - A_0||_F / ||A_0||_F (the figures' curves).

Strategies (Section 4), each applied to the source A_k, then raised to the
level: "level 1" is S(A~_k^2) and "level 2" S(A~_k^3) in the experiments'
numbering (Section 5; the prose calls S(A) level 1), plus the baseline
S(A_0) of the earlier SAM work:

* ``S(A0)``                  -- pattern of the target;
* ``global t``               -- |a_ij| scaled by the diagonals above t
                                (t = 0.1, 0.01, 0.001, 1e-4);
* ``col tau``                -- |a_ij| > (1 - tau) max_i |a_ij| (tau = 0.6, 0.7, 0.8);
* ``lfil l``                 -- the diagonal and the l - 1 largest entries per column (l = 3, 5).

Every step runs in the library (pattern, plan, build, explicit residual);
this module only loops and tabulates.

    python -m paper_2406_17656_amd.sweep --grid 64 --maps 8 [--prec f32] [--json out.json]
"""
from __future__ import annotations

import argparse
import json
import math

STRATEGIES = ([("S(A0)", {})] +
              [(f"global {t:g}", {"kind": "global", "thresh": t}) for t in (0.1, 0.01, 0.001, 1e-4)] +
              [(f"col {tau:g}", {"kind": "column", "tau": tau}) for tau in (0.6, 0.7, 0.8)] +
              [(f"lfil {l}", {"kind": "lfil", "lfil": l}) for l in (3, 5)])
LEVELS = {"level 1": 2, "level 2": 3}   # the experiments' numbering -> power of S(A~)


def run(ctx, A0, As, prec="f32", strategies=STRATEGIES, levels=LEVELS):
    """A0, As: DeviceCSC target and sources.  Returns a list of rows
    {"strategy", "level", "nnz": [per map], "rel_res": [per map]}."""
    rows = []
    P0 = {}
    for name, spec in strategies:
        for lev, power in levels.items():
            if name == "S(A0)" and lev != "level 1":
                continue
            nnz, rel = [], []
            for Ak in As:
                if name == "S(A0)":
                    if "cp" not in P0:
                        P0["cp"], P0["ri"] = ctx.pattern(A0, 1)
                    cp, ri = P0["cp"], P0["ri"]
                else:
                    cp, ri = ctx.pattern(Ak, power, **spec)
                M, _, _ = ctx.build(Ak, A0, cp, ri, prec, want_cols=False)
                r2, a02 = ctx.residual(Ak, A0, cp, ri, M, prec)
                ctx.sync_status()
                nnz.append(int(ri.numel()))
                rel.append(math.sqrt(float(r2.cpu()[0]) / float(a02.cpu()[0])))
            rows.append({"strategy": name, "level": lev if name != "S(A0)" else "-", "nnz": nnz, "rel_res": rel})
    return rows


def markdown(rows, maps_shown=(0, 1, -1)) -> str:
    n = len(rows[0]["nnz"])
    idx = sorted(set(i % n for i in maps_shown))
    head = "| Strategy | Level | " + " | ".join(f"nnz N_{i + 1}" for i in idx) + " | " + \
           " | ".join(f"rel. res. N_{i + 1}" for i in idx) + " |"
    out = [head, "|" + "---|" * (2 + 2 * len(idx))]
    for r in rows:
        out.append(f"| {r['strategy']} | {r['level']} | " + " | ".join(str(r["nnz"][i]) for i in idx) + " | " +
                   " | ".join(f"{r['rel_res'][i]:.3e}" for i in idx) + " |")
    return "\n".join(out)


def main():
    import torch  # noqa: F401  (device memory)
    import pde_inputs as P
    from .sam import Context, DeviceCSC
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--maps", type=int, default=8)
    ap.add_argument("--prec", default="f32")
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    A0h, Ash = P.config2(m=args.grid, nmat=args.maps)
    ctx = Context(0)
    A0 = DeviceCSC.from_host(A0h)
    As = [DeviceCSC.from_host(A) for A in Ash]
    rows = run(ctx, A0, As, args.prec)
    print(markdown(rows))
    if args.json:
        with open(args.json, "w") as f:
            json.dump({"grid": args.grid, "maps": args.maps, "prec": args.prec, "rows": rows}, f)
    ctx.close()


if __name__ == "__main__":
    main()
