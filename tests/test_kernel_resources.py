"""Register and scratch budgets of the compiled kernels, from the compiler's
kernel-resource-usage remarks that the library build records.  A kernel that
spills to scratch, or a numeric variant that drops to one wave per SIMD, costs
a large factor in speed without changing any result, so no parity test would
notice it."""
import json
import os
import re

import pytest

from paper_2406_17656_amd import build_lib

NUMERIC = build_lib.resource_file("sam_numeric.hip")
SYMBOLIC = build_lib.resource_file("sam_symbolic.hip")
VARIANT = re.compile(r"k_numericI([fd])Li(\d+)ELi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)E")


def load(path):
    if not os.path.exists(path):
        pytest.skip("the library has not been built in this checkout")
    with open(path) as f:
        return json.load(f)


def numeric_variants():
    out = {}
    for name, res in load(NUMERIC).items():
        m = VARIANT.search(name)
        if m:
            t, G, R, NC, TC, LPL, MODE = m.groups()
            out[(t, int(G), int(R), int(NC), int(TC), int(LPL), int(MODE))] = res
    return out


def test_every_numeric_variant_was_recorded():
    v = numeric_variants()
    assert len(v) >= 30
    assert ("f", 4, 7, 13, 1, 2, 0) in v and ("f", 16, 4, 25, 1, 1, 0) in v


# Held to three waves per SIMD on purpose: a few loop-invariant values go to
# scratch, which costs less than the third wave gains.
THREE_WAVES = {("f", 16, 4, 25, 1, 1, 0): 32}


def test_numeric_kernels_do_not_spill():
    """No variant of any mode (plain, soft-weighted forward, adjoint) spills
    to scratch, except the bounded spill of the classes held to three waves
    per SIMD."""
    bad = {k: r["ScratchSize"] for k, r in numeric_variants().items()
           if r["ScratchSize"] > THREE_WAVES.get(k, 0)}
    assert not bad, bad


def test_classes_held_to_three_waves():
    v = numeric_variants()
    for k in THREE_WAVES:
        assert v[k]["Occupancy"] == 3 and v[k]["VGPRs"] <= 168, (k, v[k])


def test_fp32_weighted_and_adjoint_kernels_hold_two_waves_per_simd():
    """The soft-weighted forward and the adjoint in FP32 keep their length-NC
    vectors in LDS and roll their long-column loops, which leaves room for two
    waves per SIMD."""
    low = {k: r["Occupancy"] for k, r in numeric_variants().items()
           if k[0] == "f" and k[6] in (1, 2) and r["Occupancy"] < 2}
    assert not low, low


def test_plain_fp32_kernels_hold_two_waves_per_simd():
    # all but the 128-row class, which holds 32 lanes x 4 rows x 32 columns
    low = {k: r["Occupancy"] for k, r in numeric_variants().items()
           if k[0] == "f" and k[6] == 0 and k[1] * k[2] < 128 and r["Occupancy"] < 2}
    assert not low, low


def test_union_kernels_do_not_spill():
    res = load(SYMBOLIC)
    unions = {n: r for n, r in res.items() if "k_union" in n}
    assert unions
    bad = {n: r["ScratchSize"] for n, r in unions.items() if r["ScratchSize"]}
    assert not bad, bad
