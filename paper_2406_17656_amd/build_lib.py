"""Builds libsam_mi355x.so (HIP for gfx950) in place, next to this file.

Every translation unit is compiled by hipcc for gfx950 with packed-FP32
instructions disabled; objects go to ``_build/`` (not committed).  Run as a
script or call ``build(force=True)``.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsam_mi355x.so")
ARCH = "gfx950"

SOURCES = ["sam_symbolic.hip", "sam_numeric.hip", "sam_aux.hip", "sam_adjoint.hip", "sam_adaptive.hip", "sam_capi.cpp",
           "sam_sequence.cpp", "sam_backward.cpp", "sam_adaptive_api.cpp", "sam_noalloc.cpp"]
HEADERS = ["sam_device.hpp", "sam_kernels.hpp", "sam_numeric_args.hpp", "sam_host.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", INCLUDE, "-I", CSRC,
]


def _stale(obj: str, src: str) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(INCLUDE, "sam.h")]
    return any(os.path.getmtime(d) > t for d in deps)


_REMARK = re.compile(r"remark: +(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]): (\S+) \[-Rpass-analysis")


def _resources(stderr: str) -> dict:
    """Per-kernel register, scratch, occupancy and LDS figures from the
    compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for m in _REMARK.finditer(stderr):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[key.split(" [")[0]] = int(val) if val.isdigit() else val
    return out


def resource_file(src: str) -> str:
    return os.path.join(OBJDIR, os.path.splitext(src)[0] + ".resources.json")


def _compile(src: str, force: bool) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    if force or _stale(obj, path):
        cmd = [HIPCC] + CFLAGS + ["-Rpass-analysis=kernel-resource-usage", "-x", "hip", "-c", path,
                                  "-o", obj + ".tmp"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        os.replace(obj + ".tmp", obj)
        with open(resource_file(src), "w") as f:
            json.dump(_resources(r.stderr), f, indent=0, sort_keys=True)
    return obj


def build(force: bool = False, jobs: int = 4) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), srcs))
    if force or not os.path.exists(LIB) or any(os.path.getmtime(o) > os.path.getmtime(LIB) for o in objs):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, LIB)
    return LIB


HOST_SOURCES = ["sam_capi.cpp", "sam_sequence.cpp", "sam_backward.cpp", "sam_adaptive_api.cpp", "sam_noalloc.cpp"]
ASAN_DIR = os.path.join(OBJDIR, "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libsam_mi355x_asan.so")


def build_host_sanitized(jobs: int = 5) -> str:
    """The library with its host code (the C ABI translation units) built
    with AddressSanitizer and UndefinedBehaviorSanitizer, linked with the
    regular kernel objects: for the host-side tests, which run without a
    GPU.  The sanitizers apply to host code only (each -fsanitize= follows
    -Xarch_host)."""
    build()
    os.makedirs(ASAN_DIR, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]

    def one(src):
        obj = os.path.join(ASAN_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + CFLAGS + san + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc (sanitized) failed for {src}:\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, HOST_SOURCES))
    kernels = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES if s not in HOST_SOURCES]
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-o", ASAN_LIB] + objs + kernels
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (sanitized) failed:\n{r.stdout}\n{r.stderr}")
    return ASAN_LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
