"""Host-side AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only):
the oracle built with both sanitizers runs its pin tests, and the library
with its C-ABI host code built with both (the kernels are the regular
objects) runs the host-side C-ABI tests.  Any report aborts the child run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_child(tests, env_extra, preload):
    if not os.path.exists(preload):
        pytest.skip(f"sanitizer runtime {preload} not found")
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] +
                       [os.path.join(ROOT, "tests", t) for t in tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error:" not in tail, tail


def test_oracle_under_asan_ubsan():
    import oracle
    lib = oracle.build(sanitize=True)
    preload = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    run_child(["test_oracle_ls.py", "test_oracle_pattern.py", "test_oracle_grad.py", "test_oracle_adaptive.py"],
              {"SAM_ORACLE_LIB": lib}, preload)


def test_capi_host_code_under_asan_ubsan():
    import glob
    from paper_2406_17656_amd import build_lib
    lib = build_lib.build_host_sanitized()
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's AddressSanitizer runtime not found")
    run_child(["test_capi_host.py"], {"SAM_MI355X_LIB": lib}, rt[-1])
