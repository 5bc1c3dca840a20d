"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The C oracle, built with gcc -fsanitize=address,undefined, labels random
  lattices of every mask (edges 1..11, so every boundary case of the scan
  and the wraps) and must agree with the normal build.
* The library's host code -- argument checks, sizing and planning, the
  server's scheduler, arena and failure bookkeeping on its simulated
  device -- built with the sanitizers on the host side only (hipcc
  -Xarch_host before each -fsanitize=), runs the ABI and simulated-server
  tests.
Each run is a child process with the sanitizer runtime preloaded; any
report fails it (UBSan set not to recover, leak checking off: the Python
interpreter and the HIP runtime are not instrumented)."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1405_1931_amd", "csrc")
SANITIZE = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _run(cmd, env_extra, timeout=300):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    p = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, timeout=timeout)
    out = p.stdout + p.stderr
    assert p.returncode == 0 and "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not found")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.exists(asan):
        pytest.skip("gcc's ASan runtime not found")
    lib = str(tmp_path / "libhk_oracle_san.so")
    subprocess.run([gcc, "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", *SANITIZE, "-o", lib,
                    os.path.join(ROOT, "oracle", "hk_oracle.c")], check=True)
    script = f"""
import sys; sys.path.insert(0, {ROOT!r})
import numpy as np, oracle
san = oracle.load({lib!r})
ref = oracle.load()
rng = np.random.default_rng(0)
for t in range(400):
    shape = tuple(int(v) for v in rng.integers(1, 12, 3))
    phi = (rng.random(shape, dtype=np.float32) - rng.uniform(0.2, 0.9)).astype(np.float32)
    m = int(rng.integers(0, 8))
    a = oracle.label(phi, m, lib=san)
    b = oracle.label(phi, m, lib=ref)
    assert a[1] == b[1] and np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2]), (shape, m)
for shape in [(1, 1, 1), (1, 1, 2), (2, 2, 2), (1, 9, 1)]:
    for m in range(8):
        for v in (1.0, -1.0):
            oracle.label(np.full(shape, v, np.float32), m, lib=san)
print("ok")
"""
    out = _run([sys.executable, "-c", script], {"LD_PRELOAD": asan})
    assert "ok" in out


def test_host_library_under_asan_ubsan(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not os.path.exists(hipcc) or not rts:
        pytest.skip("hipcc or clang's ASan runtime not found")
    lib = str(tmp_path / "libhk_san.so")
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    host_only = [f for flag in SANITIZE for f in ("-Xarch_host", flag)]
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-pthread",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_only,
                    "-I", os.path.join(ROOT, "include"), "-o", lib, *srcs], check=True, capture_output=True)
    out = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                "tests/test_abi.py", "tests/test_server_sim.py"],
               {"LD_PRELOAD": rts[0], "HK_TEST_LIB": lib})
    assert " passed" in out and " failed" not in out, out[-2000:]
    # the tests ran against the sanitizer build
    out = _run([sys.executable, "-c",
                "import sys; sys.path.insert(0, 'tests'); import conftest; from paper_1405_1931_amd import _lib; "
                "_lib.load(); print(open('/proc/self/maps').read())"],
               {"LD_PRELOAD": rts[0], "HK_TEST_LIB": lib})
    assert lib in out
