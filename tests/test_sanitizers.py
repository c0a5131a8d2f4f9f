"""CPU builds under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle (plain C, gcc) driven through every entry point on seeded inputs,
and the HIP library's host code (hipcc, sanitizers on the host side only)
through the entry points that need no GPU.  Any sanitizer report fails the
test.  No GPU is used."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-std=c99", "-g", "-O1", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall", "-o", exe,
                           os.path.join(SAN, "oracle_main.c"), os.path.join(ROOT, "oracle", "scpl_oracle.c"), "-lm"])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ok" in r.stdout


def _asan_runtime():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    base = os.path.join(rocm, "llvm", "lib", "clang")
    if not os.path.isdir(base):
        return None
    for ver in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    rt = _asan_runtime()
    if not os.path.exists(hipcc) or rt is None or shutil.which("ld") is None:
        pytest.skip("hipcc or the clang sanitizer runtime is not installed")
    lib = str(tmp_path / "libscpl_san.so")
    csrc = os.path.join(ROOT, "paper_1903_03180_amd", "csrc")
    # device code is built as usual; the sanitizers apply to the host side only
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"), "-o", lib] + \
        [os.path.join(csrc, f) for f in ("scpl_kernels.hip", "scpl_host.hip", "scpl_server.hip")]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(SAN, "host_calls.py"), lib], capture_output=True, text=True,
                       timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "ok" in r.stdout
