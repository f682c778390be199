"""The library's host code (planner, layout, argument checks, autotuner set-up)
built with AddressSanitizer and UndefinedBehaviorSanitizer on the host side only
(device code unchanged), and the C-ABI tests run against that build in a child
process that preloads the sanitizer runtime. No kernel is launched: the ABI
tests are host-only."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
                  + glob.glob("/opt/rocm/llvm/lib/clang/*/lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so"))
    return hits[-1] if hits else None


def test_abi_tests_under_host_sanitizers(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("clang sanitizer runtime not installed")
    lib = str(tmp_path / "libvalmod_san.so")
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2008_13447_amd", "csrc", "*.hip")))
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared",
                           "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                           "-I", os.path.join(ROOT, "include")] + srcs + ["-o", lib],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    env = dict(os.environ, LD_PRELOAD=rt, VALMOD_TEST_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu"], env=env, cwd=ROOT, capture_output=True,
                       text=True, timeout=900)
    assert p.returncode == 0, p.stdout[-3000:] + p.stderr[-3000:]
