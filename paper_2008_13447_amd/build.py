"""Build the VALMOD HIP library for gfx950 (in-tree, no JIT cache).

``build_native()`` compiles every ``csrc/*.hip`` source with hipcc into
``libvalmod.so`` next to this file. Packed FP32 instructions are disabled for
all device code (``-packed-fp32-ops``).
"""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libvalmod.so")
ARCH = os.environ.get("VALMOD_OFFLOAD_ARCH", "gfx950")


def hipcc_command(out: str = LIB):
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    return (["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]
            + srcs + ["-o", out])


def build_native() -> str:
    """Compile libvalmod.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(hipcc_command(tmp))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_native())
