"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host only) and driven through every entry point on small inputs, edge cases
included, in a child process that preloads the sanitizer runtimes. Any invalid
access or undefined operation aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
import sys
import numpy as np
sys.path.insert(0, ROOT)
import oracle
oracle._LIB = LIB
oracle._lib = None
oracle.build = lambda force=False: oracle._LIB
from paper_2008_13447_amd import gen

x = gen.small_random_walk(420, 7)
for L in (8, 13):
    oracle.stats(x, L)
    oracle.profile(x, L, excl_den=2, nthreads=2)
    oracle.profile(x, L, rows=[0, 5, x.shape[0] - L], nthreads=1)
oracle.pair_dist(x, 12, 3, 200)
oracle.pair_dists(x, 12, [[3, 200], [10, 300]])
oracle.pearson(x, 12, 3, 200)
oracle.lb(x, 3, 200, 10, 14)
oracle.submp_decide(np.array([1.0, 2.0, np.inf]), np.array([0.5, 3.0, 1.0]))
oracle.valid_fraction(x, 10, 12, 3)
r = oracle.valmod(x, 10, 14, k_motifs=4, k_discords=4)
oracle.valmod(x, 10, 12, excl_den=2, k_motifs=2, k_discords=2)
oracle.mth_rows(x, 12, 3, rows=[0, 50])
oracle.mth_discords(x, 10, 12, 3, 3)
oracle.motif_sets(x, r["g_motif_abl"], r["g_motif_d"][:, 0], 4.0, 16)
# flat stretches, a series barely longer than the longest window, a constant series
y = gen.small_random_walk(300, 8) + 1.0e4
y[100:160] = y[100]
oracle.valmod(y, 12, 20, k_motifs=3, k_discords=3)
oracle.mth_discords(y, 12, 14, 2, 2)
z = gen.small_random_walk(40, 9)
oracle.valmod(z, 16, 19, k_motifs=2, k_discords=2)
oracle.valmod(np.full(64, 3.0), 8, 10, k_motifs=2, k_discords=2)
print("sanitized oracle run complete")
"""


def _runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-D_GNU_SOURCE", "-shared", "-fPIC",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           os.path.join(ROOT, "oracle", "valmod_oracle.c"), "-o", lib, "-lm", "-lpthread"])
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + DRIVER
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    assert "sanitized oracle run complete" in p.stdout
