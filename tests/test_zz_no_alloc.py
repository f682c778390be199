"""The allocation-free entry point valmod_run_noalloc (static device scratch)
against valmod_run on the same plans, through the C ABI: two calls in a row,
the second with a smaller input, each compared with valmod_run's outputs
(distances within 1e-9 of d / sqrt(L), indices equal except ties) and with the
oracle."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2008_13447_amd import gen

pytestmark = pytest.mark.gpu

TOL64 = 1e-9


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_run(precision):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from oracle import compare
    from paper_2008_13447_amd import native

    oracle.build(force=False)
    L_ = native.lib()
    stream = torch.cuda.current_stream().cuda_stream
    for call, (n, lo, hi, seed) in enumerate([(3000, 40, 46, 70), (1500, 24, 30, 71)]):
        _say(f"noalloc call {call}: {precision} n={n} L={lo}..{hi}")
        x = gen.small_random_walk(n, seed, np.float32)
        v = native.Valmod(torch.from_numpy(x).cuda(), lo, hi, p=5, k_motifs=3, k_discords=3,
                          precision=precision, path="full")
        assert native.valmod_workspace_bytes(v.plan) <= (64 << 20)
        v.run()
        ref = v.result(0)
        # fresh outputs, no workspace: the static scratch of the entry point
        for t in v.out.values():
            if t is not None:
                t.fill_(-7)
        rc = L_.valmod_run_noalloc(ctypes.c_void_p(v.plan), ctypes.c_void_p(v.series.data_ptr()),
                                   ctypes.byref(v._outs), ctypes.c_void_p(stream))
        assert rc == 0, native.STATUS.get(rc, rc)
        rc = L_.valmod_run_status(ctypes.c_void_p(v.plan), ctypes.c_void_p(stream))
        assert rc == 0, native.STATUS.get(rc, rc)
        got = v.result(0)
        v.close()
        # against valmod_run's outputs (the reference entry point)
        rep = compare.check_full(x, lo, got, ref, TOL64)
        _say(f"noalloc call {call}: vs valmod_run {dict(rep)}")
        # and against the oracle
        r = oracle.valmod(x, lo, hi, k_motifs=3, k_discords=3)
        compare.check_full(x, lo, got, r, TOL64)
