"""The pass's step test against the per-cell test it replaces (CPU emulation in
the pass's precisions).

Per step and lane the pass takes the largest C_q invn_j(q) over the lane's K
cells, scales it by the row's inverse norm and raises it by the item's rounding
bound with one rounding, and compares that with the smallest threshold the
lane's cells can have (a running minimum of the column thresholds of the block,
and the row's). A cell that passes its own test (its correlation raised by the
bound, against the smaller of its two owners' thresholds) must make the step
pass, in FP32 (flat windows carry a NaN inverse norm that the maximum ignores)
and in FP64 (flat windows carry 0). The fused multiply-add is emulated exactly
(an exact product and sum in rationals, then one rounding).
"""
from fractions import Fraction

import numpy as np
import pytest


def _fma(a, b, c, dt):
    """One rounding of a * b + c in `dt` (the inputs are `dt` values)."""
    if not (np.isfinite(a) and np.isfinite(b) and np.isfinite(c)):
        return dt(np.float64(a) * np.float64(b) + np.float64(c))
    return dt(float(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))))


def _fmax(a, b, dt):
    """IEEE maxNum: a NaN operand yields the other one."""
    if np.isnan(a):
        return b
    if np.isnan(b):
        return a
    return dt(max(a, b))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_step_test_passes_whenever_a_cell_does(dt):
    g = np.random.default_rng(20081347)
    K = 8
    flat_inv = dt(np.nan) if dt is np.float32 else dt(0.0)
    trials = cells_passing = 0
    for _ in range(4000):
        C = (g.standard_normal(K) * g.uniform(0.1, 10.0)).astype(dt)
        inv = (g.uniform(0.05, 1.0, K) / g.uniform(0.5, 20.0)).astype(dt)
        inv[g.random(K) < 0.1] = flat_inv
        rinv = dt(g.uniform(0.05, 1.0) / g.uniform(0.5, 20.0))
        delta = dt(g.choice([0.0, 1e-7, 1e-3, 5e-3]))
        thr_j = g.uniform(-0.2, 1.0, K).astype(dt)
        thr_i = dt(g.uniform(-0.2, 1.0))
        # the lane's threshold: a minimum over a superset of its cells' column thresholds
        extra = g.uniform(-0.2, 1.0, int(g.integers(0, 8))).astype(dt)
        tcol = dt(min(np.min(thr_j), np.min(extra) if extra.size else np.inf))
        per_cell = [_fma(dt(C[q] * inv[q]), rinv, delta, dt) >= min(thr_j[q], thr_i) for q in range(K)]
        m = dt(np.nan)
        for q in range(K):
            m = _fmax(m, dt(C[q] * inv[q]), dt)
        step = bool(_fma(m, rinv, delta, dt) >= min(tcol, thr_i)) if not np.isnan(m) else False
        trials += 1
        cells_passing += sum(per_cell)
        if any(per_cell):
            assert step, (C, inv, rinv, delta, thr_j, thr_i)
    assert cells_passing > 100  # the sample exercises passing cells
