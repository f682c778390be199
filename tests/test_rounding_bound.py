"""The rounding bound of the diagonal recurrence against an emulation of the
pass's arithmetic (CPU).

The pass selects candidates with the co-moment recurrence of Alg.
ComputeMatrixProfile in FP32 or FP64 and widens every threshold by a per-item
bound of its rounding (valmod_rounding_bound, exported by the HIP library as a
host function). Here the recurrence of one work item is replayed with the
pass's roundings: FP64 statistics and inputs, one rounding per FMA (exact
rational arithmetic for FP64; an exact product and a 64-bit-mantissa sum for
FP32), FP32 copies of the inputs on the FP32 path. Every cell's correlation is
compared with a direct evaluation in extended precision. Items sit next to flat
stretches of a series at offset 1e4 (low-deviation windows, the case that makes
the bound large), and away from them.
"""
from fractions import Fraction

import numpy as np
import pytest


def _series():
    """1e4 + random walk (FP32) with two flat stretches (increments zeroed)."""
    g = np.random.default_rng(20080001)
    n = 4000
    inc = g.standard_normal(n)
    inc[1200:1800] = 0.0
    inc[2600:3200] = 0.0
    x = (1.0e4 + np.cumsum(inc)).astype(np.float32)
    return x.astype(np.float64)


def _stats(xs, L):
    """Window statistics as the window-prep kernel forms them (anchored sums, FP64)."""
    n = xs.shape[0]
    N = n - L + 1
    x0 = xs[:N]
    a = np.zeros(N)
    b = np.zeros(N)
    for k in range(1, L):
        d = xs[k:k + N] - x0
        a = a + d
        b = d * d + b
    m = a / L
    v = np.maximum(b / L - m * m, 0.0)
    s = np.sqrt(v)
    mu = x0 + m
    flat = s <= 2.0 ** -20 * np.maximum(1.0, np.abs(mu))
    inv = np.zeros(N)
    inv[~flat] = 1.0 / (s[~flat] * np.sqrt(float(L)))
    df = np.zeros(N)
    dg = np.zeros(N)
    df[:N - 1] = 0.5 * (xs[L:L + N - 1] - xs[:N - 1])
    dg[:N - 1] = (xs[L:L + N - 1] - mu[1:N]) + (xs[:N - 1] - mu[:N - 1])
    return a, mu, s, inv, flat, df, dg


def _exact_rho(xs, L, i, j):
    """Correlation of windows i and j evaluated directly in extended precision."""
    wi = xs[i:i + L].astype(np.longdouble)
    wj = xs[j:j + L].astype(np.longdouble)
    ci = wi - wi.sum() / L
    cj = wj - wj.sum() / L
    return float((ci * cj).sum() / np.sqrt((ci * ci).sum() * (cj * cj).sum()))


def _fma64(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _fma32(a, b, c):
    p = np.longdouble(np.float32(a)) * np.longdouble(np.float32(b))  # exact (48 bits)
    return np.float32(p + np.longdouble(np.float32(c)))


def _emulate(xs, L, i0, d0, H, BW, precision):
    """Max |rho computed - rho| over the cells of one item (rows i0..i0+H-1,
    diagonals d0..d0+BW-1), and the item's bound parameters (phi, psi, xi)."""
    a, mu, s, inv, flat, df, dg = _stats(xs, L)
    N = mu.shape[0]
    sw = s * np.sqrt(float(L))
    rows = np.arange(i0, min(i0 + H + 1, N))
    cols = np.arange(i0 + d0, min(i0 + d0 + H + BW + 1, N))
    rnf, cnf = rows[~flat[rows]], cols[~flat[cols]]
    phi = (sw[rnf].max() / sw[rnf].min()) * (sw[cnf].max() / sw[cnf].min())
    dfr, dgr, dfc, dgc = (np.abs(df[rows]).max(), np.abs(dg[rows]).max(), np.abs(df[cols]).max(),
                          np.abs(dg[cols]).max())
    psi = (dfr * dgc + dgr * dfc) / (sw[rnf].min() * sw[cnf].min())
    xi = (dfr + dfc) * max(np.abs(mu[rows]).max(), np.abs(mu[cols]).max()) / (sw[rnf].min() * sw[cnf].min())
    worst = 0.0
    f32 = precision == "fp32"
    ai = a[i0] / L
    for q in range(BW):
        d = d0 + q
        j = i0 + d
        if j >= N:
            break
        # anchor: FP64 FMA chain of the anchored products, then the co-moment
        S = 0.0
        for k in range(1, L):
            S = _fma64(xs[i0 + k] - xs[i0], xs[j + k] - xs[j], S)
        C = S - ai * a[j]
        C = np.float32(C) if f32 else C
        for r in range(H):
            i = i0 + r
            jj = i + d
            if jj >= N:
                break
            if not flat[i] and not flat[jj]:
                if f32:
                    rho = float(np.float32(np.float32(C * np.float32(inv[jj])) * np.float32(inv[i])))
                else:
                    rho = (C * inv[jj]) * inv[i]
                worst = max(worst, abs(rho - _exact_rho(xs, L, i, jj)))
            if f32:
                C = _fma32(np.float32(df[i]), np.float32(dg[jj]), C)
                C = _fma32(np.float32(df[jj]), np.float32(dg[i]), C)
            else:
                C = _fma64(df[i], dg[jj], C)
                C = _fma64(df[jj], dg[i], C)
    return worst, phi, psi, xi


ITEMS = [
    # (name, i0, d0, H, BW). Rows at the end of the first flat stretch (windows
    # with a single non-flat point, sigma down to 0.017 at level 1e4) against
    # columns at the end of the second one: phi ~ 4e4, the FP32 bound exceeds 1
    # (such items run in FP64) and the FP64 bound is ~7e-8.
    ("next to flats", 1590, 1400, 128, 16),
    ("wider item next to flats", 1595, 1405, 256, 32),
    ("random walk", 300, 500, 128, 16),
]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name,i0,d0,H,BW", ITEMS, ids=[t[0] for t in ITEMS])
def test_recurrence_error_within_bound(precision, name, i0, d0, H, BW):
    from paper_2008_13447_amd import native

    xs = _series()
    L = 200
    worst, phi, psi, xi = _emulate(xs, L, i0, d0, H, BW, precision)
    bound = native.valmod_rounding_bound(precision, H, L, phi, psi, xi)
    assert worst <= bound, (name, precision, worst, bound)
    assert worst > 0.0


def test_bound_host_function_domain():
    from paper_2008_13447_amd import native

    assert np.isnan(native.valmod_rounding_bound("fp32", 0, 100, 1.0, 1.0, 1.0))
    assert np.isnan(native.valmod_rounding_bound("fp64", 64, 100, -1.0, 1.0, 1.0))
    b32 = native.valmod_rounding_bound("fp32", 256, 100, 2.0, 3.0, 1.0)
    b64 = native.valmod_rounding_bound("fp64", 256, 100, 2.0, 3.0, 1.0)
    assert 0.0 < b64 < b32 < 1e-2
    assert native.valmod_rounding_bound("fp64", 512, 100, 2.0, 3.0, 1.0) > b64
