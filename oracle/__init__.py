"""CPU FP64 brute-force oracle for VALMOD (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product path (``paper_2008_13447_amd``)
never does, and the two share no code: only the seeded input generators of
``paper_2008_13447_amd.gen`` (which hold none of the method's arithmetic) feed
both.

The arithmetic lives in ``valmod_oracle.c`` (plain C, double precision, threads
over owner rows); this module only marshals numpy arrays through ctypes. See the
header of the C file for the definitions followed and the readings taken.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "valmod_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
FLAT_EPS = 2.0 ** -20

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (no GPU involved)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-shared", "-fPIC",
                               _SRC, "-o", tmp, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    D = ctypes.c_double
    I64 = ctypes.c_int64
    P = ctypes.c_void_p
    lib.oracle_stats.argtypes = [P, I64, I64, D, P, P, P]
    lib.oracle_stats.restype = None
    lib.oracle_pair_dist.argtypes = [P, I64, I64, I64, I64, D]
    lib.oracle_pair_dist.restype = D
    lib.oracle_pearson.argtypes = [P, I64, I64, I64, I64, D]
    lib.oracle_pearson.restype = D
    lib.oracle_profile_rows.argtypes = [P, I64, I64, I64, D, P, I64, P, P, ctypes.c_int]
    lib.oracle_profile_rows.restype = ctypes.c_int
    lib.oracle_lb.argtypes = [P, I64, I64, I64, I64, I64, D]
    lib.oracle_lb.restype = D
    lib.oracle_submp_decide.argtypes = [I64, P, P, P, P, P]
    lib.oracle_submp_decide.restype = ctypes.c_int
    lib.oracle_valmod.argtypes = [P, I64, I64, I64, I64, D, I64, I64, ctypes.c_int] + [P] * 14
    lib.oracle_valmod.restype = ctypes.c_int
    lib.oracle_pair_dists.argtypes = [P, I64, I64, D, P, I64, P]
    lib.oracle_pair_dists.restype = ctypes.c_int
    lib.oracle_valid_fraction.argtypes = [P, I64, I64, I64, I64, I64, D, P]
    lib.oracle_valid_fraction.restype = I64
    lib.oracle_mth_rows.argtypes = [P, I64, I64, I64, D, I64, P, I64, P, P]
    lib.oracle_mth_rows.restype = ctypes.c_int
    lib.oracle_mth_discords.argtypes = [P, I64, I64, I64, I64, D, I64, I64, P, P, P, P]
    lib.oracle_mth_discords.restype = ctypes.c_int
    lib.oracle_motif_sets.argtypes = [P, I64, I64, P, P, D, I64, D, I64, P, P, P]
    lib.oracle_motif_sets.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(x) -> np.ndarray:
    # float32 inputs are widened exactly
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def stats(x, L: int, flat_eps: float = FLAT_EPS):
    """(mu, sigma, flat) of every window of length L (two-pass, population sigma)."""
    x = _f64(x)
    N = x.shape[0] - L + 1
    mu = np.empty(N)
    sg = np.empty(N)
    fl = np.empty(N, dtype=np.uint8)
    _load().oracle_stats(_ptr(x), x.shape[0], L, flat_eps, _ptr(mu), _ptr(sg), _ptr(fl))
    return mu, sg, fl.astype(bool)


def pair_dist(x, L: int, i: int, j: int, flat_eps: float = FLAT_EPS) -> float:
    """Direct z-normalised Euclidean distance of windows i and j."""
    x = _f64(x)
    return _load().oracle_pair_dist(_ptr(x), x.shape[0], L, i, j, flat_eps)


def pair_dists(x, L: int, pairs, flat_eps: float = FLAT_EPS) -> np.ndarray:
    """Direct distances of many (i, j) pairs at length L (statistics formed once)."""
    x = _f64(x)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    out = np.empty(pr.shape[0])
    if pr.shape[0]:
        _load().oracle_pair_dists(_ptr(x), x.shape[0], L, flat_eps, _ptr(pr), pr.shape[0], _ptr(out))
    return out


def pearson(x, L: int, i: int, j: int, flat_eps: float = FLAT_EPS) -> float:
    x = _f64(x)
    return _load().oracle_pearson(_ptr(x), x.shape[0], L, i, j, flat_eps)


def profile(x, L: int, rows: Optional[Sequence[int]] = None, excl_den: int = 4,
            flat_eps: float = FLAT_EPS, nthreads: int = 0):
    """Exact matrix-profile entries (dist, idx) of the given owners (all if None)."""
    x = _f64(x)
    N = x.shape[0] - L + 1
    if rows is None:
        r = None
        m = N
    else:
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        m = r.shape[0]
    dist = np.empty(m)
    idx = np.empty(m, dtype=np.int64)
    rc = _load().oracle_profile_rows(_ptr(x), x.shape[0], L, excl_den, flat_eps,
                                     None if r is None else _ptr(r), m, _ptr(dist), _ptr(idx),
                                     nthreads)
    if rc != 0:
        raise ValueError("oracle_profile_rows: bad arguments")
    return dist, idx


def lb(x, o: int, c: int, b: int, L: int, flat_eps: float = FLAT_EPS) -> float:
    x = _f64(x)
    return _load().oracle_lb(_ptr(x), x.shape[0], o, c, b, L, flat_eps)


def submp_decide(min_dist, max_lb):
    """Alg. ComputeSubMP decision: (valid[], minDistAbs, minLbAbs, bBestM)."""
    a = _f64(min_dist)
    b = _f64(max_lb)
    v = np.empty(a.shape[0], dtype=np.uint8)
    md = ctypes.c_double()
    ml = ctypes.c_double()
    best = _load().oracle_submp_decide(a.shape[0], _ptr(a), _ptr(b), _ptr(v), ctypes.byref(md),
                                       ctypes.byref(ml))
    return v.astype(bool), md.value, ml.value, bool(best)


def valid_fraction(x, b: int, L: int, p: int, excl_den: int = 4, flat_eps: float = FLAT_EPS):
    """Per-owner validity of heaps of size p built at base b and tested at L."""
    x = _f64(x)
    NL = x.shape[0] - L + 1
    out = np.empty(NL, dtype=np.uint8)
    nv = _load().oracle_valid_fraction(_ptr(x), x.shape[0], b, L, p, excl_den, flat_eps, _ptr(out))
    if nv < 0:
        raise ValueError("bad arguments")
    return out, int(nv)


def valmod(x, l_min: int, l_max: int, excl_den: int = 4, k_motifs: int = 1, k_discords: int = 1,
           flat_eps: float = FLAT_EPS, nthreads: int = 0) -> Dict[str, np.ndarray]:
    """Exact variable-length run: per-length profiles, VALMP and rankings."""
    x = _f64(x)
    n = x.shape[0]
    N0 = n - l_min + 1
    nl = l_max - l_min + 1
    km, kd = k_motifs, k_discords
    o = dict(
        prof_dist=np.empty((nl, N0)), prof_idx=np.empty((nl, N0), dtype=np.int64),
        valmp_norm=np.empty(N0), valmp_dist=np.empty(N0),
        valmp_len=np.empty(N0, dtype=np.int64), valmp_idx=np.empty(N0, dtype=np.int64),
        motif_ab=np.empty((nl, km, 2), dtype=np.int64), motif_d=np.empty((nl, km)),
        discord_on=np.empty((nl, kd, 2), dtype=np.int64), discord_d=np.empty((nl, kd)),
        g_motif_abl=np.empty((km, 3), dtype=np.int64), g_motif_d=np.empty((km, 2)),
        g_discord_onl=np.empty((kd, 3), dtype=np.int64), g_discord_d=np.empty((kd, 2)),
    )
    order = ["prof_dist", "prof_idx", "valmp_norm", "valmp_dist", "valmp_len", "valmp_idx",
             "motif_ab", "motif_d", "discord_on", "discord_d", "g_motif_abl", "g_motif_d",
             "g_discord_onl", "g_discord_d"]
    rc = _load().oracle_valmod(_ptr(x), n, l_min, l_max, excl_den, flat_eps, km, kd, nthreads,
                               *[_ptr(o[k]) for k in order])
    if rc != 0:
        raise ValueError("oracle_valmod: bad arguments")
    return o


def mth_rows(x, L: int, m: int, rows: Optional[Sequence[int]] = None, excl_den: int = 4,
             flat_eps: float = FLAT_EPS):
    """The m smallest distance-profile entries (Def. m-th best match) of each
    listed owner: (dist[rows, m], idx[rows, m]), +inf / -1 where missing."""
    x = _f64(x)
    N = x.shape[0] - L + 1
    r = None if rows is None else np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    cnt = N if r is None else r.shape[0]
    d = np.empty((cnt, m))
    i = np.empty((cnt, m), dtype=np.int64)
    rc = _load().oracle_mth_rows(_ptr(x), x.shape[0], L, excl_den, flat_eps, m,
                                 None if r is None else _ptr(r), cnt, _ptr(d), _ptr(i))
    if rc != 0:
        raise ValueError("oracle_mth_rows: invalid arguments")
    return d, i


def mth_discords(x, l_min: int, l_max: int, k: int, m: int, excl_den: int = 4, flat_eps: float = FLAT_EPS):
    """Top-k m-th discords per length and across lengths (see the C header)."""
    x = _f64(x)
    nlen = l_max - l_min + 1
    on = np.empty((nlen, m, k, 2), dtype=np.int64)
    d = np.empty((nlen, m, k))
    g_onl = np.empty((m, k, 3), dtype=np.int64)
    g_d = np.empty((m, k, 2))
    rc = _load().oracle_mth_discords(_ptr(x), x.shape[0], l_min, l_max, excl_den, flat_eps, k, m, _ptr(on),
                                     _ptr(d), _ptr(g_onl), _ptr(g_d))
    if rc != 0:
        raise ValueError("oracle_mth_discords: invalid arguments")
    return {"on": on, "d": d, "g_onl": g_onl, "g_d": g_d}


def motif_sets(x, pairs_abl, pair_d, D: float, cap: int, excl_den: int = 4, flat_eps: float = FLAT_EPS):
    """Motif sets grown from the given pairs (a, b, L) with distances d, radius D * d
    (see the C header): (count[k], off[k, cap], dist[k, cap])."""
    x = _f64(x)
    pa = np.ascontiguousarray(np.asarray(pairs_abl, dtype=np.int64).reshape(-1, 3))
    pd_ = np.ascontiguousarray(np.asarray(pair_d, dtype=np.float64).reshape(-1))
    k = pa.shape[0]
    count = np.empty(k, dtype=np.int64)
    off = np.empty((k, cap), dtype=np.int64)
    dist = np.empty((k, cap))
    rc = _load().oracle_motif_sets(_ptr(x), x.shape[0], k, _ptr(pa), _ptr(pd_), float(D), excl_den, flat_eps, cap,
                                   _ptr(count), _ptr(off), _ptr(dist))
    if rc != 0:
        raise ValueError("oracle_motif_sets: invalid arguments")
    return count, off, dist
