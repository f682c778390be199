"""Pins of the oracle's greedy motif rankings against an independent brute force.

The per-length top-k motif pairs and the cross-length top-k motif pairs of the
oracle are rebuilt here from scratch: distance matrices by numpy z-normalisation
and scipy pairwise distances, the matrix profile by argmin (first minimum, so
exact ties go to the smaller index), VALMP by the strict normalised minimum over
lengths (Alg. updateVALMP), and both rankings by a plain Python greedy over the
sorted candidates (Def. data series motif pair; Sec. "Comparing Motifs of
Different Lengths"; exclusion zone ceil(L / 4), for pairs of two lengths the
zone of the longer one). Inputs with exact copies make many distances exactly
zero, so the tie-breaking order is pinned too. (The length tie-break of the
cross-length ranking is unreachable at exact ties: windows that are identical
at a length are identical at every shorter one, and VALMP keeps the shortest;
a nonzero bit-exact tie between two lengths cannot be constructed on purpose.)
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from paper_2008_13447_amd import gen


def _excl(L, den=4):
    return -(-L // den)


def _brute_profile(x, L, den=4):
    W = np.lib.stride_tricks.sliding_window_view(np.asarray(x, dtype=np.float64), L)
    Z = (W - W.mean(axis=1, keepdims=True)) / W.std(axis=1, keepdims=True)
    D = cdist(Z, Z)
    N = D.shape[0]
    ii = np.arange(N)
    D[np.abs(ii[:, None] - ii[None, :]) <= _excl(L, den)] = np.inf
    idx = np.argmin(D, axis=1)
    d = D[ii, idx]
    idx[~np.isfinite(d)] = -1
    return d, idx


def _greedy_pairs(cands, k, zone):
    """cands: sorted list of (key..., a, b, L); accept a pair unless one of its
    endpoints lies within the exclusion zone of an accepted endpoint."""
    got = []
    for c in cands:
        a, b, L = c[-3], c[-2], c[-1]
        ok = True
        for (a2, b2, L2) in got:
            e = zone(L, L2)
            if min(abs(a - a2), abs(a - b2), abs(b - a2), abs(b - b2)) <= e:
                ok = False
                break
        if ok:
            got.append((a, b, L))
        if len(got) == k:
            break
    return got


def _brute_rankings(x, lo, hi, k):
    n = x.shape[0]
    N0 = n - lo + 1
    per_len = []
    vn = np.full(N0, np.inf)
    vd = np.full(N0, np.inf)
    vl = np.zeros(N0, dtype=np.int64)
    vi = np.full(N0, -1, dtype=np.int64)
    for L in range(lo, hi + 1):
        d, idx = _brute_profile(x, L)
        N = d.shape[0]
        cands = sorted((float(d[i]), min(i, int(idx[i])), max(i, int(idx[i])), L)
                       for i in range(N) if idx[i] >= 0)
        mot = _greedy_pairs([(c[0], c[1], c[2], c[1], c[2], c[3]) for c in cands], k,
                            lambda La, Lb: _excl(max(La, Lb)))
        pair_d = {(c[1], c[2]): c[0] for c in cands}
        per_len.append([(a, b, pair_d[(a, b)]) for (a, b, _) in mot])
        dn = d * np.sqrt(1.0 / L)
        upd = dn < vn[:N]
        vn[:N][upd] = dn[upd]
        vd[:N][upd] = d[upd]
        vl[:N][upd] = L
        vi[:N][upd] = idx[upd]
    cands = sorted((float(vn[i]), int(vl[i]), i, min(i, int(vi[i])), max(i, int(vi[i])), int(vl[i]))
                   for i in range(N0) if vi[i] >= 0)
    glob = _greedy_pairs(cands, k, lambda La, Lb: _excl(max(La, Lb)))
    gdn = {}
    for c in cands:
        gdn.setdefault((c[3], c[4], c[5]), c[0])
    return per_len, glob, gdn


def _with_copies(n, seed, copies):
    """Random walk with exact (value-identical) copies of some stretches."""
    x = gen.small_random_walk(n, seed)
    for src, dst, length in copies:
        x[dst:dst + length] = x[src:src + length]
    return x


CASES = [
    ("random walk", lambda: gen.small_random_walk(420, 40), 18, 22, 6),
    ("random walk, other seed", lambda: gen.small_random_walk(360, 41), 12, 15, 8),
    ("exact copies (zero-distance ties)", lambda: _with_copies(460, 42, [(40, 250, 90), (150, 380, 60)]),
     16, 20, 7),
    ("planted pair", lambda: gen.small_planted(500, 3, 30, noise=0.05, base="walk")[0], 26, 30, 5),
]


@pytest.mark.parametrize("name,make,lo,hi,k", CASES, ids=[c[0] for c in CASES])
def test_motif_rankings_vs_brute_force(oracle_mod, name, make, lo, hi, k):
    x = make()
    out = oracle_mod.valmod(x, lo, hi, k_motifs=k, k_discords=2)
    per_len, glob, gdn = _brute_rankings(x, lo, hi, k)
    for t, L in enumerate(range(lo, hi + 1)):
        want = [(a, b) for (a, b, _) in per_len[t]]
        got = [tuple(int(v) for v in ab) for ab in out["motif_ab"][t] if ab[0] >= 0]
        assert got == want, (name, L)
        for r, (_, _, d) in enumerate(per_len[t]):
            assert abs(out["motif_d"][t, r] - d) <= 1e-10
        assert np.all(np.isnan(out["motif_d"][t, len(want):]))
    got = [tuple(int(v) for v in abl) for abl in out["g_motif_abl"] if abl[0] >= 0]
    assert got == glob, name
    for r, key in enumerate(glob):
        assert abs(out["g_motif_d"][r, 1] - gdn[key]) <= 1e-12
        assert abs(out["g_motif_d"][r, 0] - gdn[key] * np.sqrt(key[2])) <= 1e-10


def test_copies_make_exact_ties(oracle_mod):
    """The copy fixture really ranks several zero-distance pairs (ties broken
    by the smaller offsets) and spaces them by more than the exclusion zone."""
    x = _with_copies(460, 42, [(40, 250, 90), (150, 380, 60)])
    out = oracle_mod.valmod(x, 16, 20, k_motifs=7, k_discords=1)
    zeros = np.sum(out["motif_d"][0] == 0.0)
    assert zeros >= 3
    ab = out["motif_ab"][0][:zeros]
    assert np.all(np.diff(ab[:, 0]) > _excl(16))
    assert np.all(out["g_motif_d"][:3, 1] == 0.0) and np.all(out["g_motif_abl"][:3, 2] == 16)
