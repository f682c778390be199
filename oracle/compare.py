"""Element-by-element comparison of VALMOD outputs against the oracle.

Test infrastructure only. Distances are compared as length-normalised
distances dn = d / sqrt(L) within an absolute tolerance. Indices must be equal,
except where distances tie within the tolerance: a different index is accepted
iff the oracle's own distance for the reported pair is within the tolerance of
the oracle's optimum (and the pair is a legal, non-trivial one).
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np

from . import pair_dists, profile


def _excl(L: int, den: int) -> int:
    return -(-L // den)


class Report(dict):
    def merge_max(self, key, val):
        self[key] = max(self.get(key, 0.0), float(val))


def check_profile_rows(x, L: int, rows: np.ndarray, d_gpu: np.ndarray, i_gpu: np.ndarray,
                       d_ref: np.ndarray, i_ref: np.ndarray, tol: float, excl_den: int = 4,
                       rep: Optional[Report] = None, what: str = "") -> Report:
    """Compare matrix-profile entries of owners `rows` at length L."""
    rep = rep if rep is not None else Report()
    rows = np.asarray(rows)
    fin_g, fin_r = np.isfinite(d_gpu), np.isfinite(d_ref)
    bad = np.nonzero(fin_g != fin_r)[0]
    assert bad.size == 0, f"{what} L={L}: finiteness differs at owners {rows[bad[:10]]}: " \
                          f"gpu={d_gpu[bad[:10]]} ref={d_ref[bad[:10]]}"
    assert np.all(i_gpu[~fin_g] == -1), f"{what} L={L}: index set for an infinite entry"
    sq = np.sqrt(L)
    if fin_g.any():
        err = np.abs(d_gpu[fin_g] - d_ref[fin_g]) / sq
        rep.merge_max("max_dn_err", err.max())
        worst = np.argmax(err)
        assert err.max() <= tol, f"{what} L={L}: |d dn| {err.max():.3e} > {tol} at owner " \
                                 f"{rows[fin_g][worst]} (gpu {d_gpu[fin_g][worst]!r}, ref {d_ref[fin_g][worst]!r})"
    mis = np.nonzero(fin_g & (i_gpu != i_ref))[0]
    rep["idx_mismatch"] = rep.get("idx_mismatch", 0) + int(mis.size)
    if mis.size:
        e = _excl(L, excl_den)
        own = rows[mis]
        assert np.all(np.abs(i_gpu[mis] - own) > e), f"{what} L={L}: trivial neighbour reported"
        dg = pair_dists(x, L, np.stack([own, i_gpu[mis]], 1))
        gap = (dg - d_ref[mis]) / sq
        rep.merge_max("max_tie_gap", gap.max())
        assert np.all(gap <= tol), f"{what} L={L}: index mismatch beyond a tie at owners " \
                                   f"{own[gap > tol][:10]} (gap {gap.max():.3e})"
    return rep


def check_full(x, l_min: int, gpu: Dict[str, np.ndarray], ref: Dict[str, np.ndarray], tol: float,
               excl_den: int = 4) -> Report:
    """Compare every output of a full run against oracle.valmod()."""
    rep = Report()
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    nl, N0 = ref["prof_dist"].shape
    for t in range(nl):
        L = l_min + t
        N = n - L + 1
        rows = np.arange(N)
        check_profile_rows(x, L, rows, gpu["prof_dist"][t, :N], gpu["prof_idx"][t, :N].astype(np.int64),
                           ref["prof_dist"][t, :N], ref["prof_idx"][t, :N], tol, excl_den, rep, "profile")
        assert np.all(np.isinf(gpu["prof_dist"][t, N:])) and np.all(gpu["prof_idx"][t, N:] == -1), \
            f"L={L}: tail entries past N_L not cleared"
    check_valmp(x, l_min, gpu, ref, tol, excl_den, rep)
    check_rankings(x, l_min, gpu, ref, tol, excl_den, rep)
    return rep


def check_valmp(x, l_min, gpu, ref, tol, excl_den=4, rep=None) -> Report:
    rep = rep if rep is not None else Report()
    gn, rn = gpu["valmp_norm"], ref["valmp_norm"]
    fin = np.isfinite(rn)
    assert np.array_equal(np.isfinite(gn), fin), "VALMP finiteness differs"
    err = np.abs(gn[fin] - rn[fin])
    if err.size:
        rep.merge_max("valmp_dn_err", err.max())
        assert err.max() <= tol, f"VALMP normalised distance error {err.max():.3e}"
    # a different length (or neighbour) is a tie within the tolerance
    dl = np.nonzero(fin & ((gpu["valmp_len"] != ref["valmp_len"]) | (gpu["valmp_idx"] != ref["valmp_idx"])))[0]
    rep["valmp_tie_swaps"] = int(dl.size)
    for i in dl[:200]:
        L = int(gpu["valmp_len"][i])
        d = pair_dists(x, L, [[i, int(gpu["valmp_idx"][i])]])[0]
        assert abs(d * np.sqrt(1.0 / L) - rn[i]) <= tol, f"VALMP entry {i}: not a tie"
    return rep


def check_rankings(x, l_min, gpu, ref, tol, excl_den=4, rep=None) -> Report:
    """Rankings per length and across lengths. Every index that differs from the
    oracle's must be a tie under the oracle's own distances: the reported pair
    (or offset and neighbour) is legal and its oracle distance is within `tol`
    (normalised) of the oracle's value at that rank."""
    rep = rep if rep is not None else Report()
    x = np.asarray(x, dtype=np.float64)
    nl = ref["motif_d"].shape[0]
    n = x.shape[0]
    for t in range(nl):
        L = l_min + t
        sq = np.sqrt(L)
        e = _excl(L, excl_den)
        for key_d, key_i, kind in (("motif_d", "motif_ab", "motif"), ("discord_d", "discord_on", "discord")):
            dg, dr = gpu[key_d][t], ref[key_d][t]
            assert np.array_equal(np.isnan(dg), np.isnan(dr)), f"{kind} L={L}: filled slots differ"
            ok = ~np.isnan(dr)
            if ok.any():
                err = np.abs(dg[ok] - dr[ok]) / sq
                rep.merge_max(f"{kind}_dn_err", err.max())
                assert err.max() <= tol, f"{kind} L={L}: rank distances differ by {err.max():.3e}"
            ig, ir = gpu[key_i][t], ref[key_i][t]
            for r in np.nonzero(ok)[0]:
                if kind == "motif" and not np.array_equal(ig[r], ir[r]):
                    a, b = int(ig[r][0]), int(ig[r][1])
                    assert 0 <= a < b < n - L + 1 and b - a > e, f"motif L={L} rank {r}: illegal pair {ig[r]}"
                    d = pair_dists(x, L, [[a, b]])[0]
                    assert abs(d - dr[r]) / sq <= tol, f"motif L={L} rank {r}: {ig[r]} vs {ir[r]}"
                    rep["rank_tie_swaps"] = rep.get("rank_tie_swaps", 0) + 1
                if kind == "discord" and not np.array_equal(ig[r], ir[r]):
                    o, nn = int(ig[r][0]), int(ig[r][1])
                    assert abs(o - nn) > e, f"discord L={L} rank {r}: trivial neighbour {ig[r]}"
                    # the offset's exact profile value and the neighbour's distance both tie
                    d_o = ref["prof_dist"][t, o]
                    assert abs(d_o - dr[r]) / sq <= tol, f"discord L={L} rank {r}: {ig[r]} vs {ir[r]}"
                    d_nn = pair_dists(x, L, [[o, nn]])[0]
                    assert abs(d_nn - d_o) / sq <= tol, f"discord L={L} rank {r}: neighbour {nn} is not nearest"
                    rep["rank_tie_swaps"] = rep.get("rank_tie_swaps", 0) + 1
    for key_d, key_i, kind in (("g_motif_d", "g_motif_abl", "g_motif"), ("g_discord_d", "g_discord_onl", "g_discord")):
        dg, dr = gpu[key_d], ref[key_d]
        assert np.array_equal(np.isnan(dg[:, 1]), np.isnan(dr[:, 1])), f"{kind}: filled slots differ"
        ok = ~np.isnan(dr[:, 1])
        if ok.any():
            err = np.abs(dg[ok, 1] - dr[ok, 1])
            rep.merge_max(f"{kind}_dn_err", err.max())
            assert err.max() <= tol, f"{kind}: normalised distances differ by {err.max():.3e}"
        ig, ir = gpu[key_i], ref[key_i]
        for r in np.nonzero(ok)[0]:
            if np.array_equal(ig[r], ir[r]):
                continue
            u, v, L = (int(w) for w in ig[r])
            assert l_min <= L < l_min + nl, f"{kind} rank {r}: length {L} outside the range"
            sq = np.sqrt(L)
            e = _excl(L, excl_den)
            if kind == "g_motif":
                assert 0 <= u < v < n - L + 1 and v - u > e, f"{kind} rank {r}: illegal pair {ig[r]}"
                dn = pair_dists(x, L, [[u, v]])[0] / sq
            else:
                assert abs(u - v) > e, f"{kind} rank {r}: trivial neighbour {ig[r]}"
                dn = ref["prof_dist"][L - l_min, u] / sq
                d_nn = pair_dists(x, L, [[u, v]])[0] / sq
                assert abs(d_nn - dn) <= tol, f"{kind} rank {r}: neighbour {v} is not nearest"
            assert abs(dn - dr[r, 1]) <= tol, f"{kind} rank {r}: {ig[r]} vs {ir[r]} is not a tie ({dn} vs {dr[r, 1]})"
            rep["rank_tie_swaps"] = rep.get("rank_tie_swaps", 0) + 1
    return rep


def sample_rows(N: int, count: int, seed: int, extra: Sequence[int] = ()) -> np.ndarray:
    g = np.random.default_rng(seed)
    base = g.choice(N, size=min(count, N), replace=False)
    ex = [int(v) for v in extra if 0 <= int(v) < N]
    return np.unique(np.concatenate([base, np.array(ex, dtype=np.int64)])).astype(np.int64)


def check_sampled(x, l_min: int, gpu: Dict[str, np.ndarray], lengths: Sequence[int], rows_per_len: int,
                  tol: float, excl_den: int = 4, seed: int = 0, extra: Sequence[int] = (),
                  nthreads: int = 0) -> Report:
    """Compare sampled owners of the given lengths against oracle.profile()."""
    rep = Report()
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    for L in lengths:
        t = L - l_min
        N = n - L + 1
        rows = sample_rows(N, rows_per_len, seed + L, extra)
        d_ref, i_ref = profile(x, L, rows=rows, excl_den=excl_den, nthreads=nthreads)
        check_profile_rows(x, L, rows, gpu["prof_dist"][t, rows], gpu["prof_idx"][t, rows].astype(np.int64),
                           d_ref, i_ref, tol, excl_den, rep, "sampled")
    return rep


def check_paper_mode(x, l_min: int, gpu: Dict[str, np.ndarray], ref: Dict[str, np.ndarray], tol: float,
                     excl_den: int = 4) -> Report:
    """Guarantees of Alg. ComputeSubMP as published: computed profile entries are
    exact, uncomputed ones (index -2) carry a lower bound of the true entry, the
    first motif of every length and the first global motif are exact."""
    rep = Report()
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    nl = ref["prof_dist"].shape[0]
    partial = 0
    for t in range(nl):
        L = l_min + t
        N = n - L + 1
        gi = gpu["prof_idx"][t, :N].astype(np.int64)
        rows = np.nonzero(gi != -2)[0]
        check_profile_rows(x, L, rows, gpu["prof_dist"][t, rows], gi[rows], ref["prof_dist"][t, rows],
                           ref["prof_idx"][t, rows], tol, excl_den, rep, "computed")
        part = np.nonzero(gi == -2)[0]
        partial += part.size
        if part.size:
            lb, true = gpu["prof_dist"][t, part], ref["prof_dist"][t, part]
            assert np.all(lb <= true + tol * np.sqrt(L)), f"L={L}: a partial entry's bound exceeds MP_L"
        gd, rd = gpu["motif_d"][t, 0], ref["motif_d"][t, 0]
        assert abs(gd - rd) <= tol * np.sqrt(L), f"L={L}: motif distance {gd} vs {rd}"
        a, b = (int(v) for v in gpu["motif_ab"][t, 0])
        if a >= 0:
            assert abs(pair_dists(x, L, [[a, b]])[0] - rd) <= tol * np.sqrt(L), f"L={L}: motif pair not optimal"
    assert abs(gpu["g_motif_d"][0, 1] - ref["g_motif_d"][0, 1]) <= tol, "global motif differs"
    rep["partial_entries"] = partial
    return rep
