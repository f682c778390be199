"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: the closed
form of Eq. (6), an independent brute force written with numpy/scipy, the lower
bound derivation (Eq. lowerBoundFormula) minimised numerically, invariants
(symmetry, affine invariance, rank preservation), planted motifs / discords and
the worked Example 2 of the paper.
"""
import json
import os

import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial.distance import cdist

from paper_2008_13447_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _windows(x, L):
    return np.lib.stride_tricks.sliding_window_view(np.asarray(x, dtype=np.float64), L)


def _brute_mp(x, L, excl_den=4):
    """Independent brute force: numpy z-normalisation + scipy pairwise distances."""
    W = _windows(x, L)
    Z = (W - W.mean(axis=1, keepdims=True)) / W.std(axis=1, keepdims=True)
    D = cdist(Z, Z)
    N = W.shape[0]
    e = -(-L // excl_den)
    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    D[np.abs(ii - jj) <= e] = np.inf
    idx = np.argmin(D, axis=1)
    return D[np.arange(N), idx], idx, D


def test_stats_match_numpy(oracle_mod):
    x = gen.small_random_walk(300, 0) * 3.0 + 1.0e4
    for L in (5, 17, 64):
        mu, sg, fl = oracle_mod.stats(x, L)
        W = _windows(x, L)
        np.testing.assert_allclose(mu, W.mean(axis=1), rtol=1e-13)
        np.testing.assert_allclose(sg, W.std(axis=1), rtol=1e-9)
        assert not fl.any()


def test_flat_rule_special_cases(oracle_mod):
    # constant stretch at a large offset: windows inside it are flat, the others not
    x = gen.small_random_walk(200, 1) + 1.0e4
    x[60:120] = 1.0e4
    mu, sg, fl = oracle_mod.stats(x, 20)
    assert fl[60:101].all() and not fl[:40].any() and not fl[121:].any()
    d, idx = oracle_mod.profile(x, 20)
    assert np.isinf(d[60:101]).all() and (idx[60:101] == -1).all()
    assert not np.isin(idx, np.arange(60, 101)).any()  # flat windows are never neighbours


def test_closed_form_eq6(oracle_mod):
    """P1: d^2 = 2L(1 - rho) with rho from numpy's corrcoef (Eq. 6)."""
    x = gen.small_random_walk(120, 2)
    L = 16
    W = _windows(x, L)
    rng = np.random.default_rng(0)
    for _ in range(200):
        i, j = rng.integers(0, W.shape[0], 2)
        rho = np.corrcoef(W[i], W[j])[0, 1]
        d = oracle_mod.pair_dist(x, L, int(i), int(j))
        np.testing.assert_allclose(d * d, 2 * L * (1 - rho), rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(oracle_mod.pearson(x, L, int(i), int(j)), rho, atol=1e-12)


def test_symmetry_and_profile_invariants(oracle_mod):
    """P2 + P11: d(i,j) = d(j,i) exactly, MP[IP[i]] <= MP[i], dn in [0, 2]."""
    x = gen.small_random_walk(400, 3)
    L = 24
    for (i, j) in [(0, 50), (7, 311), (100, 102), (250, 30)]:
        assert oracle_mod.pair_dist(x, L, i, j) == oracle_mod.pair_dist(x, L, j, i)
    d, idx = oracle_mod.profile(x, L)
    assert (idx >= 0).all()
    assert (d[idx] <= d + 1e-12).all()
    dn = d / np.sqrt(L)
    assert (dn >= 0).all() and (dn <= 2.0 + 1e-12).all()
    e = -(-L // 4)
    assert (np.abs(idx - np.arange(idx.shape[0])) > e).all()


@pytest.mark.parametrize("excl_den", [4, 2])
def test_profile_vs_independent_brute_force(oracle_mod, excl_den):
    """The oracle's matrix profile equals an independent scipy brute force."""
    x = gen.small_random_walk(500, 4)
    for L in (8, 31, 50):
        d, idx = oracle_mod.profile(x, L, excl_den=excl_den)
        bd, bidx, _ = _brute_mp(x, L, excl_den)
        np.testing.assert_allclose(d, bd, rtol=1e-9, atol=1e-9)
        assert (idx == bidx).mean() > 0.999  # argmin ties are measure-zero here


def test_profile_rows_subset(oracle_mod):
    x = gen.small_random_walk(300, 5)
    dfull, ifull = oracle_mod.profile(x, 20)
    rows = [0, 5, 77, 280]
    d, idx = oracle_mod.profile(x, 20, rows=rows)
    np.testing.assert_array_equal(d, dfull[rows])
    np.testing.assert_array_equal(idx, ifull[rows])


def test_lb_is_minimum_of_its_definition(oracle_mod):
    """Eq. lowerBoundFinalFormula equals the numeric minimum of Eq.
    lowerBoundFormula over (mu', sigma' > 0)."""
    x = gen.small_random_walk(200, 6)
    b, L = 20, 27
    Wb = _windows(x, b)
    WL = _windows(x, L)
    for (o, c) in [(10, 60), (100, 30), (5, 150), (70, 170)]:
        zo = (Wb[o] - Wb[o].mean()) / Wb[o].std()
        tc = Wb[c]
        ratio = Wb[o].std() / WL[o].std()

        def f(v):
            a = np.exp(v[0])  # 1/sigma' > 0
            return np.sum((a * (tc - v[1]) - zo) ** 2)

        best = min(minimize(f, [np.log(1.0 / tc.std()) + s, tc.mean()], method="Nelder-Mead",
                            options=dict(xatol=1e-10, fatol=1e-12, maxiter=20000)).fun
                   for s in (-3.0, 0.0, 3.0))
        # with a -> 0 the objective tends to b (the rho <= 0 branch)
        best = min(best, float(b))
        np.testing.assert_allclose(oracle_mod.lb(x, o, c, b, L), ratio * np.sqrt(best),
                                   rtol=1e-5, atol=1e-7)


def test_lb_never_exceeds_true_distance(oracle_mod):
    """P3: LB(o, c, b -> L) <= d_L(o, c) for every pair, several k."""
    x = gen.small_random_walk(110, 7)
    b = 12
    e = 3
    for L in (13, 16, 21, 30):
        _, _, DL = _brute_mp(x, L, 4)
        NL = DL.shape[0]
        for o in range(0, NL, 3):
            for c in range(0, NL):
                if abs(o - c) <= -(-L // 4):
                    continue
                assert oracle_mod.lb(x, o, c, b, L) <= DL[o, c] + 1e-9


def test_rank_preservation(oracle_mod):
    """P4: LB^{L+1} / LB^{L} = sigma_{o,L} / sigma_{o,L+1} for every candidate."""
    x = gen.small_random_walk(150, 8)
    b, L = 16, 20
    _, sL, _ = oracle_mod.stats(x, L)
    _, sL1, _ = oracle_mod.stats(x, L + 1)
    for o in (3, 50, 90):
        ratios = [oracle_mod.lb(x, o, c, b, L + 1) / oracle_mod.lb(x, o, c, b, L)
                  for c in range(0, 120, 7) if abs(c - o) > 4]
        np.testing.assert_allclose(ratios, sL[o] / sL1[o], rtol=1e-12)


def test_affine_invariance(oracle_mod):
    """P7: MP(a*T + c) = MP(T) for a > 0."""
    x = gen.small_random_walk(300, 9)
    d0, i0 = oracle_mod.profile(x, 25)
    d1, i1 = oracle_mod.profile(3.7 * x - 250.0, 25)
    np.testing.assert_allclose(d1, d0, rtol=1e-9, atol=1e-9)
    assert (i0 == i1).mean() > 0.999


def test_planted_motif_recovered(oracle_mod):
    """P8: a planted pair in white noise is the motif pair."""
    x, (a, b) = gen.small_planted(1200, 0, 60, noise=0.05, base="noise")
    out = oracle_mod.valmod(x, 55, 60, k_motifs=1, k_discords=1)
    L = 60
    e = -(-L // 4)
    d, idx = out["prof_dist"][L - 55], out["prof_idx"][L - 55]
    assert abs(idx[a] - b) <= e
    ma, mb = out["motif_ab"][L - 55, 0]
    assert abs(ma - a) <= e and abs(mb - b) <= e
    # the cross-length top motif lands on the planted pair too
    ga, gb, gl = out["g_motif_abl"][0]
    assert abs(ga - a) <= e and abs(gb - b) <= e


def test_planted_discord_recovered(oracle_mod):
    """P9: a noise burst in a noisy sine is the top-1 discord."""
    x, c = gen.small_sine_with_discord(1500, 0, 50, 40)
    out = oracle_mod.valmod(x, 36, 40, k_motifs=1, k_discords=3)
    for t in range(5):
        L = 36 + t
        o = out["discord_on"][t, 0, 0]
        assert abs(o - c) <= L, (L, o, c)
    assert abs(out["g_discord_onl"][0, 0] - c) <= 40


def test_single_length_reduces_to_matrix_profile(oracle_mod):
    """P5: l_min = l_max gives the textbook matrix profile, VALMP = MP * sqrt(1/L)."""
    x = gen.small_random_walk(260, 10)
    L = 18
    out = oracle_mod.valmod(x, L, L, k_motifs=3, k_discords=3)
    bd, bidx, _ = _brute_mp(x, L)
    np.testing.assert_allclose(out["prof_dist"][0], bd, rtol=1e-9)
    np.testing.assert_allclose(out["valmp_norm"], bd * np.sqrt(1.0 / L), rtol=1e-9)
    assert (out["valmp_len"] == L).all()
    # top-1 motif is the pair at the global minimum (Def. motif pair)
    i = int(np.argmin(bd))
    assert set(out["motif_ab"][0, 0]) == {min(i, bidx[i]), max(i, bidx[i])}
    np.testing.assert_allclose(out["motif_d"][0, 0], bd.min(), rtol=1e-9)
    # top-1 discord is the offset with the largest NN distance (Def. m-th discord, m = 1)
    assert out["discord_on"][0, 0, 0] == int(np.argmax(bd))


def test_valmp_is_min_over_lengths_of_normalised_profiles(oracle_mod):
    """Alg. updateVALMP: VALMP[i] = min over L of MP_L[i] * sqrt(1/L), first L on ties,
    against profiles from the independent brute force."""
    x = gen.small_random_walk(240, 11)
    lmin, lmax = 10, 16
    out = oracle_mod.valmod(x, lmin, lmax, k_motifs=2, k_discords=2)
    N0 = x.shape[0] - lmin + 1
    best = np.full(N0, np.inf)
    blen = np.zeros(N0, dtype=int)
    for L in range(lmin, lmax + 1):
        bd, _, _ = _brute_mp(x, L)
        nd = bd * np.sqrt(1.0 / L)
        upd = nd < best[: nd.shape[0]] * (1 - 1e-12)
        best[: nd.shape[0]][upd] = nd[upd]
        blen[: nd.shape[0]][upd] = L
    np.testing.assert_allclose(out["valmp_norm"], best, rtol=1e-9)
    assert (out["valmp_len"] == blen).mean() > 0.99


def test_topk_rankings_are_non_trivial(oracle_mod):
    x = gen.small_random_walk(1000, 12)
    out = oracle_mod.valmod(x, 30, 34, k_motifs=5, k_discords=5)
    for t in range(5):
        L = 30 + t
        e = -(-L // 4)
        ab = out["motif_ab"][t]
        ends = ab[ab[:, 0] >= 0].ravel()
        for u in range(len(ends)):
            for v in range(u + 1, len(ends)):
                if u // 2 != v // 2:
                    assert abs(ends[u] - ends[v]) > e
        md = out["motif_d"][t]
        assert np.all(np.diff(md[np.isfinite(md)]) >= 0)
        dd = out["discord_d"][t]
        assert np.all(np.diff(dd[np.isfinite(dd)]) <= 0)
        offs = out["discord_on"][t, :, 0]
        assert all(abs(a - b) > e for a in offs for b in offs if a != b)
    # cross-length discords: rank r holds the max over L of d / sqrt(L) at rank r
    for r in range(5):
        dn = out["discord_d"][:, r] / np.sqrt(np.arange(30, 35))
        np.testing.assert_allclose(out["g_discord_d"][r, 1], dn.max(), rtol=1e-12)
        assert out["g_discord_onl"][r, 2] == 30 + int(np.argmax(dn))


def test_example2_decision_logic(oracle_mod):
    """P10: the numbers of Example 2 through the decision of Alg. ComputeSubMP."""
    g = json.load(open(os.path.join(GOLDEN, "example2_submp.json")))
    md = [p["minDist"] for p in g["profiles"]]
    ml = [p["maxLB"] for p in g["profiles"]]
    valid, mdabs, mlabs, best = oracle_mod.submp_decide(md, ml)
    assert list(valid) == [p["valid"] for p in g["profiles"]]
    assert mdabs == g["minDistAbs"] and mlabs == g["minLbAbs"] and best == g["bBestM"]


def test_valid_heaps_give_exact_minimum(oracle_mod):
    """Soundness of the lower-bound test: wherever the heap test passes, the
    heap minimum is the true matrix-profile value; p >= N-1 is always valid."""
    x = gen.small_random_walk(400, 13)
    b = 30
    for L in (31, 33, 38):
        dL, _ = oracle_mod.profile(x, L)
        for p in (1, 5, 20):
            v, nv = oracle_mod.valid_fraction(x, b, L, p)
            assert 0 < nv
            # recompute heap minima independently for the valid owners
            W = _windows(x, b)
            Z = (W - W.mean(1, keepdims=True)) / W.std(1, keepdims=True)
            R = Z @ Z.T / b
            _, _, DL = _brute_mp(x, L)
            eb = -(-b // 4)
            for o in np.nonzero(v == 1)[0][::7]:
                r = R[o].copy()
                r[np.abs(np.arange(r.shape[0]) - o) <= eb] = -np.inf
                order = np.lexsort((np.arange(r.shape[0]), -r))[:p]
                order = order[order < DL.shape[0]]
                assert np.isclose(DL[o, order].min(), dL[o], rtol=1e-9)
        v, nv = oracle_mod.valid_fraction(x, b, L, 10 ** 6)
        assert nv == (v != 2).sum()


def _brute_dist_matrix(x, L, excl_den=4):
    """Independent brute force: z-normalised windows, all pair distances, trivial
    matches masked with +inf."""
    Z = _windows(x, L)
    Z = (Z - Z.mean(axis=1, keepdims=True)) / Z.std(axis=1, keepdims=True)
    D = cdist(Z, Z)
    N = D.shape[0]
    e = -(-L // excl_den)
    ii = np.arange(N)
    D[np.abs(ii[:, None] - ii[None, :]) <= e] = np.inf
    return D


@pytest.mark.parametrize("m", [1, 3])
def test_mth_best_matches_vs_brute_force(oracle_mod, m):
    """Def. m-th best match: the m smallest entries of each distance profile,
    excluding the owner's trivial matches; j-th distances never decrease with j."""
    x = gen.small_random_walk(260, 31)
    L = 18
    D = _brute_dist_matrix(x, L)
    d, i = oracle_mod.mth_rows(x, L, m)
    order = np.lexsort((np.broadcast_to(np.arange(D.shape[1]), D.shape), D), axis=1)[:, :m]
    ref = np.take_along_axis(D, order, axis=1)
    np.testing.assert_allclose(d, ref, rtol=0, atol=1e-10)
    assert np.all(np.diff(d, axis=1) >= 0)
    # indices equal except between ties
    diff = i != order
    assert np.all(np.abs(d[diff] - ref[diff]) <= 1e-10)
    if m == 1:
        d1, i1 = oracle_mod.profile(x, L)
        np.testing.assert_allclose(d[:, 0], d1, rtol=0, atol=1e-12)


def test_mth_discords_vs_brute_force(oracle_mod):
    """Top-k m-th discords: for each j the owners by j-th best-match distance,
    greedy with the exclusion zone; across lengths the largest d / sqrt(L)."""
    x = gen.small_random_walk(240, 32)
    lo, hi, k, m = 16, 19, 3, 3
    r = oracle_mod.mth_discords(x, lo, hi, k, m)
    best = {}
    for t, L in enumerate(range(lo, hi + 1)):
        D = _brute_dist_matrix(x, L)
        S = np.sort(D, axis=1)
        e = -(-L // 4)
        for j in range(m):
            v = S[:, j]
            order = sorted(range(len(v)), key=lambda o: (-v[o], o))
            got = []
            for o in order:
                if not np.isfinite(v[o]):
                    continue
                if all(abs(o - g) > e for g in got):
                    got.append(o)
                if len(got) == k:
                    break
            for rank, o in enumerate(got):
                assert r["on"][t, j, rank, 0] == o, (L, j, rank)
                assert abs(r["d"][t, j, rank] - v[o]) <= 1e-10
                nn = r["on"][t, j, rank, 1]
                assert abs(D[o, nn] - v[o]) <= 1e-10  # the reported neighbour is at that distance
                dn = v[o] / np.sqrt(L)
                if (j, rank) not in best or dn > best[(j, rank)][0]:
                    best[(j, rank)] = (dn, o, L)
    for (j, rank), (dn, o, L) in best.items():
        assert abs(r["g_d"][j, rank, 1] - dn) <= 1e-12
        assert tuple(r["g_onl"][j, rank, [0, 2]]) == (o, L)


def test_first_discords_special_case(oracle_mod):
    """m = 1 reduces to the 1st discords of the full run."""
    x = gen.small_random_walk(300, 33)
    r = oracle_mod.mth_discords(x, 20, 24, 3, 1)
    v = oracle_mod.valmod(x, 20, 24, k_motifs=1, k_discords=3)
    np.testing.assert_array_equal(r["on"][:, 0, :, 0], v["discord_on"][:, :, 0])
    np.testing.assert_allclose(r["d"][:, 0], v["discord_d"], rtol=0, atol=1e-12)


def test_motif_sets_vs_brute_force(oracle_mod):
    """Def. data series motif set: windows within radius D * d of either center,
    taken by (distance to the nearer center, offset), trivial matches of taken
    members dropped, sets disjoint by offset; checked against an independent
    brute force and the definition's invariants."""
    x = gen.small_random_walk(900, 37)
    lo, hi, k, D, cap = 30, 34, 4, 5.0, 60
    v = oracle_mod.valmod(x, lo, hi, k_motifs=k, k_discords=1)
    pairs, pd = v["g_motif_abl"], v["g_motif_d"][:, 0]
    count, off, dist = oracle_mod.motif_sets(x, pairs, pd, D, cap)
    taken = set()
    skipped = 0
    for s in range(k):
        a, b, L = (int(t) for t in pairs[s])
        Dm = _brute_dist_matrix(x, L)
        np.fill_diagonal(Dm, 0.0)
        W = _windows(x, L)
        Z = (W - W.mean(axis=1, keepdims=True)) / W.std(axis=1, keepdims=True)
        da = np.linalg.norm(Z - Z[a], axis=1)
        db = np.linalg.norm(Z - Z[b], axis=1)
        near = np.minimum(da, db)
        r = D * pd[s]
        cand = sorted((float(near[c]), c) for c in range(len(near)) if near[c] < r)
        e = -(-L // 4)
        acc = []
        for dnear, c in cand:
            if any(abs(c - u) <= e for u in acc):
                continue
            if c in taken:
                skipped += 1
                continue
            acc.append(c)
        assert count[s] == len(acc), (s, count[s], len(acc))
        got = [int(t) for t in off[s, :min(cap, len(acc))]]
        assert got == acc[:cap]
        np.testing.assert_allclose(dist[s, :len(got)], [near[c] for c in got], rtol=0, atol=1e-10)
        assert a in acc or a in taken  # a center is a member of its own set unless an earlier set took it
        taken.update(acc)
        # invariants: members within the radius, no two members are trivial matches
        assert all(near[c] < r for c in acc)
        assert all(abs(u - w) > e for i, u in enumerate(acc) for w in acc[i + 1:])
    assert skipped > 0  # the input exercises the disjointness rule


def test_motif_sets_special_radii(oracle_mod):
    """Def. data series motif set with the strict radius: D = 0 gives empty sets;
    with an unbounded radius every non-flat window is a candidate of the first
    set, so its members are the greedy non-overlapping cover of the offsets and
    no offset is farther than the exclusion zone from a member."""
    x = gen.small_random_walk(400, 35)
    L = 20
    v = oracle_mod.valmod(x, L, L, k_motifs=2, k_discords=1)
    pairs, pd = v["g_motif_abl"], v["g_motif_d"][:, 0]
    count, off, _ = oracle_mod.motif_sets(x, pairs, pd, 0.0, 8)
    assert np.all(count == 0) and np.all(off == -1)
    N = x.shape[0] - L + 1
    e = -(-L // 4)
    count, off, dist = oracle_mod.motif_sets(x, pairs[:1], pd[:1], 1e12, N)
    mem = off[0, :count[0]]
    assert mem[0] == min(pairs[0, 0], pairs[0, 1]) and dist[0, 0] == 0.0
    assert np.all(np.diff(dist[0, :count[0]]) >= 0)
    s = np.sort(mem)
    assert np.all(np.diff(s) > e)  # pairwise non-trivial
    gaps = np.abs(np.arange(N)[:, None] - s[None, :]).min(axis=1)
    assert np.all(gaps <= e)  # maximal: every window is a trivial match of some member


def test_lb_of_candidate_flat_at_base(oracle_mod):
    """Eq. lowerBoundFinalFormula for a candidate that the flat rule excludes at
    the base length but not at L: the bound uses its real base correlation and
    stays below the true distance, while the correlation-0 convention of an
    exactly constant window would exceed it (the fixture is a scaled copy of
    the owner whose deviation at b lies just under the flat threshold)."""
    b, Lmax = 24, 30
    x, o, c, m = gen.flat_at_base_copy(600, 0, b, Lmax)
    _, sgb, flb = oracle_mod.stats(x, b)
    assert flb[c] and not flb[o]
    for L in range(b + 1, Lmax + 1):
        _, sgL, flL = oracle_mod.stats(x, L)
        assert not flL[c]
        d = oracle_mod.pair_dist(x, L, o, c)
        dp, ip = oracle_mod.profile(x, L, rows=[o])
        assert ip[0] == c and dp[0] == d and d < 1e-9
        assert oracle_mod.lb(x, o, c, b, L) <= d + 1e-12
        assert np.sqrt(b) * sgb[o] / sgL[o] > 1.0  # what correlation 0 would claim


def test_valid_heaps_exact_with_candidates_flat_at_base(oracle_mod):
    """Soundness of the heap test with windows that are flat at b and candidates
    at L: every valid owner's heap minimum is its true profile value (heaps hold
    the p best non-flat candidates at b, found here with numpy)."""
    b = 24
    x, o, c, m = gen.flat_at_base_copy(600, 0, b, 30)
    _, sgb, flb = oracle_mod.stats(x, b)
    W = _windows(x, b)
    Z = (W - W.mean(1, keepdims=True)) / W.std(1, keepdims=True)
    R = Z @ Z.T / b
    eb = -(-b // 4)
    for L in (25, 28, 30):
        dL, _ = oracle_mod.profile(x, L)
        _, _, DL = _brute_mp(x, L)
        _, _, flL = oracle_mod.stats(x, L)
        DL[:, flL] = np.inf
        for p in (1, 5):
            v, nv = oracle_mod.valid_fraction(x, b, L, p)
            assert v[o] == 0  # the copy flat at b is not covered by any certified bound
            for w in np.nonzero(v == 1)[0]:
                r = R[w].copy()
                r[np.abs(np.arange(r.shape[0]) - w) <= eb] = -np.inf
                r[flb] = -np.inf
                order = np.lexsort((np.arange(r.shape[0]), -r))[:p]
                order = order[order < DL.shape[0]]
                assert np.isclose(DL[w, order].min(), dL[w], rtol=1e-9, atol=1e-12), (L, p, w)


def test_flat_between_fixture_and_profile(oracle_mod):
    """The fixture of an owner flat only at intermediate lengths (gen.flat_between)
    is what it claims under the oracle's flat rule, and at a length past the
    constant stretch the oracle's profile row of that owner equals a numpy brute
    force (the owner is an ordinary window again)."""
    x, o = gen.flat_between(900, 1)
    x = x.astype(np.float32).astype(np.float64)
    flags = {L: bool(oracle_mod.stats(x, L)[2][o]) for L in range(30, 48)}
    assert not any(flags[L] for L in range(30, 35))
    assert all(flags[L] for L in range(35, 43))
    assert not any(flags[L] for L in range(43, 48))
    for L in (45, 47):
        dp, ip = oracle_mod.profile(x, L, rows=[o])
        d, i, D = _brute_mp(x, L)
        _, _, fl = oracle_mod.stats(x, L)
        row = D[o].copy()
        row[fl[:row.shape[0]]] = np.inf
        assert ip[0] == int(np.argmin(row)) and np.isclose(dp[0], row.min(), rtol=1e-12, atol=1e-12)
