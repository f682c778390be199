"""GPU parity at the full sizes of the large workloads, on sampled owners the
oracle can compute one by one, and the recompute path forced by small candidate
lists.

- The 2^21-point precision-stress series (level 1e4, 20 flat stretches, 5
  planted pairs of length 300) over its whole range 200..400 on the FP32 path:
  at lengths 200, 300 and 400, random owners, owners at both edges of every flat
  stretch (the windows that route work to the FP64 kernel), the planted offsets
  and every reported motif and discord endpoint.
- All 512 series of the batched workload in one plan: sampled owners of every
  series at l_min, the middle length and l_max.
- Collecting lists of 1 or 3 entries: nearly every owner overflows and is
  recomputed by a row scan, and the outputs stay exact.
"""
import os
import sys

import numpy as np
import pytest

from paper_2008_13447_amd import gen

pytestmark = pytest.mark.gpu

TOL64 = 1e-9


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle

    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="module")
def config5_fp32():
    torch = _torch()
    from paper_2008_13447_amd import native

    w = gen.config5()
    _say(f"config5 n={w.n} L={w.l_min}..{w.l_max} fp32 (whole range)")
    g = native.run_valmod(torch.from_numpy(w.x).cuda(), w.l_min, w.l_max, p=w.p, k_motifs=w.k_motifs,
                          k_discords=w.k_discords, precision="fp32")
    _say(f"config5 GPU done, stats sums {g['stats'].sum(axis=0).tolist()}")
    return w, g


def _flat_edges(w, L):
    """Owners at both edges of every flat stretch: windows that start just
    before it, end inside it, start inside it or leave it."""
    out = []
    for s, ln in w.flats:
        out += [s - L, s - L + 1, s - L // 2, s - 1, s, s + 1, s + ln - L, s + ln - L + 1, s + ln - L // 2,
                s + ln - 1, s + ln]
    return out


@pytest.mark.parametrize("L", [200, 300, 400])
def test_config5_whole_range_sampled(oracle_mod, config5_fp32, L):
    from oracle import compare

    w, g = config5_fp32
    t = L - w.l_min
    extra = [a for (a, b, _) in w.planted_motifs] + [b for (a, b, _) in w.planted_motifs]
    extra += _flat_edges(w, L)
    extra += [int(v) for v in np.concatenate([g["motif_ab"][t].ravel(), g["discord_on"][t].ravel()]) if v >= 0]
    rep = compare.check_sampled(w.x, w.l_min, g, [L], 64, TOL64, extra=extra)
    _say(f"config5 L={L}: {dict(rep)}")
    # planted pairs (length 300) are each other's neighbours there
    if L == 300:
        e = -(-L // 4)
        for a, b, _ in w.planted_motifs:
            assert abs(int(g["prof_idx"][t, a]) - b) <= e
    # windows inside a flat stretch are +inf / -1
    for s, ln in w.flats:
        if ln > L + 2:
            assert np.isinf(g["prof_dist"][t, s + 1:s + ln - L]).all()
            assert (g["prof_idx"][t, s + 1:s + ln - L] == -1).all()


def test_config5_reported_pairs_and_rankings(oracle_mod, config5_fp32):
    """Every reported motif pair and discord neighbour at 200, 300 and 400 is at
    the reported distance; the global rankings point at legal pairs."""
    import oracle

    w, g = config5_fp32
    for L in (200, 300, 400):
        t = L - w.l_min
        pairs, got = [], []
        for (a, b), d in zip(g["motif_ab"][t], g["motif_d"][t]):
            if a >= 0:
                pairs.append((a, b))
                got.append(d)
        for (o, nn), d in zip(g["discord_on"][t], g["discord_d"][t]):
            if o >= 0 and nn >= 0:
                pairs.append((o, nn))
                got.append(d)
        ref = oracle.pair_dists(w.x, L, pairs)
        assert (np.abs(ref - np.asarray(got)) / np.sqrt(L) <= TOL64).all(), L
    for (a, b, L), (d, dn) in zip(g["g_motif_abl"], g["g_motif_d"]):
        if a >= 0:
            assert b - a > -(-L // 4)
            assert abs(oracle.pair_dist(w.x, int(L), int(a), int(b)) - d) / np.sqrt(L) <= TOL64


def test_batched_all_series_sampled(oracle_mod):
    """All 512 series of the batched workload in one plan (FP32 path, 4 lanes):
    8 sampled owners of every series at l_min, the middle length and l_max."""
    torch = _torch()
    from oracle import compare
    from paper_2008_13447_amd import native

    ws = gen.config4(512)
    _say(f"batched: {len(ws)} series, n {min(w.n for w in ws)}..{max(w.n for w in ws)}")
    v = native.Valmod([torch.from_numpy(w.x).cuda() for w in ws], [w.l_min for w in ws], [w.l_max for w in ws],
                      p=10, k_motifs=10, k_discords=10, precision="fp32", lanes=4)
    v.run()
    _say("batched GPU done")
    worst = 0.0
    for s, w in enumerate(ws):
        g = v.result(s)
        mid = (w.l_min + w.l_max) // 2
        rep = compare.check_sampled(w.x, w.l_min, g, [w.l_min, mid, w.l_max], 8, TOL64, seed=s)
        worst = max(worst, rep.get("max_dn_err", 0.0))
        if s % 64 == 0:
            _say(f"series {s}: {dict(rep)}")
    v.close()
    _say(f"batched: worst |d dn| {worst:.3g}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cap", [1, 3])
def test_overflowing_lists_are_recomputed(oracle_mod, monkeypatch, precision, cap):
    """Collecting lists of `cap` entries (a test hook read when the plan is
    built): owners with more candidates above their threshold overflow and are
    recomputed by a row scan; the outputs match the oracle."""
    _torch()
    from oracle import compare

    monkeypatch.setenv("VALMOD_COLLECT_CAP", str(cap))
    x = gen.small_random_walk(2500, 80, np.float32)
    lo, hi = 30, 38
    _say(f"collect cap {cap} {precision}")
    from paper_2008_13447_amd import native

    g = native.run_valmod(_torch().from_numpy(x).cuda(), lo, hi, p=5, k_motifs=3, k_discords=3,
                          precision=precision)
    r = oracle_mod.valmod(x, lo, hi, k_motifs=3, k_discords=3)
    compare.check_full(x, lo, g, r, TOL64)
    recomputed = int(g["stats"][:, 2].sum())
    _say(f"collect cap {cap} {precision}: {recomputed} owners recomputed")
    assert recomputed > 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mfma_and_valu_contractions_agree(oracle_mod, monkeypatch, precision):
    """The anchor table and the row recompute on FP64 matrix cores give the
    outputs of the VALU kernels (VALMOD_MFMA=0), and both match the oracle, on
    the path that recomputes every failing window."""
    torch = _torch()
    from oracle import compare
    from paper_2008_13447_amd import native

    x = gen.small_random_walk(3000, 81, np.float32)
    lo, hi = 40, 48
    outs = []
    for mfma in ("1", "0"):
        monkeypatch.setenv("VALMOD_MFMA", mfma)
        _say(f"contractions mfma={mfma} {precision}")
        outs.append(native.run_valmod(torch.from_numpy(x).cuda(), lo, hi, p=5, k_motifs=3, k_discords=3,
                                      precision=precision, path="recompute"))
    r = oracle_mod.valmod(x, lo, hi, k_motifs=3, k_discords=3)
    for g in outs:
        compare.check_full(x, lo, g, r, TOL64)
    assert int(outs[0]["stats"][:, 2].sum()) > 0  # rows were recomputed
