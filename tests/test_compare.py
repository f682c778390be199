"""The comparator accepts the oracle's own outputs and rejects index changes
that are not ties (CPU; the mistakes are planted in a copy of the oracle's
output, never in a GPU result)."""
import copy

import numpy as np
import pytest

from paper_2008_13447_amd import gen


@pytest.fixture(scope="module")
def case(oracle_mod):
    x = gen.small_random_walk(400, 50)
    lo, hi = 20, 23
    r = oracle_mod.valmod(x, lo, hi, k_motifs=4, k_discords=4)
    return x, lo, r


def test_oracle_output_passes(case):
    from oracle import compare

    x, lo, r = case
    rep = compare.check_full(x, lo, copy.deepcopy(r), r, 1e-9)
    assert rep.get("rank_tie_swaps", 0) == 0 and rep["idx_mismatch"] == 0


@pytest.mark.parametrize("what", ["g_motif", "g_discord", "discord_nn", "motif", "profile_idx"])
def test_non_ties_are_rejected(case, what):
    from oracle import compare

    x, lo, r = case
    g = copy.deepcopy(r)
    if what == "g_motif":
        a, b, L = g["g_motif_abl"][0]
        g["g_motif_abl"][0] = (a, b + 7, L)  # another pair of the same length
    elif what == "g_discord":
        o, nn, L = g["g_discord_onl"][0]
        g["g_discord_onl"][0] = (o + 31, nn, L)
    elif what == "discord_nn":
        o, nn = g["discord_on"][1, 0]
        g["discord_on"][1, 0] = (o, nn + 40 if nn + 40 < 360 else nn - 40)
    elif what == "motif":
        g["motif_ab"][2, 1, 1] += 9
    else:
        i = 100
        g["prof_idx"][0, i] = g["prof_idx"][0, i] + 13
    with pytest.raises(AssertionError):
        compare.check_full(x, lo, g, r, 1e-9)
