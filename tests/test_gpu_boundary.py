"""GPU tests of the run contract of the C ABI: valmod_run enqueues and returns,
valmod_run_status waits and reports the device status word, a NULL output is
skipped (the run still computes what the other outputs need), and the lower
bound of a candidate flat at the base length (Eq. lowerBoundFinalFormula)."""
import ctypes
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


def _valmod(x, lo, hi, **kw):
    torch = _torch()
    from paper_2008_13447_amd import native

    return native.Valmod(torch.from_numpy(np.ascontiguousarray(x)).cuda(), lo, hi, **kw)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_runs_enqueue_and_status_waits(oracle_mod, precision):
    """Two runs enqueued back to back (partial profiles: the call waits inside
    for its sweep counters), one status read: the outputs are the oracle's."""
    from oracle import compare

    x = gen.small_random_walk(1500, 60, np.float32)
    lo, hi = 30, 36
    _say(f"async runs {precision} n=1500 L={lo}..{hi}")
    v = _valmod(x, lo, hi, p=5, k_motifs=3, k_discords=3, precision=precision, path="recompute")
    v.run(sync=False)
    v.run(sync=False)
    v.status()
    g = v.result(0)
    v.close()
    r = oracle_mod.valmod(x, lo, hi, k_motifs=3, k_discords=3)
    compare.check_full(x, lo, g, r, TOL64)


def test_status_reports_non_finite_input():
    """A NaN in the input sets the device status word: the run is enqueued
    (VALMOD_OK) and valmod_run_status returns VALMOD_E_DEVICE."""
    from paper_2008_13447_amd import native

    x = gen.small_random_walk(800, 61, np.float32)
    x[400] = np.nan
    _say("non-finite input n=800")
    v = _valmod(x, 20, 22, p=5)
    v.run(sync=False)
    rc = native.lib().valmod_run_status(ctypes.c_void_p(v.plan), None)
    assert rc == -6, native.STATUS.get(rc, rc)
    # the status stays readable, and a clean input clears it
    v.series.copy_(v.series.nan_to_num(0.0))
    v.run()
    v.close()


@pytest.mark.parametrize("skip", [
    ("prof_dist", "prof_idx"),
    ("prof_dist", "prof_idx", "valmp_norm", "valmp_dist", "valmp_len", "valmp_idx"),
    ("motif_ab", "motif_d", "discord_on", "discord_d", "stats"),
], ids=["profiles", "profiles+valmp", "per-length rankings"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_skipped_outputs(oracle_mod, skip, precision):
    """Outputs passed as NULL are not written; the rest match the oracle (the
    rankings need the per-length profiles, which the run keeps in its workspace;
    more lengths than the workspace keeps rows for at once)."""
    from oracle import compare

    x = gen.small_random_walk(1200, 62, np.float32)
    lo, hi = 20, 60  # 41 lengths: the rankings run on two groups of rows
    _say(f"skipped outputs {skip} {precision}")
    v = _valmod(x, lo, hi, p=5, k_motifs=4, k_discords=4, precision=precision, skip=skip)
    v.run()
    g = v.result(0)
    v.close()
    r = oracle_mod.valmod(x, lo, hi, k_motifs=4, k_discords=4)
    for key in skip:
        assert g[key] is None
    if "prof_dist" not in skip:
        for t in range(hi - lo + 1):
            N = x.shape[0] - (lo + t) + 1
            compare.check_profile_rows(x, lo + t, np.arange(N), g["prof_dist"][t, :N],
                                       g["prof_idx"][t, :N].astype(np.int64), r["prof_dist"][t, :N],
                                       r["prof_idx"][t, :N], TOL64)
    if "valmp_norm" not in skip:
        compare.check_valmp(x, lo, g, r, TOL64)
    if "motif_d" not in skip:
        # per-length rankings (the discord tie check reads the oracle's profiles)
        gg = dict(g)
        gg["prof_dist"] = r["prof_dist"]
        gg["g_motif_abl"], gg["g_motif_d"] = r["g_motif_abl"], r["g_motif_d"]
        gg["g_discord_onl"], gg["g_discord_d"] = r["g_discord_onl"], r["g_discord_d"]
        compare.check_rankings(x, lo, gg, r, TOL64)
    # cross-length rankings are always compared
    gr = {k: r[k] for k in ("motif_ab", "motif_d", "discord_on", "discord_d")}
    gr.update({k: g[k] for k in ("g_motif_abl", "g_motif_d", "g_discord_onl", "g_discord_d")})
    gr["prof_dist"] = r["prof_dist"]
    compare.check_rankings(x, lo, gr, r, TOL64)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("p", [1, 5])
def test_candidate_flat_at_base_length(oracle_mod, precision, p):
    """A scaled copy of an owner whose deviation at the base length lies just
    under the flat threshold becomes its exact neighbour (distance 0) a length
    later; partial profiles (forced row recompute path) never saw it, and the
    sweep's bound must not certify the owner's stored minimum."""
    from oracle import compare

    b, hi = 24, 30
    x, o, c, m = gen.flat_at_base_copy(600, 0, b, hi)
    _say(f"flat-at-base copy {precision} p={p}")
    v = _valmod(x, b, hi, p=p, k_motifs=2, k_discords=2, precision=precision, path="recompute")
    v.run()
    g = v.result(0)
    v.close()
    r = oracle_mod.valmod(x, b, hi, k_motifs=2, k_discords=2)
    compare.check_full(x, b, g, r, TOL64)
    for t in range(1, hi - b + 1):
        assert g["prof_idx"][t, o] == c and g["prof_dist"][t, o] < 1e-6
