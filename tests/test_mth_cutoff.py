"""The pruning cutoff of the m-th discords (CPU, plain Python).

Per length and column j, the Top-k m-th discords are taken greedily: owners by
their j-th best-match distance, descending (ties to the smaller offset), each
accepted unless it lies within the exclusion zone e of an owner already accepted
(Defs. m-th discord and Top-k m-th discord). With partial profiles (Alg.
Topkm_nextLength) only some owners have certified distances; the others have
upper bounds. The HIP path ranks the certified owners with twice the exclusion
zone, takes the k-th accepted distance tau, and leaves out every uncertified
owner whose upper bound lies below tau. The claim it relies on: whatever the
uncertified owners' true distances are (at most their bounds), the greedy over
all owners accepts the same owners whether or not those below tau take part.
Here that is checked by brute force on random instances, and a concrete case
shows why the zone must be doubled.
"""
import random

import pytest


def greedy(vals, e, k):
    """Accepted (value, offset) pairs of the greedy ranking; vals maps offset -> value."""
    order = sorted(vals.items(), key=lambda t: (-t[1], t[0]))
    got = []
    for o, v in order:
        if len(got) == k:
            break
        if all(abs(o - a) > e for a, _ in got):
            got.append((o, v))
    return got


def cutoff(certified, e, k):
    """tau: the k-th accepted value with twice the zone, or None if fewer than k."""
    got = greedy(certified, 2 * e, k)
    return got[-1][1] if len(got) == k else None


def pruned_ranking(certified, bounds, truth, e, k):
    """The ranking the HIP path reports: certified owners, plus the uncertified
    ones whose bound reaches tau (at their true value, as the recompute gives)."""
    tau = cutoff(certified, e, k)
    kept = dict(certified)
    for o, u in bounds.items():
        if tau is None or not (u < tau):
            kept[o] = truth[o]
    return greedy(kept, e, k)


def test_doubled_zone_is_needed():
    """A recomputed owner X can exclude two certified owners of the single-zone
    ranking at once; then an owner Y below that ranking's k-th value enters the
    top k, and a single-zone cutoff would have dropped it."""
    e, k = 60, 3
    certified = {0: 10.0, 100: 9.0, 200: 8.0, 500: 1.0}
    truth = {150: 9.5, 400: 5.0}
    bounds = dict(truth)
    full = greedy({**certified, **truth}, e, k)
    assert [o for o, _ in full] == [0, 150, 400]
    single = greedy(certified, e, k)[-1][1]
    assert single == 8.0 and truth[400] < single  # a single-zone cutoff prunes Y
    assert pruned_ranking(certified, bounds, truth, e, k) == full


@pytest.mark.parametrize("seed", range(40))
def test_pruned_ranking_equals_full_ranking(seed):
    """Random instances, dense enough that a cutoff from the single zone gives a
    wrong ranking in about 3 of 1000 of them (a dozen per run of this test)."""
    rng = random.Random(20080913 + seed)
    for _ in range(100):
        n = rng.randint(10, 60)
        e = rng.randint(1, 8)
        k = rng.randint(1, 6)
        levels = rng.randint(3, 30)  # few levels: many ties
        truth = {o: float(rng.randint(0, levels)) for o in range(n)}
        owners = [o for o in range(n) if rng.random() < 0.95]  # the rest: no entry (flat windows)
        certified, bounds = {}, {}
        for o in owners:
            if rng.random() < 0.5:
                certified[o] = truth[o]
            else:
                bounds[o] = truth[o] + rng.choice([0.0, 0.5, 2.0, float(levels)])
        full = greedy({o: truth[o] for o in owners}, e, k)
        assert pruned_ranking(certified, bounds, truth, e, k) == full, (n, e, k)
