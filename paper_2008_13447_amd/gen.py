"""Seeded synthetic input series for VALMOD workloads.

This module only draws numbers: it holds none of the method's arithmetic, so
both the CPU oracle (tests) and the HIP path consume the same inputs from here.

The paper evaluates on real recordings (GAP, CAP/EEG, ECG, EMG, ASTRO; §7
datasets) that are not available; the generators below stand in for them with
the shapes of the paper's parameter grid (Table "tableParameters": series of
0.1M-1M points, length ranges of 100+, p between 5 and 150).

Every generator takes its seed explicitly and uses numpy's PCG64, drawing in
float64 and casting to the stated dtype at the end.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

SEED_BASE = 13447
BATCH_SEED_BASE = 13447000


@dataclasses.dataclass
class Workload:
    """One series plus the VALMOD parameters it is run with."""

    name: str
    x: np.ndarray  # float32 or float64 series
    l_min: int
    l_max: int
    p: int
    k_motifs: int
    k_discords: int
    excl_den: int = 4
    planted_motifs: List[Tuple[int, int, int]] = dataclasses.field(default_factory=list)  # (a, b, length)
    planted_discords: List[Tuple[int, int]] = dataclasses.field(default_factory=list)  # (offset, length)
    flats: List[Tuple[int, int]] = dataclasses.field(default_factory=list)  # (start, length)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_walk(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """x_t = cumsum(N(0, 1))."""
    g = _rng(seed)
    return np.cumsum(g.standard_normal(n)).astype(dtype)


def _place_disjoint(g: np.random.Generator, n: int, lengths: List[int], gap: int,
                    forbidden: Optional[List[Tuple[int, int]]] = None,
                    max_tries: int = 100000) -> List[int]:
    """Draw start offsets for segments of the given lengths so that no two
    segments (nor a forbidden interval) come within `gap` of each other."""
    taken: List[Tuple[int, int]] = list(forbidden or [])
    starts = []
    for ln in lengths:
        for _ in range(max_tries):
            s = int(g.integers(0, n - ln))
            ok = all(s + ln + gap <= a or a + la + gap <= s for a, la in taken)
            if ok:
                taken.append((s, ln))
                starts.append(s)
                break
        else:  # pragma: no cover - only on absurd parameters
            raise RuntimeError("could not place disjoint segments")
    return starts


def plant_motif_pairs(x: np.ndarray, g: np.random.Generator, count: int, length: int,
                      noise: float, forbidden=None) -> List[Tuple[int, int, int]]:
    """Plant `count` motif pairs of `length` points into x (float64, in place).

    Pattern P = cumsum(N(0,1)); instance A at a: x[a:a+len] = x[a] + (P - P0);
    instance B at b: alpha*(P - P0) + x[b] + beta + N(0, noise^2), with
    alpha ~ U[0.5, 2] and beta ~ U[-5, 5]. Placements are disjoint with a gap of
    two pattern lengths.
    """
    n = x.shape[0]
    starts = _place_disjoint(g, n, [length] * (2 * count), 2 * length, forbidden)
    out = []
    for m in range(count):
        a, b = starts[2 * m], starts[2 * m + 1]
        pat = np.cumsum(g.standard_normal(length))
        pat = pat - pat[0]
        alpha = g.uniform(0.5, 2.0)
        beta = g.uniform(-5.0, 5.0)
        x[a:a + length] = x[a] + pat
        x[b:b + length] = alpha * pat + x[b] + beta + g.normal(0.0, noise, length)
        out.append((min(a, b), max(a, b), length))
    return out


def config1() -> Workload:
    """Plain FP64 case: n=2,048 random walk, lengths 32..40, p=5, top-1."""
    x = random_walk(2048, SEED_BASE + 1, np.float64)
    return Workload("rw2048_l32-40_fp64", x, 32, 40, 5, 1, 1)


def config2() -> Workload:
    """n=65,536 FP32 random walk with 3 planted motif pairs (length 150,
    noise 0.05) and one planted discord (Gaussian bump), lengths 100..200, p=10."""
    g = _rng(SEED_BASE + 2)
    n = 65536
    x = np.cumsum(g.standard_normal(n))
    # discord first, so motif placements avoid it
    c = int(g.integers(0, n - 150))
    motifs = plant_motif_pairs(x, g, 3, 150, 0.05, forbidden=[(c, 150)])
    t = np.arange(150, dtype=np.float64)
    x[c:c + 150] += 20.0 * np.exp(-((t - 75.0) ** 2) / (2.0 * 25.0 ** 2))
    return Workload("rw65536_planted_l100-200", x.astype(np.float32), 100, 200, 10, 10, 10,
                    planted_motifs=motifs, planted_discords=[(c, 150)])


def sensor_like(n: int, seed: int) -> np.ndarray:
    """Sum of 4 sinusoids (periods log-uniform in [200, 2000], random phase,
    amplitude 1) + AR(1) noise (phi=0.9, innovation sd 0.3) + random-walk drift
    (step sd 0.02). Returned as float64."""
    from scipy.signal import lfilter

    g = _rng(seed)
    t = np.arange(n, dtype=np.float64)
    periods = np.exp(g.uniform(np.log(200.0), np.log(2000.0), 4))
    phases = g.uniform(0.0, 2.0 * np.pi, 4)
    x = np.zeros(n)
    for per, ph in zip(periods, phases):
        x += np.sin(2.0 * np.pi * t / per + ph)
    e = lfilter([1.0], [1.0, -0.9], g.normal(0.0, 0.3, n))
    drift = np.cumsum(g.normal(0.0, 0.02, n))
    return x + e + drift


def config3() -> Workload:
    """n=2^20 FP32 sensor-like series, lengths 256..384, p=20, top-10."""
    x = sensor_like(1 << 20, SEED_BASE + 3)
    return Workload("sensor1M_l256-384", x.astype(np.float32), 256, 384, 20, 10, 10)


def config4_params(count: int = 512) -> List[Tuple[int, int, int, int]]:
    """(seed, n, l_min, l_max) for each batched series: n ~ U{4096..131072},
    l_min ~ U{32..256}, l_max = floor(1.5 * l_min)."""
    out = []
    for s in range(count):
        g = _rng(BATCH_SEED_BASE + s)
        n = int(g.integers(4096, 131072 + 1))
        lmin = int(g.integers(32, 256 + 1))
        out.append((BATCH_SEED_BASE + s, n, lmin, (3 * lmin) // 2))
    return out


def config4(count: int = 512) -> List[Workload]:
    """Batched random walks (float32), p=10, top-10 each."""
    out = []
    for seed, n, lmin, lmax in config4_params(count):
        g = _rng(seed)
        g.integers(4096, 131072 + 1)  # replay the parameter draws
        g.integers(32, 256 + 1)
        x = np.cumsum(g.standard_normal(n)).astype(np.float32)
        out.append(Workload(f"batch{seed - BATCH_SEED_BASE}", x, lmin, lmax, 10, 10, 10))
    return out


def config5(n: int = 1 << 21) -> Workload:
    """Precision stress: 1e4 + random walk with 20 flat segments (increments
    zeroed, plus N(0, 1e-6^2) value noise) and 5 planted motif pairs of length
    300, lengths 200..400, p=20, top-10. Cast to float32."""
    g = _rng(SEED_BASE + 5)
    steps = g.standard_normal(n)
    flat_lens = [int(v) for v in g.integers(500, 5000 + 1, 20)]
    flat_starts = _place_disjoint(g, n, flat_lens, 1000)
    for s, ln in zip(flat_starts, flat_lens):
        steps[s + 1:s + ln] = 0.0
    x = 1.0e4 + np.cumsum(steps)
    for s, ln in zip(flat_starts, flat_lens):
        x[s:s + ln] += g.normal(0.0, 1.0e-6, ln)
    flats = list(zip(flat_starts, flat_lens))
    motifs = plant_motif_pairs(x, g, 5, 300, 0.05, forbidden=flats)
    return Workload("rw2M_offset1e4_flats_l200-400", x.astype(np.float32), 200, 400, 20, 10, 10,
                    planted_motifs=motifs, flats=flats)


def small_random_walk(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Tiny random-walk fixture for unit tests."""
    return random_walk(n, SEED_BASE + 100 + seed, dtype)


def small_planted(n: int, seed: int, length: int, noise: float = 0.05,
                  base: str = "noise") -> Tuple[np.ndarray, Tuple[int, int]]:
    """Tiny fixture with one planted motif pair in white noise or a random walk."""
    g = _rng(SEED_BASE + 200 + seed)
    x = g.standard_normal(n) if base == "noise" else np.cumsum(g.standard_normal(n))
    (a, b, _), = plant_motif_pairs(x, g, 1, length, noise)
    return x, (a, b)


def small_sine_with_discord(n: int, seed: int, period: int, length: int,
                            noise: float = 0.05) -> Tuple[np.ndarray, int]:
    """Tiny fixture: a noisy sine with one planted anomaly of `length` points."""
    g = _rng(SEED_BASE + 300 + seed)
    t = np.arange(n, dtype=np.float64)
    x = np.sin(2.0 * np.pi * t / period) + g.normal(0.0, noise, n)
    c = int(g.integers(length, n - 2 * length))
    x[c:c + length] = g.normal(0.0, 1.0, length)
    return x, c


def flat_at_base_copy(n: int, seed: int, b: int, L: int, flat_eps: float = 2.0 ** -20,
                      near_noise: float = 0.1) -> Tuple[np.ndarray, int, int, int]:
    """Random walk with one owner window o of length L, a scaled copy of it at c
    whose deviation over the first b points lies just under the flat threshold
    (|mean| < 1) while its last L - b points make it non-flat, and a noisy copy
    of o at m (a close candidate that is not flat). Returns (x, o, c, m)."""
    g = _rng(SEED_BASE + 400 + seed)
    x = np.cumsum(g.standard_normal(n))
    w = g.standard_normal(L)
    w[:b] = (w[:b] - w[:b].mean()) / w[:b].std()
    w[b:] = 3.0 * np.where(g.standard_normal(L - b) >= 0.0, 1.0, -1.0)
    o, m, c = n // 5, 2 * n // 5, 3 * n // 5
    x[o:o + L] = x[o] + w
    x[m:m + L] = x[m] + w + g.normal(0.0, near_noise, L)
    x[c:c + L] = 0.9 * flat_eps * w
    return x, o, c, m


def flat_between(n: int, seed: int, hold: int = 42, h: float = 5.68e-6,
                 level: float = 0.5) -> Tuple[np.ndarray, int]:
    """Sensor-like series with one owner window o that is not flat at the
    shortest lengths, flat at intermediate ones and not flat again once it
    reaches past a constant stretch: x[o] = level + h, x[o+1 .. o+hold-1] = level
    (deviation h sqrt(L - 1) / L against the flat threshold 2^-20 max(1, |mean|)),
    then the series resumes from `level`. With the defaults o is not flat for
    L <= 34, flat for 35 <= L <= hold and not flat beyond. Returns (x, o)."""
    x = sensor_like(n, SEED_BASE + 500 + seed)
    o = n // 2
    tail = x[o + hold:] - x[o + hold] + level + 0.3
    x[o:o + hold] = level
    x[o] = level + h
    x[o + hold:] = tail
    return x, o


WORKLOADS = {1: config1, 2: config2, 3: config3, 5: config5}
