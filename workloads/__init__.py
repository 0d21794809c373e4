"""Seeded synthetic workloads for the matrix-profile join.

This module only draws data: it holds none of the join's arithmetic and is
shared by the tests, the benchmark and the smoke check so that the oracle and
the GPU library are fed identical inputs.  The recipes follow the workload
shapes of the matrix-profile literature that the tsmp paper times and
demonstrates (random walks, Section 4; physiological signals, Section 3.4):

* ``random_walk``      cumulative sum of N(0, 1) steps, drawn in float64.
* ``paper_walk``       the +-1 random walk of the paper's speed test (n=40000).
* ``planted_walk``     random walk with planted motif pairs (a white N(0,1)
                       pattern, each copy scaled by U(0.5, 2) plus N(0, 0.05^2)
                       noise, written into the walk's increments so the window
                       is an offset copy) and additive N(0, 3^2) discord
                       bursts, all windows >= 2m apart.
* ``ecg_like``         beats made of five Gaussian bumps, beat length
                       round(250 * U(0.9, 1.1)), two-sinusoid baseline wander,
                       N(0, 0.02^2) noise.
* ``ragged_batch``     many random walks of uneven lengths and window sizes.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def random_walk(n: int, seed, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.standard_normal(n)).astype(dtype)


def paper_walk(n: int = 40000, seed: int = 2018, dtype=np.float64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.choice(np.array([-1.0, 1.0]), size=n)).astype(dtype)


@dataclass
class Planted:
    T: np.ndarray
    m: int
    motif_pairs: list = field(default_factory=list)   # [(pos_a, pos_b), ...]
    discords: list = field(default_factory=list)      # [pos, ...]


def _spaced_positions(rng, n, m, count, gap):
    """count window starts in [0, n-m], pairwise at least `gap` apart."""
    for _ in range(1000):
        pos = np.sort(rng.integers(0, n - m + 1, size=count))
        if count < 2 or np.min(np.diff(pos)) >= gap:
            return [int(p) for p in rng.permutation(pos)]
    raise RuntimeError("could not place planted windows")


def planted_walk(n: int, m: int, seed, n_motifs: int = 8, n_discords: int = 4,
                 dtype=np.float32) -> Planted:
    """Motif copies are planted in the increments of the walk, so that each
    planted window is an offset copy of s*p + e and the walk stays continuous
    around it (an overwrite would leave level jumps whose straddling windows
    form spurious step-shaped motifs).  A discord burst overwrites its window
    with N(0, 3^2) noise around the walk's level at the window start."""
    rng = np.random.default_rng(seed)
    steps = rng.standard_normal(n)
    pos = _spaced_positions(rng, n, m, 2 * n_motifs + n_discords, 2 * m)
    pairs = []
    for k in range(n_motifs):
        pat = rng.standard_normal(m)
        a, b = pos[2 * k], pos[2 * k + 1]
        for p in (a, b):
            w = rng.uniform(0.5, 2.0) * pat + rng.normal(0.0, 0.05, m)
            steps[p + 1:p + m] = np.diff(w)
        pairs.append((min(a, b), max(a, b)))
    T = np.cumsum(steps)
    disc = []
    for k in range(n_discords):
        p = pos[2 * n_motifs + k]
        T[p:p + m] = T[p] + rng.normal(0.0, 3.0, m)
        disc.append(p)
    return Planted(T.astype(dtype), m, pairs, sorted(disc))


def ecg_like(n: int, seed, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    # (centre, width, amplitude) of the P, Q, R, S, T waves, as beat fractions
    bumps = ((0.20, 0.025, 0.12), (0.36, 0.008, -0.15), (0.40, 0.010, 1.0),
             (0.44, 0.010, -0.25), (0.65, 0.040, 0.30))
    out = np.empty(n)
    t = 0
    while t < n:
        L = int(round(250 * rng.uniform(0.9, 1.1)))
        x = (np.arange(L) + 0.5) / L
        beat = np.zeros(L)
        for c, w, a in bumps:
            beat += a * np.exp(-0.5 * ((x - c) / w) ** 2)
        e = min(n, t + L)
        out[t:e] = beat[:e - t]
        t = e
    tt = np.arange(n)
    ph = rng.uniform(0, 2 * np.pi, 2)
    out += 0.10 * np.sin(2 * np.pi * tt / 2800 + ph[0]) + 0.05 * np.sin(2 * np.pi * tt / 900 + ph[1])
    out += rng.normal(0.0, 0.02, n)
    return out.astype(dtype)


@dataclass
class Ragged:
    series: list        # list of 1-D arrays
    m: list             # window per series
    ez: list            # exclusion zone per series

    def concat(self):
        off = np.zeros(len(self.series) + 1, dtype=np.int64)
        off[1:] = np.cumsum([s.size for s in self.series])
        return np.concatenate(self.series), off


def ragged_batch(nseries: int, seed, nmin: int = 2048, nmax: int = 65536,
                 windows=(32, 64, 128), dtype=np.float32) -> Ragged:
    rng = np.random.default_rng(seed)
    lens = rng.integers(nmin, nmax + 1, size=nseries)
    ms = rng.choice(np.asarray(windows), size=nseries)
    series = [np.cumsum(rng.standard_normal(int(L))).astype(dtype) for L in lens]
    ms = [int(x) for x in ms]
    return Ragged(series, ms, [x // 4 for x in ms])


def walk_batch(nseries: int, n: int, seed, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.standard_normal((nseries, n)), axis=1).astype(dtype)


def regime_series(n: int, seed, dtype=np.float64):
    """Three regimes of about n/3 samples each: a sine of period 40, a
    sawtooth of period 55 and a two-level pulse of period 70, every cycle
    with its own amplitude U(0.8, 1.2) and N(0, 0.05^2) noise.  Returns the
    series and the two regime boundaries (semantic-segmentation input)."""
    rng = np.random.default_rng(seed)
    b1, b2 = n // 3 + int(rng.integers(-n // 20, n // 20)), 2 * n // 3 + int(rng.integers(-n // 20, n // 20))
    out = np.empty(n)
    t = 0
    while t < n:
        reg = 0 if t < b1 else (1 if t < b2 else 2)
        p = (40, 55, 70)[reg]
        u = np.arange(p) / p
        cyc = (np.sin(2 * np.pi * u), 2.0 * u - 1.0, np.where(u < 0.3, 1.0, -0.4))[reg]
        e = min(n, t + p, b1 if t < b1 else (b2 if t < b2 else n))
        out[t:e] = rng.uniform(0.8, 1.2) * cyc[:e - t]
        t = e
    out += rng.normal(0.0, 0.05, n)
    return out.astype(dtype), (b1, b2)


def evolving_chain(n: int, m: int, k: int, seed, dtype=np.float64):
    """A random walk with k planted windows that morph step by step from one
    random smooth shape into another (copy t is (1 - t/(k-1)) A + t/(k-1) B
    plus N(0, 0.01^2), scaled to the local walk), spaced evenly: each copy's
    nearest neighbours to the left and right are the copies before and after
    it, so they form one chain.  Returns the series and the positions."""
    rng = np.random.default_rng(seed)
    T = np.cumsum(rng.standard_normal(n))
    u = np.arange(m) / m

    def shape():
        f = sum(rng.normal() * np.sin(2 * np.pi * (h * u + rng.random())) / h for h in range(1, 6))
        return (f - f.mean()) / f.std()

    A, Bs = shape(), shape()
    gap = n // (k + 1)
    pos = [gap * (t + 1) - m // 2 for t in range(k)]
    for t, p in enumerate(pos):
        w = (1 - t / (k - 1)) * A + t / (k - 1) * Bs + rng.normal(0.0, 0.01, m)
        T[p:p + m] = T[p] + 5.0 * w
    return T.astype(dtype), pos


# ---- the five benchmark workloads -----------------------------------------

def selfjoin_small():
    """Plain FP64 self-join: n=4096 random walk, m=64, ez=16."""
    return random_walk(4096, 1, np.float64), 64, 16


def selfjoin_large(n: int = 1 << 20):
    """n=2^20 float32 random walk with 8 planted motif pairs and 4 discords,
    m=256, ez=64."""
    return planted_walk(n, 256, 2), 64


def abjoin_ecg(n: int = 1 << 19):
    """Two n=2^19 float32 ECG-like series, m=128."""
    return ecg_like(n, 31), ecg_like(n, 32), 128


def batch_ragged(nseries: int = 512):
    """512 random walks, lengths U{2048..65536}, m in {32, 64, 128}, ez=m/4."""
    return ragged_batch(nseries, 4)


def diff_batch(nseries: int = 64, n: int = 16384):
    """64 float32 random walks of n=16384 for the differentiable profile,
    m=100, ez=25."""
    return walk_batch(nseries, n, 5), 100, 25
