"""GPU parity of the self-join against the FP64 oracle (through the C ABI)."""

import numpy as np
import pytest
import torch

from oracle import cimpl
from oracle import mp_oracle as O
from tests.parity import compare_profile
from workloads import random_walk, selfjoin_small

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _run(T, m, ez, precision, slots=0, reseed=0, finalize=True):
    import paper_1904_12626_amd as mpx
    Tg = torch.from_numpy(np.ascontiguousarray(T)).to(DEV)
    P, I = mpx.selfjoin(Tg, m, ez, precision=precision, tile_slots=slots, reseed_rows=reseed,
                        fp64_finalize=finalize)
    torch.cuda.synchronize()
    return P.cpu().numpy(), I.cpu().numpy()


def test_dpp_wave_shift_direction():
    """The sweep moves column data with a DPP wave shift: lane L must read
    lane L+1 (checked here through a tiny join whose answer depends on it)."""
    T = random_walk(700, 3, np.float64)
    P, I = _run(T, 16, 4, "f64")
    Po, Io = cimpl.selfjoin(T, 16, 4)
    compare_profile(T, 16, P, I, Po, Io, 1e-9, ez=4, where="dpp")


@pytest.mark.parametrize("precision,tol", [("f64", 1e-9), ("f32", 1e-3 * 8.0)])
def test_selfjoin_small_random_walk(precision, tol):
    """n=4096 float64 random walk, m=64, ez=16: full oracle."""
    T, m, ez = selfjoin_small()
    P, I = _run(T, m, ez, precision)
    Po, Io = cimpl.selfjoin(T, m, ez)
    maxd, nd = compare_profile(T, m, P, I, Po, Io, tol, ez=ez, where=precision)
    print(f"{precision}: max|dP|={maxd:.3e}, index differences (ties) {nd}")


@pytest.mark.parametrize("n,m,ez,dtype,precision,slots", [
    (300, 7, 1, np.float64, "f64", 8),
    (1000, 2, 0, np.float64, "f64", 8),
    (2500, 33, 8, np.float32, "f32", 8),
    (2500, 33, 8, np.float32, "f32", 16),
    (5000, 100, 25, np.float32, "f64", 8),
    (1300, 64, 16, np.float64, "f32", 16),
    (3100, 40, 10, np.float32, "f32", 12),
    (129, 64, 16, np.float64, "f64", 8),
    (64, 64, 0, np.float64, "f64", 8),        # one window: no neighbour
    (90, 64, 26, np.float64, "f32", 8),       # l = 27 = ez + 1: no neighbour
    (91, 64, 26, np.float64, "f32", 8),       # l = 28: exactly one admissible pair
])
def test_selfjoin_shapes(n, m, ez, dtype, precision, slots):
    T = random_walk(n, n * 7 + m, dtype)
    tol = 1e-9 if precision == "f64" else 1e-3 * np.sqrt(m)
    if dtype == np.float32:   # P is returned in the input dtype
        tol = max(tol, 2.0 ** -23 * 2 * np.sqrt(m))
    P, I = _run(T, m, ez, precision, slots)
    Po, Io = cimpl.selfjoin(T.astype(np.float64), m, ez)
    compare_profile(T.astype(np.float64), m, P, I, Po, Io, tol, ez=ez, where=f"{n},{m},{ez}")


@pytest.mark.parametrize("reseed", [64, 256, 1024])
def test_tiling_does_not_change_the_answer(reseed):
    """Traversal order is free (the paper's modes return equal results): other
    tile heights give the same P and, up to ties, the same I."""
    T, m, ez = selfjoin_small()
    P, I = _run(T, m, ez, "f64", reseed=reseed)
    P0, I0 = _run(T, m, ez, "f64")
    np.testing.assert_allclose(P, P0, atol=1e-9)
    Po, Io = cimpl.selfjoin(T, m, ez)
    compare_profile(T, m, P, I, Po, Io, 1e-9, ez=ez)


def test_raw_key_profile_without_fp64_finalize():
    T, m, ez = selfjoin_small()
    P, I = _run(T, m, ez, "f32", finalize=False)
    Po, Io = cimpl.selfjoin(T, m, ez)
    compare_profile(T, m, P, I, Po, Io, 1e-3 * np.sqrt(m), ez=ez)


def test_deterministic_reruns():
    T = random_walk(20000, 11, np.float32)
    a = _run(T, 128, 32, "f32")
    b = _run(T, 128, 32, "f32")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_affine_invariance_large_offset():
    """P(aT + b) = P(T); b = 1e6 stresses the FP32 sweep (the series itself
    is first rounded to float32, the oracle sees the same values)."""
    T = random_walk(6000, 17, np.float64)
    m, ez = 50, 13
    T2 = (-0.5 * T + 1e6).astype(np.float32).astype(np.float64)
    P, I = _run(T2, m, ez, "f32")
    Po, Io = cimpl.selfjoin(T2, m, ez)
    compare_profile(T2, m, P, I, Po, Io, 1e-3 * np.sqrt(m), ez=ez)


def test_constant_and_nonfinite_windows():
    rng = np.random.default_rng(8)
    m, ez = 16, 4
    T = np.cumsum(rng.standard_normal(3000))
    T[500:500 + 2 * m] = 2.0          # constant windows
    T[1500:1500 + m + 3] = -7.0       # more constant windows
    T[2200] = np.nan                  # invalid windows
    T[2600] = np.inf
    for prec in ("f64", "f32"):
        P, I = _run(T, m, ez, prec)
        Po, Io = O.selfjoin(T, m, ez)
        compare_profile(T, m, P, I, Po, Io, 1e-9 if prec == "f64" else 1e-3 * np.sqrt(m), ez=ez,
                        where=prec)


def test_invalid_neighbour_rescan():
    """A row whose every admissible valid neighbour is anti-correlated
    (P > sqrt(2m)) must not pick an invalid window: the sweep scores pairs
    with an invalid column like rho = 0, so such rows go through the exact
    rescan."""
    m, ez = 3, 1
    rng = np.random.default_rng(0)
    T = rng.standard_normal(10)
    T[int(rng.integers(3, 9))] = np.nan
    Po, Io = O.selfjoin(T, m, ez)
    assert Po[0] > np.sqrt(2 * m)          # the case this test is about
    for prec in ("f64", "f32"):
        P, I = _run(T, m, ez, prec)
        compare_profile(T, m, P, I, Po, Io, 1e-9 if prec == "f64" else 1e-3 * np.sqrt(m), ez=ez)


def test_sine_profile_is_zero():
    t = np.arange(4000)
    T = np.sin(2 * np.pi * t / 97)
    P, I = _run(T, 64, 16, "f32")
    assert np.max(P) < 1e-3


@pytest.mark.parametrize("m,precision", [(64, "f64"), (64, "f32"), (256, "f64"), (256, "f32")])
def test_paper_walk_with_exact_ties(m, precision):
    """The paper's speed-test input, a +-1 random walk of n = 40000, with the
    steps of one window copied to two more places: the three windows differ
    only by an offset, so each has two partners at distance exactly 0 (a tie
    the tie rule decides).  Every row: admissible, and the reported P is the
    exact FP64 distance of the reported pair within the tolerance; the three
    copies find each other at 0; sampled rows against the oracle."""
    from workloads import paper_walk
    T = paper_walk()
    steps = np.diff(T)
    a, b, c = 5000, 20000, 33000
    steps[b:b + m - 1] = steps[a:a + m - 1]
    steps[c:c + m - 1] = steps[a:a + m - 1]
    T = np.concatenate([[T[0]], T[0] + np.cumsum(steps)])
    n, ez = T.size, m // 2
    l = n - m + 1
    Th = T if precision == "f64" else T.astype(np.float32).astype(np.float64)
    dt = np.float64 if precision == "f64" else np.float32
    P, I = _run(Th.astype(dt), m, ez, precision)
    P = P.astype(np.float64)
    tol = 1e-9 if precision == "f64" else 1e-3 * np.sqrt(m)
    assert np.all(np.isfinite(P)) and np.all(np.abs(I - np.arange(l)) > ez) and np.all((I >= 0) & (I < l))
    for w in (a, b, c):
        assert P[w] <= tol and I[w] in {a, b, c} - {w}, (w, P[w], I[w])
    rng = np.random.default_rng(40 + m)
    for i in rng.choice(l, 200, replace=False):
        assert abs(P[i] - O.pair_distance(Th, int(i), Th, int(I[i]), m)) <= tol
    rows = np.unique(np.concatenate([rng.choice(l, 125, replace=False), [a, b, c]]))
    Po, Io = cimpl.selfjoin_rows(Th, m, ez, rows)
    compare_profile(Th, m, P[rows], I[rows], Po, Io, tol, ez=ez, where=f"m={m} {precision}", rows=rows)
    assert Io[np.searchsorted(rows, b)] == a   # the oracle's tie rule: the smallest index


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("m", [2048, 2304])
def test_long_window(precision, m):
    """Windows of 2048 and 2304 samples (eight and nine times the largest
    elsewhere): long FP64 seeds, and in the FP32 sweep a cross product of
    size ~m sigma^2 carried over whole tiles; 2304 is past the window
    statistics' and the finalize's LDS tile, so they read the series from
    global memory.  Sampled rows against the oracle; every row admissible
    and consistent with its reported pair."""
    n, ez = 24000, m // 4
    T = random_walk(n, 91, np.float32)
    Th = T.astype(np.float64)
    # the FP64 path on float64 input (P comes back in the input's type)
    P, I = _run(Th if precision == "f64" else T, m, ez, precision)
    P = P.astype(np.float64)
    l = n - m + 1
    tol = 1e-9 if precision == "f64" else 1e-3 * np.sqrt(m)
    assert np.all(np.isfinite(P)) and np.all(np.abs(I - np.arange(l)) > ez) and np.all((I >= 0) & (I < l))
    assert np.all(P <= 2 * np.sqrt(m) + tol)
    rng = np.random.default_rng(92)
    rows = np.unique(np.concatenate([rng.choice(l, 90, replace=False), [0, l - 1]]))
    for i in rows[:30]:
        assert abs(P[i] - O.pair_distance(Th, int(i), Th, int(I[i]), m)) <= tol
    Po, Io = cimpl.selfjoin_rows(Th, m, ez, rows)
    compare_profile(Th, m, P[rows], I[rows], Po, Io, tol, ez=ez, where=f"m={m} {precision}", rows=rows)


def test_exact_tie_order_of_the_fp64_sweep():
    """Exact ties (integer +-1 walk, m = 64: every quantity of the FP64
    sweep is a dyadic rational computed without rounding up to the key, so
    equal distances give bitwise equal keys).  Copies of one window's steps
    at a, a2 = a + 100 and c: all three windows differ by an offset only.
      row a: right partners a2 and c (distance 0) in different strips ->
             the packed global minimum takes the smallest index, a2;
      row a2: left partner a and right partner c -> a (the packed minimum
             across the row and column paths takes the smaller index);
      row c: left partners a and a2.  With tiles of 64 rows their cells lie
             in different tiles, whose column minima meet in the packed
             minimum: a.  With 4096-row tiles both cells share a tile, where
             the in-wave minimum orders equal keys by their diagonal code,
             not by index: either copy may come out (both at P = 0).
    The oracle takes the smallest index: a2, a, a."""
    from workloads import paper_walk
    T = paper_walk()
    m, ez = 64, 32
    steps = np.diff(T)
    a, a2 = 5000, 5100
    # c chosen so that offsets c - a2 and c - a fall in one strip of the
    # FP64 sweep (W = 512 offsets, strips start at ez + 1)
    W = 512
    s = (30000 - a - (ez + 1)) // W
    c = a + ez + 1 + s * W + 150
    assert (c - a2 - (ez + 1)) // W == (c - a - (ez + 1)) // W
    for p in (a2, c):
        steps[p:p + m - 1] = steps[a:a + m - 1]
    T = np.concatenate([[T[0]], T[0] + np.cumsum(steps)])
    Po, Io = cimpl.selfjoin_rows(T, m, ez, np.array([a, a2, c]))
    assert list(Io) == [a2, a, a] and list(Po) == [0.0, 0.0, 0.0]
    P, I = _run(T, m, ez, "f64", reseed=64)
    assert P[a] == 0.0 and P[a2] == 0.0 and P[c] == 0.0
    assert (I[a], I[a2], I[c]) == (a2, a, a)
    assert a // 4096 == a2 // 4096
    P, I = _run(T, m, ez, "f64", reseed=4096)
    assert P[a] == 0.0 and P[a2] == 0.0 and P[c] == 0.0
    assert (I[a], I[a2]) == (a2, a) and I[c] in (a, a2)


def test_joins_in_flight_on_two_streams():
    """Two self-joins in flight at once on two streams, each call with its own
    workspace and outputs, return bitwise what the same joins return one after
    the other: nothing is shared between calls."""
    import paper_1904_12626_amd as mpx
    TA, TB = random_walk(6000, 21, np.float32), random_walk(5000, 22, np.float64)
    a, b = torch.from_numpy(TA).to(DEV), torch.from_numpy(TB).to(DEV)
    PA0, IA0 = mpx.selfjoin(a, 50, 12)
    PB0, IB0 = mpx.selfjoin(b, 64, 16, precision="f64")
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    outs = []
    for _ in range(4):
        with torch.cuda.stream(s1):
            ra = mpx.selfjoin(a, 50, 12, stream=s1)
        with torch.cuda.stream(s2):
            rb = mpx.selfjoin(b, 64, 16, precision="f64", stream=s2)
        outs.append((ra, rb))
    torch.cuda.synchronize()
    for (PA, IA), (PB, IB) in outs:
        assert torch.equal(PA, PA0) and torch.equal(IA, IA0)
        assert torch.equal(PB, PB0) and torch.equal(IB, IB0)
    Po, Io = cimpl.selfjoin(TB, 64, 16)
    compare_profile(TB, 64, PB0.cpu().numpy(), IB0.cpu().numpy(), Po, Io, 1e-9, ez=16, where="two streams")


@pytest.mark.parametrize("scale", [1e-18, 1e-10, 1e10, 1e18, 1e19])
def test_scale_invariance_fp32(scale):
    """The z-normalised profile does not depend on the scale of the series.
    The FP32 sweep's cross products (about m sigma^2 unscaled) would leave
    FP32's range at both ends; each series' records carry a power of two
    that keeps them near 1."""
    T = random_walk(3000, 43, np.float64)
    m, ez = 64, 16
    P, I = _run(T * scale, m, ez, "f32")
    Po, Io = cimpl.selfjoin(T, m, ez)
    compare_profile(T, m, P, I, Po, Io, 1e-3 * np.sqrt(m), ez=ez, where=f"scale {scale:g}")


@pytest.mark.parametrize("precision,tol", [("f32", 1e-3), ("f64", 1e-9)])
@pytest.mark.parametrize("scale", [1e-150, 1e140])
def test_magnitudes_near_the_fp64_limits(scale, precision, tol):
    """Series whose squared window sums are still finite in FP64 (the seeds
    and the oracle form them from raw samples).  At 1e-150 the spread of the
    samples asks for a power of two beyond 2^500, which is clamped there; the
    scaled records are still far inside FP32's range."""
    T = random_walk(2500, 47, np.float64)
    m, ez = 40, 10
    P, I = _run(T * scale, m, ez, precision)
    Po, Io = cimpl.selfjoin(T, m, ez)
    compare_profile(T, m, P, I, Po, Io, tol * np.sqrt(m), ez=ez,
                    where=f"scale {scale:g} {precision}")


def test_regimes_of_very_different_magnitude():
    """A series whose first half moves by 1e-12 and second half by 1e10: the
    FP32 sweep's per-series power of two leaves room for both (the small
    windows keep their precision, the large ones do not overflow)."""
    rng = np.random.default_rng(80)
    n = 4000
    T = np.concatenate([np.cumsum(rng.standard_normal(n // 2)) * 1e-12,
                        np.cumsum(rng.standard_normal(n // 2)) * 1e10])
    m, ez = 48, 12
    P, I = _run(T, m, ez, "f32")
    Po, Io = cimpl.selfjoin(T, m, ez)
    compare_profile(T, m, P, I, Po, Io, 1e-3 * np.sqrt(m), ez=ez, where="regimes")
