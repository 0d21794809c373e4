"""Pins of the FP64 CPU oracle against facts fixed outside the oracle itself:
values the paper prints, library special cases (scipy z-score + cdist, the
Pearson identity through numpy.corrcoef), a pure-Python rendering of the
definition on tiny inputs, closed forms, invariants and metamorphic
relations.  Each test names the slip it would catch."""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial.distance import cdist
from scipy.stats import zscore

from oracle import cimpl
from oracle import mp_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- paper sizes

def test_paper_printed_sizes():
    """Profile size n-m+1 and ez = ceil(frac*m) as printed by the paper
    (an off-by-one in l or a round-half-even zone fails here)."""
    with open(os.path.join(GOLDEN, "paper_sizes.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        if c["n"] is not None:
            assert O.profile_length(c["n"], c["m"]) == c["profile_size"], c["cite"]
        assert O.exclusion_zone(c["m"], Fraction(c["frac"])) == c["ez"], c["cite"]


# ------------------------------------------------------- definition, tiny cases

def _pure_python_selfjoin(T, m, ez):
    """The definition written with Python floats and loops only."""
    n = len(T)
    l = n - m + 1

    def z(i):
        w = [float(x) for x in T[i:i + m]]
        mu = sum(w) / m
        sd = math.sqrt(sum((x - mu) ** 2 for x in w) / m)
        return [(x - mu) / sd for x in w]

    Z = [z(i) for i in range(l)]
    P, I = [], []
    for i in range(l):
        best, arg = math.inf, -1
        for j in range(l):
            if abs(i - j) <= ez:
                continue
            d = math.sqrt(sum((a - b) ** 2 for a, b in zip(Z[i], Z[j])))
            if d < best:
                best, arg = d, j
        P.append(best)
        I.append(arg)
    return np.array(P), np.array(I)


@pytest.mark.parametrize("seed,n,m,ez", [(0, 24, 3, 1), (1, 40, 8, 2), (2, 33, 2, 0), (3, 50, 8, 4)])
def test_oracle_equals_pure_python(seed, n, m, ez):
    T = np.random.default_rng(seed).standard_normal(n).cumsum()
    P, I = O.selfjoin(T, m, ez)
    P2, I2 = _pure_python_selfjoin(T, m, ez)
    np.testing.assert_allclose(P, P2, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(I, I2)


@pytest.mark.parametrize("seed,n,m", [(0, 64, 2), (1, 64, 3), (2, 60, 8), (3, 45, 8)])
def test_distance_matrix_matches_scipy_and_corrcoef(seed, n, m):
    """D from the oracle == cdist of scipy z-scores (ddof=0) == sqrt(2m(1-rho))
    from numpy.corrcoef (a wrong std convention or dropped term fails)."""
    T = np.random.default_rng(seed).standard_normal(n).cumsum()
    W = np.lib.stride_tricks.sliding_window_view(T, m)
    D = O.distance_matrix(T, m)
    Zs = zscore(W, axis=1, ddof=0)
    np.testing.assert_allclose(D, cdist(Zs, Zs), rtol=0, atol=1e-12)
    rho = np.corrcoef(W)
    Dp = np.sqrt(np.maximum(2 * m * (1 - rho), 0.0))
    np.testing.assert_allclose(D, Dp, rtol=0, atol=1e-6)


def test_selfjoin_is_rowmin_of_distance_matrix_with_zone():
    T = np.random.default_rng(7).standard_normal(80).cumsum()
    m, ez = 8, 2
    D = O.distance_matrix(T, m)
    l = D.shape[0]
    ii, jj = np.meshgrid(np.arange(l), np.arange(l), indexing="ij")
    D[np.abs(ii - jj) <= ez] = np.inf
    P, I = O.selfjoin(T, m, ez)
    np.testing.assert_allclose(P, D.min(axis=1), atol=1e-12)
    np.testing.assert_array_equal(I, D.argmin(axis=1))


def test_exclusion_zone_boundary_is_inclusive():
    """|i-j| <= ez is excluded, |i-j| = ez+1 is admissible: an exact repeat
    at distance p is found when ez = p-1 and skipped when ez = p."""
    rng = np.random.default_rng(11)
    m, p = 12, 5
    base = rng.standard_normal(p)
    T = np.concatenate([np.tile(base, 8), rng.standard_normal(60).cumsum() + 40])
    P, I = O.selfjoin(T, m, p - 1)
    assert P[0] < 1e-7 and I[0] == p
    P, I = O.selfjoin(T, m, p)
    assert P[0] < 1e-7 and I[0] == 2 * p


# ------------------------------------------------------------------ closed forms

def test_bounds_attained_population_std():
    """d(w, -w) = 2 sqrt(m) exactly and d(w, a*w+b) = 0: only the
    population-std z-normalisation gives both."""
    rng = np.random.default_rng(3)
    m = 16
    w = rng.standard_normal(m)
    T = np.concatenate([w, rng.standard_normal(10), -w, rng.standard_normal(10), 3 * w + 7])
    j1, j2 = m + 10, 2 * m + 20
    assert abs(O.pair_distance(T, 0, T, j1, m) - 2 * math.sqrt(m)) < 1e-12
    assert O.pair_distance(T, 0, T, j2, m) < 1e-12


def test_planted_copy_points_both_ways():
    rng = np.random.default_rng(5)
    m = 32
    T = rng.standard_normal(600).cumsum()
    T[400:400 + m] = 0.5 * T[100:100 + m] - 9.0
    P, I = O.selfjoin(T, m, m // 4)
    assert P[100] < 1e-7 and P[400] < 1e-7
    assert I[100] == 400 and I[400] == 100


def test_sine_integer_period_profile_is_zero():
    p, m = 37, 20
    t = np.arange(400)
    T = np.sin(2 * np.pi * t / p)
    P, I = O.selfjoin(T, m, m // 4)
    assert np.max(P) < 1e-6
    assert np.all(np.abs(np.abs(np.arange(len(P)) - I) % p) == 0)


# --------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(4))
def test_selfjoin_invariants(seed):
    rng = np.random.default_rng(seed)
    n, m = 300, int(rng.integers(4, 40))
    ez = m // 4
    T = rng.standard_normal(n).cumsum()
    P, I = O.selfjoin(T, m, ez)
    l = n - m + 1
    assert P.shape == (l,)
    assert np.all(P >= 0) and np.all(P <= 2 * math.sqrt(m) + 1e-12)
    assert np.all(np.abs(np.arange(l) - I) > ez)
    assert np.all((I >= 0) & (I < l))
    for i in range(0, l, 7):
        assert abs(P[i] - O.pair_distance(T, i, T, I[i], m)) < 1e-12
    assert np.all(P[I] <= P + 1e-12)


def test_affine_invariance_and_reversal():
    rng = np.random.default_rng(9)
    m, ez = 16, 4
    T = rng.standard_normal(250).cumsum()
    P, I = O.selfjoin(T, m, ez)
    P2, I2 = O.selfjoin(-0.37 * T + 1e6, m, ez)
    np.testing.assert_allclose(P, P2, atol=1e-6)
    Pr, _ = O.selfjoin(T[::-1].copy(), m, ez)
    np.testing.assert_allclose(Pr[::-1], P, atol=1e-10)


def test_abjoin_properties():
    rng = np.random.default_rng(4)
    m = 10
    A = rng.standard_normal(120).cumsum()
    B = rng.standard_normal(90).cumsum()
    Pab, Iab, Pba, Iba = O.abjoin(A, B, m)
    assert abs(Pab.min() - Pba.min()) < 1e-12
    for i in range(0, Pab.size, 5):
        assert abs(Pab[i] - O.pair_distance(A, i, B, Iab[i], m)) < 1e-12
    for j in range(0, Pba.size, 5):
        assert abs(Pba[j] - O.pair_distance(A, Iba[j], B, j, m)) < 1e-12
    # joined with itself: every window finds itself at distance 0
    Pss, Iss, _, _ = O.abjoin(A, A, m)
    assert np.max(Pss) < 1e-7
    np.testing.assert_array_equal(Iss, np.arange(Pss.size))


# ------------------------------------------------------- degenerate windows

def test_constant_windows():
    """Reading: a constant window z-normalises to zero, so d(const, x) =
    sqrt(m) and d(const, const) = 0."""
    rng = np.random.default_rng(2)
    m = 8
    T = rng.standard_normal(200).cumsum()
    T[50:50 + m] = 3.0
    T[150:150 + m] = -1.0
    assert O.pair_distance(T, 50, T, 150, m) == 0.0
    assert abs(O.pair_distance(T, 50, T, 10, m) - math.sqrt(m)) < 1e-12
    P, I = O.selfjoin(T, m, 2)
    assert P[50] == 0.0 and I[50] == 150
    assert P[150] == 0.0 and I[150] == 50
    Pc, Ic = cimpl.selfjoin(T, m, 2)
    np.testing.assert_allclose(Pc, P, atol=1e-12)
    np.testing.assert_array_equal(Ic, I)


def test_non_finite_windows_are_invalid():
    rng = np.random.default_rng(6)
    m, ez = 8, 2
    T = rng.standard_normal(150).cumsum()
    T[70] = np.nan
    T[100] = np.inf
    P, I = O.selfjoin(T, m, ez)
    bad = np.zeros(P.size, bool)
    for q in (70, 100):
        bad[max(0, q - m + 1):q + 1] = True
    assert np.all(np.isinf(P[bad])) and np.all(I[bad] == -1)
    assert np.all(np.isfinite(P[~bad]))
    assert not np.any(bad[I[~bad]])
    Pc, Ic = cimpl.selfjoin(T, m, ez)
    np.testing.assert_allclose(Pc, P, atol=1e-12)
    np.testing.assert_array_equal(Ic, I)


def test_no_admissible_neighbour():
    T = np.random.default_rng(1).standard_normal(20)
    P, I = O.selfjoin(T, 8, 20)
    assert np.all(np.isinf(P)) and np.all(I == -1)


# ------------------------------------------------------------ C vs numpy

@pytest.mark.parametrize("seed,n,m,ez", [(0, 700, 32, 8), (1, 513, 17, 5), (2, 300, 2, 0)])
def test_c_oracle_matches_numpy_oracle(seed, n, m, ez):
    T = np.random.default_rng(seed).standard_normal(n).cumsum()
    P, I = O.selfjoin(T, m, ez)
    Pc, Ic = cimpl.selfjoin(T, m, ez)
    np.testing.assert_allclose(Pc, P, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(Ic, I)
    rows = np.array([0, 5, n - m, (n - m) // 2])
    Pr, Ir = O.selfjoin_rows(T, m, ez, rows, chunk=97)
    np.testing.assert_allclose(Pr, P[rows], atol=1e-12)
    np.testing.assert_array_equal(Ir, I[rows])


def test_c_abjoin_matches_numpy():
    rng = np.random.default_rng(12)
    A = rng.standard_normal(300).cumsum()
    B = rng.standard_normal(260).cumsum()
    m = 16
    Pab, Iab, Pba, Iba = O.abjoin(A, B, m)
    P1, I1 = cimpl.abjoin_rows(A, B, m, np.arange(Pab.size))
    P2, I2 = cimpl.abjoin_rows(B, A, m, np.arange(Pba.size))
    np.testing.assert_allclose(P1, Pab, atol=1e-12)
    np.testing.assert_array_equal(I1, Iab)
    np.testing.assert_allclose(P2, Pba, atol=1e-12)
    np.testing.assert_array_equal(I2, Iba)


# ------------------------------------------------------------- gradient

def test_reference_gradient_matches_finite_differences():
    rng = np.random.default_rng(21)
    n, m, ez = 120, 12, 3
    T = rng.standard_normal(n).cumsum()
    P, I = O.selfjoin(T, m, ez)
    g = O.reference_gradient(T, m, I, np.ones_like(P))
    h = 1e-6
    for t in rng.choice(n, 25, replace=False):
        Tp, Tm = T.copy(), T.copy()
        Tp[t] += h
        Tm[t] -= h
        fd = (O.profile_sum_loss(Tp, m, I) - O.profile_sum_loss(Tm, m, I)) / (2 * h)
        assert abs(fd - g[t]) <= 1e-5 * max(1.0, abs(fd)), (t, fd, g[t])


def test_reference_gradient_invariants():
    """L is invariant to T -> aT + b, so sum(g) = 0 and T.g = 0."""
    rng = np.random.default_rng(22)
    n, m = 200, 16
    T = rng.standard_normal(n).cumsum()
    P, I = O.selfjoin(T, m, 4)
    gP = rng.uniform(0.5, 1.5, P.size)
    g = O.reference_gradient(T, m, I, gP)
    scale = np.abs(g).sum()
    assert abs(g.sum()) < 1e-12 * scale
    assert abs((T * g).sum()) < 1e-10 * scale * np.abs(T).max()


def test_gradient_fd_through_the_argmin():
    """Central differences of sum(P) with the argmin recomputed agree with
    the fixed-index gradient wherever the index does not flip."""
    rng = np.random.default_rng(23)
    n, m, ez = 90, 10, 2
    T = rng.standard_normal(n).cumsum()
    P, I = O.selfjoin(T, m, ez)
    g = O.reference_gradient(T, m, I, np.ones_like(P))
    h, checked = 1e-5, 0
    for t in rng.permutation(n):
        Tp, Tm = T.copy(), T.copy()
        Tp[t] += h
        Tm[t] -= h
        Pp, Ip = O.selfjoin(Tp, m, ez)
        Pm, Im = O.selfjoin(Tm, m, ez)
        if not (np.array_equal(Ip, I) and np.array_equal(Im, I)):
            continue
        fd = (Pp.sum() - Pm.sum()) / (2 * h)
        assert abs(fd - g[t]) <= 1e-4 * max(1.0, abs(fd))
        checked += 1
        if checked == 12:
            break
    assert checked >= 6


# ------------------------------------------------------------- motifs

def test_top_motifs_recover_planted_pairs():
    """Planted noisy pairs are the top motifs (a member may shift by a few
    samples: a window sliding one step keeps most of the copy)."""
    from workloads import planted_walk
    for seed in (123, 77):
        pw = planted_walk(6000, 64, seed=seed, n_motifs=3, n_discords=2, dtype=np.float64)
        P, I = cimpl.selfjoin(pw.T, pw.m, pw.m // 4)
        found = [tuple(sorted(p)) for p in O.top_motifs(P, I, pw.m, 3)]
        for a, b in pw.motif_pairs:
            assert any(abs(a - x) <= pw.m // 8 and abs(b - y) <= pw.m // 8 for x, y in found)


def test_top_discords_recover_planted_bursts():
    """Windows overwritten by white noise are the top discords (the masked
    argmax of P lands within m of each burst)."""
    from workloads import planted_walk
    for seed in (123, 77):
        pw = planted_walk(6000, 64, seed=seed, n_motifs=3, n_discords=2, dtype=np.float64)
        P, _ = cimpl.selfjoin(pw.T, pw.m, pw.m // 4)
        for d in O.top_discords(P, pw.m, 2):
            assert min(abs(d - b) for b in pw.discords) <= pw.m


def test_top_discord_on_corrupted_sine():
    """A sine with one cycle replaced by noise: the top discord overlaps the
    corruption, and the motif pairs lie a whole number of periods apart."""
    p, m = 50, 40
    t = np.arange(3000)
    T = np.sin(2 * np.pi * t / p)
    T[1500:1550] = np.random.default_rng(0).standard_normal(50)
    P, I = O.selfjoin(T, m, m // 4)
    d = O.top_discords(P, m, 1)[0]
    assert 1500 - m < d < 1550
    for i, j in O.top_motifs(P, I, m, 3):
        assert abs(i - j) % p == 0


# ----------------------------------------------- restricted and one-sided joins

def _pure_python_restricted(T, m, ez, allowed, side):
    """Definition by loops: every pair through pair_distance."""
    l = len(T) - m + 1
    P = np.full(l, np.inf)
    I = np.full(l, -1, dtype=np.int64)
    for i in range(l):
        for j in range(l):
            k = j - i
            if abs(k) <= ez or not allowed[abs(k)]:
                continue
            if (side == "right" and k < 0) or (side == "left" and k > 0):
                continue
            d = O.pair_distance(T, i, T, j, m)
            if d < P[i]:
                P[i], I[i] = d, j
    return P, I


@pytest.mark.parametrize("side", ["both", "left", "right"])
def test_restricted_join_equals_loops(side):
    rng = np.random.default_rng(40)
    T = np.cumsum(rng.standard_normal(70))
    m, ez = 8, 2
    l = len(T) - m + 1
    allowed = rng.random(l) < 0.4
    P, I = O.selfjoin_restricted(T, m, ez, allowed, side)
    Pl, Il = _pure_python_restricted(T, m, ez, allowed, side)
    np.testing.assert_allclose(P, Pl, rtol=0, atol=1e-12)
    assert np.array_equal(I, Il)
    Pc, Ic = cimpl.selfjoin_rows_restricted(T, m, ez, np.arange(l), allowed, side)
    np.testing.assert_allclose(Pc, P, rtol=0, atol=1e-12)
    assert np.array_equal(Ic, I)


def test_left_right_profiles_compose_the_profile():
    """min(left, right) is the profile, the left one winning ties (its index
    is the smaller); no left neighbour for i <= ez, no right one for
    i >= l - 1 - ez."""
    T = np.cumsum(np.random.default_rng(41).standard_normal(400))
    m, ez = 20, 5
    P, I = O.selfjoin(T, m, ez)
    PL, IL = O.selfjoin_restricted(T, m, ez, side="left")
    PR, IR = O.selfjoin_restricted(T, m, ez, side="right")
    right = (IL < 0) | ((IR >= 0) & (PR < PL))
    assert np.array_equal(np.where(right, PR, PL), P)
    assert np.array_equal(np.where(right, IR, IL), I)
    l = P.size
    assert np.all(np.isinf(PL[:ez + 1])) and np.all(IL[:ez + 1] == -1)
    assert np.all(np.isinf(PR[l - 1 - ez:])) and np.all(IR[l - 1 - ez:] == -1)
    assert np.all(IL[ez + 1:] < np.arange(ez + 1, l) - ez)
    assert np.all(IR[:l - 1 - ez] > np.arange(l - 1 - ez) + ez)


def test_restricted_join_is_monotone_and_exact_on_its_offsets():
    """More offsets never raise P; P[i] = d(i, I[i]) with |i - I[i]| allowed;
    the full offset set gives the self-join."""
    rng = np.random.default_rng(42)
    T = np.cumsum(rng.standard_normal(500))
    m, ez = 24, 6
    l = T.size - m + 1
    a = rng.random(l) < 0.2
    b = a | (rng.random(l) < 0.3)
    Pa, Ia = O.selfjoin_restricted(T, m, ez, a)
    Pb, _ = O.selfjoin_restricted(T, m, ez, b)
    assert np.all(Pb <= Pa)
    for i in rng.choice(l, 20, replace=False):
        if Ia[i] >= 0:
            assert a[abs(i - Ia[i])] and abs(i - Ia[i]) > ez
            assert abs(Pa[i] - O.pair_distance(T, i, T, int(Ia[i]), m)) < 1e-12
    Pf, If = O.selfjoin_restricted(T, m, ez, np.ones(l, dtype=bool))
    P, I = O.selfjoin(T, m, ez)
    assert np.array_equal(Pf, P) and np.array_equal(If, I)


def test_one_sided_profiles_of_a_sine():
    """A sine of integer period p > ez repeats exactly p samples away: the
    left profile vanishes from i = p on, the right one up to i = l - 1 - p."""
    p, m, ez = 25, 20, 5
    T = np.sin(2 * np.pi * np.arange(300) / p)
    PL, IL = O.selfjoin_restricted(T, m, ez, side="left")
    PR, IR = O.selfjoin_restricted(T, m, ez, side="right")
    l = T.size - m + 1
    assert np.all(PL[p:] < 1e-6) and np.all((np.arange(l) - IL)[p:] % p == 0)
    assert np.all(PR[:l - p] < 1e-6) and np.all((IR - np.arange(l))[:l - p] % p == 0)


# ------------------------------------------- segmentation and chains

def test_arc_curve_counts_spanning_arcs():
    rng = np.random.default_rng(70)
    l = 60
    I = rng.integers(-3, l + 3, l)
    I[5] = 5                                      # self arc: none
    ac = O.arc_curve(I)
    for x in range(l):
        want = sum(1 for i in range(l) if 0 <= I[i] < l and I[i] != i and min(i, I[i]) <= x < max(i, I[i]))
        assert ac[x] == want


def test_random_arcs_follow_the_ideal_arc_curve():
    """For arcs to uniformly random other windows, the expected count at x
    under 'min <= x < max' is 2(x+1)(l-1-x)/(l-1) (which the corrected
    curve's 2x(l-x)/l approximates); the mean of many draws agrees within
    its standard error."""
    rng = np.random.default_rng(71)
    l, draws = 120, 3000
    acc = np.zeros(l)
    acc2 = np.zeros(l)
    for _ in range(draws):
        j = rng.integers(0, l - 1, l)
        j = j + (j >= np.arange(l))              # uniform over the others
        a = O.arc_curve(j)
        acc += a
        acc2 += a * a
    mean = acc / draws
    se = np.sqrt(np.maximum(acc2 / draws - mean ** 2, 1e-12) / draws)
    x = np.arange(l)
    want = 2.0 * (x + 1) * (l - 1 - x) / (l - 1)
    assert np.all(np.abs(mean - want) <= 5 * se + 1e-9)


def test_fluss_finds_regime_changes():
    import workloads as W
    T, (b1, b2) = W.regime_series(6000, 7)
    m = 60
    P, I = cimpl.selfjoin(T, m, m // 2)
    cac = O.corrected_arc_curve(I, 5 * m)
    assert np.all(cac[:5 * m] == 1) and np.all(cac[-5 * m:] == 1) and np.all((cac >= 0) & (cac <= 1))
    seg = sorted(O.fluss_segments(cac, 2, 5 * m))
    assert abs(seg[0] - b1) <= m and abs(seg[1] - b2) <= m


def test_chains_by_hand():
    # windows 0..9; confirmed links 1->4->7 and 2->5; 3->6 is not confirmed
    # (IL[6] = 0); 8 -> 9 confirmed
    IL = np.array([-1, -1, -1, -1, 1, 2, 0, 4, -1, 8])
    IR = np.array([3, 4, 5, 6, 7, -1, 9, -1, 9, -1])
    nxt, length, count, best = O.chains(IL, IR, min_len=2)
    assert list(nxt) == [-1, 4, 5, -1, 7, -1, -1, -1, 9, -1]
    assert list(length) == [1, 3, 2, 1, 2, 1, 1, 1, 2, 1]
    assert count == 3 and best == [1, 4, 7]
    assert O.chains(IL, IR, min_len=3)[2] == 1


def test_chains_partition_the_windows_and_follow_an_evolving_pattern():
    import workloads as W
    T, pos = W.evolving_chain(8000, 64, 8, 2)
    m, ez = 64, 16
    rows = np.arange(T.size - m + 1)
    _, IL = cimpl.selfjoin_rows_restricted(T, m, ez, rows, None, "left")
    _, IR = cimpl.selfjoin_rows_restricted(T, m, ez, rows, None, "right")
    nxt, length, count, best = O.chains(IL, IR)
    # every window lies on exactly one chain: chain lengths at the first
    # windows add up to l, and no window has two confirmed predecessors
    heads = [i for i in rows if not (0 <= IL[i] < i and nxt[IL[i]] == i)]
    assert sum(int(length[h]) for h in heads) == rows.size
    succ = nxt[nxt >= 0]
    assert np.unique(succ).size == succ.size
    for p in pos:
        assert any(abs(b - p) <= m // 8 for b in best), (p, best)


def test_ab_reference_gradient_matches_finite_differences():
    """Central differences (h = 1e-6) of the weighted AB loss with fixed
    indices on every coordinate of A and B."""
    rng = np.random.default_rng(100)
    A = np.cumsum(rng.standard_normal(60))
    B = np.cumsum(rng.standard_normal(45))
    m = 8
    Pab, Iab, Pba, Iba = O.abjoin(A, B, m)
    wab = rng.uniform(0.5, 1.5, Iab.size)
    wba = rng.uniform(0.5, 1.5, Iba.size)
    gA, gB = O.reference_gradient_ab(A, B, m, Iab, wab, Iba, wba)
    h = 1e-6
    for X, gX, isA in ((A, gA, True), (B, gB, False)):
        for t in range(X.size):
            Xp, Xm = X.copy(), X.copy()
            Xp[t] += h
            Xm[t] -= h
            if isA:
                fd = (O.abjoin_sum_loss(Xp, B, m, Iab, wab, Iba, wba) - O.abjoin_sum_loss(Xm, B, m, Iab, wab, Iba, wba)) / (2 * h)
            else:
                fd = (O.abjoin_sum_loss(A, Xp, m, Iab, wab, Iba, wba) - O.abjoin_sum_loss(A, Xm, m, Iab, wab, Iba, wba)) / (2 * h)
            assert abs(fd - gX[t]) <= 1e-6 * max(1.0, abs(fd)), (isA, t, fd, gX[t])
    # each row's contribution is shift invariant: the gradients sum to zero
    assert abs(gA.sum() + gB.sum()) < 1e-9


# ------------------------------------------- SiMPle and multidimensional

def test_simple_join_is_plain_euclidean():
    """SiMPle = Euclidean distance of raw windows (all dimensions stacked):
    scipy cdist on the concatenated windows, row minimum outside the zone;
    and it is not shift invariant, unlike the z-normalised profile."""
    rng = np.random.default_rng(120)
    T = np.cumsum(rng.standard_normal((3, 150)), axis=1)
    m, ez = 10, 3
    l = 150 - m + 1
    X = np.concatenate([np.lib.stride_tricks.sliding_window_view(T[d], m) for d in range(3)], axis=1)
    Dm = cdist(X, X)
    Dm[np.abs(np.arange(l)[:, None] - np.arange(l)[None, :]) <= ez] = np.inf
    P, I = O.simple_join(T, m, ez)
    np.testing.assert_allclose(P, Dm.min(axis=1), rtol=0, atol=1e-10)
    assert np.array_equal(I, Dm.argmin(axis=1))
    P2, _ = O.simple_join(T + 5.0, m, ez)
    np.testing.assert_allclose(P2, P, atol=1e-9)       # a common offset cancels
    P3, _ = O.simple_join(T * np.array([[1.0], [1.0], [3.0]]), m, ez)
    assert not np.allclose(P3, P)
    # AB form
    B = np.cumsum(rng.standard_normal((3, 90)), axis=1)
    Pab, Iab = O.simple_join(T, m, TB=B)
    XB = np.concatenate([np.lib.stride_tricks.sliding_window_view(B[d], m) for d in range(3)], axis=1)
    np.testing.assert_allclose(Pab, cdist(X, XB).min(axis=1), rtol=0, atol=1e-10)


def test_mstomp_one_dimension_is_the_profile_and_loops_agree():
    rng = np.random.default_rng(121)
    T = np.cumsum(rng.standard_normal(200))
    m, ez = 12, 3
    P, I = O.mstomp(T[None, :], m, ez)
    P1, I1 = O.selfjoin(T, m, ez)
    np.testing.assert_allclose(P[0], P1, rtol=0, atol=1e-12)
    assert np.array_equal(I[0], I1)
    # pair-by-pair loops on a 3-dimensional series
    T3 = np.cumsum(rng.standard_normal((3, 60)), axis=1)
    m = 6
    P, I = O.mstomp(T3, m, 2)
    l = 60 - m + 1
    for i in range(0, l, 7):
        best = np.full(3, np.inf)
        arg = np.full(3, -1)
        for j in range(l):
            if abs(i - j) <= 2:
                continue
            ds = np.sort([O.pair_distance(T3[d], i, T3[d], j, m) for d in range(3)])
            for k in range(3):
                v = ds[:k + 1].mean()
                if v < best[k]:
                    best[k], arg[k] = v, j
        np.testing.assert_allclose(P[:, i], best, rtol=0, atol=1e-12)
        assert np.array_equal(I[:, i], arg)


def test_mstomp_finds_a_motif_living_in_some_dimensions():
    """A pattern planted in dimensions 0 and 2 only: the 2-dimensional
    profile pairs the copies; using every dimension (k = 3) does not."""
    rng = np.random.default_rng(122)
    n, m = 800, 32
    T = np.cumsum(rng.standard_normal((3, n)), axis=1)
    pat = rng.standard_normal((2, m)) * 3
    for p in (150, 600):
        T[0, p:p + m] = T[0, p] + pat[0] + rng.normal(0, 0.05, m)
        T[2, p:p + m] = T[2, p] + pat[1] + rng.normal(0, 0.05, m)
    P, I = O.mstomp(T, m, m // 4)
    assert abs(int(I[1, 150]) - 600) <= 2 and abs(int(I[1, 600]) - 150) <= 2
    assert P[1, 150] < 0.5 * np.median(P[1])
    assert P[2, 150] > P[1, 150]


def _two_readings_series():
    """Two dimensions, m = 4, three valid windows separated by NaN samples
    (windows over a NaN are invalid, so rows 0, 5 and 10 see only each
    other).  Built from the Walsh patterns w1 = [1,1,-1,-1], w2 = [1,-1,-1,1],
    w3 = [1,-1,1,-1]: zero mean, population std 1, mutually orthogonal, so
    z-normalisation leaves them as they are and d^2 = 2m(1 - rho) = 8(1 - rho).
      window 0  (query)  dim 1: w3,                dim 2: w3
      window 5  (A)      dim 1: w3,                dim 2: -w3
      window 10 (B)      dim 1: c w3 + s w1,       dim 2: c w3 + s w2
    with c = 7/32, s = sqrt(1 - c^2) (zero mean, std 1, rho with w3 = c)."""
    c = 7.0 / 32.0
    s = np.sqrt(1.0 - c * c)
    w1 = np.array([1.0, 1.0, -1.0, -1.0])
    w2 = np.array([1.0, -1.0, -1.0, 1.0])
    w3 = np.array([1.0, -1.0, 1.0, -1.0])
    nan = np.array([np.nan])
    d1 = np.concatenate([w3, nan, w3, nan, c * w3 + s * w1])
    d2 = np.concatenate([w3, nan, -w3, nan, c * w3 + s * w2])
    return np.stack([d1, d2])


def test_mstomp_hand_worked_case_fixes_the_mean_of_distances():
    """Pins the k-dimensional distance as the mean of the k smallest
    per-dimension distances (Section 3.3.5 reading), not the root of the
    mean of squared distances, on a case where the two choose different
    neighbours.  By hand (d^2 = 8(1 - rho)):
      row 0 vs A: dim 1 rho = 1 -> 0;  dim 2 rho = -1 -> 4
      row 0 vs B: both dims rho = c = 7/32 -> d^2 = 8 * 25/32 = 6.25 -> 2.5
      k = 1: min(0, 2.5) = 0 at A (window 5)
      k = 2: mean of distances A (0 + 4)/2 = 2.0 < B 2.5 -> P = 2.0, I = 5
             (the other reading: A sqrt(16/2) = 2.83 > B 2.5 would give 2.5, I = 10)
      row 10 (B) vs 0: (2.5, 2.5); vs A: dim 1 rho = c -> 2.5, dim 2
             rho = -c -> d^2 = 8 * 39/32 = 9.75 -> 3.1225
      k = 1: 2.5 at both -> the smaller index 0; k = 2: 2.5 (row 0) < 2.811 -> I = 0
      row 5 (A) vs 0: (0, 4); vs B: (2.5, 3.1225) -> k = 1: 0 at 0;
             k = 2: 2.0 at 0 (vs 2.811)
    Every other window holds a NaN: +inf, -1."""
    T = _two_readings_series()
    P, I = O.mstomp(T, 4, 0)
    l = T.shape[1] - 3
    assert P.shape == (2, l)
    want = {0: ((0.0, 5), (2.0, 5)), 5: ((0.0, 0), (2.0, 0)), 10: ((2.5, 0), (2.5, 0))}
    for i in range(l):
        for k in range(2):
            if i in want:
                p, j = want[i][k]
                assert abs(P[k, i] - p) < 1e-12, (i, k, P[k, i], p)
                assert I[k, i] == j, (i, k, I[k, i], j)
            else:
                assert P[k, i] == np.inf and I[k, i] == -1
    # the per-dimension distances the derivation uses
    assert abs(O.pair_distance(T[0], 10, T[0], 5, 4) - 2.5) < 1e-12
    assert abs(O.pair_distance(T[1], 10, T[1], 5, 4) - np.sqrt(9.75)) < 1e-12
