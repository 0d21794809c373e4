"""Multidimensional joins on the GPU: SiMPle (raw Euclidean over all
dimensions) and the k-dimensional profiles, against the FP64 oracle."""

import numpy as np
import pytest
import torch

from oracle import mp_oracle as O

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _simple_dist(A, i, B, j, m):
    return float(np.sqrt(((A[:, i:i + m] - B[:, j:j + m]) ** 2).sum()))


def _multi_dist(T, i, j, m, k):
    ds = np.sort([O.pair_distance(T[d], i, T[d], j, m) for d in range(T.shape[0])])
    return float(ds[:k].mean())


def _compare(P, I, Po, Io, dist, rtol, ez=None, where="", rows=None):
    """P within rtol (relative, 1e-12 absolute floor); a different index is
    accepted when admissible and its exact distance is within the tolerance
    of the oracle's minimum (near-ties).  With `rows`, entry e of the arrays
    belongs to window rows[e]."""
    P, I = np.asarray(P, dtype=np.float64), np.asarray(I)
    fin = np.isfinite(Po)
    assert np.array_equal(np.isfinite(P), fin), where
    assert np.all(I[~fin] == -1), where
    tol = rtol * np.maximum(1.0, np.abs(Po[fin]))
    assert np.all(np.abs(P[fin] - Po[fin]) <= tol), (where, np.max(np.abs(P[fin] - Po[fin])))
    for i in np.nonzero(fin & (I != Io))[0]:
        row = int(rows[i]) if rows is not None else int(i)
        j = int(I[i])
        if ez is not None:
            assert abs(row - j) > ez, where
        assert dist(row, j) <= Po[i] * (1 + rtol) + 1e-12, (where, row, j, Io[i])


@pytest.mark.parametrize("D,dtype", [(1, np.float64), (3, np.float64), (2, np.float32), (5, np.float64)])
def test_simple_selfjoin(D, dtype):
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(130 + D)
    n, m, ez = 2000, 24, 6
    T = np.cumsum(rng.standard_normal((D, n)), axis=1).astype(dtype)
    P, I = mpx.mdjoin(torch.from_numpy(T).to(DEV), m, ez, mode="simple")
    T64 = T.astype(np.float64)
    Po, Io = O.simple_join(T64, m, ez)
    _compare(P.cpu().numpy(), I.cpu().numpy(), Po, Io, lambda i, j: _simple_dist(T64, i, T64, j, m), 1e-6, ez,
             f"D={D}")


def test_simple_abjoin():
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(140)
    A = np.cumsum(rng.standard_normal((2, 1700)), axis=1)
    B = np.cumsum(rng.standard_normal((2, 1300)), axis=1)
    m = 20
    Pab, Iab, Pba, Iba = [x.cpu().numpy() for x in mpx.mdjoin(torch.from_numpy(A).to(DEV), m,
                                                               B=torch.from_numpy(B).to(DEV))]
    Po, Io = O.simple_join(A, m, TB=B)
    _compare(Pab, Iab, Po, Io, lambda i, j: _simple_dist(A, i, B, j, m), 1e-6, where="ab")
    Po, Io = O.simple_join(B, m, TB=A)
    _compare(Pba, Iba, Po, Io, lambda i, j: _simple_dist(B, i, A, j, m), 1e-6, where="ba")


@pytest.mark.parametrize("D", [1, 2, 3])
def test_multidimensional_profiles(D):
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(150 + D)
    n, m, ez = 1200, 20, 5
    T = np.cumsum(rng.standard_normal((D, n)), axis=1)
    P, I = mpx.mdjoin(torch.from_numpy(T).to(DEV), m, ez, mode="multi")
    P, I = P.cpu().numpy(), I.cpu().numpy()
    Po, Io = O.mstomp(T, m, ez)
    for k in range(D):
        _compare(P[k], I[k], Po[k], Io[k], lambda i, j, k=k: _multi_dist(T, i, j, m, k + 1), 1e-6, ez, f"k={k + 1}")
    if D == 1:
        P1, I1 = mpx.selfjoin(torch.from_numpy(T[0]).to(DEV), m, ez, precision="f64")
        np.testing.assert_allclose(P[0], P1.cpu().numpy(), rtol=1e-9, atol=1e-9)


def test_degenerate_windows_and_planted_motif():
    """Constant stretches in one dimension, a NaN in another, and a motif
    planted in dimensions 0 and 2 of 3."""
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(160)
    n, m, ez = 1500, 32, 8
    T = np.cumsum(rng.standard_normal((3, n)), axis=1)
    T[1, 300:380] = 2.0
    T[2, 900] = np.nan
    pat = rng.standard_normal((2, m)) * 3
    for p in (150, 1100):
        T[0, p:p + m] = T[0, p] + pat[0] + rng.normal(0, 0.05, m)
        T[2, p:p + m] = T[2, p] + pat[1] + rng.normal(0, 0.05, m)
    P, I = [x.cpu().numpy() for x in mpx.mdjoin(torch.from_numpy(T).to(DEV), m, ez, mode="multi")]
    Po, Io = O.mstomp(T, m, ez)
    for k in range(3):
        _compare(P[k], I[k], Po[k], Io[k], lambda i, j, k=k: _multi_dist(T, i, j, m, k + 1), 1e-6, ez, f"k={k + 1}")
    assert abs(int(I[1, 150]) - 1100) <= 2
    Ps, Is = [x.cpu().numpy() for x in mpx.mdjoin(torch.from_numpy(T).to(DEV), m, ez, mode="simple")]
    Po, Io = O.simple_join(T, m, ez)
    _compare(Ps, Is, Po, Io, lambda i, j: _simple_dist(T, i, T, j, m), 1e-6, ez, "simple")


@pytest.mark.parametrize("mode", ["simple", "multi"])
def test_eight_dimensions(mode):
    """The largest supported dimension count."""
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(180)
    D, n, m, ez = 8, 700, 16, 4
    T = np.cumsum(rng.standard_normal((D, n)), axis=1)
    P, I = [x.cpu().numpy() for x in mpx.mdjoin(torch.from_numpy(T).to(DEV), m, ez, mode=mode)]
    if mode == "simple":
        Po, Io = O.simple_join(T, m, ez)
        _compare(P, I, Po, Io, lambda i, j: _simple_dist(T, i, T, j, m), 1e-6, ez, "simple D=8")
    else:
        Po, Io = O.mstomp(T, m, ez)
        for k in (0, 3, 7):
            _compare(P[k], I[k], Po[k], Io[k], lambda i, j, k=k: _multi_dist(T, i, j, m, k + 1), 1e-6, ez, f"k={k + 1}")


@pytest.mark.parametrize("mode,D", [("simple", 4), ("simple", 6), ("simple", 7), ("multi", 4), ("multi", 5),
                                    ("multi", 6), ("multi", 7)])
def test_remaining_dimension_counts(mode, D):
    """Dimension counts not covered above: the kernel's slot count and
    whether a row's records are staged in LDS or loaded per row both depend
    on the mode and D."""
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(190 + D + (10 if mode == "multi" else 0))
    n, m, ez = 640, 16, 4
    dtype = np.float32 if D % 2 else np.float64
    T = np.cumsum(rng.standard_normal((D, n)), axis=1).astype(dtype)
    P, I = [x.cpu().numpy() for x in mpx.mdjoin(torch.from_numpy(T).to(DEV), m, ez, mode=mode)]
    T64 = T.astype(np.float64)
    if mode == "simple":
        Po, Io = O.simple_join(T64, m, ez)
        _compare(P, I, Po, Io, lambda i, j: _simple_dist(T64, i, T64, j, m), 1e-6, ez, f"simple D={D}")
    else:
        Po, Io = O.mstomp(T64, m, ez)
        for k in range(D):
            _compare(P[k], I[k], Po[k], Io[k], lambda i, j, k=k: _multi_dist(T64, i, j, m, k + 1), 1e-6, ez,
                     f"D={D} k={k + 1}")


def test_simple_abjoin_float32_and_short_series():
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(181)
    A = np.cumsum(rng.standard_normal((2, 300)), axis=1).astype(np.float32)
    B = np.cumsum(rng.standard_normal((2, 40)), axis=1).astype(np.float32)   # lB = 9: one partial strip
    m = 32
    out = [x.cpu().numpy() for x in mpx.mdjoin(torch.from_numpy(A).to(DEV), m, B=torch.from_numpy(B).to(DEV))]
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    Po, Io = O.simple_join(A64, m, TB=B64)
    _compare(out[0], out[1], Po, Io, lambda i, j: _simple_dist(A64, i, B64, j, m), 1e-6, where="ab")
    Po, Io = O.simple_join(B64, m, TB=A64)
    _compare(out[2], out[3], Po, Io, lambda i, j: _simple_dist(B64, i, A64, j, m), 1e-6, where="ba")


@pytest.mark.parametrize("mode", ["simple", "multi"])
def test_benchmark_size_sampled_rows(mode):
    """The benchmark's multidimensional join (3-dimensional float32 walk,
    n=2^18, m=128, ez=32: thousands of strips of several diagonals per lane)
    on sampled rows against the oracle, plus invariants on every row."""
    import paper_1904_12626_amd as mpx
    n, m, ez = 1 << 18, 128, 32
    T = np.cumsum(np.random.default_rng(7).standard_normal((3, n)), axis=1).astype(np.float32)
    P, I = [x.cpu().numpy() for x in mpx.mdjoin(torch.from_numpy(T).to(DEV), m, ez, mode=mode)]
    T64 = T.astype(np.float64)
    l = n - m + 1
    rows = np.sort(np.random.default_rng(9).choice(l, 8, replace=False))
    if mode == "simple":
        assert np.all(np.isfinite(P)) and np.all(np.abs(I - np.arange(l)) > ez)
        Po, Io = O.simple_join(T64, m, ez, rows=rows)
        _compare(P[rows], I[rows], Po[rows], Io[rows], lambda i, j: _simple_dist(T64, i, T64, j, m), 1e-6, ez,
                 "simple", rows=rows)
    else:
        assert np.all(np.isfinite(P)) and np.all(np.abs(I - np.arange(l)[None, :]) > ez)
        assert np.all(np.diff(P, axis=0) >= -1e-3)   # mean of the k smallest grows with k
        Po, Io = O.mstomp(T64, m, ez, rows=rows)
        for k in range(3):
            _compare(P[k][rows], I[k][rows], Po[k][rows], Io[k][rows],
                     lambda i, j, k=k: _multi_dist(T64, i, j, m, k + 1), 1e-6, ez, f"k={k + 1}", rows=rows)


def test_multi_hand_worked_case():
    """The two-dimensional case whose k = 2 neighbour differs between the
    mean of distances and the root of the mean of squared distances (see the
    oracle pin): the GPU profile follows the mean of distances."""
    import paper_1904_12626_amd as mpx
    from tests.test_oracle_pins import _two_readings_series
    T = _two_readings_series()
    P, I = mpx.mdjoin(torch.from_numpy(T).to(DEV), 4, 0, mode="multi")
    P, I = P.double().cpu().numpy(), I.cpu().numpy()
    Po, Io = O.mstomp(T, 4, 0)
    assert np.array_equal(np.isfinite(P), np.isfinite(Po))
    fin = np.isfinite(Po)
    assert np.max(np.abs(P[fin] - Po[fin])) < 1e-9
    # row 10, k = 1: windows 0 and 5 tie exactly at 2.5 (both are left
    # partners, where the column minimum may keep the larger index); every
    # other entry has a unique minimum
    tie = np.zeros_like(I, dtype=bool)
    tie[0, 10] = True
    assert np.array_equal(I[~tie], Io[~tie])
    assert I[0, 10] in (0, 5)
    assert I[1, 0] == 5 and abs(P[1, 0] - 2.0) < 1e-9


@pytest.mark.parametrize("scale", [1e-25, 1e15, 1e19])
def test_simple_keys_cover_any_magnitude(scale):
    """SiMPle distances carry the data's units (P(aT) = a P(T)), and its
    candidates are merged as 32-bit patterns of the FP64 squared distance
    that cover 2^-511 .. 2^511, so series far outside float's range still
    get the oracle's neighbours."""
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(150)
    n, m, ez = 1500, 24, 6
    T = np.cumsum(rng.standard_normal((3, n)), axis=1)
    P, I = mpx.mdjoin(torch.from_numpy(T * scale).to(DEV), m, ez, mode="simple")
    Po, Io = O.simple_join(T, m, ez)
    _compare(P.cpu().numpy() / scale, I.cpu().numpy(), Po, Io, lambda i, j: _simple_dist(T, i, T, j, m), 1e-6, ez,
             f"scale {scale:g}")
