"""Parity at the benchmark sizes, in the launch configuration bench.py times.

The FP64 oracle is exact on every row it computes, so large joins are
checked on sampled rows (plus every planted window) against it, and in full
against the library's FP64 sweep, whose own parity is established on the
small cases.  Tolerance 1e-3*sqrt(m) on P; indices equal up to near-ties."""

import math

import numpy as np
import pytest
import torch

from oracle import cimpl
from oracle import mp_oracle as O
from tests.parity import compare_profile
import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _np(x):
    return x.double().cpu().numpy() if x.is_floating_point() else x.cpu().numpy()


def _invariants(T64, m, ez, P, I, rng, nsample=64, tol=None):
    """Invariants every self-join profile satisfies: 0 <= P <= 2 sqrt(m),
    admissible indices, P[i] = d(i, I[i]) (sampled) and P[I[i]] <= P[i]:
    window i is an admissible candidate of its own neighbour j = I[i], so
    j's nearest distance is at most d(j, i) = P[i] (exact in FP64, within
    `tol` for the FP32 sweep)."""
    l = P.size
    fin = np.isfinite(P)
    assert fin.all()
    assert np.all(P >= 0) and np.all(P <= 2 * math.sqrt(m) + 1e-3)
    assert np.all((I >= 0) & (I < l))
    if ez is not None:
        assert np.all(np.abs(np.arange(l) - I) > ez)
    for i in rng.choice(l, nsample, replace=False):
        assert abs(P[i] - O.pair_distance(T64, int(i), T64, int(I[i]), m)) < 1e-4
    if ez is not None and tol is not None:
        excess = P[I] - P
        assert excess.max() <= tol, (int(np.argmax(excess)), float(excess.max()))


def test_selfjoin_large_planted_walk():
    """n=2^20 float32 planted random walk, m=256, ez=64 (the benchmark join)."""
    import paper_1904_12626_amd as mpx
    pw, ez = W.selfjoin_large()
    m = pw.m
    Tg = torch.from_numpy(pw.T).to(DEV)
    P32, I32 = mpx.selfjoin(Tg, m, ez)
    P64, I64 = mpx.selfjoin(Tg, m, ez, precision="f64")
    Praw, _ = mpx.selfjoin(Tg, m, ez, fp64_finalize=False)
    # the reversed series: P_rev[l-1-i] = P[i] (the distance is invariant
    # under reversing both windows)
    Prev32, _ = mpx.selfjoin(torch.flip(Tg, [0]).contiguous(), m, ez)
    Prev64, _ = mpx.selfjoin(torch.flip(Tg, [0]).contiguous(), m, ez, precision="f64")
    torch.cuda.synchronize()
    P32, I32, P64, I64, Praw = _np(P32), _np(I32), _np(P64), _np(I64), _np(Praw)
    Prev32, Prev64 = _np(Prev32)[::-1], _np(Prev64)[::-1]
    tol = 1e-3 * math.sqrt(m)
    T64 = pw.T.astype(np.float64)
    rng = np.random.default_rng(0)
    # FP32-mixed vs FP64 GPU path over the whole profile
    assert np.max(np.abs(P32 - P64)) <= tol
    assert np.max(np.abs(Praw - P64)) <= tol
    assert np.mean(I32 == I64) > 0.99
    assert np.max(np.abs(Prev64 - P64)) <= 1e-9
    assert np.max(np.abs(Prev32 - P32)) <= tol
    # exact oracle rows: 256 random rows and every planted window
    rows = list(rng.choice(P32.size, 256, replace=False))
    for a, b in pw.motif_pairs:
        rows += [a, b]
    rows += list(pw.discords)
    rows = np.array(sorted(set(int(r) for r in rows)))
    Po, Io = cimpl.selfjoin_rows(T64, m, ez, rows)
    for P, I, where in ((P32, I32, "f32"), (P64, I64, "f64")):
        for r, po, io in zip(rows, Po, Io):
            if I[r] != io:
                assert abs(r - I[r]) > ez
                assert O.pair_distance(T64, int(r), T64, int(I[r]), m) <= po + tol, (where, r)
        assert np.max(np.abs(P[rows] - Po)) <= tol, where
    _invariants(T64, m, ez, P32, I32, rng, tol=tol)
    _invariants(T64, m, ez, P64, I64, rng, tol=1e-9)
    # planted motif pairs are the top motifs, re-measured in FP64
    idx, dist = mpx.recheck(Tg, m, torch.from_numpy(P32.astype(np.float32)).to(DEV),
                            torch.from_numpy(I32).to(DEV), 8, 4)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    found = [tuple(sorted(p)) for p in idx[:16].reshape(8, 2)]
    for a, b in pw.motif_pairs:
        assert any(abs(a - x) <= m // 8 and abs(b - y) <= m // 8 for x, y in found), (a, b, found)
    for q, (i, j) in enumerate(idx[:16].reshape(8, 2)):
        assert abs(dist[q] - O.pair_distance(T64, int(i), T64, int(j), m)) < 1e-9
    # noisy planted pairs: d ~ sqrt(m * 0.05^2 * (s_a^-2 + s_b^-2)) in [0.57, 2.26]
    assert np.all(dist[:8] > 0.3) and np.all(dist[:8] < 3.0)
    # discords: the white-noise bursts have no match anywhere, and neither
    # do windows that straddle a planted motif copy (its pattern is white
    # noise too, matched only at its own twin); each of the top-4 discords
    # lands within m of a planted window, and every burst is among the top 5
    planted = list(pw.discords) + [x for pr in pw.motif_pairs for x in pr]
    for q, p in enumerate(idx[16:20]):
        assert min(abs(int(p) - b) for b in planted) <= m, (p, planted)
        assert abs(dist[8 + q] - O.pair_distance(T64, int(p), T64, int(I32[p]), m)) < 1e-9
    top5 = O.top_discords(P32, m, 5)
    for b in pw.discords:
        assert min(abs(int(p) - b) for p in top5) <= m, (b, top5)


def test_abjoin_ecg_full():
    """Two n=2^19 float32 ECG-like series, m=128: both directions."""
    import paper_1904_12626_amd as mpx
    A, B, m = W.abjoin_ecg()
    Ag, Bg = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    out32 = [_np(x) for x in mpx.abjoin(Ag, Bg, m)]
    out64 = [_np(x) for x in mpx.abjoin(Ag, Bg, m, precision="f64")]
    tol = 1e-3 * math.sqrt(m)
    assert np.max(np.abs(out32[0] - out64[0])) <= tol
    assert np.max(np.abs(out32[2] - out64[2])) <= tol
    assert abs(out32[0].min() - out32[2].min()) <= tol
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    rng = np.random.default_rng(3)
    ra = rng.choice(out32[0].size, 256, replace=False)
    rb = rng.choice(out32[2].size, 256, replace=False)
    Po, Io = cimpl.abjoin_rows(A64, B64, m, ra)
    for r, po, io in zip(ra, Po, Io):
        for P, I in ((out32[0], out32[1]), (out64[0], out64[1])):
            assert abs(P[r] - po) <= tol
            if I[r] != io:
                assert O.pair_distance(A64, int(r), B64, int(I[r]), m) <= po + tol
    Po, Io = cimpl.abjoin_rows(B64, A64, m, rb)
    for r, po, io in zip(rb, Po, Io):
        for P, I in ((out32[2], out32[3]), (out64[2], out64[3])):
            assert abs(P[r] - po) <= tol
            if I[r] != io:
                assert O.pair_distance(B64, int(r), A64, int(I[r]), m) <= po + tol


def test_batch_ragged_full():
    """512 float32 random walks, lengths U{2048..65536}, m in {32,64,128},
    ez = m/4, one launch sequence; five graph replays equal the eager run."""
    import paper_1904_12626_amd as mpx
    rb = W.batch_ragged()
    Tc, _ = rb.concat()
    plan = mpx.BatchPlan([s.size for s in rb.series], rb.m, rb.ez, dtype=torch.float32, device=DEV)
    Tg = torch.from_numpy(Tc).to(DEV)
    P, I = plan.run(Tg)
    torch.cuda.synchronize()
    Ph, Ih = _np(P), _np(I)
    Ps, Is = plan.split(Ph), plan.split(Ih)
    lens = np.array([s.size for s in rb.series])
    rng = np.random.default_rng(4)
    # full oracle on the 8 shortest series
    for s in np.argsort(lens)[:8]:
        T64 = rb.series[s].astype(np.float64)
        m, ez = rb.m[s], rb.ez[s]
        Po, Io = cimpl.selfjoin(T64, m, ez)
        compare_profile(T64, m, Ps[s], Is[s], Po, Io, 1e-3 * math.sqrt(m), ez=ez, where=f"series {s}")
    # sampled rows on 8 random series
    for s in rng.choice(len(rb.series), 8, replace=False):
        T64 = rb.series[s].astype(np.float64)
        m, ez = rb.m[s], rb.ez[s]
        rows = rng.choice(Ps[s].size, 8, replace=False)
        Po, Io = cimpl.selfjoin_rows(T64, m, ez, rows)
        assert np.max(np.abs(Ps[s][rows] - Po)) <= 1e-3 * math.sqrt(m)
    # a few series against single joins: within the tolerance with automatic
    # tiling, and bitwise with the same tile height (= reseed interval)
    pick = rng.choice(len(rb.series), 3, replace=False)
    for s in pick:
        P1, I1 = mpx.selfjoin(torch.from_numpy(rb.series[s]).to(DEV), rb.m[s], rb.ez[s])
        torch.cuda.synchronize()
        assert np.max(np.abs(_np(P1) - Ps[s])) <= 1e-3 * math.sqrt(rb.m[s])
    fixed = mpx.BatchPlan([s.size for s in rb.series], rb.m, rb.ez, dtype=torch.float32, device=DEV,
                          reseed_rows=1024)
    Pf, If = fixed.run(Tg)
    Pfs, Ifs = fixed.split(_np(Pf)), fixed.split(_np(If))
    for s in pick:
        P1, I1 = mpx.selfjoin(torch.from_numpy(rb.series[s]).to(DEV), rb.m[s], rb.ez[s], reseed_rows=1024)
        torch.cuda.synchronize()
        assert np.array_equal(_np(P1), Pfs[s]) and np.array_equal(_np(I1), Ifs[s])
    # graph capture and replay
    Pg = torch.empty_like(P)
    Ig = torch.empty_like(I)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run(Tg, Pg, Ig)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(Tg, Pg, Ig)
    for rep in range(5):
        Pg.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(_np(Pg), Ph) and np.array_equal(_np(Ig), Ih), rep


def test_differentiable_batch_full():
    """64 float32 walks of n=16384, m=100, ez=25; L = sum(P); kernel gradient
    vs the FP64 reference gradient on sampled series and central differences
    (h=1e-3) on 32 coordinates, redrawn where the argmin flips."""
    import paper_1904_12626_amd as mpx
    T, m, ez = W.diff_batch()
    Tg = torch.from_numpy(T).to(DEV).requires_grad_(True)
    P, I = mpx.matrix_profile(Tg, m, ez)
    P.sum().backward()
    g = Tg.grad.double().cpu().numpy()
    Ih = I.cpu().numpy()
    rng = np.random.default_rng(5)
    for b in rng.choice(T.shape[0], 3, replace=False):
        ref = O.reference_gradient(T[b].astype(np.float64), m, Ih[b], np.ones(Ih.shape[1]))
        err = np.max(np.abs(g[b] - ref)) / np.max(np.abs(ref))
        assert err <= 1e-4, (b, err)
    # central differences of the fixed-index loss (only rows touching t move);
    # a coordinate is redrawn when the FP64 profile's argmin changes at T +- h
    checked = flips = 0
    base = {}
    while checked < 32:
        b, t = int(rng.integers(T.shape[0])), int(rng.integers(T.shape[1]))
        T64 = T[b].astype(np.float64)
        h = 1e-3
        if b not in base:
            base[b] = mpx.selfjoin(torch.from_numpy(T64).to(DEV), m, ez, precision="f64")[1].cpu().numpy()
        flip = False
        for sgn in (1, -1):
            Tp = T64.copy()
            Tp[t] += sgn * h
            _, Ip = mpx.selfjoin(torch.from_numpy(Tp).to(DEV), m, ez, precision="f64")
            flip |= not np.array_equal(Ip.cpu().numpy(), base[b])
        if flip:
            flips += 1
            assert flips < 64
            continue
        rows = [i for i in range(Ih.shape[1]) if (i <= t < i + m) or (Ih[b, i] <= t < Ih[b, i] + m)]

        def loss(x):
            return sum(O.pair_distance(x, i, x, int(Ih[b, i]), m) for i in rows)

        Tp, Tm = T64.copy(), T64.copy()
        Tp[t] += h
        Tm[t] -= h
        fd = (loss(Tp) - loss(Tm)) / (2 * h)
        assert abs(fd - g[b, t]) <= 1e-3 * max(1.0, abs(fd)), (b, t, fd, g[b, t])
        checked += 1
    print(f"FD checked {checked} coordinates, redrawn {flips}")


def test_left_right_segmentation_chains_full():
    """The benchmark self-join (n=2^20, m=256) split into left and right
    profiles by one sweep; sampled rows of each side against the oracle;
    the combined profile against the plain self-join; arc curve, boundaries
    and chains of the GPU indices against the oracle on the same indices."""
    import paper_1904_12626_amd as mpx
    pw, ez = W.selfjoin_large()
    m = pw.m
    Tg = torch.from_numpy(pw.T).to(DEV)
    P, I, PL, IL, PR, IR = [_np(x) for x in mpx.left_right_profiles(Tg, m, ez)]
    P1, I1 = [_np(x) for x in mpx.selfjoin(Tg, m, ez)]
    tol = 1e-3 * math.sqrt(m)
    assert np.max(np.abs(P - P1)) <= tol
    T64 = pw.T.astype(np.float64)
    rng = np.random.default_rng(6)
    rows = np.sort(rng.choice(P.size, 24, replace=False))
    for side, Ps, Is in (("left", PL, IL), ("right", PR, IR)):
        Po, Io = cimpl.selfjoin_rows_restricted(T64, m, ez, rows, None, side)
        fin = np.isfinite(Po)
        assert np.array_equal(np.isfinite(Ps[rows]), fin)
        assert np.max(np.abs(Ps[rows][fin] - Po[fin])) <= tol, side
    cac, seg = mpx.fluss(torch.from_numpy(I).to(DEV), m, k=3)
    want = O.corrected_arc_curve(I, 5 * m)
    np.testing.assert_allclose(cac.cpu().numpy(), want, rtol=1e-15, atol=0)
    assert list(seg.cpu().numpy()) == O.fluss_segments(want, 3, 5 * m)
    ch = mpx.chains(torch.from_numpy(IL).to(DEV), torch.from_numpy(IR).to(DEV))
    nxt, length, count, best = O.chains(IL, IR)
    assert np.array_equal(ch["next"].cpu().numpy(), nxt) and np.array_equal(ch["length"].cpu().numpy(), length)
    assert ch["count"] == count and ch["best"] == best


def test_stream_append_full():
    """The streaming benchmark: the FP64 stream of the first n - 8192 samples
    of the n=2^20 planted walk (m=256, ez=64), then the last 8192 samples
    appended 512 at a time (batches of up to 63 windows across ~2300
    workgroups, re-seeds included).  Sampled appended rows, random old rows
    and old rows whose neighbour is now an appended window, against the
    oracle on the grown series."""
    import paper_1904_12626_amd as mpx
    pw, ez = W.selfjoin_large()
    m = pw.m
    T = pw.T
    n = T.size
    n0 = n - 8192
    s = mpx.SelfJoinStream(torch.from_numpy(T[:n0]).to(DEV), m, ez, n_max=n)
    for a in range(n0, n, 512):
        s.append(torch.from_numpy(T[a:a + 512]).to(DEV))
    P, I = _np(s.P), _np(s.I)
    l, l0 = n - m + 1, n0 - m + 1
    assert P.size == l
    rng = np.random.default_rng(8)
    moved = np.nonzero(I[:l0] >= l0)[0]         # old rows that took an appended window
    rows = np.unique(np.concatenate([rng.choice(np.arange(l0, l), 24, replace=False),
                                     rng.choice(l0, 24, replace=False),
                                     rng.permutation(moved)[:16]]))
    T64 = T.astype(np.float64)
    Po, Io = cimpl.selfjoin_rows(T64, m, ez, rows)
    compare_profile(T64, m, P[rows], I[rows], Po, Io, 1e-6, ez=None, where="stream", rows=rows)
    assert np.all(np.abs(I[rows] - rows) > ez)
    assert moved.size > 0


def _near_repeats(n, m, seed, triples=8):
    """The n = 2^20 planted walk with `triples` groups of three windows
    written into its increments: a random-walk window w at p1, the exact
    offset copy w + 3 at p2, and a near copy w + a e at p3 whose distance to
    w is 0.02 .. 0.05 (e white noise, its component along w removed)."""
    pw = W.planted_walk(n, m, 2)
    rng = np.random.default_rng(seed)
    T = pw.T.astype(np.float64)
    steps = np.diff(T, prepend=0.0)
    pos = rng.permutation(rng.choice(np.arange(2 * m, n - 2 * m, 4 * m), 3 * triples, replace=False))
    groups = []
    for k in range(triples):
        p1, p2, p3 = (int(x) for x in pos[3 * k:3 * k + 3])
        w = np.cumsum(rng.standard_normal(m))
        wc = w - w.mean()
        e = rng.standard_normal(m)
        e -= e.mean()
        e -= (e @ wc) / (wc @ wc) * wc
        target = 0.02 + 0.03 * k / max(1, triples - 1)
        a = target * w.std() / np.linalg.norm(e)
        for p, win in ((p1, w), (p2, w + 3.0), (p3, w + a * e)):
            steps[p + 1:p + m] = np.diff(win)
        groups.append((p1, p2, p3))
    return np.cumsum(steps).astype(np.float32), groups


def test_near_repeats_full():
    """FP32 keys at the default tile height (R = 4104 rows between FP64
    seeds) cannot order candidates whose keys differ by less than their
    drift: an exact repeat (d ~ 1e-4 after float32 rounding) and a near
    repeat at d = 0.02 .. 0.05 can swap, and the FP64 finalize would then
    report the near one, beyond the tolerance.  Rows whose raw key is below
    the key-error floor are re-found by the exact FP64 scan; those rows must
    match the oracle."""
    import paper_1904_12626_amd as mpx
    n, m, ez = 1 << 20, 256, 64
    T, groups = _near_repeats(n, m, 123)
    Tg = torch.from_numpy(T).to(DEV)
    P, I = (_np(x) for x in mpx.selfjoin(Tg, m, ez))
    Praw, _ = (_np(x) for x in mpx.selfjoin(Tg, m, ez, fp64_finalize=False))
    rows = np.array(sorted(x for g in groups for x in g), dtype=np.int64)
    T64 = T.astype(np.float64)
    Po, Io = cimpl.selfjoin_rows(T64, m, ez, rows)
    tol = 1e-3 * math.sqrt(m)
    compare_profile(T64, m, P[rows], I[rows], Po, Io, tol, ez=ez, where="near repeats", rows=rows)
    assert np.all(Po < 0.06)
    # the raw FP32 keys of these rows are off by up to several tolerances
    # (what the exact re-scan is for), the reported P is exact
    print("raw FP32 |dP| on the repeat rows:", float(np.max(np.abs(Praw[rows] - Po))))
    assert np.max(np.abs(P[rows] - Po)) <= 1e-6
