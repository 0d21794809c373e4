"""Backward kernel: dL/dT through each row's argmin pair, against the FP64
reference gradient and central finite differences."""

import numpy as np
import pytest
import torch

from oracle import mp_oracle as O
from workloads import walk_batch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_backward_matches_reference_gradient():
    import paper_1904_12626_amd as mpx
    B, n, m, ez = 4, 700, 20, 5
    T = walk_batch(B, n, 5, np.float64)
    Tg = torch.from_numpy(T).to(DEV).requires_grad_(True)
    P, I = mpx.matrix_profile(Tg, m, ez, precision="f64")
    w = torch.from_numpy(np.random.default_rng(1).uniform(0.5, 1.5, P.shape)).to(DEV)
    (P * w).sum().backward()
    g = Tg.grad.cpu().numpy()
    Ih = I.cpu().numpy()
    wh = w.cpu().numpy()
    for b in range(B):
        ref = O.reference_gradient(T[b], m, Ih[b], wh[b])
        np.testing.assert_allclose(g[b], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_backward_float32_against_fd():
    import paper_1904_12626_amd as mpx
    B, n, m, ez = 2, 600, 16, 4
    T = walk_batch(B, n, 6, np.float32)
    Tg = torch.from_numpy(T).to(DEV).requires_grad_(True)
    P, I = mpx.matrix_profile(Tg, m, ez)
    P.sum().backward()
    g = Tg.grad.cpu().numpy().astype(np.float64)
    Ih = I.cpu().numpy()
    T64 = T.astype(np.float64)
    rng = np.random.default_rng(2)
    h = 1e-3
    for _ in range(12):
        b, t = int(rng.integers(B)), int(rng.integers(n))
        Tp, Tm = T64[b].copy(), T64[b].copy()
        Tp[t] += h
        Tm[t] -= h
        fd = (O.profile_sum_loss(Tp, m, Ih[b]) - O.profile_sum_loss(Tm, m, Ih[b])) / (2 * h)
        assert abs(fd - g[b, t]) <= 1e-3 * max(1.0, abs(fd)), (b, t, fd, g[b, t])
    ref = O.reference_gradient(T64[0], m, Ih[0], np.ones(Ih.shape[1]))
    np.testing.assert_allclose(g[0], ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())


def _batch(lengths, ms, seed, dtype):
    rng = np.random.default_rng(seed)
    return [np.cumsum(rng.standard_normal(n)).astype(dtype) for n in lengths]


def test_backward_ragged_deterministic():
    """Ragged batch, different windows per series: the gradient matches the
    FP64 reference per series and two runs are bitwise equal."""
    import paper_1904_12626_amd as mpx
    lengths, ms = [900, 333, 1500, 64], [24, 16, 40, 8]
    zs = [m // 4 for m in ms]
    series = _batch(lengths, ms, 11, np.float64)
    Tg = torch.from_numpy(np.concatenate(series)).to(DEV)
    plan = mpx.BatchPlan(lengths, ms, zs, dtype=torch.float64, device=DEV, precision="f64")
    P, I = plan.run(Tg)
    gP = torch.from_numpy(np.random.default_rng(12).uniform(-1, 2, P.shape)).to(DEV)
    g1 = plan.backward(Tg, I, gP).clone()
    g2 = plan.backward(Tg, I, gP)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    gs = np.split(g1.cpu().numpy(), np.cumsum(lengths)[:-1])
    Is, gPs = plan.split(I.cpu().numpy()), plan.split(gP.cpu().numpy())
    for s in range(len(lengths)):
        ref = O.reference_gradient(series[s], ms[s], Is[s], gPs[s])
        np.testing.assert_allclose(gs[s], ref, rtol=1e-9, atol=1e-9 * max(1.0, np.abs(ref).max()))


def test_backward_hub_constant_and_nan_windows():
    """A hand-made index with hub neighbours (half the rows point at one
    window), out-of-range and negative entries, a constant stretch and a NaN
    sample, exact repeats and a self pair: the kernel takes the same
    subgradient-0 rules as the reference."""
    import paper_1904_12626_amd as mpx
    n, m = 1200, 32
    T = np.cumsum(np.random.default_rng(21).standard_normal(n))
    T[300:400] = 2.5              # constant windows 300..368
    T[800] = np.nan               # windows 769..800 invalid
    T[600:640] = T[100:140]       # exact repeats: d(100, 600) = d(101, 601) = 0
    l = n - m + 1
    rng = np.random.default_rng(22)
    I = rng.integers(0, l, l)
    I[::2] = 500                  # hub
    I[1::7] = 123                 # second hub
    I[5::11] = -1
    I[3::13] = l + 5              # outside the series: ignored
    I[100], I[101], I[413] = 600, 601, 413   # zero distance, self pair
    gP = rng.uniform(0.5, 1.5, l)
    plan = mpx.BatchPlan([n], [m], [m // 4], dtype=torch.float64, device=DEV, precision="f64")
    Tg = torch.from_numpy(T).to(DEV)
    g = plan.backward(Tg, torch.from_numpy(I).to(DEV), torch.from_numpy(gP).to(DEV))
    g = g.cpu().numpy()
    Iref = np.where(I >= l, -1, I)
    ref = O.reference_gradient(T, m, Iref, gP)
    assert np.all(np.isfinite(g))
    bad = np.flatnonzero(np.abs(g - ref) > 1e-9 * np.abs(ref).max() + 1e-9 * np.abs(ref))
    assert bad.size == 0, (bad[:70].tolist(), g[bad[:8]].tolist(), ref[bad[:8]].tolist())


def test_backward_degenerate_series():
    """A batch mixing a one-window series, a series with no admissible
    neighbour (l = ez + 1), an all-constant series and an ordinary walk:
    the forward gives (+inf, -1) on the first three, and the backward gives
    exact zeros there (no row, no bucket edge, no own edge) and the
    reference gradient on the walk."""
    import paper_1904_12626_amd as mpx
    m = 16
    lengths = [m, m + 4, 60, 700]
    zs = [4, 4, 4, 4]
    rng = np.random.default_rng(51)
    series = [np.cumsum(rng.standard_normal(lengths[0])), np.cumsum(rng.standard_normal(lengths[1])),
              np.full(lengths[2], 3.25), np.cumsum(rng.standard_normal(lengths[3]))]
    Tg = torch.from_numpy(np.concatenate(series)).to(DEV)
    plan = mpx.BatchPlan(lengths, [m] * 4, zs, dtype=torch.float64, device=DEV, precision="f64")
    P, I = plan.run(Tg)
    Ps, Is = plan.split(P.cpu().numpy()), plan.split(I.cpu().numpy())
    assert np.all(np.isinf(Ps[0])) and np.all(Is[0] == -1)
    assert np.all(np.isinf(Ps[1])) and np.all(Is[1] == -1)
    gP = torch.from_numpy(np.random.default_rng(52).uniform(0.5, 1.5, P.shape)).to(DEV)
    g = plan.backward(Tg, I, gP).cpu().numpy()
    gs = np.split(g, np.cumsum(lengths)[:-1])
    for s in range(3):
        assert np.all(gs[s] == 0.0), s
    Ih, gPs = Is[3], plan.split(gP.cpu().numpy())[3]
    ref = O.reference_gradient(series[3], m, Ih, gPs)
    np.testing.assert_allclose(gs[3], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_backward_after_forward_matches_backward(dtype):
    """mp_backward_after_forward (window statistics and distances taken from
    the forward) against mp_backward (both recomputed from the samples) on a
    ragged batch with a NaN sample and a constant stretch: equal up to the
    rounding of rho = 1 - d^2/(2m) (and of d stored in a float P), and
    bitwise repeatable."""
    import paper_1904_12626_amd as mpx
    lengths, ms = [900, 333, 1500, 64], [24, 16, 40, 8]
    zs = [m // 4 for m in ms]
    series = _batch(lengths, ms, 61, dtype)
    series[2][400:470] = 0.75
    series[0][500] = np.nan
    Tg = torch.from_numpy(np.concatenate(series)).to(DEV)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    plan = mpx.BatchPlan(lengths, ms, zs, dtype=tdt, device=DEV, precision="f64" if dtype == np.float64 else "f32")
    assert plan.reuses_forward
    P, I = plan.run(Tg)
    gP = torch.from_numpy(np.random.default_rng(62).uniform(-1, 2, P.shape).astype(dtype)).to(DEV)
    full = plan.backward(Tg, I, gP).clone()
    fast = plan.backward_after_forward(Tg, I, P, gP).clone()
    again = plan.backward_after_forward(Tg, I, P, gP)
    torch.cuda.synchronize()
    assert torch.equal(fast, again)
    a, b = full.double().cpu().numpy(), fast.double().cpu().numpy()
    assert np.all(np.isfinite(b))
    tol = 1e-11 if dtype == np.float64 else 2e-5
    np.testing.assert_allclose(b, a, rtol=tol, atol=tol * np.abs(a).max())


def test_abjoin_backward_after_forward():
    """The AB-join plan's layout: dL/dA and dL/dB from the forward's state
    equal the full backward's."""
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(63)
    A, Bs, m = np.cumsum(rng.standard_normal(1500)), np.cumsum(rng.standard_normal(900)), 32
    plan = mpx.ABJoinPlan(A.size, Bs.size, m, dtype=torch.float64, device=DEV, precision="f64")
    Tg = torch.from_numpy(np.concatenate([A, Bs])).to(DEV)
    P, I = plan.run(Tg)
    gP = torch.from_numpy(rng.uniform(0.5, 1.5, P.shape)).to(DEV)
    full = plan.backward(Tg, I, gP).clone()
    fast = plan.backward_after_forward(Tg, I, P, gP)
    a, b = full.cpu().numpy(), fast.cpu().numpy()
    np.testing.assert_allclose(b, a, rtol=1e-11, atol=1e-11 * np.abs(a).max())


def test_autograd_falls_back_when_another_forward_intervened():
    """Two forwards on one plan before the first one's backward: the
    workspace then holds the second forward's statistics, so the first
    backward recomputes them (and is still the reference gradient); the
    second backward may reuse them."""
    import paper_1904_12626_amd as mpx
    B, n, m, ez = 2, 600, 20, 5
    T1 = walk_batch(B, n, 64, np.float64)
    T2 = walk_batch(B, n, 65, np.float64)
    plan = mpx.BatchPlan([n] * B, [m] * B, [ez] * B, dtype=torch.float64, device=DEV, precision="f64")
    x1 = torch.from_numpy(T1).to(DEV).requires_grad_(True)
    x2 = torch.from_numpy(T2).to(DEV).requires_grad_(True)
    P1, I1 = mpx.matrix_profile(x1, m, ez, plan=plan)
    P2, I2 = mpx.matrix_profile(x2, m, ez, plan=plan)
    P1.sum().backward()
    P2.sum().backward()
    for x, T, Ih in ((x1, T1, I1), (x2, T2, I2)):
        g = x.grad.cpu().numpy()
        Ih = Ih.cpu().numpy()
        for b in range(B):
            ref = O.reference_gradient(T[b], m, Ih[b], np.ones(Ih.shape[1]))
            np.testing.assert_allclose(g[b], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_backward_after_forward_needs_fp64_finalize():
    import paper_1904_12626_amd as mpx
    plan = mpx.BatchPlan([500], [16], [4], dtype=torch.float32, device=DEV, fp64_finalize=False)
    assert not plan.reuses_forward
    T = torch.from_numpy(walk_batch(1, 500, 66, np.float32).reshape(-1)).to(DEV)
    P, I = plan.run(T)
    with pytest.raises(mpx.MPError):
        plan.backward_after_forward(T, I, P, torch.ones_like(P))
    x = T.view(1, -1).clone().requires_grad_(True)
    Pa, _ = mpx.matrix_profile(x, 16, 4, plan=plan)
    Pa.sum().backward()           # takes mp_backward
    assert torch.isfinite(x.grad).all()


def test_backward_long_window():
    """m = 2100 is past the LDS tile of the window statistics and the
    coefficients: both read the series from global memory.  Against the FP64
    reference gradient."""
    import paper_1904_12626_amd as mpx
    B, n, m, ez = 2, 5200, 2100, 525
    T = walk_batch(B, n, 41, np.float64)
    Tg = torch.from_numpy(T).to(DEV).requires_grad_(True)
    P, I = mpx.matrix_profile(Tg, m, ez, precision="f64")
    w = torch.from_numpy(np.random.default_rng(42).uniform(0.5, 1.5, P.shape)).to(DEV)
    (P * w).sum().backward()
    g = Tg.grad.cpu().numpy()
    Ih, wh = I.cpu().numpy(), w.cpu().numpy()
    for b in range(B):
        ref = O.reference_gradient(T[b], m, Ih[b], wh[b])
        np.testing.assert_allclose(g[b], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_gather_flat_and_buffer_loads_agree(dtype):
    """The gather reads source samples with buffer loads (arrays under 2 GiB,
    out-of-window lanes may read past either end of the array) or flat loads
    (forced here; the path of larger arrays): bitwise the same gradient, on a
    ragged batch whose first and last series put window edges at both ends
    of the array, with a NaN sample, a constant stretch and a hub."""
    import paper_1904_12626_amd as mpx
    lengths, ms = [700, 90, 1300, 400], [24, 10, 40, 16]
    zs = [m // 4 for m in ms]
    series = _batch(lengths, ms, 31, dtype)
    series[2][500:560] = 1.25
    series[2][900] = np.nan
    Tc = np.concatenate(series)
    Tg = torch.from_numpy(Tc).to(DEV)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    prec = "f64" if dtype == np.float64 else "f32"
    buf = mpx.BatchPlan(lengths, ms, zs, dtype=tdt, device=DEV, precision=prec)
    flat = mpx.BatchPlan(lengths, ms, zs, dtype=tdt, device=DEV, precision=prec, flat_loads=True)
    P, I = buf.run(Tg)
    I = I.clone()
    Ih = I.cpu().numpy()
    off = 0
    for n, m in zip(lengths, ms):   # a hub in every series: the first window
        Ih[off:off + n - m + 1:3] = 0
        off += n - m + 1
    I = torch.from_numpy(Ih).to(DEV)
    gP = torch.from_numpy(np.random.default_rng(32).uniform(0.5, 1.5, P.shape).astype(dtype)).to(DEV)
    g_buf = buf.backward(Tg, I, gP).clone()
    g_flat = flat.backward(Tg, I, gP)
    torch.cuda.synchronize()
    assert torch.equal(g_buf, g_flat)
    if dtype == np.float64:
        gs = np.split(g_buf.cpu().numpy(), np.cumsum(lengths)[:-1])
        Is, gPs = buf.split(Ih), buf.split(gP.cpu().numpy())
        for s in range(len(lengths)):
            ref = O.reference_gradient(series[s], ms[s], Is[s], gPs[s])
            np.testing.assert_allclose(gs[s], ref, rtol=1e-9, atol=1e-9 * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("precision,dtype", [("f64", np.float64), ("f32", np.float32)])
def test_abjoin_plan_and_backward(precision, dtype):
    """AB-join as a plan: profiles equal mp_abjoin's; the backward gives
    [dL/dA | dL/dB] equal to the FP64 reference gradient."""
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(110)
    A = np.cumsum(rng.standard_normal(1500)).astype(dtype)
    Bs = np.cumsum(rng.standard_normal(1100)).astype(dtype)
    m = 32
    Ag, Bg = torch.from_numpy(A).to(DEV), torch.from_numpy(Bs).to(DEV)
    plan = mpx.ABJoinPlan(A.size, Bs.size, m, dtype=Ag.dtype, device=DEV, precision=precision)
    P, I = plan.run(torch.cat([Ag, Bg]))
    Pab, Iab, Pba, Iba = mpx.abjoin(Ag, Bg, m, precision=precision)
    lA = A.size - m + 1
    assert torch.equal(P[:lA], Pab) and torch.equal(I[:lA], Iab)
    assert torch.equal(P[lA:], Pba) and torch.equal(I[lA:], Iba)
    w = torch.from_numpy(rng.uniform(0.5, 1.5, P.numel())).to(DEV, Ag.dtype)
    Ax = Ag.clone().requires_grad_(True)
    Bx = Bg.clone().requires_grad_(True)
    pab, iab, pba, iba = mpx.abjoin_profile(Ax, Bx, m, precision=precision)
    (torch.cat([pab, pba]) * w).sum().backward()
    wh = w.double().cpu().numpy()
    gA, gB = O.reference_gradient_ab(A.astype(np.float64), Bs.astype(np.float64), m, iab.cpu().numpy(), wh[:lA],
                                     iba.cpu().numpy(), wh[lA:])
    tol = 1e-9 if precision == "f64" else 1e-4
    for g, ref in ((Ax.grad, gA), (Bx.grad, gB)):
        g = g.double().cpu().numpy()
        np.testing.assert_allclose(g, ref, rtol=tol, atol=tol * np.abs(ref).max())


def test_forward_backward_graph_replay_equals_eager():
    """The differentiable profile's forward and backward (dL/dP = 1, that is
    L = sum(P), given as a static ones tensor so that no reduction kernel is
    captured) in one captured graph: four replays, each after its outputs
    are overwritten and with unrelated eager work in between, equal the eager
    step bitwise."""
    import paper_1904_12626_amd as mpx
    B, n, m, ez = 8, 3000, 50, 12
    T = np.cumsum(np.random.default_rng(77).standard_normal((B, n)), axis=1).astype(np.float32)
    Tg = torch.from_numpy(T).to(DEV)
    plan = mpx.BatchPlan([n] * B, [m] * B, [ez] * B, dtype=torch.float32, device=DEV)
    ones = torch.ones((B, n - m + 1), dtype=torch.float32, device=DEV)
    x0 = Tg.clone().requires_grad_(True)
    P0, I0 = mpx.MatrixProfileFn.apply(x0, plan)
    P0.backward(ones)
    torch.cuda.synchronize()
    P0, I0, g0 = P0.detach().cpu(), I0.cpu(), x0.grad.cpu()
    xs = Tg.clone().requires_grad_(True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):   # warm-up outside the graph (no reference kept)
        mpx.MatrixProfileFn.apply(xs, plan)[0].backward(ones)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    xs.grad = None
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        Pg, Ig = mpx.MatrixProfileFn.apply(xs, plan)
        Pg.backward(ones)
    gx = xs.grad
    for rep in range(4):
        with torch.no_grad():
            Pg.fill_(-1.0)
            gx.fill_(float("nan"))
        Ig.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Pg.detach().cpu(), P0), rep
        assert torch.equal(Ig.cpu(), I0), rep
        assert torch.equal(gx.cpu(), g0), rep
        _ = (Tg * 2).sum().item()   # unrelated eager work between replays



def test_backward_large_hub_is_fast_and_exact():
    """One window named as nearest neighbour by 90 % of 100 000 rows (a hub,
    as periodic or ECG-like series produce) plus a second hub of 3000 rows:
    the bucket of each is ordered by a workgroup sort, O(h log^2 h), not by
    per-row counting, O(h^2).  Gradient against the FP64 reference, two
    runs bitwise equal, and the backward well under a second."""
    import time
    import paper_1904_12626_amd as mpx
    n, m = 100_000, 64
    T = np.cumsum(np.random.default_rng(31).standard_normal(n))
    l = n - m + 1
    rng = np.random.default_rng(32)
    I = rng.integers(0, l, l)
    I[rng.random(l) < 0.9] = 777
    I[5::30] = 50_000
    I[777] = 901
    gP = rng.uniform(0.5, 1.5, l)
    plan = mpx.BatchPlan([n], [m], [m // 4], dtype=torch.float64, device=DEV, precision="f64")
    Tg = torch.from_numpy(T).to(DEV)
    Ig, gPg = torch.from_numpy(I).to(DEV), torch.from_numpy(gP).to(DEV)
    g1 = plan.backward(Tg, Ig, gPg).clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g2 = plan.backward(Tg, Ig, gPg)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert torch.equal(g1, g2)
    assert dt < 0.5, dt
    ref = O.reference_gradient(T, m, I, gP)
    g = g1.cpu().numpy()
    np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
