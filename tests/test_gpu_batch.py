"""Batched self-joins: one launch sequence for many series of uneven
lengths and windows; equal to a loop of single joins; graph replay equal to
the eager run."""

import numpy as np
import pytest
import torch

from oracle import cimpl
from tests.parity import compare_profile
from workloads import ragged_batch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _plan(rb, **kw):
    import paper_1904_12626_amd as mpx
    return mpx.BatchPlan([s.size for s in rb.series], rb.m, rb.ez, dtype=torch.float32, device=DEV, **kw)


def test_batch_matches_oracle_and_single_joins():
    import paper_1904_12626_amd as mpx
    rb = ragged_batch(12, 40, nmin=300, nmax=3000)
    Tc, _ = rb.concat()
    plan = _plan(rb)
    P, I = plan.run(torch.from_numpy(Tc).to(DEV))
    torch.cuda.synchronize()
    Ps, Is = plan.split(P.cpu().numpy()), plan.split(I.cpu().numpy())
    for s, (T, m, ez) in enumerate(zip(rb.series, rb.m, rb.ez)):
        T64 = T.astype(np.float64)
        Po, Io = cimpl.selfjoin(T64, m, ez)
        tol = 1e-3 * np.sqrt(m)
        compare_profile(T64, m, Ps[s], Is[s], Po, Io, tol, ez=ez, where=f"series {s}")
        P1, I1 = mpx.selfjoin(torch.from_numpy(T).to(DEV), m, ez)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(P1.cpu().numpy(), Ps[s])
        np.testing.assert_array_equal(I1.cpu().numpy(), Is[s])


def test_batch_graph_replay_equals_eager():
    rb = ragged_batch(16, 41, nmin=500, nmax=4000)
    Tc, _ = rb.concat()
    plan = _plan(rb)
    Tg = torch.from_numpy(Tc).to(DEV)
    P0, I0 = plan.run(Tg)
    torch.cuda.synchronize()
    P0, I0 = P0.cpu().numpy(), I0.cpu().numpy()
    Pg = torch.empty(plan.profile_length, dtype=torch.float32, device=DEV)
    Ig = torch.empty(plan.profile_length, dtype=torch.int64, device=DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(Tg, Pg, Ig)        # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(Tg, Pg, Ig)
    for rep in range(4):
        Pg.fill_(-1.0)
        Ig.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(Pg.cpu().numpy(), P0), rep
        assert np.array_equal(Ig.cpu().numpy(), I0), rep
        _ = (Tg * 2).sum().item()   # unrelated eager work between replays


def test_batch_float64_fp64_sweep():
    import paper_1904_12626_amd as mpx
    rb = ragged_batch(5, 42, nmin=200, nmax=2000, dtype=np.float64)
    Tc, _ = rb.concat()
    plan = mpx.BatchPlan([s.size for s in rb.series], rb.m, rb.ez, dtype=torch.float64, device=DEV,
                         precision="f64")
    P, I = plan.run(torch.from_numpy(Tc).to(DEV))
    torch.cuda.synchronize()
    Ps, Is = plan.split(P.cpu().numpy()), plan.split(I.cpu().numpy())
    for s, (T, m, ez) in enumerate(zip(rb.series, rb.m, rb.ez)):
        Po, Io = cimpl.selfjoin(T, m, ez)
        compare_profile(T, m, Ps[s], Is[s], Po, Io, 1e-9, ez=ez)


def test_batch_of_series_at_different_magnitudes():
    """Series of one batch each carry their own power of two in the sweep's
    records: a batch of walks scaled by 1e-18, 1 and 1e19 gives each series
    the oracle's profile."""
    import paper_1904_12626_amd as mpx
    from workloads import random_walk
    lens, ms, ezs, scales = [2000, 1700, 2500], [32, 48, 40], [8, 12, 10], [1e-18, 1.0, 1e19]
    Ts = [random_walk(n, 60 + k, np.float64) for k, n in enumerate(lens)]
    plan = mpx.BatchPlan(lens, ms, ezs, dtype=torch.float64, device=DEV)
    P, I = plan.run(torch.from_numpy(np.concatenate([T * a for T, a in zip(Ts, scales)])).to(DEV))
    torch.cuda.synchronize()
    Ps, Is = plan.split(P.cpu().numpy()), plan.split(I.cpu().numpy())
    for s, (T, m, ez) in enumerate(zip(Ts, ms, ezs)):
        Po, Io = cimpl.selfjoin(T, m, ez)
        compare_profile(T, m, Ps[s], Is[s], Po, Io, 1e-3 * np.sqrt(m), ez=ez, where=f"series {s}")


def test_batch_of_more_series_than_plan_threads():
    """1100 series, more than the plan kernel's 1024 threads, so that some
    threads set a second series' power of two.  Magnitudes cycle through
    1e-25 (whose FP32 cross products would underflow unscaled), 1 and 1e19,
    and every series is checked against the oracle."""
    import paper_1904_12626_amd as mpx
    from workloads import random_walk
    ns = 1100
    scales = [1e-25, 1.0, 1e19]
    lens = [150 + (k % 7) * 10 for k in range(ns)]
    Ts = [random_walk(n, 1000 + k, np.float64) for k, n in enumerate(lens)]
    m, ez = 16, 4
    plan = mpx.BatchPlan(lens, [m] * ns, [ez] * ns, dtype=torch.float64, device=DEV)
    Tcat = np.concatenate([T * scales[k % 3] for k, T in enumerate(Ts)])
    P, I = plan.run(torch.from_numpy(Tcat).to(DEV))
    torch.cuda.synchronize()
    Ps, Is = plan.split(P.cpu().numpy()), plan.split(I.cpu().numpy())
    for s, T in enumerate(Ts):
        Po, Io = cimpl.selfjoin(T, m, ez)
        compare_profile(T, m, Ps[s], Is[s], Po, Io, 1e-3 * np.sqrt(m), ez=ez, where=f"series {s}")
