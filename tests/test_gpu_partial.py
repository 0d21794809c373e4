"""Self-joins restricted to chunks of diagonal offsets (the anytime mode) and
left/right profiles, against the FP64 oracle's restricted join."""

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


def _allowed(l, ez, width, chunks):
    """Offsets k = |i - j| covered by the chosen chunks."""
    a = np.zeros(l, dtype=bool)
    for c in chunks:
        lo, hi = ez + 1 + c * width, min(ez + (c + 1) * width, l - 1)
        a[lo:hi + 1] = True
    return a


@pytest.mark.parametrize("precision,slots", [("f64", 8), ("f32", 8), ("f32", 12)])
def test_chunk_subset_matches_restricted_oracle(precision, slots):
    import paper_1904_12626_amd as mpx
    T, m, ez = W.selfjoin_small()
    n, l = T.size, T.size - m + 1
    count, width = mpx.selfjoin_chunks(n, m, ez, precision=precision, tile_slots=slots)
    assert width == 64 * slots and count == math.ceil((l - 1 - ez) / width)
    rng = np.random.default_rng(50 + slots)
    chunks = list(rng.permutation(count)[:max(1, count // 3)])
    plan = mpx.SelfJoinPlan(n, m, ez, dtype=torch.float64, device=DEV, chunks=chunks, precision=precision,
                            tile_slots=slots)
    P, I = plan.run(torch.from_numpy(T).to(DEV))
    torch.cuda.synchronize()
    allowed = _allowed(l, ez, width, chunks)
    Po, Io = cimpl.selfjoin_rows_restricted(T, m, ez, np.arange(l), allowed)
    compare_profile(T, m, _np(P), _np(I), Po, Io, 1e-3 * math.sqrt(m), ez=ez, where=precision)
    Ih = _np(I)
    ok = Ih >= 0
    assert np.all(allowed[np.abs(Ih[ok] - np.arange(l)[ok])])


def test_all_chunks_in_random_order_equal_the_selfjoin_bitwise():
    import paper_1904_12626_amd as mpx
    T, m, ez = W.selfjoin_small()
    Tg = torch.from_numpy(T.astype(np.float32)).to(DEV)
    count, _ = mpx.selfjoin_chunks(T.size, m, ez)
    order = mpx.anytime_order(count, 3)
    plan = mpx.SelfJoinPlan(T.size, m, ez, dtype=torch.float32, device=DEV, chunks=order, reseed_rows=1024)
    P, I = plan.run(Tg)
    P1, I1 = mpx.selfjoin(Tg, m, ez, reseed_rows=1024)
    torch.cuda.synchronize()
    assert torch.equal(P, P1) and torch.equal(I, I1)


def test_empty_chunk_set_gives_no_neighbours():
    import paper_1904_12626_amd as mpx
    T, m, ez = W.selfjoin_small()
    plan = mpx.SelfJoinPlan(T.size, m, ez, dtype=torch.float64, device=DEV, chunks=[], precision="f64")
    P, I = plan.run(torch.from_numpy(T).to(DEV))
    assert torch.all(torch.isinf(P)) and torch.all(I == -1)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_left_right_profiles(precision):
    import paper_1904_12626_amd as mpx
    T, m, ez = W.selfjoin_small()
    l = T.size - m + 1
    dt = torch.float64 if precision == "f64" else torch.float32
    Th = T if precision == "f64" else T.astype(np.float32).astype(np.float64)
    P, I, PL, IL, PR, IR = [_np(x) for x in mpx.left_right_profiles(torch.from_numpy(Th).to(DEV, dt), m, ez,
                                                                    precision=precision)]
    tol = 1e-3 * math.sqrt(m)
    rows = np.arange(l)
    for side, Pg, Ig in (("left", PL, IL), ("right", PR, IR)):
        Po, Io = cimpl.selfjoin_rows_restricted(Th, m, ez, rows, None, side)
        compare_profile(Th, m, Pg, Ig, Po, Io, tol, ez=ez, where=side)
    assert np.all(IL[IL >= 0] < rows[IL >= 0]) and np.all(IR[IR >= 0] > rows[IR >= 0])
    Po, Io = cimpl.selfjoin(Th, m, ez)
    compare_profile(Th, m, P, I, Po, Io, tol, ez=ez, where="combined")
    # the combined profile is the better side, left on equal distances
    right = (IL < 0) | ((IR >= 0) & (PR < PL))
    assert np.array_equal(P, np.where(right, PR, PL)) and np.array_equal(I, np.where(right, IR, IL))


def test_restricted_and_one_sided_with_constant_and_invalid_windows():
    """Constant stretches and a NaN: the degenerate-window rules (constant
    partners at distance 0 or sqrt(m), invalid windows never chosen) are
    applied inside the chunk set and on one side only."""
    import paper_1904_12626_amd as mpx
    n, m, ez = 3000, 32, 8
    T = np.cumsum(np.random.default_rng(60).standard_normal(n))
    T[400:470] = 1.0                # constant windows 400..438
    T[2100:2160] = -4.0             # constant windows 2100..2128
    T[1500] = np.nan                # windows 1469..1500 invalid
    l = n - m + 1
    Tg = torch.from_numpy(T).to(DEV)
    count, width = mpx.selfjoin_chunks(n, m, ez, precision="f64")
    chunks = [c for c in range(count) if c % 2 == 1]
    allowed = _allowed(l, ez, width, chunks)
    plan = mpx.SelfJoinPlan(n, m, ez, dtype=torch.float64, device=DEV, chunks=chunks, precision="f64")
    P, I = plan.run(Tg)
    Po, Io = O.selfjoin_restricted(T, m, ez, allowed)
    compare_profile(T, m, _np(P), _np(I), Po, Io, 1e-9, ez=ez, where="chunks")
    out = [_np(x) for x in mpx.left_right_profiles(Tg, m, ez, precision="f64")]
    for side, Pg, Ig in (("left", out[2], out[3]), ("right", out[4], out[5])):
        Po, Io = O.selfjoin_restricted(T, m, ez, side=side)
        compare_profile(T, m, Pg, Ig, Po, Io, 1e-9, ez=ez, where=side)
    out = [_np(x) for x in mpx.left_right_profiles(Tg, m, ez, precision="f64", chunks=chunks)]
    for side, Pg, Ig in (("left", out[2], out[3]), ("right", out[4], out[5])):
        Po, Io = O.selfjoin_restricted(T, m, ez, allowed, side=side)
        compare_profile(T, m, Pg, Ig, Po, Io, 1e-9, ez=ez, where="chunks " + side)


def test_backward_of_a_restricted_plan():
    import paper_1904_12626_amd as mpx
    T, m, ez = W.selfjoin_small()
    count, _ = mpx.selfjoin_chunks(T.size, m, ez, precision="f64")
    plan = mpx.SelfJoinPlan(T.size, m, ez, dtype=torch.float64, device=DEV, chunks=[0, count - 1], precision="f64")
    Tg = torch.from_numpy(T).to(DEV)
    P, I = plan.run(Tg)
    g = plan.backward(Tg, I, torch.ones_like(P))
    ref = O.reference_gradient(T, m, _np(I), np.ones(P.numel()))
    np.testing.assert_allclose(_np(g), ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
