"""Incrementally updated self-join against the oracle's self-join of the
grown series."""

import math

import numpy as np
import pytest
import torch

from oracle import cimpl
from oracle import mp_oracle as O
from tests.parity import compare_profile

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_stream_matches_selfjoin_of_the_grown_series(dtype):
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(170)
    n_total, n0, m, ez = 3000, 1800, 40, 10
    T = np.cumsum(rng.standard_normal(n_total)).astype(dtype)
    s = mpx.SelfJoinStream(torch.from_numpy(T[:n0]).to(DEV), m, ez, n_max=n_total)
    T64 = T.astype(np.float64)
    n = n0
    for k in (1, 7, 150, 1, 1041):       # the last append crosses a re-seed point
        s.append(torch.from_numpy(T[n:n + k]).to(DEV))
        n += k
        P, I = s.P.double().cpu().numpy(), s.I.cpu().numpy()
        Po, Io = cimpl.selfjoin(T64[:n], m, ez)
        tol = 1e-9 if dtype == np.float64 else 1e-3 * math.sqrt(m)
        compare_profile(T64[:n], m, P, I, Po, Io, tol, ez=ez, where=f"n={n}")
    assert n == n_total


def test_stream_degenerate_windows():
    """Constant stretch and a NaN arriving in the stream."""
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(171)
    n_total, n0, m, ez = 1500, 600, 24, 6
    T = np.cumsum(rng.standard_normal(n_total))
    T[700:760] = 3.0
    T[1000] = np.nan
    s = mpx.SelfJoinStream(torch.from_numpy(T[:n0]).to(DEV), m, ez, n_max=n_total)
    n = n0
    for k in (200, 300, 400):
        s.append(torch.from_numpy(T[n:n + k]).to(DEV))
        n += k
        Po, Io = O.selfjoin(T[:n], m, ez)
        compare_profile(T[:n], m, s.P.cpu().numpy(), s.I.cpu().numpy(), Po, Io, 1e-9, ez=ez, where=f"n={n}")


@pytest.mark.parametrize("ez,chunks", [(0, (1, 5, 3, 64, 2)), (2, (9, 1, 40)), (70, (200, 333))])
def test_stream_batch_shapes(ez, chunks):
    """Batch sizes from one window (ez = 0: no halo) to several workgroups
    with a halo, and a window longer than the first strip."""
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(172 + ez)
    m = 8 if ez < 70 else 96
    n0 = 700
    n_total = n0 + sum(chunks)
    T = np.cumsum(rng.standard_normal(n_total))
    s = mpx.SelfJoinStream(torch.from_numpy(T[:n0]).to(DEV), m, ez, n_max=n_total)
    n = n0
    for k in chunks:
        s.append(torch.from_numpy(T[n:n + k]).to(DEV))
        n += k
        Po, Io = cimpl.selfjoin(T[:n], m, ez)
        compare_profile(T[:n], m, s.P.cpu().numpy(), s.I.cpu().numpy(), Po, Io, 1e-9, ez=ez, where=f"n={n}")
