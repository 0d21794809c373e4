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
