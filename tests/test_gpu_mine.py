"""Semantic segmentation (arc curve, corrected arc curve, boundaries) and
time series chains on the GPU, against the oracle on the same indices."""

import numpy as np
import pytest
import torch

from oracle import mp_oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _check_fluss(I, m, k, zone):
    import paper_1904_12626_amd as mpx
    cac, seg = mpx.fluss(torch.from_numpy(I).to(DEV), m, k=k, zone=zone)
    cac, seg = cac.cpu().numpy(), seg.cpu().numpy()
    want = O.corrected_arc_curve(I, zone)
    np.testing.assert_allclose(cac, want, rtol=1e-15, atol=0)
    assert list(seg) == O.fluss_segments(want, k, zone)
    return seg


def test_fluss_on_regime_changes():
    import paper_1904_12626_amd as mpx
    T, (b1, b2) = W.regime_series(6000, 7)
    m = 60
    _, I = mpx.selfjoin(torch.from_numpy(T).to(DEV), m, m // 2, precision="f64")
    seg = sorted(_check_fluss(I.cpu().numpy(), m, 2, 5 * m))
    assert abs(seg[0] - b1) <= m and abs(seg[1] - b2) <= m


@pytest.mark.parametrize("seed", [0, 1])
def test_fluss_arbitrary_indices(seed):
    """Random indices with out-of-range, negative and self entries; more
    picks than fit (trailing -1); zone 0."""
    rng = np.random.default_rng(80 + seed)
    l = 5000
    I = rng.integers(-5, l + 5, l)
    I[::97] = np.arange(0, l, 97)
    _check_fluss(I, 10, 7, 300)
    _check_fluss(I, 10, 3, 0)
    seg = _check_fluss(I[:700], 10, 5, 150)
    assert seg[-1] == -1


def test_chains_on_an_evolving_pattern():
    import paper_1904_12626_amd as mpx
    T, pos = W.evolving_chain(8000, 64, 8, 2)
    m, ez = 64, 16
    P, I, PL, IL, PR, IR = mpx.left_right_profiles(torch.from_numpy(T).to(DEV), m, ez, precision="f64")
    ch = mpx.chains(IL, IR, min_len=3)
    nxt, length, count, best = O.chains(IL.cpu().numpy(), IR.cpu().numpy(), 3)
    assert np.array_equal(ch["next"].cpu().numpy(), nxt)
    assert np.array_equal(ch["length"].cpu().numpy(), length)
    assert ch["count"] == count and ch["best"] == best
    for p in pos:
        assert any(abs(b - p) <= m // 8 for b in best)


def test_chains_arbitrary_links():
    """Random left/right indices (mostly unconfirmed links, some long
    confirmed runs planted) against the oracle, bit for bit."""
    import paper_1904_12626_amd as mpx
    rng = np.random.default_rng(90)
    l = 20000
    IL = np.full(l, -1, dtype=np.int64)
    IR = np.full(l, -1, dtype=np.int64)
    for i in range(l):
        if rng.random() < 0.7:
            IR[i] = rng.integers(i + 1, l) if i + 1 < l else -1
        if rng.random() < 0.7 and i > 0:
            IL[i] = rng.integers(0, i)
    for start in rng.choice(l - 2000, 30, replace=False):
        v = int(start)
        for _ in range(int(rng.integers(2, 40))):
            w = v + int(rng.integers(1, 50))
            if w >= l:
                break
            IR[v], IL[w] = w, v
            v = w
    ch = mpx.chains(torch.from_numpy(IL).to(DEV), torch.from_numpy(IR).to(DEV), min_len=4)
    nxt, length, count, best = O.chains(IL, IR, 4)
    assert np.array_equal(ch["next"].cpu().numpy(), nxt)
    assert np.array_equal(ch["length"].cpu().numpy(), length)
    assert ch["count"] == count and ch["best"] == best
