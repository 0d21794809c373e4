"""FP64 recheck of the top motif pairs and discords."""

import numpy as np
import pytest
import torch

from oracle import cimpl
from oracle import mp_oracle as O
from workloads import planted_walk

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_recheck_matches_oracle_extraction():
    import paper_1904_12626_amd as mpx
    pw = planted_walk(8000, 64, seed=123, n_motifs=3, n_discords=2, dtype=np.float32)
    m, ez = pw.m, pw.m // 4
    Tg = torch.from_numpy(pw.T).to(DEV)
    P, I = mpx.selfjoin(Tg, m, ez)
    idx, dist = mpx.recheck(Tg, m, P, I, 3, 2)
    torch.cuda.synchronize()
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    Ph, Ih = P.cpu().numpy().astype(np.float64), I.cpu().numpy()
    mot = O.top_motifs(Ph, Ih, m, 3)
    dis = O.top_discords(Ph, m, 2)
    assert [tuple(x) for x in idx[:6].reshape(3, 2)] == [tuple(p) for p in mot]
    assert list(idx[6:]) == dis
    T64 = pw.T.astype(np.float64)
    for q, (i, j) in enumerate(mot):
        assert abs(dist[q] - O.pair_distance(T64, i, T64, j, m)) < 1e-9
    for q, i in enumerate(dis):
        assert abs(dist[3 + q] - O.pair_distance(T64, i, T64, int(Ih[i]), m)) < 1e-9
    # the planted pairs are the motifs
    found = sorted(tuple(sorted(p)) for p in mot)
    for a, b in pw.motif_pairs:
        assert any(abs(a - x) <= m // 8 and abs(b - y) <= m // 8 for x, y in found)
