"""Comparison rules between the GPU library and the FP64 oracle.

P must agree within `tol` element by element.  I must equal the oracle's
index, except where several neighbours are (near-)tied: a GPU index is
accepted when it is admissible and its exact FP64 distance is within `tol`
of the oracle's minimum (several answers are then correct; only the
distance is unique)."""

import numpy as np

from oracle import mp_oracle as O


def compare_profile(TA, m, P, I, Po, Io, tol, TB=None, ez=None, where="", rows=None):
    P = np.asarray(P, dtype=np.float64)
    I = np.asarray(I)
    Po = np.asarray(Po, dtype=np.float64)
    Io = np.asarray(Io)
    TB = TA if TB is None else TB
    fin_o = np.isfinite(Po)
    assert np.array_equal(np.isfinite(P), fin_o), f"{where}: finiteness differs at {np.nonzero(np.isfinite(P) != fin_o)[0][:10]}"
    assert np.all(I[~fin_o] == -1) and np.all(Io[~fin_o] == -1), where
    d = np.abs(P[fin_o] - Po[fin_o])
    maxd = float(d.max()) if d.size else 0.0
    assert maxd <= tol, f"{where}: max |dP| = {maxd} > {tol} at {np.nonzero(fin_o)[0][np.argmax(d)]}"
    diff = np.nonzero(fin_o & (I != Io))[0]
    for i in diff:
        row = int(rows[i]) if rows is not None else int(i)
        j = int(I[i])
        assert j >= 0, f"{where}: row {row} has no index"
        if ez is not None:
            assert abs(row - j) > ez, f"{where}: row {row} index {j} inside the exclusion zone"
        dj = O.pair_distance(TA, row, TB, j, m)
        assert dj <= Po[i] + tol, f"{where}: row {row}: GPU index {j} at {dj} vs oracle {Io[i]} at {Po[i]}"
    return maxd, int(diff.size)
