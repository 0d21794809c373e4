"""mpx: exact matrix-profile similarity joins on AMD MI355X (gfx950).

The matrix profile (tsmp, arXiv 1904.12626, Section 2) holds, for every
length-m window of a series, the z-normalised Euclidean distance to its
nearest non-trivial neighbour, and the profile index its position.  This
package computes it with hand-written HIP kernels behind a C ABI
(include/mp.h, libmpx.so); Python only marshals arguments.

    P, I = mpx.selfjoin(T, m, ez)                 # Section 3.2 self-join
    Pab, Iab, Pba, Iba = mpx.abjoin(A, B, m)      # Section 3.2 AB-join
    plan = mpx.BatchPlan(lengths, windows, zones) # many joins, one launch
    P, I = mpx.MatrixProfileFn.apply(T, plan)     # differentiable profile
"""

from ._binding import (  # noqa: F401
    EXPORTS, LIB_PATH, MPError, BatchPlan, abjoin, abjoin_cells, exclusion_zone, lib, make_options,
    recheck, selfjoin, selfjoin_cells, timing_enable, timing_query,
)
from .autograd import MatrixProfileFn, matrix_profile  # noqa: F401

__all__ = [
    "selfjoin", "abjoin", "BatchPlan", "recheck", "MatrixProfileFn", "matrix_profile",
    "exclusion_zone", "selfjoin_cells", "abjoin_cells", "MPError", "lib",
]
