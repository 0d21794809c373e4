"""mpx: exact matrix-profile similarity joins on AMD MI355X (gfx950).

The matrix profile (tsmp, arXiv 1904.12626, Section 2) holds, for every
length-m window of a series, the z-normalised Euclidean distance to its
nearest non-trivial neighbour, and the profile index its position.  This
package computes it with hand-written HIP kernels behind a C ABI
(include/mp.h, libmpx.so); Python only marshals arguments.

    P, I = mpx.selfjoin(T, m, ez)                 # Section 3.2 self-join
    Pab, Iab, Pba, Iba = mpx.abjoin(A, B, m)      # Section 3.2 AB-join
    plan = mpx.BatchPlan(lengths, windows, zones) # many joins, one launch
    P, I = mpx.matrix_profile(T_batch, m, ez)     # differentiable profile
    P, I, chunks = mpx.anytime_selfjoin(T, m, ez, fraction=0.05)  # Sections 3.3.1/3.3.3
    P, I, PL, IL, PR, IR = mpx.left_right_profiles(T, m, ez)      # left/right profiles
    cac, boundaries = mpx.fluss(I, m, k=2)        # Section 3.4.2 segmentation
    ch = mpx.chains(IL, IR)                       # Section 3.4.3 chains
    P, I = mpx.mdjoin(T_multi, m, ez, mode="simple")  # Section 3.3.4 SiMPle
    P, I = mpx.mdjoin(T_multi, m, ez, mode="multi")   # Section 3.3.5 k-dim profiles
    s = mpx.SelfJoinStream(T, m, ez, n_max=N); s.append(x)  # incremental (Section 2)
"""

from ._binding import (  # noqa: F401
    EXPORTS, LIB_PATH, MPError, ABJoinPlan, BatchPlan, SelfJoinPlan, SelfJoinStream, abjoin, abjoin_cells, anytime_order, chains, fluss,
    anytime_selfjoin, exclusion_zone, left_right_profiles, lib, make_options, mdjoin, recheck, selfjoin,
    selfjoin_cells, selfjoin_noalloc, selfjoin_chunks, timing_enable, timing_query,
)
from .autograd import MatrixProfileFn, abjoin_profile, matrix_profile  # noqa: F401

__all__ = [
    "selfjoin", "abjoin", "BatchPlan", "recheck", "MatrixProfileFn", "matrix_profile",
    "exclusion_zone", "selfjoin_cells", "abjoin_cells", "MPError", "lib", "SelfJoinPlan",
    "selfjoin_chunks", "anytime_order", "anytime_selfjoin", "left_right_profiles", "fluss", "chains",
    "ABJoinPlan", "abjoin_profile", "mdjoin", "SelfJoinStream", "selfjoin_noalloc",
]
