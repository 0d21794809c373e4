"""Plain FP64 CPU oracle for the exact matrix-profile similarity join.

TEST INFRASTRUCTURE ONLY.  This module is imported by ``tests/``, by the
package's smoke check and by the CPU-baseline leg of ``bench.py``; the
product path never imports, calls or links it, and it shares no code,
constants or helpers with the HIP library.

What it computes, and where the paper states it (tsmp, Bischoff &
Rodrigues, arXiv 1904.12626):

* Section 2 ("The matrix profile"): the matrix profile is the vector of
  Euclidean distances from every subsequence of a sliding-window join to its
  nearest neighbour, i.e. the smallest non-trivial entry of each row of the
  full distance matrix; the profile index holds the position of that
  neighbour.  The method is exact (no false positives or dismissals), so the
  brute-force row minimum *is* the definition, and that is what this module
  writes out.
* Section 3.3 (brute force is O(n^2 m)) and 3.3.4 (SiMPle is the one mode
  that skips z-normalisation): every other mode compares z-normalised
  windows.
* Section 3.2: one series gives a self-join, two give an AB-join; the
  exclusion zone is a fraction of the window size that suppresses trivial
  matches in self-joins.  The printed sessions in Section 3.4 (profile sizes
  9922 and 855, exclusion zones 40 and 13) fix the profile length n-m+1 and
  the rounding of the zone upwards.

Readings taken where the paper is silent (each is listed in the design
notes and pinned by a test):

1. sigma is the population standard deviation (ddof=0), so ||z||^2 = m and
   0 <= d <= 2 sqrt(m).
2. ez = ceil(frac * m); pairs with |i - j| <= ez are excluded.
3. Ties go to the smallest index (strict "<" scan in increasing j).
4. A constant window (all values equal) has the zero vector as its
   z-normalised form: d(const, x) = sqrt(m), d(const, const) = 0.
5. A window holding a non-finite value is invalid: its P is +inf, its I is
   -1, and it is never anybody's neighbour.
6. P holds distances, not squared distances; I is 0-based.

Every distance here is computed in the *direct difference form*
``sqrt(sum((z_i - z_j)**2))`` from explicitly z-normalised windows.
"""

from __future__ import annotations

from fractions import Fraction

import numpy as np

__all__ = [
    "profile_length",
    "exclusion_zone",
    "window_stats",
    "znormalize",
    "pair_distance",
    "distance_matrix",
    "selfjoin",
    "selfjoin_restricted",
    "selfjoin_rows",
    "abjoin",
    "abjoin_rows",
    "top_motifs",
    "arc_curve",
    "corrected_arc_curve",
    "fluss_segments",
    "chains",
    "top_discords",
    "reference_gradient",
    "profile_sum_loss",
    "reference_gradient_ab",
    "abjoin_sum_loss",
    "simple_join",
    "mstomp",
]


# --------------------------------------------------------------------------
# Sizes (Section 3.2 exclusion zone; Section 3.4 printed sessions)
# --------------------------------------------------------------------------

def profile_length(n: int, m: int) -> int:
    """Number of length-m windows of a length-n series: n - m + 1."""
    return int(n) - int(m) + 1


def exclusion_zone(m: int, frac) -> int:
    """ez = ceil(frac * m), evaluated exactly (Section 3.2; the printed
    sessions give 80 * 1/2 -> 40 and 50 * 1/4 = 12.5 -> 13)."""
    f = Fraction(frac).limit_denominator(1 << 20) if isinstance(frac, float) else Fraction(frac)
    v = f * int(m)
    return int(-((-v.numerator) // v.denominator))


# --------------------------------------------------------------------------
# Window statistics and z-normalisation (Section 3.3.4: z-normalised modes)
# --------------------------------------------------------------------------

def _windows(T: np.ndarray, m: int) -> np.ndarray:
    return np.lib.stride_tricks.sliding_window_view(T, m)


def window_stats(T, m: int, chunk: int = 1 << 16):
    """Two-pass FP64 mean and population std of every window.

    Returns (mu, sigma, valid, const):  valid is False for windows holding a
    non-finite value; const is True for windows whose m values are all
    bitwise equal (max == min).  mu/sigma of invalid windows are NaN.
    """
    T = np.asarray(T, dtype=np.float64)
    l = profile_length(T.shape[0], m)
    mu = np.empty(l)
    sig = np.empty(l)
    valid = np.empty(l, dtype=bool)
    const = np.empty(l, dtype=bool)
    W = _windows(T, m)
    for s in range(0, l, chunk):
        w = W[s:s + chunk]
        fin = np.isfinite(w).all(axis=1)
        with np.errstate(invalid="ignore", over="ignore"):
            mean = w.mean(axis=1)
            dev = w - mean[:, None]
            sd = np.sqrt((dev * dev).mean(axis=1))
            cst = w.max(axis=1) == w.min(axis=1)
        mean[~fin] = np.nan
        sd[~fin] = np.nan
        mu[s:s + chunk] = mean
        sig[s:s + chunk] = sd
        valid[s:s + chunk] = fin
        const[s:s + chunk] = cst & fin
    return mu, sig, valid, const


def znormalize(T, m: int):
    """Matrix Z[l, m] of z-normalised windows (rows of invalid windows are
    NaN, rows of constant windows are zero)."""
    T = np.asarray(T, dtype=np.float64)
    mu, sig, valid, const = window_stats(T, m)
    W = _windows(T, m)
    Z = np.full(W.shape, np.nan)
    ok = valid & ~const
    Z[ok] = (W[ok] - mu[ok, None]) / sig[ok, None]
    Z[const] = 0.0
    return Z, valid


def pair_distance(TA, i: int, TB, j: int, m: int) -> float:
    """Distance between window i of TA and window j of TB, direct form."""
    a = np.asarray(TA, dtype=np.float64)[i:i + m]
    b = np.asarray(TB, dtype=np.float64)[j:j + m]
    if not (np.isfinite(a).all() and np.isfinite(b).all()):
        return np.inf

    def z(w):
        if w.max() == w.min():
            return np.zeros_like(w)
        mu = w.mean()
        return (w - mu) / np.sqrt(((w - mu) ** 2).mean())

    d = z(a) - z(b)
    return float(np.sqrt((d * d).sum()))


# --------------------------------------------------------------------------
# Brute force joins (Section 2: row minima of the distance matrix)
# --------------------------------------------------------------------------

def distance_matrix(TA, m: int, TB=None) -> np.ndarray:
    """Full distance matrix D[i, j] = ||z(TA_i) - z(TB_j)|| (inf where a
    window is invalid).  Small inputs only."""
    ZA, vA = znormalize(TA, m)
    ZB, vB = (ZA, vA) if TB is None else znormalize(TB, m)
    diff = ZA[:, None, :] - ZB[None, :, :]
    D = np.sqrt((diff * diff).sum(axis=2))
    D[~vA, :] = np.inf
    D[:, ~vB] = np.inf
    return D


def _row_min(drow: np.ndarray):
    """Strict-'<' scan in increasing index == first argmin."""
    if drow.size == 0:
        return np.inf, -1
    j = int(np.argmin(drow))
    if not np.isfinite(drow[j]):
        return np.inf, -1
    return float(drow[j]), j


def selfjoin(T, m: int, ez: int, block: int = 64):
    """Self-join matrix profile (P, I): P[i] = min over |i-j| > ez of d(i, j).

    Brute force over all pairs in the direct difference form, O(l^2 m).
    """
    Z, valid = znormalize(T, m)
    l = Z.shape[0]
    P = np.full(l, np.inf)
    I = np.full(l, -1, dtype=np.int64)
    Zv = np.where(valid[:, None], Z, 0.0)
    idx = np.arange(l)
    for s in range(0, l, block):
        rows = idx[s:s + block]
        diff = Zv[None, :, :] - Zv[rows, None, :]
        D = np.sqrt((diff * diff).sum(axis=2))
        D[:, ~valid] = np.inf
        D[np.abs(rows[:, None] - idx[None, :]) <= ez] = np.inf
        for r, i in enumerate(rows):
            if valid[i]:
                P[i], I[i] = _row_min(D[r])
    return P, I


def selfjoin_restricted(T, m: int, ez: int, allowed=None, side: str = "both", block: int = 64):
    """Self-join over a subset of the candidates: P[i] = min of d(i, j) over
    |i-j| > ez with j on `side` of i ("right": j > i, "left": j < i,
    "both") and allowed[|i-j|] (a boolean array over offsets 0..l-1; None =
    every offset).

    The anytime modes of Section 3.3 (STAMP, SCRIMP) return this profile for
    the offsets processed so far; the left and right profiles used by time
    series chains (Section 3.4.3) are its two one-sided cases.  Brute force
    in the direct difference form, like `selfjoin`.
    """
    if side not in ("both", "left", "right"):
        raise ValueError("side must be 'both', 'left' or 'right'")
    Z, valid = znormalize(T, m)
    l = Z.shape[0]
    allow = np.ones(l, dtype=bool) if allowed is None else np.asarray(allowed, dtype=bool)
    P = np.full(l, np.inf)
    I = np.full(l, -1, dtype=np.int64)
    Zv = np.where(valid[:, None], Z, 0.0)
    idx = np.arange(l)
    for s in range(0, l, block):
        rows = idx[s:s + block]
        diff = Zv[None, :, :] - Zv[rows, None, :]
        D = np.sqrt((diff * diff).sum(axis=2))
        D[:, ~valid] = np.inf
        off = idx[None, :] - rows[:, None]          # j - i
        D[np.abs(off) <= ez] = np.inf
        D[~allow[np.abs(off)]] = np.inf
        if side == "right":
            D[off < 0] = np.inf
        elif side == "left":
            D[off > 0] = np.inf
        for r, i in enumerate(rows):
            if valid[i]:
                P[i], I[i] = _row_min(D[r])
    return P, I


def selfjoin_rows(T, m: int, ez: int, rows, chunk: int = 1 << 15):
    """Exact P[i], I[i] of a self-join for the listed rows only (the full
    row minimum, so these entries equal the full join's).  Windows are
    z-normalised chunk by chunk, never all at once."""
    return _join_rows(T, T, m, rows, ez, chunk)


def abjoin(A, B, m: int):
    """AB-join: P_AB[i] = min_j d(A_i, B_j) with index, and P_BA[j] =
    min_i d(A_i, B_j) with index.  No exclusion zone (Section 3.2 gives the
    zone for self-joins only)."""
    D = distance_matrix(A, m, B)
    lA, lB = D.shape
    Pab = np.full(lA, np.inf)
    Iab = np.full(lA, -1, dtype=np.int64)
    Pba = np.full(lB, np.inf)
    Iba = np.full(lB, -1, dtype=np.int64)
    for i in range(lA):
        Pab[i], Iab[i] = _row_min(D[i])
    for j in range(lB):
        Pba[j], Iba[j] = _row_min(D[:, j])
    return Pab, Iab, Pba, Iba


def abjoin_rows(A, B, m: int, rows, chunk: int = 1 << 15):
    """Exact P_AB[i], I_AB[i] for the listed rows of A (swap A and B to get
    entries of P_BA)."""
    return _join_rows(A, B, m, rows, None, chunk)


def _join_rows(TA, TB, m, rows, ez, chunk):
    TA = np.asarray(TA, dtype=np.float64)
    TB = np.asarray(TB, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    muA, sgA, vA, cA = window_stats(TA, m)
    if TB is TA:
        muB, sgB, vB, cB = muA, sgA, vA, cA
    else:
        muB, sgB, vB, cB = window_stats(TB, m)
    WA = _windows(TA, m)
    WB = _windows(TB, m)
    lB = WB.shape[0]
    zr = np.zeros((rows.size, m))
    for r, i in enumerate(rows):
        if vA[i] and not cA[i]:
            zr[r] = (WA[i] - muA[i]) / sgA[i]
    best = np.full(rows.size, np.inf)
    arg = np.full(rows.size, -1, dtype=np.int64)
    jidx = np.arange(lB)
    for s in range(0, lB, chunk):
        e = min(lB, s + chunk)
        w = WB[s:e]
        ok = vB[s:e] & ~cB[s:e]
        zc = np.zeros(w.shape)
        zc[ok] = (w[ok] - muB[s:e][ok, None]) / sgB[s:e][ok, None]
        for r, i in enumerate(rows):
            if not vA[i]:
                continue
            diff = zc - zr[r]
            d = np.sqrt((diff * diff).sum(axis=1))
            d[~vB[s:e]] = np.inf
            if ez is not None:
                d[np.abs(jidx[s:e] - i) <= ez] = np.inf
            j = int(np.argmin(d))
            if d[j] < best[r]:           # strict: earlier chunks win ties
                best[r] = d[j]
                arg[r] = s + j
    best[arg < 0] = np.inf
    return best, arg


# --------------------------------------------------------------------------
# Motifs and discords read off the profile (Section 2 properties; the
# find_motif call of Section 3.2.1/3.4.1 with masking around each find)
# --------------------------------------------------------------------------

def top_motifs(P, I, m: int, k: int):
    """Repeatedly take the pair (i, I[i]) at the smallest finite P, then mask
    every index within m of either member; k times."""
    P = np.array(P, dtype=np.float64)
    I = np.asarray(I)
    out = []
    for _ in range(k):
        cand = np.where(np.isfinite(P), P, np.inf)
        i = int(np.argmin(cand))
        if not np.isfinite(cand[i]) or I[i] < 0:
            break
        j = int(I[i])
        out.append((i, j))
        for c in (i, j):
            P[max(0, c - m):c + m + 1] = np.inf
    return out


def top_discords(P, m: int, k: int):
    """Repeatedly take the largest finite P, masking within m of it."""
    P = np.array(P, dtype=np.float64)
    out = []
    for _ in range(k):
        cand = np.where(np.isfinite(P), P, -np.inf)
        i = int(np.argmax(cand))
        if not np.isfinite(cand[i]):
            break
        out.append(i)
        P[max(0, i - m):i + m + 1] = np.nan
    return out


# --------------------------------------------------------------------------
# Data-mining passes over a profile index: semantic segmentation
# (Section 3.4.2, FLUSS after Gharghabi et al. 2017) and time series chains
# (Section 3.4.3, after Zhu et al. 2018)
# --------------------------------------------------------------------------

def arc_curve(I):
    """AC[x] = number of windows i whose arc to I[i] spans x, i.e.
    min(i, I[i]) <= x < max(i, I[i]).  Entries < 0, >= l or equal to i draw
    no arc.  (+1 at the arc's start, -1 at its end, then a running sum.)"""
    I = np.asarray(I, dtype=np.int64)
    l = I.size
    marks = np.zeros(l + 1, dtype=np.int64)
    for i in range(l):
        j = int(I[i])
        if j < 0 or j >= l or j == i:
            continue
        marks[min(i, j)] += 1
        marks[max(i, j)] -= 1
    return np.cumsum(marks[:l])


def corrected_arc_curve(I, zone: int):
    """CAC[x] = min(AC[x] / IAC[x], 1) with IAC[x] = 2x(l - x)/l, the
    expected arc count when every arc ends at a uniformly random position;
    1 within `zone` of either end."""
    ac = arc_curve(I).astype(np.float64)
    l = ac.size
    cac = np.ones(l)
    for x in range(zone, l - zone):
        ideal = 2.0 * x * (l - x) / l
        if ideal > 0:
            cac[x] = min(ac[x] / ideal, 1.0)
    return cac


def fluss_segments(cac, k: int, zone: int):
    """k boundaries: repeatedly the smallest CAC (first index on ties)
    outside the edge zones and farther than `zone` from earlier picks; -1
    once nothing is left."""
    cac = np.asarray(cac, dtype=np.float64)
    l = cac.size
    picks = []
    for _ in range(k):
        best, arg = np.inf, -1
        for x in range(zone, l - zone):
            if any(abs(x - c) <= zone for c in picks if c >= 0):
                continue
            if cac[x] < best:
                best, arg = cac[x], x
        picks.append(arg)
    return picks


def chains(IL, IR, min_len: int = 3):
    """Chains from the left and right profile indices.  The link i -> IR[i]
    holds when IL[IR[i]] == i; the links form disjoint increasing paths.
    Returns (next, length, count, best): the confirmed successor of every
    window (-1 if none), the number of windows from i to its chain's end,
    the number of chains (counted at their first window) with at least
    min_len windows, and the longest chain (the earliest on equal lengths)."""
    IL = np.asarray(IL, dtype=np.int64)
    IR = np.asarray(IR, dtype=np.int64)
    l = IL.size
    nxt = np.full(l, -1, dtype=np.int64)
    for i in range(l):
        j = int(IR[i])
        if i < j < l and IL[j] == i:
            nxt[i] = j
    length = np.ones(l, dtype=np.int64)
    for i in range(l - 1, -1, -1):
        if nxt[i] >= 0:
            length[i] = 1 + length[nxt[i]]
    count, best_head, best_len = 0, -1, 0
    for i in range(l):
        p = int(IL[i])
        if 0 <= p < i and nxt[p] == i:
            continue                       # not the first window of its chain
        if length[i] >= min_len:
            count += 1
        if length[i] > best_len:
            best_head, best_len = i, int(length[i])
    best = []
    v = best_head
    while v >= 0 and len(best) < best_len:
        best.append(v)
        v = int(nxt[v])
    return nxt, length, count, best


# --------------------------------------------------------------------------
# Gradient of sum-type losses through the profile (not in the paper; the
# closed form below is derived from the direct distance and pinned against
# central finite differences by the tests)
# --------------------------------------------------------------------------

def reference_gradient(T, m: int, I, gP):
    """dL/dT for L with dL/dP = gP, holding the index I fixed.

    For the row i -> j = I[i] with distance d > 0 and Pearson correlation
    rho = z_i . z_j / m, differentiating d = ||z_i - z_j|| through the
    z-normalisation z = (x - mean) / sigma (whose Jacobian is
    (Id - 11^T/m - z z^T/m) / sigma) gives

        dd/dT[i:i+m] = (rho * z_i - z_j) / (sigma_i * d)
        dd/dT[j:j+m] = (rho * z_j - z_i) / (sigma_j * d)

    Rows with I[i] < 0, non-finite P, d == 0 or a constant window on either
    side contribute nothing (the subgradient 0 is taken there).
    """
    T = np.asarray(T, dtype=np.float64)
    gP = np.asarray(gP, dtype=np.float64)
    I = np.asarray(I)
    g = np.zeros_like(T)
    for i in range(I.shape[0]):
        j = int(I[i])
        if j < 0 or gP[i] == 0.0:
            continue
        a = T[i:i + m]
        b = T[j:j + m]
        if not (np.isfinite(a).all() and np.isfinite(b).all()):
            continue
        if a.max() == a.min() or b.max() == b.min():
            continue
        sa = np.sqrt(((a - a.mean()) ** 2).mean())
        sb = np.sqrt(((b - b.mean()) ** 2).mean())
        za = (a - a.mean()) / sa
        zb = (b - b.mean()) / sb
        diff = za - zb
        d = np.sqrt((diff * diff).sum())
        if d == 0.0:
            continue
        rho = (za * zb).sum() / m
        g[i:i + m] += gP[i] * (rho * za - zb) / (sa * d)
        g[j:j + m] += gP[i] * (rho * zb - za) / (sb * d)
    return g


def profile_sum_loss(T, m: int, I) -> float:
    """L = sum_i d(i, I[i]) with the index held fixed (the quantity whose
    finite differences pin reference_gradient)."""
    T = np.asarray(T, dtype=np.float64)
    tot = 0.0
    for i in range(len(I)):
        j = int(I[i])
        if j < 0:
            continue
        tot += pair_distance(T, i, T, j, m)
    return tot


def reference_gradient_ab(A, B, m: int, Iab, gPab, Iba, gPba):
    """(dL/dA, dL/dB) for an AB-join loss with dL/dP_ab = gPab and
    dL/dP_ba = gPba, indices held fixed: row i of A with neighbour j = Iab[i]
    of B adds gPab[i] * dd(A_i, B_j) -- (rho z_a - z_b)/(sigma_a d) on
    A[i:i+m] and (rho z_b - z_a)/(sigma_b d) on B[j:j+m] -- and row j of B
    with neighbour Iba[j] of A the same with the roles swapped.  Same
    subgradient-0 rules as reference_gradient."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    gA = np.zeros_like(A)
    gB = np.zeros_like(B)

    def add(X, gX, i, Y, gY, j, g):
        a = X[i:i + m]
        b = Y[j:j + m]
        if g == 0.0 or not (np.isfinite(a).all() and np.isfinite(b).all()):
            return
        if a.max() == a.min() or b.max() == b.min():
            return
        sa = np.sqrt(((a - a.mean()) ** 2).mean())
        sb = np.sqrt(((b - b.mean()) ** 2).mean())
        za = (a - a.mean()) / sa
        zb = (b - b.mean()) / sb
        d = np.sqrt(((za - zb) ** 2).sum())
        if d == 0.0:
            return
        rho = (za * zb).sum() / m
        gX[i:i + m] += g * (rho * za - zb) / (sa * d)
        gY[j:j + m] += g * (rho * zb - za) / (sb * d)

    for i in range(len(Iab)):
        if Iab[i] >= 0:
            add(A, gA, i, B, gB, int(Iab[i]), float(gPab[i]))
    for j in range(len(Iba)):
        if Iba[j] >= 0:
            add(B, gB, j, A, gA, int(Iba[j]), float(gPba[j]))
    return gA, gB


def abjoin_sum_loss(A, B, m: int, Iab, wab, Iba, wba) -> float:
    """L = sum_i wab[i] d(A_i, B_Iab[i]) + sum_j wba[j] d(B_j, A_Iba[j]),
    indices held fixed."""
    tot = 0.0
    for i in range(len(Iab)):
        if Iab[i] >= 0:
            tot += wab[i] * pair_distance(A, i, B, int(Iab[i]), m)
    for j in range(len(Iba)):
        if Iba[j] >= 0:
            tot += wba[j] * pair_distance(B, j, A, int(Iba[j]), m)
    return tot


# --------------------------------------------------------------------------
# Non-normalised (SiMPle) and multidimensional (mSTOMP) joins, Sections
# 3.3.4 and 3.3.5.  T has shape [D, n]: D dimensions sampled together; a
# window is invalid when any dimension holds a non-finite value in it.
# --------------------------------------------------------------------------

def _md_windows(T, m):
    T = np.atleast_2d(np.asarray(T, dtype=np.float64))
    D, n = T.shape
    l = n - m + 1
    W = np.stack([_windows(T[d], m) for d in range(D)])      # [D, l, m]
    valid = np.isfinite(W).all(axis=(0, 2))
    return W, valid


def simple_join(TA, m: int, ez=None, TB=None, rows=None):
    """SiMPle profile: P[i] = min_j sqrt(sum_d ||A_i^d - B_j^d||^2) over all
    dimensions, no z-normalisation (Section 3.3.4).  Self-join (TB None,
    pairs with |i - j| <= ez excluded) or AB-join (no zone).  Brute force;
    `rows` limits the rows computed (entries of the others stay +inf / -1)."""
    WA, vA = _md_windows(TA, m)
    WB, vB = (WA, vA) if TB is None else _md_windows(TB, m)
    lA, lB = WA.shape[1], WB.shape[1]
    XA = np.where(vA[None, :, None], WA, 0.0).transpose(1, 0, 2).reshape(lA, -1)
    XB = np.where(vB[None, :, None], WB, 0.0).transpose(1, 0, 2).reshape(lB, -1)
    P = np.full(lA, np.inf)
    I = np.full(lA, -1, dtype=np.int64)
    jidx = np.arange(lB)
    for i in (range(lA) if rows is None else rows):
        if not vA[i]:
            continue
        diff = XB - XA[i]
        d = np.sqrt((diff * diff).sum(axis=1))
        d[~vB] = np.inf
        if TB is None:
            d[np.abs(jidx - i) <= ez] = np.inf
        P[i], I[i] = _row_min(d)
    return P, I


def mstomp(T, m: int, ez: int, rows=None):
    """Multidimensional profiles (Section 3.3.5): for every pair the
    z-normalised distance of each dimension (constant windows normalise to
    zero), sorted ascending; the k-dimensional distance is the mean of the k
    smallest; P[k-1][i] = min over |i - j| > ez of it, k = 1 .. D.
    Returns P, I of shape [D, l] (`rows` limits the rows computed)."""
    W, valid = _md_windows(T, m)
    D, l, _ = W.shape
    Z = np.zeros_like(W)
    for d in range(D):
        mu = W[d].mean(axis=1)
        sg = np.sqrt(((W[d] - mu[:, None]) ** 2).mean(axis=1))
        const = W[d].max(axis=1) == W[d].min(axis=1)
        ok = valid & ~const
        Z[d, ok] = (W[d, ok] - mu[ok, None]) / sg[ok, None]
    P = np.full((D, l), np.inf)
    I = np.full((D, l), -1, dtype=np.int64)
    jidx = np.arange(l)
    for i in (range(l) if rows is None else rows):
        if not valid[i]:
            continue
        dist = np.sqrt(((Z - Z[:, i:i + 1, :]) ** 2).sum(axis=2))   # [D, l]
        dist = np.sort(dist, axis=0)
        avg = np.cumsum(dist, axis=0) / np.arange(1, D + 1)[:, None]
        avg[:, ~valid] = np.inf
        avg[:, np.abs(jidx - i) <= ez] = np.inf
        for k in range(D):
            P[k, i], I[k, i] = _row_min(avg[k])
    return P, I
