"""ctypes wrapper of the C + OpenMP brute-force oracle (mp_oracle.c).

TEST INFRASTRUCTURE ONLY (tests/, the smoke check, the CPU-baseline leg of
bench.py).  ``build_oracle()`` compiles the shared library with gcc.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mp_oracle.c")
_LIB = os.path.join(_HERE, "libmp_oracle.so")
_lib = None


def build_oracle() -> str:
    """Compile mp_oracle.c -> libmp_oracle.so (gcc, OpenMP, strict IEEE)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_oracle()
    lib = ctypes.CDLL(_LIB)
    d, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.mpo_selfjoin_rows.argtypes = [d, i64, i32, i64, d, i64, d, d]
    lib.mpo_selfjoin_rows.restype = ctypes.c_int
    lib.mpo_selfjoin_rows_restricted.argtypes = [d, i64, i32, i64, d, i32, d, i64, d, d]
    lib.mpo_selfjoin_rows_restricted.restype = ctypes.c_int
    lib.mpo_abjoin_rows.argtypes = [d, i64, d, i64, i32, d, i64, d, d]
    lib.mpo_abjoin_rows.restype = ctypes.c_int
    lib.mpo_window_stats.argtypes = [d, i64, i32, d, d, d]
    lib.mpo_window_stats.restype = None
    lib.mpo_max_threads.argtypes = []
    lib.mpo_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().mpo_max_threads())


def selfjoin_rows(T, m: int, ez: int, rows):
    lib = _load()
    T = np.ascontiguousarray(T, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    P = np.empty(rows.size)
    I = np.empty(rows.size, dtype=np.int64)
    rc = lib.mpo_selfjoin_rows(_p(T), T.size, m, ez, _p(rows), rows.size, _p(P), _p(I))
    if rc != 0:
        raise ValueError("mpo_selfjoin_rows: bad arguments")
    return P, I


def abjoin_rows(A, B, m: int, rows):
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    P = np.empty(rows.size)
    I = np.empty(rows.size, dtype=np.int64)
    rc = lib.mpo_abjoin_rows(_p(A), A.size, _p(B), B.size, m, _p(rows), rows.size, _p(P), _p(I))
    if rc != 0:
        raise ValueError("mpo_abjoin_rows: bad arguments")
    return P, I


_SIDES = {"both": 0, "right": 1, "left": 2}


def selfjoin_rows_restricted(T, m: int, ez: int, rows, allowed=None, side: str = "both"):
    """Self-join entries for `rows` over the candidates j on `side` of i
    ("right": j > i, "left": j < i) whose offset |i - j| has allowed[k]
    (boolean array of l entries; None = every offset)."""
    lib = _load()
    T = np.ascontiguousarray(T, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    l = T.size - m + 1
    al = None
    if allowed is not None:
        al = np.ascontiguousarray(np.asarray(allowed, dtype=bool).astype(np.uint8))
        if al.size != l:
            raise ValueError("allowed must have l entries")
    P = np.empty(rows.size)
    I = np.empty(rows.size, dtype=np.int64)
    rc = lib.mpo_selfjoin_rows_restricted(_p(T), T.size, m, ez, None if al is None else _p(al), _SIDES[side],
                                          _p(rows), rows.size, _p(P), _p(I))
    if rc != 0:
        raise ValueError("mpo_selfjoin_rows_restricted: bad arguments")
    return P, I


def selfjoin(T, m: int, ez: int):
    n = np.asarray(T).shape[0]
    return selfjoin_rows(T, m, ez, np.arange(n - m + 1))


def window_stats(T, m: int):
    lib = _load()
    T = np.ascontiguousarray(T, dtype=np.float64)
    l = T.size - m + 1
    mu = np.empty(l)
    sg = np.empty(l)
    fl = np.empty(l, dtype=np.int8)
    lib.mpo_window_stats(_p(T), T.size, m, _p(mu), _p(sg), _p(fl))
    return mu, sg, (fl & 1).astype(bool), (fl & 2).astype(bool)
