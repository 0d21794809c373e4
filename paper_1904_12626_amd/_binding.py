"""ctypes binding of libmpx.so (include/mp.h).

Argument marshalling only: every step of the join runs in the library's HIP
kernels.  torch supplies device memory (outputs and workspace) and the
current stream.  The binding refuses to run when the library is missing.
"""

from __future__ import annotations

import ctypes
import math
import os
from fractions import Fraction
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpx.so")

MP_OK, MP_EINVAL, MP_EWORKSPACE, MP_ELAUNCH, MP_EUNSUPPORTED, MP_ETOOLARGE = 0, -1, -2, -3, -4, -5
MP_NOALLOC_SCRATCH_BYTES = 64 << 20
MP_F64, MP_F32 = 0, 1
MP_PREC_F64, MP_PREC_F32 = 0, 1
MP_FLAG_FP64_FINALIZE = 1
MP_FLAG_FLAT_LOADS = 2

# every symbol include/mp.h declares
EXPORTS = (
    "mp_selfjoin_workspace", "mp_selfjoin", "mp_abjoin_workspace", "mp_abjoin",
    "mp_batch_plan_create", "mp_batch_plan_workspace", "mp_batch_plan_profile_length",
    "mp_batch_plan_cells", "mp_batch_plan_upload", "mp_batch", "mp_batch_plan_destroy",
    "mp_backward", "mp_recheck_workspace", "mp_recheck", "mp_strerror", "mp_abi_version",
    "mp_selfjoin_cells", "mp_abjoin_cells", "mp_timing_enable", "mp_timing_query",
    "mp_selfjoin_chunks", "mp_selfjoin_plan_create", "mp_anytime_order",
    "mp_fluss_workspace", "mp_fluss", "mp_chains_workspace", "mp_chains", "mp_abjoin_plan_create",
    "mp_mdjoin_workspace", "mp_mdjoin", "mp_mdjoin_cells",
    "mp_stream_workspace", "mp_stream_init", "mp_stream_append", "mp_selfjoin_noalloc",
    "mp_backward_after_forward",
)


class MPError(RuntimeError):
    def __init__(self, where: str, status: int, msg: str):
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


class mp_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("reseed_rows", ctypes.c_int32),
                ("tile_slots", ctypes.c_int32), ("flags", ctypes.c_int32)]


_lib = None


def lib():
    """Load libmpx.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(hipcc, gfx950); there is no fallback implementation")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    op = ctypes.POINTER(mp_options)
    sig = {
        "mp_selfjoin_workspace": (sz, [i64, i32, i32, op]),
        "mp_selfjoin": (ctypes.c_int, [vp, i64, i32, i32, i32, op, vp, vp, vp, sz, vp]),
        "mp_selfjoin_noalloc": (ctypes.c_int, [vp, i64, i32, i32, i32, op, vp, vp, vp]),
        "mp_abjoin_workspace": (sz, [i64, i64, i32, i32, op]),
        "mp_abjoin": (ctypes.c_int, [vp, i64, vp, i64, i32, i32, op, vp, vp, vp, vp, vp, sz, vp]),
        "mp_batch_plan_create": (ctypes.c_int, [i32, vp, vp, vp, i32, op, ctypes.POINTER(vp)]),
        "mp_batch_plan_workspace": (sz, [vp]),
        "mp_batch_plan_profile_length": (i64, [vp]),
        "mp_batch_plan_cells": (i64, [vp]),
        "mp_batch_plan_upload": (ctypes.c_int, [vp, vp, sz, vp]),
        "mp_batch": (ctypes.c_int, [vp, vp, vp, vp, vp, sz, vp]),
        "mp_batch_plan_destroy": (None, [vp]),
        "mp_backward": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, sz, vp]),
        "mp_backward_after_forward": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "mp_recheck_workspace": (sz, [i64, i32]),
        "mp_recheck": (ctypes.c_int, [vp, i64, i32, i32, vp, vp, i32, i32, vp, vp, vp, sz, vp]),
        "mp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "mp_abi_version": (ctypes.c_int, []),
        "mp_selfjoin_cells": (i64, [i64, i32, i32]),
        "mp_abjoin_cells": (i64, [i64, i64, i32]),
        "mp_selfjoin_chunks": (i64, [i64, i32, i32, op, ctypes.POINTER(i64)]),
        "mp_selfjoin_plan_create": (ctypes.c_int, [i64, i32, i32, i32, op, i32, i64, vp, ctypes.POINTER(vp)]),
        "mp_anytime_order": (ctypes.c_int, [i64, ctypes.c_uint64, vp]),
        "mp_abjoin_plan_create": (ctypes.c_int, [i64, i64, i32, i32, op, ctypes.POINTER(vp)]),
        "mp_mdjoin_workspace": (sz, [i32, i32, i64, i64, i32]),
        "mp_mdjoin": (ctypes.c_int, [i32, i32, vp, i64, vp, i64, i32, i32, i32, vp, vp, vp, vp, vp, sz, vp]),
        "mp_mdjoin_cells": (i64, [i32, i64, i64, i32, i32]),
        "mp_stream_workspace": (sz, [i64, i32]),
        "mp_stream_init": (ctypes.c_int, [vp, i64, i64, i32, i32, i32, vp, vp, vp, sz, vp]),
        "mp_stream_append": (ctypes.c_int, [vp, i64, i64, i64, i32, i32, i32, vp, vp, vp, sz, vp]),
        "mp_fluss_workspace": (sz, [i64]),
        "mp_fluss": (ctypes.c_int, [vp, i64, i64, i32, vp, vp, vp, sz, vp]),
        "mp_chains_workspace": (sz, [i64]),
        "mp_chains": (ctypes.c_int, [vp, vp, i64, i32, vp, vp, vp, vp, vp, sz, vp]),
        "mp_timing_enable": (ctypes.c_int, [ctypes.c_int]),
        "mp_timing_query": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(where: str, status: int):
    if status != MP_OK:
        raise MPError(where, status, lib().mp_strerror(status).decode())


def exclusion_zone(m: int, frac=Fraction(1, 2)) -> int:
    """ez = ceil(frac * m) (the tsmp exclusion_zone argument is a fraction of
    the window; default 1/2)."""
    f = Fraction(frac).limit_denominator(1 << 20) if isinstance(frac, float) else Fraction(frac)
    v = f * int(m)
    return int(math.ceil(v))


def make_options(precision: str = "f32", reseed_rows: int = 0, tile_slots: int = 0,
                 fp64_finalize: bool = True, flat_loads: bool = False) -> mp_options:
    if precision not in ("f32", "f64"):
        raise ValueError("precision must be 'f32' or 'f64'")
    flags = (MP_FLAG_FP64_FINALIZE if fp64_finalize else 0) | (MP_FLAG_FLAT_LOADS if flat_loads else 0)
    return mp_options(MP_PREC_F32 if precision == "f32" else MP_PREC_F64, int(reseed_rows),
                      int(tile_slots), flags)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return MP_F64
    if t.dtype == torch.float32:
        return MP_F32
    raise TypeError(f"series must be float32 or float64, got {t.dtype}")


def _series(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dim() != 1:
        raise ValueError(f"{name} must be 1-D")
    return t.contiguous()


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def selfjoin(T: torch.Tensor, m: int, ez: int | None = None, *, exclusion_zone_frac=Fraction(1, 2),
             precision: str = "f32", reseed_rows: int = 0, tile_slots: int = 0,
             fp64_finalize: bool = True, stream=None, workspace: torch.Tensor | None = None):
    """Self-join matrix profile of a 1-D series: returns (P, I) on T's device.

    ez defaults to ceil(exclusion_zone_frac * m).  P has T's dtype, I is int64;
    invalid rows are (+inf, -1).  Enqueued on `stream` (default: current)."""
    T = _series(T, "T")
    L = lib()
    n = T.numel()
    if ez is None:
        ez = exclusion_zone(m, exclusion_zone_frac)
    dt = _dtype_code(T)
    opt = make_options(precision, reseed_rows, tile_slots, fp64_finalize)
    ws_bytes = L.mp_selfjoin_workspace(n, m, dt, ctypes.byref(opt))
    if ws_bytes == 0:
        _check("mp_selfjoin", MP_EINVAL if (m < 2 or n < m) else MP_EUNSUPPORTED)
    l = n - m + 1
    P = torch.empty(l, dtype=T.dtype, device=T.device)
    I = torch.empty(l, dtype=torch.int64, device=T.device)
    ws = workspace if workspace is not None else torch.empty(ws_bytes, dtype=torch.uint8, device=T.device)
    _check("mp_selfjoin", L.mp_selfjoin(_ptr(T), n, m, int(ez), dt, ctypes.byref(opt), _ptr(P), _ptr(I),
                                        _ptr(ws), ws.numel(), _stream(stream)))
    return P, I


def selfjoin_noalloc(T: torch.Tensor, m: int, ez: int | None = None, *, P: torch.Tensor, I: torch.Tensor,
                     exclusion_zone_frac=Fraction(1, 2), precision: str = "f32", reseed_rows: int = 0,
                     tile_slots: int = 0, fp64_finalize: bool = True, stream=None):
    """Self-join into caller-given P (T's dtype) and I (int64), both of length
    n - m + 1, through mp_selfjoin_noalloc: nothing is allocated, the
    library's fixed per-device scratch serves as the workspace (jobs whose
    workspace exceeds MP_NOALLOC_SCRATCH_BYTES raise MPError with
    MP_ETOOLARGE).  Calls on one device must be ordered on one stream."""
    T = _series(T, "T")
    n = T.numel()
    l = n - m + 1
    if ez is None:
        ez = exclusion_zone(m, exclusion_zone_frac)
    for t, name, dt_ in ((P, "P", T.dtype), (I, "I", torch.int64)):
        if not isinstance(t, torch.Tensor) or t.device != T.device or t.dtype != dt_ or t.numel() != l \
                or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt_} tensor of {l} entries on {T.device}")
    opt = make_options(precision, reseed_rows, tile_slots, fp64_finalize)
    _check("mp_selfjoin_noalloc", lib().mp_selfjoin_noalloc(_ptr(T), n, m, int(ez), _dtype_code(T),
                                                            ctypes.byref(opt), _ptr(P), _ptr(I),
                                                            _stream(stream)))
    return P, I


def abjoin(A: torch.Tensor, B: torch.Tensor, m: int, *, precision: str = "f32", reseed_rows: int = 0,
           tile_slots: int = 0, fp64_finalize: bool = True, stream=None):
    """AB-join: returns (P_ab, I_ab, P_ba, I_ba); I_ab indexes B, I_ba indexes A."""
    A = _series(A, "A")
    B = _series(B, "B")
    if A.dtype != B.dtype or A.device != B.device:
        raise ValueError("A and B must share dtype and device")
    L = lib()
    dt = _dtype_code(A)
    opt = make_options(precision, reseed_rows, tile_slots, fp64_finalize)
    nA, nB = A.numel(), B.numel()
    ws_bytes = L.mp_abjoin_workspace(nA, nB, m, dt, ctypes.byref(opt))
    if ws_bytes == 0:
        _check("mp_abjoin", MP_EINVAL)
    lA, lB = nA - m + 1, nB - m + 1
    Pab = torch.empty(lA, dtype=A.dtype, device=A.device)
    Iab = torch.empty(lA, dtype=torch.int64, device=A.device)
    Pba = torch.empty(lB, dtype=A.dtype, device=A.device)
    Iba = torch.empty(lB, dtype=torch.int64, device=A.device)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=A.device)
    _check("mp_abjoin", L.mp_abjoin(_ptr(A), nA, _ptr(B), nB, m, dt, ctypes.byref(opt), _ptr(Pab), _ptr(Iab),
                                    _ptr(Pba), _ptr(Iba), _ptr(ws), ws.numel(), _stream(stream)))
    return Pab, Iab, Pba, Iba


class BatchPlan:
    """Host plan of many self-joins of uneven lengths and windows
    (mp_batch_plan_*).  `run` enqueues only kernels and may be captured into
    a CUDA/HIP graph once `upload` has completed."""

    def __init__(self, lengths, windows, zones, dtype=torch.float32, device="cuda", *,
                 precision: str = "f32", reseed_rows: int = 0, tile_slots: int = 0,
                 fp64_finalize: bool = True, flat_loads: bool = False):
        L = lib()
        self.lengths = [int(x) for x in lengths]
        self.windows = [int(x) for x in windows]
        self.zones = [int(x) for x in zones]
        ns = len(self.lengths)
        if not (ns == len(self.windows) == len(self.zones)) or ns == 0:
            raise ValueError("lengths, windows and zones must be non-empty and of equal length")
        self.dtype = dtype
        self.device = torch.device(device)
        dt = MP_F64 if dtype == torch.float64 else MP_F32
        off = (ctypes.c_int64 * (ns + 1))()
        acc = 0
        for i, n in enumerate(self.lengths):
            off[i] = acc
            acc += n
        off[ns] = acc
        self.total_n = acc
        self.t_off = [off[i] for i in range(ns + 1)]
        mm = (ctypes.c_int32 * ns)(*self.windows)
        ee = (ctypes.c_int32 * ns)(*self.zones)
        self._opt = make_options(precision, reseed_rows, tile_slots, fp64_finalize, flat_loads)
        h = ctypes.c_void_p()
        _check("mp_batch_plan_create", L.mp_batch_plan_create(ns, off, mm, ee, dt, ctypes.byref(self._opt),
                                                              ctypes.byref(h)))
        self.p_off = []
        acc = 0
        for n, m in zip(self.lengths, self.windows):
            self.p_off.append(acc)
            acc += n - m + 1
        self.p_off.append(acc)
        self._setup(h)

    def _setup(self, h):
        L = lib()
        self._h = h
        self.forward_count = 0   # mp_batch calls on this plan's workspace so far
        self.profile_length = int(L.mp_batch_plan_profile_length(h))
        self.cells = int(L.mp_batch_plan_cells(h))
        self.ws_bytes = int(L.mp_batch_plan_workspace(h))
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.upload()

    def upload(self, stream=None):
        _check("mp_batch_plan_upload", lib().mp_batch_plan_upload(self._h, _ptr(self.workspace), self.ws_bytes,
                                                                   _stream(stream)))
        (stream or torch.cuda.current_stream()).synchronize()

    def run(self, T_cat: torch.Tensor, P_cat=None, I_cat=None, stream=None):
        T_cat = _series(T_cat, "T_cat")
        if T_cat.numel() != self.total_n or T_cat.dtype != self.dtype:
            raise ValueError("T_cat does not match the plan")
        if P_cat is None:
            P_cat = torch.empty(self.profile_length, dtype=self.dtype, device=T_cat.device)
        if I_cat is None:
            I_cat = torch.empty(self.profile_length, dtype=torch.int64, device=T_cat.device)
        _check("mp_batch", lib().mp_batch(self._h, _ptr(T_cat), _ptr(P_cat), _ptr(I_cat), _ptr(self.workspace),
                                          self.ws_bytes, _stream(stream)))
        self.forward_count += 1
        return P_cat, I_cat

    @property
    def reuses_forward(self) -> bool:
        """Whether backward_after_forward applies: the plan finalizes P in
        FP64 and gives the plain profile (not left/right)."""
        return bool(self._opt.flags & MP_FLAG_FP64_FINALIZE) and getattr(self, "sides", "both") == "both"

    def backward_after_forward(self, T_cat, I_cat, P_cat, gP_cat, gT_cat=None, stream=None):
        """mp_backward_after_forward: the backward of the last `run` on this
        plan (same T_cat, its P_cat and I_cat), reusing the forward's window
        statistics and distances.  The caller guarantees no other `run`
        happened in between (`forward_count` tells)."""
        T_cat = _series(T_cat, "T_cat")
        gP_cat = gP_cat.contiguous().to(self.dtype)
        if gT_cat is None:
            gT_cat = torch.empty_like(T_cat)
        _check("mp_backward_after_forward",
               lib().mp_backward_after_forward(self._h, _ptr(T_cat), _ptr(I_cat.contiguous()), _ptr(P_cat.contiguous()),
                                               _ptr(gP_cat), _ptr(gT_cat), _ptr(self.workspace), self.ws_bytes,
                                               _stream(stream)))
        return gT_cat

    def backward(self, T_cat, I_cat, gP_cat, gT_cat=None, stream=None):
        T_cat = _series(T_cat, "T_cat")
        gP_cat = gP_cat.contiguous().to(self.dtype)
        if gT_cat is None:
            gT_cat = torch.empty_like(T_cat)
        _check("mp_backward", lib().mp_backward(self._h, _ptr(T_cat), _ptr(I_cat.contiguous()), _ptr(gP_cat),
                                                _ptr(gT_cat), _ptr(self.workspace), self.ws_bytes,
                                                _stream(stream)))
        return gT_cat

    def split(self, X_cat):
        return [X_cat[self.p_off[i]:self.p_off[i + 1]] for i in range(len(self.lengths))]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.mp_batch_plan_destroy(h)
            self._h = None


class ABJoinPlan(BatchPlan):
    """AB-join as a batch plan (mp_abjoin_plan_create): `run(T_cat)` with
    T_cat = [A | B] returns (P, I) = ([P_ab | P_ba], [I_ab | I_ba]);
    `backward` gives [dL/dA | dL/dB]."""

    def __init__(self, nA, nB, m, dtype=torch.float32, device="cuda", *, precision: str = "f32",
                 reseed_rows: int = 0, tile_slots: int = 0, fp64_finalize: bool = True):
        L = lib()
        self.lengths, self.windows, self.zones = [int(nA), int(nB)], [int(m), int(m)], [-1, -1]
        self.dtype = dtype
        self.device = torch.device(device)
        self.total_n = int(nA) + int(nB)
        self.t_off = [0, int(nA), int(nA) + int(nB)]
        dt = MP_F64 if dtype == torch.float64 else MP_F32
        self._opt = make_options(precision, reseed_rows, tile_slots, fp64_finalize)
        h = ctypes.c_void_p()
        _check("mp_abjoin_plan_create", L.mp_abjoin_plan_create(int(nA), int(nB), int(m), dt,
                                                                ctypes.byref(self._opt), ctypes.byref(h)))
        lA, lB = int(nA) - int(m) + 1, int(nB) - int(m) + 1
        self.p_off = [0, lA, lA + lB]
        self._setup(h)


def selfjoin_chunks(n: int, m: int, ez: int, *, precision: str = "f32", tile_slots: int = 0):
    """(number of chunks, chunk width W) of a self-join's diagonal offsets
    ez+1 .. l-1 (mp_selfjoin_chunks)."""
    opt = make_options(precision, 0, tile_slots)
    w = ctypes.c_int64()
    c = lib().mp_selfjoin_chunks(int(n), int(m), int(ez), ctypes.byref(opt), ctypes.byref(w))
    if c < 0:
        raise ValueError("invalid self-join arguments")
    return int(c), int(w.value)


def anytime_order(count: int, seed: int):
    """Random order of `count` chunk numbers (mp_anytime_order), host list."""
    arr = (ctypes.c_int64 * max(1, int(count)))()
    _check("mp_anytime_order", lib().mp_anytime_order(int(count), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                                      arr))
    return [int(arr[i]) for i in range(int(count))]


class SelfJoinPlan(BatchPlan):
    """Self-join plan restricted to a set of diagonal chunks and/or giving the
    left and right profiles (mp_selfjoin_plan_create).  `run(T)` returns
    (P, I) of length l (sides="both") or 3l ([P | P_left | P_right],
    sides="lr")."""

    def __init__(self, n, m, ez, dtype=torch.float32, device="cuda", *, sides: str = "both", chunks=None,
                 precision: str = "f32", reseed_rows: int = 0, tile_slots: int = 0, fp64_finalize: bool = True):
        if sides not in ("both", "lr"):
            raise ValueError("sides must be 'both' or 'lr'")
        L = lib()
        self.lengths, self.windows, self.zones = [int(n)], [int(m)], [int(ez)]
        self.dtype = dtype
        self.device = torch.device(device)
        self.total_n = int(n)
        self.t_off = [0, int(n)]
        self.sides = sides
        self.chunks = None if chunks is None else [int(c) for c in chunks]
        dt = MP_F64 if dtype == torch.float64 else MP_F32
        self._opt = make_options(precision, reseed_rows, tile_slots, fp64_finalize)
        if chunks is None:
            arr, nch = None, 0
        else:
            chunks = [int(c) for c in chunks]
            nch = len(chunks)
            arr = (ctypes.c_int64 * max(1, nch))(*chunks)
        h = ctypes.c_void_p()
        _check("mp_selfjoin_plan_create",
               L.mp_selfjoin_plan_create(int(n), int(m), int(ez), dt, ctypes.byref(self._opt),
                                         1 if sides == "lr" else 0, nch, arr, ctypes.byref(h)))
        l = int(n) - int(m) + 1
        self.p_off = [0, l]
        self._setup(h)


def left_right_profiles(T: torch.Tensor, m: int, ez: Optional[int] = None, *,
                        exclusion_zone_frac=Fraction(1, 2), chunks=None, stream=None, **opts):
    """Profile and left/right profiles of one self-join sweep:
    (P, I, P_left, I_left, P_right, I_right)."""
    T = _series(T, "T")
    if ez is None:
        ez = exclusion_zone(m, exclusion_zone_frac)
    plan = SelfJoinPlan(T.numel(), m, ez, dtype=T.dtype, device=T.device, sides="lr", chunks=chunks, **opts)
    P, I = plan.run(T, stream=stream)
    l = T.numel() - m + 1
    return P[:l], I[:l], P[l:2 * l], I[l:2 * l], P[2 * l:], I[2 * l:]


def anytime_selfjoin(T: torch.Tensor, m: int, ez: Optional[int] = None, *, fraction: float = 0.05,
                     seed: int = 0, exclusion_zone_frac=Fraction(1, 2), stream=None, **opts):
    """Best-so-far self-join after a random `fraction` of the diagonal chunks
    (at least one when fraction > 0): returns (P, I, chunks used)."""
    T = _series(T, "T")
    if ez is None:
        ez = exclusion_zone(m, exclusion_zone_frac)
    count, _ = selfjoin_chunks(T.numel(), m, ez, precision=opts.get("precision", "f32"),
                               tile_slots=opts.get("tile_slots", 0))
    k = 0 if fraction <= 0 else min(count, max(1, int(math.ceil(fraction * count))))
    chunks = anytime_order(count, seed)[:k]
    plan = SelfJoinPlan(T.numel(), m, ez, dtype=T.dtype, device=T.device, chunks=chunks, **opts)
    P, I = plan.run(T, stream=stream)
    return P, I, chunks


class SelfJoinStream:
    """Incrementally updated self-join (mp_stream_init / mp_stream_append):
    the profile of everything appended so far, exact (FP64 state).
    `append(x)` adds samples; `P`, `I` are views of the current profile."""

    def __init__(self, T: torch.Tensor, m: int, ez: Optional[int] = None, *, n_max: int,
                 exclusion_zone_frac=Fraction(1, 2), stream=None):
        T = _series(T, "T")
        self.m = int(m)
        self.ez = exclusion_zone(m, exclusion_zone_frac) if ez is None else int(ez)
        self.n_max = int(n_max)
        self.dtype = T.dtype
        self.n = T.numel()
        if self.n > self.n_max:
            raise ValueError("initial series longer than n_max")
        L = lib()
        dev = T.device
        self.T = torch.empty(self.n_max, dtype=T.dtype, device=dev)
        self.T[:self.n].copy_(T)
        lmax = self.n_max - self.m + 1
        self._P = torch.empty(lmax, dtype=T.dtype, device=dev)
        self._I = torch.empty(lmax, dtype=torch.int64, device=dev)
        self.ws_bytes = int(L.mp_stream_workspace(self.n_max, self.m))
        if self.ws_bytes == 0:
            raise MPError("mp_stream_workspace", MP_EINVAL, "invalid arguments")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        _check("mp_stream_init", L.mp_stream_init(_ptr(self.T), self.n, self.n_max, self.m, self.ez,
                                                  _dtype_code(T), _ptr(self._P), _ptr(self._I), _ptr(self.ws),
                                                  self.ws_bytes, _stream(stream)))

    def append(self, x: torch.Tensor, stream=None):
        x = x.reshape(-1).to(self.T.device, self.dtype)
        k = x.numel()
        if self.n + k > self.n_max:
            raise ValueError("stream capacity n_max exceeded")
        self.T[self.n:self.n + k].copy_(x)
        _check("mp_stream_append", lib().mp_stream_append(_ptr(self.T), self.n, self.n + k, self.n_max, self.m,
                                                          self.ez, _dtype_code(self.T), _ptr(self._P),
                                                          _ptr(self._I), _ptr(self.ws), self.ws_bytes,
                                                          _stream(stream)))
        self.n += k

    @property
    def P(self):
        return self._P[:self.n - self.m + 1]

    @property
    def I(self):
        return self._I[:self.n - self.m + 1]


MP_MD_SIMPLE, MP_MD_MULTI = 0, 1


def _md_series(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dim() == 1:
        t = t.unsqueeze(0)
    if t.dim() != 2:
        raise ValueError(f"{name} must be [D, n] (or 1-D)")
    return t.contiguous()


def mdjoin(A: torch.Tensor, m: int, ez: Optional[int] = None, B: Optional[torch.Tensor] = None, *,
           mode: str = "simple", exclusion_zone_frac=Fraction(1, 2), stream=None):
    """Multidimensional joins of [D, n] series (mp_mdjoin).
    mode="simple": SiMPle (Section 3.3.4), raw Euclidean distance over all
    dimensions; returns (P, I) for a self-join or (P_ab, I_ab, P_ba, I_ba)
    with B.  mode="multi": the D multidimensional profiles of Section 3.3.5
    (self-join), P and I of shape [D, l], row k-1 = k dimensions."""
    A = _md_series(A, "A")
    D, nA = A.shape
    if mode not in ("simple", "multi"):
        raise ValueError("mode must be 'simple' or 'multi'")
    md = MP_MD_SIMPLE if mode == "simple" else MP_MD_MULTI
    dt = _dtype_code(A)
    L = lib()
    lA = nA - m + 1
    if B is None:
        if ez is None:
            ez = exclusion_zone(m, exclusion_zone_frac)
        np_ = D if md == MP_MD_MULTI else 1
        P = torch.empty(np_ * lA, dtype=A.dtype, device=A.device)
        I = torch.empty(np_ * lA, dtype=torch.int64, device=A.device)
        ws_bytes = int(L.mp_mdjoin_workspace(md, D, nA, 0, m))
        if ws_bytes == 0:
            raise MPError("mp_mdjoin_workspace", MP_EINVAL, "invalid arguments")
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=A.device)
        _check("mp_mdjoin", L.mp_mdjoin(md, D, _ptr(A), nA, None, 0, m, int(ez), dt, _ptr(P), _ptr(I), None, None,
                                        _ptr(ws), ws_bytes, _stream(stream)))
        if md == MP_MD_MULTI:
            return P.view(D, lA), I.view(D, lA)
        return P, I
    B = _md_series(B, "B")
    if B.shape[0] != D or B.dtype != A.dtype:
        raise ValueError("A and B must have the same dimensions and dtype")
    nB = B.shape[1]
    lB = nB - m + 1
    Pab = torch.empty(lA, dtype=A.dtype, device=A.device)
    Iab = torch.empty(lA, dtype=torch.int64, device=A.device)
    Pba = torch.empty(lB, dtype=A.dtype, device=A.device)
    Iba = torch.empty(lB, dtype=torch.int64, device=A.device)
    ws_bytes = int(L.mp_mdjoin_workspace(md, D, nA, nB, m))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=A.device)
    _check("mp_mdjoin", L.mp_mdjoin(md, D, _ptr(A), nA, _ptr(B), nB, m, -1, dt, _ptr(Pab), _ptr(Iab), _ptr(Pba),
                                    _ptr(Iba), _ptr(ws), ws_bytes, _stream(stream)))
    return Pab, Iab, Pba, Iba


def fluss(I: torch.Tensor, m: int, k: int = 2, zone: Optional[int] = None, stream=None):
    """Corrected arc curve of a profile index and k segment boundaries
    (mp_fluss; Section 3.4.2).  `zone` defaults to 5 m.  Returns
    (cac float64[l], segments int64[k])."""
    if not isinstance(I, torch.Tensor) or not I.is_cuda or I.dtype != torch.int64 or I.dim() != 1:
        raise TypeError("I must be a 1-D int64 CUDA (HIP) tensor")
    I = I.contiguous()
    l = I.numel()
    zone = 5 * int(m) if zone is None else int(zone)
    L = lib()
    cac = torch.empty(l, dtype=torch.float64, device=I.device)
    seg = torch.empty(max(1, k), dtype=torch.int64, device=I.device)
    ws_bytes = int(L.mp_fluss_workspace(l))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=I.device)
    _check("mp_fluss", L.mp_fluss(_ptr(I), l, zone, int(k), _ptr(cac), _ptr(seg), _ptr(ws), ws_bytes,
                                  _stream(stream)))
    return cac, seg[:k]


def chains(IL: torch.Tensor, IR: torch.Tensor, min_len: int = 3, stream=None):
    """Time series chains from left/right profile indices (mp_chains;
    Section 3.4.3).  Returns a dict: next, length (int64[l] tensors),
    count (chains with >= min_len windows), best (the longest chain's
    windows, a host list)."""
    for t, name in ((IL, "IL"), (IR, "IR")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int64 or t.dim() != 1:
            raise TypeError(f"{name} must be a 1-D int64 CUDA (HIP) tensor")
    if IL.numel() != IR.numel():
        raise ValueError("IL and IR differ in length")
    IL, IR = IL.contiguous(), IR.contiguous()
    l = IL.numel()
    L = lib()
    nxt = torch.empty(l, dtype=torch.int64, device=IL.device)
    length = torch.empty(l, dtype=torch.int64, device=IL.device)
    summary = torch.empty(3, dtype=torch.int64, device=IL.device)
    best = torch.empty(l, dtype=torch.int64, device=IL.device)
    ws_bytes = int(L.mp_chains_workspace(l))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=IL.device)
    _check("mp_chains", L.mp_chains(_ptr(IL), _ptr(IR), l, int(min_len), _ptr(nxt), _ptr(length), _ptr(summary),
                                    _ptr(best), _ptr(ws), ws_bytes, _stream(stream)))
    cnt, head, blen = (int(v) for v in summary.cpu().tolist())
    return {"next": nxt, "length": length, "count": cnt, "best": best[:blen].cpu().tolist()}


def recheck(T: torch.Tensor, m: int, P: torch.Tensor, I: torch.Tensor, k_motifs: int, k_discords: int,
            stream=None):
    """FP64 recheck of the best motif pairs and discords of a profile.
    Returns (idx int64[2*k_motifs + k_discords], dist float64[k_motifs + k_discords])."""
    T = _series(T, "T")
    L = lib()
    dt = _dtype_code(T)
    n = T.numel()
    out_idx = torch.empty(2 * k_motifs + k_discords, dtype=torch.int64, device=T.device)
    out_dist = torch.empty(k_motifs + k_discords, dtype=torch.float64, device=T.device)
    ws_bytes = L.mp_recheck_workspace(n, m)
    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=T.device)
    _check("mp_recheck", L.mp_recheck(_ptr(T), n, m, dt, _ptr(P.contiguous()), _ptr(I.contiguous()),
                                      k_motifs, k_discords, _ptr(out_idx), _ptr(out_dist), _ptr(ws),
                                      ws.numel(), _stream(stream)))
    return out_idx, out_dist


def timing_enable(on: bool = True):
    """Record HIP events around the sweep kernel and the whole launch
    sequence of every join call (benchmark use)."""
    _check("mp_timing_enable", lib().mp_timing_enable(1 if on else 0))


def timing_query():
    """(sweep_ms, total_ms, calls) summed over the calls since the last query."""
    a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check("mp_timing_query", lib().mp_timing_query(ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)))
    return a.value, b.value, n.value


def selfjoin_cells(n: int, m: int, ez: int) -> int:
    return int(lib().mp_selfjoin_cells(n, m, ez))


def abjoin_cells(nA: int, nB: int, m: int) -> int:
    return int(lib().mp_abjoin_cells(nA, nB, m))
