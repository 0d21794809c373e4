"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/mp.h declares, and rejects bad arguments before it
touches a device."""

import ctypes
import os
import re

import pytest

from paper_1904_12626_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mp_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert sorted(B.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.mp_abi_version() == 1


def test_strerror():
    lib = B.lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.mp_strerror(s)
    assert b"scratch" in lib.mp_strerror(B.MP_ETOOLARGE)


def test_cell_counts():
    # self-join: (l-ez-1)(l-ez)/2 admissible pairs; AB-join: lA*lB
    assert B.selfjoin_cells(4096, 64, 16) == 8066136
    assert B.selfjoin_cells(1 << 20, 256, 64) == 549420844896
    assert B.abjoin_cells(1 << 19, 1 << 19, 128) == 274744753921
    assert B.selfjoin_cells(64, 64, 0) == 0


def test_cell_counts_by_enumeration():
    """The library's pair counts (self-join, AB-join, batch plans) equal a
    direct enumeration of the admissible pairs on small random shapes."""
    import numpy as np
    rng = np.random.default_rng(11)
    lib = B.lib()
    for _ in range(60):
        m = int(rng.integers(2, 20))
        n = int(rng.integers(m, m + 80))
        ez = int(rng.integers(0, 30))
        l = n - m + 1
        i, j = np.triu_indices(l, 1)
        assert B.selfjoin_cells(n, m, ez) == int(np.count_nonzero(j - i > ez)), (n, m, ez)
        nB = int(rng.integers(m, m + 60))
        assert B.abjoin_cells(n, nB, m) == l * (nB - m + 1)
    lengths, windows, zones = [50, 120, 33, 7, 90], [8, 16, 4, 7, 30], [2, 4, 1, 0, 40]
    want = 0
    for n, m, ez in zip(lengths, windows, zones):
        l = n - m + 1
        i, j = np.triu_indices(l, 1)
        want += int(np.count_nonzero(j - i > ez))
    h = ctypes.c_void_p()
    off = (ctypes.c_int64 * (len(lengths) + 1))(*np.concatenate([[0], np.cumsum(lengths)]).tolist())
    m_arr = (ctypes.c_int32 * len(lengths))(*windows)
    z_arr = (ctypes.c_int32 * len(lengths))(*zones)
    assert lib.mp_batch_plan_create(len(lengths), off, m_arr, z_arr, B.MP_F32, None, ctypes.byref(h)) == 0
    assert lib.mp_batch_plan_cells(h) == want
    lib.mp_batch_plan_destroy(h)


def test_workspace_queries():
    lib = B.lib()
    opt = B.make_options("f32")
    assert lib.mp_selfjoin_workspace(4096, 64, B.MP_F32, ctypes.byref(opt)) > 0
    assert lib.mp_selfjoin_workspace(10, 64, B.MP_F32, ctypes.byref(opt)) == 0   # n < m
    assert lib.mp_selfjoin_workspace(4096, 1, B.MP_F32, ctypes.byref(opt)) == 0  # m < 2
    opt16 = B.make_options("f64", tile_slots=16)
    assert lib.mp_selfjoin_workspace(4096, 64, B.MP_F64, ctypes.byref(opt16)) == 0
    opt12 = B.make_options("f32", tile_slots=12)
    assert lib.mp_selfjoin_workspace(4096, 64, B.MP_F32, ctypes.byref(opt12)) > 0
    assert lib.mp_abjoin_workspace(1000, 900, 32, B.MP_F64, None) > 0
    assert lib.mp_recheck_workspace(1000, 32) >= 969


@pytest.mark.parametrize("args,expect", [
    (dict(n=100, m=1, ez=0), B.MP_EINVAL),
    (dict(n=10, m=20, ez=0), B.MP_EINVAL),
    (dict(n=100, m=10, ez=-1), B.MP_EINVAL),
])
def test_selfjoin_rejects_bad_sizes(args, expect):
    lib = B.lib()
    fake = ctypes.c_void_p(1 << 20)
    st = lib.mp_selfjoin(fake, args["n"], args["m"], args["ez"], B.MP_F32, None, fake, fake, fake,
                         1 << 30, None)
    assert st == expect


def test_selfjoin_rejects_null_and_misaligned():
    lib = B.lib()
    ok = ctypes.c_void_p(1 << 20)
    assert lib.mp_selfjoin(None, 100, 10, 2, B.MP_F32, None, ok, ok, ok, 1 << 30, None) == B.MP_EINVAL
    odd = ctypes.c_void_p((1 << 20) + 2)
    assert lib.mp_selfjoin(odd, 100, 10, 2, B.MP_F32, None, ok, ok, ok, 1 << 30, None) == B.MP_EINVAL
    # workspace: null, misaligned, too small
    assert lib.mp_selfjoin(ok, 100, 10, 2, B.MP_F32, None, ok, ok, None, 1 << 30, None) == B.MP_EWORKSPACE
    assert lib.mp_selfjoin(ok, 100, 10, 2, B.MP_F32, None, ok, ok, ctypes.c_void_p((1 << 20) + 64), 1 << 30,
                           None) == B.MP_EWORKSPACE
    assert lib.mp_selfjoin(ok, 100, 10, 2, B.MP_F32, None, ok, ok, ok, 16, None) == B.MP_EWORKSPACE


def test_bad_options():
    lib = B.lib()
    ok = ctypes.c_void_p(1 << 20)
    for opt in (B.mp_options(7, 0, 0, 1), B.mp_options(1, 100, 0, 1), B.mp_options(1, 0, 10, 1),
                B.mp_options(1, 0, 0, 8)):
        assert lib.mp_selfjoin(ok, 1000, 10, 2, B.MP_F32, ctypes.byref(opt), ok, ok, ok, 1 << 30,
                               None) == B.MP_EINVAL
    opt = B.mp_options(0, 0, 16, 1)
    assert lib.mp_selfjoin(ok, 1000, 10, 2, B.MP_F64, ctypes.byref(opt), ok, ok, ok, 1 << 30,
                           None) == B.MP_EUNSUPPORTED


def test_option_flags():
    """Known flags (FP64 finalize, flat loads) are accepted, any other bit is
    refused before anything is enqueued."""
    lib = B.lib()
    for flags in (0, B.MP_FLAG_FP64_FINALIZE, B.MP_FLAG_FLAT_LOADS,
                  B.MP_FLAG_FP64_FINALIZE | B.MP_FLAG_FLAT_LOADS):
        opt = B.mp_options(1, 0, 0, flags)
        assert lib.mp_selfjoin_workspace(1000, 10, B.MP_F32, ctypes.byref(opt)) > 0
    off = (ctypes.c_int64 * 3)(0, 100, 350)
    m = (ctypes.c_int32 * 2)(8, 16)
    ez = (ctypes.c_int32 * 2)(2, 4)
    h = ctypes.c_void_p()
    opt = B.mp_options(1, 0, 0, B.MP_FLAG_FLAT_LOADS)
    assert lib.mp_batch_plan_create(2, off, m, ez, B.MP_F32, ctypes.byref(opt), ctypes.byref(h)) == 0
    lib.mp_batch_plan_destroy(h)
    for bad in (4, 8, 1 << 30):
        opt = B.mp_options(1, 0, 0, bad)
        assert lib.mp_selfjoin_workspace(1000, 10, B.MP_F32, ctypes.byref(opt)) == 0
        assert lib.mp_batch_plan_create(2, off, m, ez, B.MP_F32, ctypes.byref(opt), ctypes.byref(h)) == B.MP_EINVAL


def test_batch_plan_host_side():
    lib = B.lib()
    off = (ctypes.c_int64 * 4)(0, 100, 350, 1000)
    m = (ctypes.c_int32 * 3)(8, 16, 32)
    ez = (ctypes.c_int32 * 3)(2, 4, 8)
    h = ctypes.c_void_p()
    assert lib.mp_batch_plan_create(3, off, m, ez, B.MP_F32, None, ctypes.byref(h)) == 0
    assert lib.mp_batch_plan_profile_length(h) == (100 - 7) + (250 - 15) + (650 - 31)
    cells = sum(B.selfjoin_cells(n, mm, e) for n, mm, e in ((100, 8, 2), (250, 16, 4), (650, 32, 8)))
    assert lib.mp_batch_plan_cells(h) == cells
    assert lib.mp_batch_plan_workspace(h) > 0
    lib.mp_batch_plan_destroy(h)
    bad = (ctypes.c_int64 * 4)(0, 100, 90, 1000)   # a series shorter than its window
    assert lib.mp_batch_plan_create(3, bad, m, ez, B.MP_F32, None, ctypes.byref(h)) == B.MP_EINVAL


def test_exclusion_zone_rule():
    from fractions import Fraction
    assert B.exclusion_zone(80, Fraction(1, 2)) == 40
    assert B.exclusion_zone(50, Fraction(1, 4)) == 13
    assert B.exclusion_zone(64, 0.25) == 16


def test_selfjoin_chunks_and_restricted_plans():
    lib = B.lib()
    opt = B.make_options("f32", tile_slots=8)
    w = ctypes.c_int64()
    # l = 4033, offsets 17 .. 4032 -> 4016 offsets in chunks of 512
    assert lib.mp_selfjoin_chunks(4096, 64, 16, ctypes.byref(opt), ctypes.byref(w)) == 8
    assert w.value == 512
    assert lib.mp_selfjoin_chunks(100, 64, 40, None, None) == 0      # l = 37 <= ez + 1
    assert lib.mp_selfjoin_chunks(10, 64, 4, None, None) == -1
    h = ctypes.c_void_p()
    ch = (ctypes.c_int64 * 3)(5, 0, 7)
    assert lib.mp_selfjoin_plan_create(4096, 64, 16, B.MP_F32, ctypes.byref(opt), 0, 3, ch, ctypes.byref(h)) == 0
    assert lib.mp_batch_plan_profile_length(h) == 4033
    lib.mp_batch_plan_destroy(h)
    assert lib.mp_selfjoin_plan_create(4096, 64, 16, B.MP_F32, ctypes.byref(opt), 1, 0, None, ctypes.byref(h)) == 0
    assert lib.mp_batch_plan_profile_length(h) == 3 * 4033
    assert lib.mp_batch_plan_cells(h) == B.selfjoin_cells(4096, 64, 16)
    lib.mp_batch_plan_destroy(h)
    for bad in ((8,), (2, 2), (-1,)):
        arr = (ctypes.c_int64 * len(bad))(*bad)
        assert lib.mp_selfjoin_plan_create(4096, 64, 16, B.MP_F32, ctypes.byref(opt), 0, len(bad), arr,
                                           ctypes.byref(h)) == B.MP_EINVAL
    assert lib.mp_selfjoin_plan_create(4096, 64, 16, B.MP_F32, None, 2, 0, None, ctypes.byref(h)) == B.MP_EINVAL


def test_restricted_plan_cells_are_the_chunk_cells():
    """Cells of a chunk plan = admissible pairs whose offset is in the chunks."""
    lib = B.lib()
    opt = B.make_options("f32", tile_slots=8)
    n, m, ez, W = 4096, 64, 16, 512
    l = n - m + 1
    chunks = [1, 6, 3]
    arr = (ctypes.c_int64 * 3)(*chunks)
    h = ctypes.c_void_p()
    assert lib.mp_selfjoin_plan_create(n, m, ez, B.MP_F32, ctypes.byref(opt), 0, 3, arr, ctypes.byref(h)) == 0
    want = sum(l - k for c in chunks for k in range(ez + 1 + c * W, min(ez + (c + 1) * W, l - 1) + 1))
    assert lib.mp_batch_plan_cells(h) == want
    lib.mp_batch_plan_destroy(h)


def test_anytime_order_is_a_seeded_permutation():
    a = B.anytime_order(1000, 7)
    assert sorted(a) == list(range(1000))
    assert a == B.anytime_order(1000, 7)
    assert a != B.anytime_order(1000, 8)
    assert B.anytime_order(0, 1) == []


def test_new_entry_points_reject_bad_arguments():
    lib = B.lib()
    ok = ctypes.c_void_p(1 << 20)
    # multidimensional joins: D out of range, window too long, AB form of the k-dim profiles
    assert lib.mp_mdjoin_workspace(B.MP_MD_SIMPLE, 9, 1000, 0, 16) == 0
    assert lib.mp_mdjoin_workspace(B.MP_MD_SIMPLE, 0, 1000, 0, 16) == 0
    assert lib.mp_mdjoin_workspace(B.MP_MD_SIMPLE, 3, 10, 0, 16) == 0
    assert lib.mp_mdjoin_workspace(B.MP_MD_MULTI, 3, 1000, 0, 16) > 0
    assert lib.mp_mdjoin(B.MP_MD_MULTI, 3, ok, 1000, ctypes.c_void_p((1 << 20) + 4096), 1000, 16, 4, B.MP_F32,
                         ok, ok, ok, ok, ok, 1 << 30, None) == B.MP_EUNSUPPORTED
    assert lib.mp_mdjoin(7, 3, ok, 1000, None, 0, 16, 4, B.MP_F32, ok, ok, None, None, ok, 1 << 30,
                         None) == B.MP_EINVAL
    assert lib.mp_mdjoin_cells(3, 4096, 0, 64, 16) == B.selfjoin_cells(4096, 64, 16)
    assert lib.mp_mdjoin_cells(2, 1000, 900, 32, 0) == B.abjoin_cells(1000, 900, 32)
    # segmentation and chains
    assert lib.mp_fluss(ok, 1000, 10, 65, ok, ok, ok, 1 << 30, None) == B.MP_EINVAL
    assert lib.mp_fluss(ok, 1000, -1, 2, ok, ok, ok, 1 << 30, None) == B.MP_EINVAL
    assert lib.mp_fluss(ok, 1000, 10, 2, ok, None, ok, 1 << 30, None) == B.MP_EINVAL
    assert lib.mp_fluss(ok, 1000, 10, 2, ok, ok, ok, 8, None) == B.MP_EWORKSPACE
    assert lib.mp_chains(ok, ok, 1000, 0, ok, ok, ok, ok, ok, 1 << 30, None) == B.MP_EINVAL
    assert lib.mp_chains(ok, None, 1000, 3, ok, ok, ok, ok, ok, 1 << 30, None) == B.MP_EINVAL
    # streaming: capacity, order of sizes, workspace
    assert lib.mp_stream_workspace(100, 200) == 0
    assert lib.mp_stream_workspace(5000, 64) > 0
    assert lib.mp_stream_init(ok, 6000, 5000, 64, 16, B.MP_F32, ok, ok, ok, 1 << 30, None) == B.MP_EINVAL
    assert lib.mp_stream_append(ok, 3000, 2000, 5000, 64, 16, B.MP_F32, ok, ok, ok, 1 << 30, None) == B.MP_EINVAL
    assert lib.mp_stream_append(ok, 3000, 6000, 5000, 64, 16, B.MP_F32, ok, ok, ok, 1 << 30, None) == B.MP_EINVAL
    assert lib.mp_stream_append(ok, 3000, 3100, 5000, 64, 16, B.MP_F32, ok, ok, ok, 64, None) == B.MP_EWORKSPACE
    # plans: AB plan sizes, left/right plans refuse the backward
    h = ctypes.c_void_p()
    assert lib.mp_abjoin_plan_create(1000, 900, 32, B.MP_F32, None, ctypes.byref(h)) == 0
    assert lib.mp_batch_plan_profile_length(h) == (1000 - 31) + (900 - 31)
    assert lib.mp_batch_plan_cells(h) == B.abjoin_cells(1000, 900, 32)
    lib.mp_batch_plan_destroy(h)
    assert lib.mp_abjoin_plan_create(10, 900, 32, B.MP_F32, None, ctypes.byref(h)) == B.MP_EINVAL
    assert lib.mp_selfjoin_plan_create(4096, 64, 16, B.MP_F32, None, 1, 0, None, ctypes.byref(h)) == 0
    assert lib.mp_backward(h, ok, ok, ok, ok, ok, 1 << 40, None) == B.MP_EUNSUPPORTED
    lib.mp_batch_plan_destroy(h)
    # the backward's window limit (2^30 samples), checked before any device call
    m = (1 << 30) + 1
    assert lib.mp_selfjoin_plan_create(m + 9, m, 0, B.MP_F32, None, 0, 0, None, ctypes.byref(h)) == 0
    assert lib.mp_backward(h, ok, ok, ok, ok, ok, 1 << 40, None) == B.MP_EUNSUPPORTED
    assert lib.mp_backward_after_forward(h, ok, ok, ok, ok, ok, ok, 1 << 40, None) == B.MP_EUNSUPPORTED
    lib.mp_batch_plan_destroy(h)


def test_noalloc_selfjoin_host_checks():
    """mp_selfjoin_noalloc checks sizes, pointers and its scratch limit on
    the host, before any device call."""
    lib = B.lib()
    ok = ctypes.c_void_p(1 << 20)
    opt = B.make_options("f32")
    # the FP32 workspace of n = 2^20, m = 256 fits the fixed scratch, 2^21 does not
    assert lib.mp_selfjoin_workspace(1 << 20, 256, B.MP_F32, ctypes.byref(opt)) <= B.MP_NOALLOC_SCRATCH_BYTES
    assert lib.mp_selfjoin_workspace(1 << 21, 256, B.MP_F32, ctypes.byref(opt)) > B.MP_NOALLOC_SCRATCH_BYTES
    assert lib.mp_selfjoin_noalloc(ok, 1 << 21, 256, 64, B.MP_F32, ctypes.byref(opt), ok, ok,
                                   None) == B.MP_ETOOLARGE
    assert lib.mp_selfjoin_noalloc(ok, 100, 1, 0, B.MP_F32, None, ok, ok, None) == B.MP_EINVAL
    assert lib.mp_selfjoin_noalloc(None, 100, 10, 2, B.MP_F32, None, ok, ok, None) == B.MP_EINVAL
    assert lib.mp_selfjoin_noalloc(ok, 100, 10, 2, B.MP_F32, None, ctypes.c_void_p((1 << 20) + 2), ok,
                                   None) == B.MP_EINVAL
