"""The self-join entry point that allocates nothing (mp_selfjoin_noalloc):
called through the C ABI, it must give bitwise the P and I of mp_selfjoin
(same kernels, its workspace being the library's fixed per-device scratch),
on consecutive calls of different sizes that share that scratch."""

import ctypes

import numpy as np
import pytest
import torch

from paper_1904_12626_amd import _binding as B
from workloads import random_walk

pytestmark = pytest.mark.gpu


def _with_workspace(T, m, ez, opt):
    L = B.lib()
    n = T.numel()
    l = n - m + 1
    dt = B.MP_F64 if T.dtype == torch.float64 else B.MP_F32
    ws_bytes = L.mp_selfjoin_workspace(n, m, dt, ctypes.byref(opt))
    assert 0 < ws_bytes <= B.MP_NOALLOC_SCRATCH_BYTES
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=T.device)
    P = torch.empty(l, dtype=T.dtype, device=T.device)
    I = torch.empty(l, dtype=torch.int64, device=T.device)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.mp_selfjoin(B._ptr(T), n, m, ez, dt, ctypes.byref(opt), B._ptr(P), B._ptr(I), B._ptr(ws),
                         ws_bytes, st) == B.MP_OK
    return P, I


def _no_alloc(T, m, ez, opt):
    L = B.lib()
    n = T.numel()
    l = n - m + 1
    dt = B.MP_F64 if T.dtype == torch.float64 else B.MP_F32
    # outputs start as garbage so that a skipped write would show
    P = torch.full((l,), 12345.0, dtype=T.dtype, device=T.device)
    I = torch.full((l,), -7, dtype=torch.int64, device=T.device)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.mp_selfjoin_noalloc(B._ptr(T), n, m, ez, dt, ctypes.byref(opt), B._ptr(P), B._ptr(I), st) == B.MP_OK
    return P, I


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_noalloc_matches_selfjoin_on_two_calls(precision):
    dev = torch.device("cuda:0")
    opt = B.make_options(precision)
    cases = [(60000, 128, 32, 11), (9000, 64, 16, 12)]   # the second call is smaller
    results = []
    for n, m, ez, seed in cases:
        print(f"noalloc {precision}: n={n} m={m} ez={ez} seed={seed}", flush=True)
        T = torch.from_numpy(random_walk(n, seed, np.float32)).to(dev)
        Pn, In = _no_alloc(T, m, ez, opt)
        torch.cuda.synchronize()
        Pw, Iw = _with_workspace(T, m, ez, opt)
        torch.cuda.synchronize()
        results.append((Pn.cpu(), In.cpu(), Pw.cpu(), Iw.cpu()))
    for (Pn, In, Pw, Iw), (n, m, ez, _) in zip(results, cases):
        assert torch.equal(In, Iw), f"n={n}: indices differ"
        assert torch.equal(Pn, Pw), f"n={n}: profiles differ"
        assert bool(torch.all(In >= 0)) and bool(torch.all(torch.isfinite(Pn)))


def test_noalloc_python_wrapper_and_limit():
    dev = torch.device("cuda:0")
    T = torch.from_numpy(random_walk(5000, 3, np.float64)).to(dev)
    l = 5000 - 32 + 1
    P = torch.empty(l, dtype=torch.float64, device=dev)
    I = torch.empty(l, dtype=torch.int64, device=dev)
    B.selfjoin_noalloc(T, 32, 8, P=P, I=I, precision="f64")
    Pw, Iw = B.selfjoin(T, 32, 8, precision="f64")
    torch.cuda.synchronize()
    assert torch.equal(P, Pw) and torch.equal(I, Iw)
    # a job beyond the fixed scratch is refused before anything is enqueued
    big = torch.empty(1 << 21, dtype=torch.float32, device=dev)
    Pb = torch.empty((1 << 21) - 255, dtype=torch.float32, device=dev)
    Ib = torch.empty((1 << 21) - 255, dtype=torch.int64, device=dev)
    with pytest.raises(B.MPError) as e:
        B.selfjoin_noalloc(big, 256, 64, P=Pb, I=Ib)
    assert e.value.status == B.MP_ETOOLARGE
