"""The no-allocation product efie_zx_flush64_noalloc against efie_zx_flush64,
called through the C ABI: same kernels, so the results must agree bit for bit,
on two calls in a row (the second smaller, on the scratch the first left)."""
import ctypes

import numpy as np
import pytest

import paper_2310_15644_amd as P

from .gpu_common import flush

pytestmark = pytest.mark.gpu


def _call_ws(L, torch, Z, X, Y, n, nrhs, stream):
    nb = ctypes.c_size_t()
    assert L.efie_zx_flush64_workspace_size(n, nrhs, ctypes.byref(nb)) == 0
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=Z.device)
    off = (-ws.data_ptr()) % 256
    rc = L.efie_zx_flush64(ctypes.c_void_p(Z.data_ptr()), n, ctypes.c_void_p(X.data_ptr()),
                           ctypes.c_void_p(Y.data_ptr()), nrhs, ctypes.c_void_p(ws.data_ptr() + off), nb.value, stream)
    assert rc == 0, L.efie_last_error()
    torch.cuda.synchronize()


def _call_noalloc(L, Z, X, Y, n, nrhs, stream):
    rc = L.efie_zx_flush64_noalloc(ctypes.c_void_p(Z.data_ptr()), n, ctypes.c_void_p(X.data_ptr()),
                                   ctypes.c_void_p(Y.data_ptr()), nrhs, stream)
    assert rc == 0, L.efie_last_error()


def test_zx_flush64_noalloc_matches_workspace_call():
    import torch

    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    L = P.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    mx = ctypes.c_int64()
    assert L.efie_zx_flush64_noalloc_max(ctypes.byref(mx)) == 0
    assert mx.value == 64 << 20
    g = torch.Generator(device=dev).manual_seed(7)
    # a first call that fills much of the scratch, then a smaller one (ragged sizes)
    for n, nrhs in ((3001, 160), (517, 37)):
        flush(f"zx_flush64_noalloc n={n} nrhs={nrhs}")
        Z = torch.randn((n, n), dtype=torch.complex64, device=dev, generator=g)
        X = torch.randn((nrhs, n), dtype=torch.complex128, device=dev, generator=g)
        Yw = torch.empty_like(X)
        Yn = torch.full_like(X, float("nan"))
        _call_ws(L, torch, Z, X, Yw, n, nrhs, stream)
        _call_noalloc(L, Z, X, Yn, n, nrhs, stream)
        torch.cuda.synchronize()
        assert torch.equal(Yn, Yw)
        # and the product itself, against the FP64 product of the stored values
        ref = (Z.to(torch.complex128) @ X.T).T
        err = float((Yn - ref).abs().max() / ref.abs().max())
        flush(f"  bit-identical to efie_zx_flush64; rel err vs FP64 {err:.2e}")
        assert err <= 1e-5
    # sizes beyond the scratch are rejected on the host before any device work
    # (4096 x 2049 x 8 bytes > 64 MiB; the buffers passed are never touched)
    rc = L.efie_zx_flush64_noalloc(ctypes.c_void_p(Z.data_ptr()), 4096, ctypes.c_void_p(X.data_ptr()),
                                   ctypes.c_void_p(Yn.data_ptr()), 2049, stream)
    assert rc == -1 and b"exceed" in L.efie_last_error()
