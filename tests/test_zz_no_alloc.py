"""GPU: the allocation-free single-image entry point against fge_estimate_foreground.

fge_estimate_foreground_noalloc keeps its workspace in a file-scope device array of the library;
its results must be bit-identical to the workspace-taking call on the same inputs, for two calls
in a row (the second smaller, so it runs on what the first left in the array), in both storage
types.  Both are called through ctypes on the raw C symbols.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2006_14970_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need an MI355X"
    from paper_2006_14970_amd import fge
    fge.load()
    lib = ctypes.CDLL(fge.LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.fge_estimate_foreground_noalloc.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp]
    lib.fge_estimate_foreground_noalloc.restype = ctypes.c_int
    lib.fge_estimate_foreground.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.fge_estimate_foreground.restype = ctypes.c_int
    lib.fge_workspace_bytes.argtypes = [i32, i32, vp]
    lib.fge_workspace_bytes.restype = ctypes.c_size_t
    return torch, fge, lib


def _inputs(torch, fge, p, s):
    dt = fge.storage_dtype(p)
    I = torch.from_numpy(np.ascontiguousarray(s.I)).to(dt).cuda()
    a = torch.from_numpy(np.ascontiguousarray(s.alpha)).to(dt).cuda()
    return I, a


def _with_workspace(torch, lib, p, I, a):
    _, H, W = I.shape
    F = torch.empty_like(I)
    B = torch.empty_like(I)
    need = lib.fge_workspace_bytes(H, W, ctypes.addressof(p))
    ws = torch.empty(max(1, need), dtype=torch.uint8, device="cuda")
    st = lib.fge_estimate_foreground(I.data_ptr(), a.data_ptr(), H, W, ctypes.addressof(p),
                                     F.data_ptr(), B.data_ptr(), ws.data_ptr(), need,
                                     torch.cuda.current_stream().cuda_stream)
    assert st == 0, st
    return F, B


def _noalloc(torch, lib, p, I, a):
    _, H, W = I.shape
    F = torch.full_like(I, 0.25)
    B = torch.full_like(I, 0.75)
    st = lib.fge_estimate_foreground_noalloc(I.data_ptr(), a.data_ptr(), H, W,
                                             ctypes.addressof(p), F.data_ptr(), B.data_ptr(),
                                             torch.cuda.current_stream().cuda_stream)
    assert st == 0, st
    return F, B


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_noalloc_matches_workspace_call_twice(gpu, storage):
    torch, fge, lib = gpu
    p = fge.default_params(storage=fge.F16 if storage == "f16" else fge.F32)
    # a large image first (most of the scratch array in use), then a smaller non-square one
    for W, H, seed in ((1920, 1080, 11), (700, 301, 12)):
        print(f"noalloc {storage} {H}x{W}", flush=True)
        s = synth.smooth(W, H, seed=seed)
        I, a = _inputs(torch, fge, p, s)
        F1, B1 = _noalloc(torch, lib, p, I, a)
        F2, B2 = _with_workspace(torch, lib, p, I, a)
        torch.cuda.synchronize()
        assert torch.equal(F1, F2) and torch.equal(B1, B2), (storage, W, H)
        if W * H <= 1 << 18:
            Fo, Bo = oracle.ml(s.I, s.alpha)
            err = max(float(np.abs(F1.double().cpu().numpy() - Fo).max()),
                      float(np.abs(B1.double().cpu().numpy() - Bo).max()))
            assert err <= (2e-3 if storage == "f16" else 1e-4), err


def test_noalloc_rejects_oversize_and_jacobi(gpu):
    torch, fge, lib = gpu
    p = fge.default_params()
    H, W = 3072, 4096          # float32 workspace of 92.6 MiB, above the 64 MiB array
    assert lib.fge_workspace_bytes(H, W, ctypes.addressof(p)) > 64 << 20
    big = 1 << 36
    assert lib.fge_estimate_foreground_noalloc(big, 2 * big, H, W, ctypes.addressof(p), 3 * big,
                                               4 * big, None) == fge.FGE_EWORKSPACE
    pj = fge.default_params(order=fge.JACOBI)
    assert lib.fge_estimate_foreground_noalloc(big, 2 * big, 64, 64, ctypes.addressof(pj),
                                               3 * big, 4 * big, None) == fge.FGE_EUNSUPPORTED
