"""Python binding of libfge (include/fge.h): argument marshalling only.

Every step of the estimation runs in the HIP kernels of ``libfge.so``; this module checks tensor
shapes and dtypes, takes device pointers and the current torch stream, and calls the C ABI.  It
raises :class:`FgeError` if the library is missing or a call fails -- there is no fallback.

Images are planar torch tensors on the GPU: ``I`` is (3, H, W), ``alpha`` is (H, W), both
float32 or float16 (the storage type); ``F`` and ``B`` come back as (3, H, W) of the same type.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfge.so")

FGE_OK, FGE_EINVAL, FGE_ENOMEM, FGE_EHIP, FGE_EUNSUPPORTED, FGE_EWORKSPACE = 0, -1, -2, -3, -4, -5
F32, F16 = 0, 1
REDBLACK = 0
KERNEL_AUTO, KERNEL_FUSED, KERNEL_NAIVE = 0, 1, 2
MAX_LEVELS = 16


class FgeError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _lib().fge_status_string(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{what}: {msg}" if what else msg)


class Params(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_uint32),
        ("omega", ctypes.c_float),
        ("eps_r", ctypes.c_float),
        ("small_size", ctypes.c_int32),
        ("iters_small", ctypes.c_int32),
        ("iters_big", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("strip_rows", ctypes.c_int32),
        ("coarse_max_px", ctypes.c_int32),
        ("tile_max_px", ctypes.c_int32),
    ]


_LIB = None


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"libfge.so not found at {LIB_PATH}: build it with "
            "`python -m paper_2006_14970_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    pp = ctypes.POINTER(Params)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.fge_default_params.argtypes = [pp]
    lib.fge_default_params.restype = None
    lib.fge_status_string.argtypes = [ctypes.c_int]
    lib.fge_status_string.restype = ctypes.c_char_p
    lib.fge_version.argtypes = []
    lib.fge_version.restype = i32
    lib.fge_num_levels.argtypes = [i32, i32]
    lib.fge_num_levels.restype = i32
    lib.fge_level_size.argtypes = [i32, i32, i32]
    lib.fge_level_size.restype = i32
    lib.fge_plan.argtypes = [i32, i32, pp, i32, ip, ip, ip, ip, ip]
    lib.fge_plan.restype = ctypes.c_int
    lib.fge_workspace_bytes.argtypes = [i32, i32, pp]
    lib.fge_workspace_bytes.restype = sz
    lib.fge_estimate_foreground.argtypes = [vp, vp, i32, i32, pp, vp, vp, vp, sz, vp]
    lib.fge_estimate_foreground.restype = ctypes.c_int
    lib.fge_profile_start.argtypes = [i32]
    lib.fge_profile_start.restype = ctypes.c_int
    lib.fge_profile_stop.argtypes = [ctypes.POINTER(ctypes.c_double), ip, i32]
    lib.fge_profile_stop.restype = ctypes.c_int
    _LIB = lib
    return lib


def load():
    """Load libfge.so (raises if it is missing)."""
    return _lib()


def _check(status: int, what: str):
    if status != FGE_OK:
        raise FgeError(status, what)


def default_params(**overrides) -> Params:
    """The paper's defaults (omega 0.1, eps_r 5e-3, 32 / 10 / 2) with optional overrides,
    e.g. ``default_params(storage=F16)``."""
    p = Params()
    _lib().fge_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def num_levels(W: int, H: int) -> int:
    return _lib().fge_num_levels(W, H)


def level_size(full: int, level: int, n_levels: int) -> int:
    return _lib().fge_level_size(full, level, n_levels)


@dataclass
class PlanInfo:
    levels: list          # [(w, h, iters)] for l = 1..n
    n_coarse: int         # leading levels run by the LDS-resident coarse kernel


def plan(W: int, H: int, params: Params | None = None) -> PlanInfo:
    arr = ctypes.c_int32 * MAX_LEVELS
    w, h, it = arr(), arr(), arr()
    n, nc = ctypes.c_int32(), ctypes.c_int32()
    st = _lib().fge_plan(W, H, ctypes.byref(params) if params else None, MAX_LEVELS, w, h, it,
                         ctypes.byref(n), ctypes.byref(nc))
    _check(st, "fge_plan")
    return PlanInfo([(w[i], h[i], it[i]) for i in range(n.value)], nc.value)


def workspace_bytes(W: int, H: int, params: Params | None = None) -> int:
    return _lib().fge_workspace_bytes(W, H, ctypes.byref(params) if params else None)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def storage_dtype(params: Params):
    import torch
    return torch.float16 if params.storage == F16 else torch.float32


def estimate_foreground(I, alpha, params: Params | None = None, F=None, B=None, workspace=None,
                        stream=None):
    """Algorithm 1 on the GPU.  Returns (F, B); the work is enqueued on `stream` (default: the
    current torch stream) and the call does not synchronise."""
    import torch
    p = params if params is not None else default_params()
    dt = storage_dtype(p)
    if I.dim() != 3 or I.shape[0] != 3:
        raise ValueError("I must be (3, H, W)")
    _, H, W = I.shape
    if tuple(alpha.shape) != (H, W):
        raise ValueError("alpha must be (H, W) matching I")
    for name, t in (("I", I), ("alpha", alpha)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor of dtype {dt}")
    if F is None:
        F = torch.empty((3, H, W), dtype=dt, device=I.device)
    if B is None:
        B = torch.empty((3, H, W), dtype=dt, device=I.device)
    for name, t in (("F", F), ("B", B)):
        if tuple(t.shape) != (3, H, W) or t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{name} must be a contiguous (3, H, W) CUDA tensor of dtype {dt}")
    need = workspace_bytes(W, H, p)
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=I.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else None
    ws_len = workspace.numel() * workspace.element_size() if workspace is not None else 0
    st = _lib().fge_estimate_foreground(I.data_ptr(), alpha.data_ptr(), W, H, ctypes.byref(p),
                                        F.data_ptr(), B.data_ptr(), ws_ptr, ws_len,
                                        _stream_ptr(stream))
    _check(st, "fge_estimate_foreground")
    return F, B


def profile_start(capacity: int = 4096):
    """Record HIP events around every kernel launch of the following calls."""
    _check(_lib().fge_profile_start(capacity), "fge_profile_start")


def profile_stop(max_levels: int = MAX_LEVELS):
    """Stop recording; returns (ms_per_level, launches_per_level), level 0 = finest."""
    ms = (ctypes.c_double * max_levels)()
    cnt = (ctypes.c_int32 * max_levels)()
    _check(_lib().fge_profile_stop(ms, cnt, max_levels), "fge_profile_stop")
    return list(ms), list(cnt)
