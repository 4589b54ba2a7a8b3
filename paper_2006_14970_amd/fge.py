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
FGE_EBUDGET, FGE_ECANCELED = -6, -7
F32, F16, U8, F64 = 0, 1, 2, 3
REDBLACK, JACOBI = 0, 1
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


class LevelOptions(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_uint32),
        ("resize", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("max_sweeps", ctypes.c_int32),
        ("passes", ctypes.c_int32),
    ]


RESIZE_NEAREST, RESIZE_SMOOTH = 0, 1


class CfParams(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_uint32),
        ("storage", ctypes.c_int32),
        ("omega", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("warm_start", ctypes.c_int32),
    ]


class CfInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("channel_iterations", ctypes.c_int32 * 3),
        ("breakdown", ctypes.c_int32),
        ("rel_residual", ctypes.c_double * 3),
        ("recursive_rel_residual", ctypes.c_double * 3),
        ("device_ms", ctypes.c_double),
    ]


class TuneEntry(ctypes.Structure):
    _fields_ = [
        ("strip_rows", ctypes.c_int32),
        ("tile_max_px", ctypes.c_int32),
        ("ms", ctypes.c_float),
        ("status", ctypes.c_int32),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_uint32),
        ("max_active", ctypes.c_int32),
        ("pipeline_depth", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("budget_bytes", ctypes.c_uint64),
        ("tick_table_bytes", ctypes.c_uint64),
    ]


class ServerResult(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("ticks", ctypes.c_int32),
        ("submit_ms", ctypes.c_double),
        ("admit_ms", ctypes.c_double),
        ("ready_ms", ctypes.c_double),
        ("latency_ms", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("ticks", ctypes.c_int64),
        ("launches", ctypes.c_int64),
        ("mixed_ticks", ctypes.c_int64),
        ("admitted_while_busy", ctypes.c_int64),
        ("peak_active", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("peak_charged_bytes", ctypes.c_uint64),
        ("peak_arena_bytes", ctypes.c_uint64),
        ("mean_active", ctypes.c_double),
        ("failed", ctypes.c_int64),
        ("cancelled", ctypes.c_int64),
    ]


class ServerSim(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_uint32),
        ("manual", ctypes.c_int32),
        ("us_per_launch", ctypes.c_double),
        ("us_per_mpx", ctypes.c_double),
        ("fail_launch_tick", ctypes.c_int32),
        ("fail_device_tick", ctypes.c_int32),
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
    # libfge needs libamdhip64.so.7, the soname of PyTorch's bundled HIP runtime too: loading
    # torch first makes the library bind to that same runtime, so the streams and device memory
    # the binding passes in belong to the runtime that executes the calls.  (Loaded the other way
    # round, the process would end up with the system runtime under torch.)
    import torch  # noqa: F401
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
    bp = ctypes.c_void_p
    vpp = ctypes.POINTER(ctypes.c_void_p)
    lib.fge_batch_create.argtypes = [i32, ip, ip, pp, ctypes.POINTER(ctypes.c_void_p)]
    lib.fge_batch_create.restype = ctypes.c_int
    lib.fge_batch_destroy.argtypes = [bp]
    lib.fge_batch_destroy.restype = None
    lib.fge_batch_workspace_bytes.argtypes = [bp]
    lib.fge_batch_workspace_bytes.restype = sz
    lib.fge_batch_steps.argtypes = [bp]
    lib.fge_batch_steps.restype = i32
    lib.fge_batch_launch_count.argtypes = [bp]
    lib.fge_batch_launch_count.restype = i32
    for name in ("fge_batch_run", "fge_batch_capture"):
        f = getattr(lib, name)
        f.argtypes = [bp, vpp, vpp, vpp, vpp, vp, sz, vp]
        f.restype = ctypes.c_int
    lib.fge_batch_replay.argtypes = [bp, vp]
    lib.fge_batch_replay.restype = ctypes.c_int
    lib.fge_batch_workspace_bytes_for.argtypes = [i32, ip, ip, pp]
    lib.fge_batch_workspace_bytes_for.restype = sz
    lib.fge_estimate_foreground_batch.argtypes = [i32, vpp, vpp, ip, ip, pp, vpp, vpp, vp, sz, vp]
    lib.fge_estimate_foreground_batch.restype = ctypes.c_int
    lib.fge_profile_start.argtypes = [i32]
    lib.fge_profile_start.restype = ctypes.c_int
    lib.fge_profile_stop.argtypes = [ctypes.POINTER(ctypes.c_double), ip, i32]
    lib.fge_profile_stop.restype = ctypes.c_int
    lib.fge_energy_workspace_bytes.argtypes = [i32, i32]
    lib.fge_energy_workspace_bytes.restype = sz
    lib.fge_energy.argtypes = [vp, vp, vp, vp, i32, i32, pp, vp, vp, sz, vp]
    lib.fge_energy.restype = ctypes.c_int
    lib.fge_quality_workspace_bytes.argtypes = [i32, i32]
    lib.fge_quality_workspace_bytes.restype = sz
    lib.fge_quality.argtypes = [vp, vp, vp, i32, i32, i32, ctypes.c_double, vp, vp, sz, vp]
    lib.fge_quality.restype = ctypes.c_int
    lib.fge_composite.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp]
    lib.fge_composite.restype = ctypes.c_int
    lib.fge_hwc_to_planar.argtypes = [vp, i32, i32, i32, i32, vp, vp, i32, vp]
    lib.fge_hwc_to_planar.restype = ctypes.c_int
    lib.fge_planar_to_hwc.argtypes = [vp, i32, i32, i32, vp, i32, vp]
    lib.fge_planar_to_hwc.restype = ctypes.c_int
    lib.fge_converge_workspace_bytes.argtypes = [i32, i32, pp]
    lib.fge_converge_workspace_bytes.restype = sz
    lib.fge_estimate_foreground_converge.argtypes = [vp, vp, i32, i32, pp, ctypes.c_double, i32,
                                                     vp, vp, vp, vp, sz, vp]
    lib.fge_estimate_foreground_converge.restype = ctypes.c_int
    lib.fge_converge_passes_workspace_bytes.argtypes = [i32, i32, pp]
    lib.fge_converge_passes_workspace_bytes.restype = sz
    lib.fge_estimate_foreground_converge_passes.argtypes = [vp, vp, i32, i32, pp, ctypes.c_double,
                                                            i32, vp, vp, ip, vp, sz, vp]
    lib.fge_estimate_foreground_converge_passes.restype = ctypes.c_int
    op = ctypes.POINTER(LevelOptions)
    lib.fge_levels_workspace_bytes.argtypes = [i32, i32, pp, op]
    lib.fge_levels_workspace_bytes.restype = sz
    lib.fge_estimate_foreground_levels.argtypes = [vp, vp, i32, i32, pp, op, vp, vp, vp, vp, sz, vp]
    lib.fge_estimate_foreground_levels.restype = ctypes.c_int
    cfp = ctypes.POINTER(CfParams)
    lib.fge_cf_default_params.argtypes = [cfp]
    lib.fge_cf_default_params.restype = None
    lib.fge_cf_workspace_bytes.argtypes = [i32, i32]
    lib.fge_cf_workspace_bytes.restype = sz
    lib.fge_closed_form.argtypes = [vp, vp, i32, i32, cfp, vp, vp, vp, sz, vp,
                                    ctypes.POINTER(CfInfo)]
    lib.fge_closed_form.restype = ctypes.c_int
    tp = ctypes.POINTER(TuneEntry)
    lib.fge_tune_candidates.argtypes = []
    lib.fge_tune_candidates.restype = i32
    lib.fge_tune_workspace_bytes.argtypes = [i32, i32, pp]
    lib.fge_tune_workspace_bytes.restype = sz
    lib.fge_autotune.argtypes = [vp, vp, i32, i32, pp, vp, vp, vp, sz, vp, i32, pp, tp, i32, ip]
    lib.fge_autotune.restype = ctypes.c_int
    lib.fge_batch_tune_workspace_bytes.argtypes = [i32, ip, ip, pp]
    lib.fge_batch_tune_workspace_bytes.restype = sz
    lib.fge_batch_autotune.argtypes = [i32, vpp, vpp, ip, ip, pp, vpp, vpp, vp, sz, vp, i32, pp,
                                       tp, i32, ip]
    lib.fge_batch_autotune.restype = ctypes.c_int
    cp = ctypes.POINTER(ServerConfig)
    lib.fge_server_default_config.argtypes = [cp]
    lib.fge_server_default_config.restype = None
    lib.fge_server_request_bytes.argtypes = [i32, i32, pp]
    lib.fge_server_request_bytes.restype = sz
    lib.fge_server_reserved_bytes.argtypes = [cp]
    lib.fge_server_reserved_bytes.restype = sz
    lib.fge_server_create.argtypes = [pp, cp, vp, sz, vp, ctypes.POINTER(ctypes.c_void_p)]
    lib.fge_server_create.restype = ctypes.c_int
    lib.fge_server_submit.argtypes = [vp, ctypes.c_int64, vp, vp, i32, i32, vp, vp]
    lib.fge_server_submit.restype = ctypes.c_int
    lib.fge_server_poll.argtypes = [vp, ctypes.POINTER(ServerResult), i32]
    lib.fge_server_poll.restype = i32
    lib.fge_server_drain.argtypes = [vp]
    lib.fge_server_drain.restype = ctypes.c_int
    lib.fge_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.fge_server_get_stats.restype = ctypes.c_int
    lib.fge_server_destroy.argtypes = [vp]
    lib.fge_server_destroy.restype = None
    lib.fge_server_cancel.argtypes = [vp, ctypes.c_int64]
    lib.fge_server_cancel.restype = ctypes.c_int
    simp = ctypes.POINTER(ServerSim)
    lib.fge_server_sim_default.argtypes = [simp]
    lib.fge_server_sim_default.restype = None
    lib.fge_server_create_simulated.argtypes = [pp, cp, sz, simp, ctypes.POINTER(ctypes.c_void_p)]
    lib.fge_server_create_simulated.restype = ctypes.c_int
    lib.fge_server_sim_step.argtypes = [vp, i32, ctypes.c_double]
    lib.fge_server_sim_step.restype = i32
    lib.fge_server_sim_inflight.argtypes = [vp]
    lib.fge_server_sim_inflight.restype = i32
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


def num_levels(H: int, W: int) -> int:
    return _lib().fge_num_levels(H, W)


def level_size(full: int, level: int, n_levels: int) -> int:
    return _lib().fge_level_size(full, level, n_levels)


@dataclass
class PlanInfo:
    levels: list          # [(w, h, iters)] for l = 1..n
    n_coarse: int         # leading levels run by the LDS-resident coarse kernel


def plan(H: int, W: int, params: Params | None = None) -> PlanInfo:
    arr = ctypes.c_int32 * MAX_LEVELS
    w, h, it = arr(), arr(), arr()
    n, nc = ctypes.c_int32(), ctypes.c_int32()
    st = _lib().fge_plan(H, W, ctypes.byref(params) if params else None, MAX_LEVELS, w, h, it,
                         ctypes.byref(n), ctypes.byref(nc))
    _check(st, "fge_plan")
    return PlanInfo([(w[i], h[i], it[i]) for i in range(n.value)], nc.value)


def workspace_bytes(H: int, W: int, params: Params | None = None) -> int:
    return _lib().fge_workspace_bytes(H, W, ctypes.byref(params) if params else None)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _on_stream(fn):
    """Run a binding function with `stream` (when given) as torch's current stream, so that every
    tensor it allocates -- outputs and scratch workspaces -- comes from that stream's pool of
    PyTorch's caching allocator.  A scratch tensor dropped on return is then only handed out again
    to work ordered after what was enqueued on `stream`; tensors allocated on another stream and
    used on `stream` could be reused while the kernels still run.  Tensors the caller passes in
    follow PyTorch's usual rule: ready before the call, and kept (or record_stream'ed) by the
    caller while `stream` uses them."""
    import functools
    import inspect
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapper(*args, **kwargs):
        stream = sig.bind(*args, **kwargs).arguments.get("stream")
        if stream is None:
            return fn(*args, **kwargs)
        import torch
        with torch.cuda.stream(stream):
            return fn(*args, **kwargs)
    return wrapper


def storage_dtype(params: Params):
    import torch
    return torch.float16 if params.storage == F16 else torch.float32


@_on_stream
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
    need = workspace_bytes(H, W, p)
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=I.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else None
    ws_len = workspace.numel() * workspace.element_size() if workspace is not None else 0
    st = _lib().fge_estimate_foreground(I.data_ptr(), alpha.data_ptr(), H, W, ctypes.byref(p),
                                        F.data_ptr(), B.data_ptr(), ws_ptr, ws_len,
                                        _stream_ptr(stream))
    _check(st, "fge_estimate_foreground")
    return F, B


def cf_default_params(**overrides) -> CfParams:
    """Defaults of the closed-form solve (omega 1, eps 5e-3, tol 1e-6, 20000 iterations,
    float32), with optional overrides."""
    p = CfParams()
    _lib().fge_cf_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def cf_workspace_bytes(H: int, W: int) -> int:
    return _lib().fge_cf_workspace_bytes(H, W)


@_on_stream
def closed_form(I, alpha, params: CfParams | None = None, F=None, B=None, workspace=None,
                stream=None):
    """The closed-form solve of eq. 2 (fge_closed_form): block-Jacobi preconditioned CG in
    float64 on the device.  Returns (F, B, info) with info a dict of the iteration counts and
    residuals.  Blocks until the solve has finished.  With params.warm_start the solve starts
    from the F, B passed in."""
    import torch
    p = params if params is not None else cf_default_params()
    dt = {F16: torch.float16, F64: torch.float64}.get(p.storage, torch.float32)
    if I.dim() != 3 or I.shape[0] != 3:
        raise ValueError("I must be (3, H, W)")
    _, H, W = I.shape
    if tuple(alpha.shape) != (H, W):
        raise ValueError("alpha must be (H, W) matching I")
    for name, t in (("I", I), ("alpha", alpha)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor of dtype {dt}")
    if p.warm_start and (F is None or B is None):
        raise ValueError("warm_start needs the starting F and B")
    if F is None:
        F = torch.empty((3, H, W), dtype=dt, device=I.device)
    if B is None:
        B = torch.empty((3, H, W), dtype=dt, device=I.device)
    for name, t in (("F", F), ("B", B)):
        if tuple(t.shape) != (3, H, W) or t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{name} must be a contiguous (3, H, W) CUDA tensor of dtype {dt}")
    need = cf_workspace_bytes(H, W)
    if workspace is None:
        workspace = torch.empty(max(1, need), dtype=torch.uint8, device=I.device)
    info = CfInfo()
    st = _lib().fge_closed_form(I.data_ptr(), alpha.data_ptr(), H, W, ctypes.byref(p),
                                F.data_ptr(), B.data_ptr(), workspace.data_ptr(),
                                workspace.numel() * workspace.element_size(), _stream_ptr(stream),
                                ctypes.byref(info))
    _check(st, "fge_closed_form")
    return F, B, {
        "iterations": info.iterations,
        "converged": bool(info.converged),
        "channel_iterations": list(info.channel_iterations),
        "breakdown": bool(info.breakdown),
        "rel_residual": list(info.rel_residual),
        "recursive_rel_residual": list(info.recursive_rel_residual),
        "device_ms": info.device_ms,
    }


def profile_start(capacity: int = 4096):
    """Record HIP events around every kernel launch of the following calls."""
    _check(_lib().fge_profile_start(capacity), "fge_profile_start")


def profile_stop(max_levels: int = MAX_LEVELS):
    """Stop recording; returns (ms_per_level, launches_per_level), level 0 = finest."""
    ms = (ctypes.c_double * max_levels)()
    cnt = (ctypes.c_int32 * max_levels)()
    _check(_lib().fge_profile_stop(ms, cnt, max_levels), "fge_profile_stop")
    return list(ms), list(cnt)


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr()
    return arr


class Batch:
    """A batch plan for images of shapes [(H, W), ...], height first as in the C ABI
    (fge_batch_create).  Every image follows its own level plan, so its result is bit-identical
    to estimate_foreground's."""

    def __init__(self, shapes, params: Params | None = None):
        self.shapes = [(int(h), int(w)) for h, w in shapes]
        self.params = params if params is not None else default_params()
        n = len(self.shapes)
        H = (ctypes.c_int32 * n)(*[h for h, _ in self.shapes])
        W = (ctypes.c_int32 * n)(*[w for _, w in self.shapes])
        handle = ctypes.c_void_p()
        _check(_lib().fge_batch_create(n, H, W, ctypes.byref(self.params), ctypes.byref(handle)),
               "fge_batch_create")
        self._h = handle
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            _lib().fge_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self) -> int:
        return _lib().fge_batch_workspace_bytes(self._h)

    @property
    def steps(self) -> int:
        return _lib().fge_batch_steps(self._h)

    @property
    def launch_count(self) -> int:
        return _lib().fge_batch_launch_count(self._h)

    def _args(self, Is, alphas, Fs, Bs, workspace):
        import torch
        dt = storage_dtype(self.params)
        n = len(self.shapes)
        if not (len(Is) == len(alphas) == n):
            raise ValueError("one I and one alpha per image")
        if Fs is None:
            Fs = [torch.empty((3, h, w), dtype=dt, device=Is[0].device) for h, w in self.shapes]
        if Bs is None:
            Bs = [torch.empty((3, h, w), dtype=dt, device=Is[0].device) for h, w in self.shapes]
        for (h, w), I, a, F, B in zip(self.shapes, Is, alphas, Fs, Bs):
            for name, t, shp in (("I", I, (3, h, w)), ("alpha", a, (h, w)), ("F", F, (3, h, w)),
                                 ("B", B, (3, h, w))):
                if tuple(t.shape) != shp or t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                    raise ValueError(f"{name} must be a contiguous CUDA tensor {shp} of dtype {dt}")
        if workspace is None:
            workspace = torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8,
                                    device=Is[0].device)
        return Fs, Bs, workspace

    @_on_stream
    def run(self, Is, alphas, Fs=None, Bs=None, workspace=None, stream=None):
        """Enqueue the batch; returns (Fs, Bs).  Does not synchronise."""
        Fs, Bs, workspace = self._args(Is, alphas, Fs, Bs, workspace)
        st = _lib().fge_batch_run(self._h, _ptr_array(Is), _ptr_array(alphas), _ptr_array(Fs),
                                  _ptr_array(Bs), workspace.data_ptr(),
                                  workspace.numel(), _stream_ptr(stream))
        _check(st, "fge_batch_run")
        self._keep = (Is, alphas, Fs, Bs, workspace)
        return Fs, Bs

    @_on_stream
    def capture(self, Is, alphas, Fs=None, Bs=None, workspace=None, stream=None):
        """Capture one run with these buffers into a hipGraph; replay() launches it."""
        Fs, Bs, workspace = self._args(Is, alphas, Fs, Bs, workspace)
        st = _lib().fge_batch_capture(self._h, _ptr_array(Is), _ptr_array(alphas),
                                      _ptr_array(Fs), _ptr_array(Bs), workspace.data_ptr(),
                                      workspace.numel(), _stream_ptr(stream))
        _check(st, "fge_batch_capture")
        self._graph_keep = (Is, alphas, Fs, Bs, workspace)
        return Fs, Bs

    def replay(self, stream=None):
        _check(_lib().fge_batch_replay(self._h, _stream_ptr(stream)), "fge_batch_replay")


def server_config(**overrides) -> ServerConfig:
    """fge_server_default_config with optional overrides, e.g. ``server_config(max_active=8)``."""
    c = ServerConfig()
    _lib().fge_server_default_config(ctypes.byref(c))
    for k, v in overrides.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


def server_request_bytes(H: int, W: int, params: Params | None = None) -> int:
    """Footprint an H x W request is charged against a server's budget."""
    return _lib().fge_server_request_bytes(H, W, ctypes.byref(params) if params else None)


def server_reserved_bytes(config: ServerConfig | None = None) -> int:
    return _lib().fge_server_reserved_bytes(ctypes.byref(config) if config else None)


def server_sim(**overrides) -> ServerSim:
    """fge_server_sim_default with optional overrides, e.g. ``server_sim(fail_launch_tick=3)``."""
    m = ServerSim()
    _lib().fge_server_sim_default(ctypes.byref(m))
    for k, v in overrides.items():
        if not hasattr(m, k):
            raise KeyError(k)
        setattr(m, k, v)
    return m


class Server:
    """Continuous-batching request server (fge_server_*).  `arena` is a CUDA uint8 tensor the
    server carves its tick tables and the requests' workspaces from; `stream` the torch stream
    every launch goes to.  Inputs must be complete on the device before they are submitted."""

    def __init__(self, params: Params | None = None, config: ServerConfig | None = None,
                 arena=None, arena_bytes: int | None = None, stream=None):
        import torch
        self.params = params if params is not None else default_params()
        self.config = config if config is not None else server_config()
        if arena is None:
            if arena_bytes is None:
                raise ValueError("give an arena tensor or arena_bytes")
            arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
        if not arena.is_cuda or arena.dtype != torch.uint8 or not arena.is_contiguous():
            raise ValueError("arena must be a contiguous CUDA uint8 tensor")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.arena = arena
        handle = ctypes.c_void_p()
        _check(_lib().fge_server_create(ctypes.byref(self.params), ctypes.byref(self.config),
                                        arena.data_ptr(), arena.numel(),
                                        ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(handle)), "fge_server_create")
        self._h = handle
        self._held = {}

    def submit(self, rid: int, I, alpha, F=None, B=None):
        """Queue request `rid` with tensors I (3, H, W) and alpha (H, W); returns (F, B), which
        hold the result once poll() has reported the request."""
        import torch
        dt = storage_dtype(self.params)
        if I.dim() != 3 or I.shape[0] != 3:
            raise ValueError("I must be (3, H, W)")
        _, H, W = I.shape
        if F is None:
            F = torch.empty((3, H, W), dtype=dt, device=I.device)
        if B is None:
            B = torch.empty((3, H, W), dtype=dt, device=I.device)
        for name, t, shp in (("I", I, (3, H, W)), ("alpha", alpha, (H, W)), ("F", F, (3, H, W)),
                             ("B", B, (3, H, W))):
            if tuple(t.shape) != shp or t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous CUDA tensor {shp} of dtype {dt}")
        self.submit_ptrs(rid, I.data_ptr(), alpha.data_ptr(), H, W, F.data_ptr(), B.data_ptr())
        self._held[rid] = (I, alpha, F, B)
        return F, B

    def submit_ptrs(self, rid: int, I: int, alpha: int, H: int, W: int, F: int, B: int):
        """Raw form: device addresses the caller keeps alive until the request completes."""
        _check(_lib().fge_server_submit(self._h, rid, I, alpha, H, W, F, B), "fge_server_submit")

    def cancel(self, rid: int) -> bool:
        """Cancel a request still queued; False if it was admitted, completed or unknown."""
        st = _lib().fge_server_cancel(self._h, rid)
        if st not in (FGE_OK, FGE_EINVAL):
            raise FgeError(st, "fge_server_cancel")
        if st == FGE_OK:
            self._held.pop(rid, None)
        return st == FGE_OK

    @classmethod
    def simulated(cls, params: Params | None = None, config: ServerConfig | None = None,
                  arena_bytes: int = 1 << 30, sim: ServerSim | None = None):
        """A server on the host model of the device (fge_server_create_simulated): submit with
        submit_ptrs (addresses are only stored), drive it with step() in manual mode."""
        self = cls.__new__(cls)
        self.params = params if params is not None else default_params()
        self.config = config if config is not None else server_config()
        self.stream = None
        self.arena = None
        self._held = {}
        handle = ctypes.c_void_p()
        _check(_lib().fge_server_create_simulated(ctypes.byref(self.params),
                                                  ctypes.byref(self.config), arena_bytes,
                                                  ctypes.byref(sim) if sim is not None else None,
                                                  ctypes.byref(handle)),
               "fge_server_create_simulated")
        self._h = handle
        return self

    def step(self, complete: int = 0, advance_ms: float = 0.0) -> int:
        """Manual simulated server: complete the oldest `complete` ticks, run the scheduler;
        returns the ticks it enqueued (raises if the server has failed)."""
        n = _lib().fge_server_sim_step(self._h, complete, advance_ms)
        if n < 0:
            raise FgeError(n, "fge_server_sim_step")
        return n

    def inflight(self) -> int:
        return _lib().fge_server_sim_inflight(self._h)

    def poll(self, cap: int = 4096):
        """Completed requests since the last poll: a list of ServerResult records."""
        buf = (ServerResult * cap)()
        n = _lib().fge_server_poll(self._h, buf, cap)
        if n < 0:
            raise FgeError(n, "fge_server_poll")
        out = [buf[i] for i in range(n)]
        for r in out:
            self._held.pop(r.id, None)
        return out

    def drain(self):
        _check(_lib().fge_server_drain(self._h), "fge_server_drain")

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib().fge_server_get_stats(self._h, ctypes.byref(st)), "fge_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_ if k != "reserved0"}

    def close(self):
        if getattr(self, "_h", None):
            _lib().fge_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- autotuner ---------------------------------------------------------------------------------

def _tune_key(kind: str, params: Params, sizes) -> str:
    import hashlib
    import torch
    fields = {k: getattr(params, k) for k, _ in Params._fields_
              if k not in ("strip_rows", "tile_max_px")}
    h = hashlib.sha1(repr((kind, sorted(fields.items()), list(sizes))).encode()).hexdigest()[:16]
    return f"{torch.cuda.get_device_name()}|{kind}|{h}"


def _cache_get(cache_path, key):
    import json
    if not cache_path or not os.path.exists(cache_path):
        return None
    with open(cache_path) as f:
        return json.load(f).get(key)


def _cache_put(cache_path, key, value):
    import json
    if not cache_path:
        return
    data = {}
    if os.path.exists(cache_path):
        with open(cache_path) as f:
            data = json.load(f)
    data[key] = value
    tmp = cache_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, cache_path)


def _tuned(params: Params, strip_rows: int, tile_max_px: int) -> Params:
    q = Params()
    ctypes.pointer(q)[0] = params
    q.strip_rows = strip_rows
    q.tile_max_px = tile_max_px
    return q


def _entries(buf, n):
    return [{"strip_rows": buf[i].strip_rows, "tile_max_px": buf[i].tile_max_px,
             "ms": buf[i].ms, "status": buf[i].status} for i in range(n)]


@_on_stream
def autotune(I, alpha, params: Params | None = None, reps: int = 3, stream=None,
             cache_path: str | None = None):
    """Search strip height and tile threshold for this image size on the device (fge_autotune).
    Returns (best_params, entries); with `cache_path`, a JSON file keyed by device, parameters and
    size answers repeated calls without running anything."""
    import torch
    p = params if params is not None else default_params()
    _, H, W = I.shape
    key = _tune_key("single", p, [(H, W)])
    hit = _cache_get(cache_path, key)
    if hit is not None:
        return _tuned(p, hit["strip_rows"], hit["tile_max_px"]), hit.get("entries", [])
    dt = storage_dtype(p)
    F = torch.empty((3, H, W), dtype=dt, device=I.device)
    B = torch.empty_like(F)
    need = _lib().fge_tune_workspace_bytes(H, W, ctypes.byref(p))
    ws = torch.empty(max(1, need), dtype=torch.uint8, device=I.device)
    nc = _lib().fge_tune_candidates()
    buf = (TuneEntry * nc)()
    n = ctypes.c_int32()
    best = Params()
    _check(_lib().fge_autotune(I.data_ptr(), alpha.data_ptr(), H, W, ctypes.byref(p), F.data_ptr(),
                               B.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(stream), reps,
                               ctypes.byref(best), buf, nc, ctypes.byref(n)), "fge_autotune")
    ent = _entries(buf, n.value)
    _cache_put(cache_path, key, {"strip_rows": best.strip_rows, "tile_max_px": best.tile_max_px,
                                 "entries": ent})
    return best, ent


@_on_stream
def autotune_batch(shapes, Is, alphas, params: Params | None = None, reps: int = 3, stream=None,
                   cache_path: str | None = None):
    """The same search for a batch of shapes [(H, W), ...] (fge_batch_autotune)."""
    import torch
    p = params if params is not None else default_params()
    shapes = [(int(h), int(w)) for h, w in shapes]
    key = _tune_key("batch", p, shapes)
    hit = _cache_get(cache_path, key)
    if hit is not None:
        return _tuned(p, hit["strip_rows"], hit["tile_max_px"]), hit.get("entries", [])
    n = len(shapes)
    H = (ctypes.c_int32 * n)(*[h for h, _ in shapes])
    W = (ctypes.c_int32 * n)(*[w for _, w in shapes])
    dt = storage_dtype(p)
    Fs = [torch.empty((3, h, w), dtype=dt, device=Is[0].device) for h, w in shapes]
    Bs = [torch.empty_like(f) for f in Fs]
    need = _lib().fge_batch_tune_workspace_bytes(n, H, W, ctypes.byref(p))
    if need == 0:
        raise FgeError(FGE_EINVAL, "fge_batch_tune_workspace_bytes")
    ws = torch.empty(need, dtype=torch.uint8, device=Is[0].device)
    nc = _lib().fge_tune_candidates()
    buf = (TuneEntry * nc)()
    cnt = ctypes.c_int32()
    best = Params()
    _check(_lib().fge_batch_autotune(n, _ptr_array(Is), _ptr_array(alphas), H, W, ctypes.byref(p),
                                     _ptr_array(Fs), _ptr_array(Bs), ws.data_ptr(), ws.numel(),
                                     _stream_ptr(stream), reps, ctypes.byref(best), buf, nc,
                                     ctypes.byref(cnt)), "fge_batch_autotune")
    ent = _entries(buf, cnt.value)
    _cache_put(cache_path, key, {"strip_rows": best.strip_rows, "tile_max_px": best.tile_max_px,
                                 "entries": ent})
    return best, ent


# ---- reporting and layout ----------------------------------------------------------------------

def _dtype_code(dt):
    import torch
    codes = {torch.float32: F32, torch.float16: F16, torch.uint8: U8}
    if dt not in codes:
        raise ValueError(f"unsupported dtype {dt}")
    return codes[dt]


def _torch_dtype(code):
    import torch
    return {F32: torch.float32, F16: torch.float16, U8: torch.uint8}[code]


@_on_stream
def energy(I, alpha, F, B, params: Params | None = None, stream=None, out=None):
    """Energy E of (F, B) and the compositing residual, reduced on the device (fge_energy).
    Returns a float64 CUDA tensor of 6: E, data term, smoothness term, mean and max |residual|
    over fractional pixels, their count.  Does not synchronise."""
    import torch
    p = params if params is not None else default_params()
    _, H, W = I.shape
    dt = storage_dtype(p)
    for name, t, shp in (("I", I, (3, H, W)), ("alpha", alpha, (H, W)), ("F", F, (3, H, W)),
                         ("B", B, (3, H, W))):
        if tuple(t.shape) != shp or t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor {shp} of dtype {dt}")
    if out is None:
        out = torch.empty(6, dtype=torch.float64, device=I.device)
    ws = torch.empty(_lib().fge_energy_workspace_bytes(H, W), dtype=torch.uint8, device=I.device)
    _check(_lib().fge_energy(I.data_ptr(), alpha.data_ptr(), F.data_ptr(), B.data_ptr(), H, W,
                             ctypes.byref(p), out.data_ptr(), ws.data_ptr(), ws.numel(),
                             _stream_ptr(stream)), "fge_energy")
    return out


@_on_stream
def hwc_to_planar(img, dtype=None, stream=None):
    """(H, W, 3|4) CUDA tensor (uint8, float32 or float16) -> (I (3, H, W), alpha (H, W) or None)
    in `dtype` (default float32); uint8 maps to v / 255 (fge_hwc_to_planar)."""
    import torch
    dtype = dtype or torch.float32
    if img.dim() != 3 or img.shape[2] not in (3, 4) or not img.is_cuda or not img.is_contiguous():
        raise ValueError("img must be a contiguous CUDA tensor (H, W, 3|4)")
    H, W, C = img.shape
    I = torch.empty((3, H, W), dtype=dtype, device=img.device)
    a = torch.empty((H, W), dtype=dtype, device=img.device) if C == 4 else None
    _check(_lib().fge_hwc_to_planar(img.data_ptr(), _dtype_code(img.dtype), C, H, W, I.data_ptr(),
                                    a.data_ptr() if a is not None else None, _dtype_code(dtype),
                                    _stream_ptr(stream)), "fge_hwc_to_planar")
    return I, a


@_on_stream
def planar_to_hwc(planes, dtype=None, stream=None):
    """(3, H, W) CUDA tensor -> (H, W, 3) in `dtype` (default uint8: round(clamp(v) * 255))."""
    import torch
    dtype = dtype or torch.uint8
    if planes.dim() != 3 or planes.shape[0] != 3 or not planes.is_cuda or not planes.is_contiguous():
        raise ValueError("planes must be a contiguous CUDA tensor (3, H, W)")
    _, H, W = planes.shape
    out = torch.empty((H, W, 3), dtype=dtype, device=planes.device)
    _check(_lib().fge_planar_to_hwc(planes.data_ptr(), _dtype_code(planes.dtype), H, W,
                                    out.data_ptr(), _dtype_code(dtype), _stream_ptr(stream)),
           "fge_planar_to_hwc")
    return out


@_on_stream
def estimate_foreground_converge(I, alpha, params: Params | None = None, tol: float = 1e-4,
                                 max_sweeps: int = 100, F=None, B=None, stream=None):
    """Algorithm 1's "while not converged" level loop on the device (fge_estimate_foreground_converge):
    per level, sweep until the level energy changes by at most `tol` (relative) or `max_sweeps`.
    Returns (F, B, sweeps), sweeps an int32 CUDA tensor of the per-level counts.  tol < 0 runs the
    fixed counts.  Does not synchronise."""
    import torch
    p = params if params is not None else default_params()
    dt = storage_dtype(p)
    _, H, W = I.shape
    for name, t in (("I", I), ("alpha", alpha)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor of dtype {dt}")
    if tuple(alpha.shape) != (H, W):
        raise ValueError("alpha must be (H, W) matching I")
    if F is None:
        F = torch.empty((3, H, W), dtype=dt, device=I.device)
    if B is None:
        B = torch.empty((3, H, W), dtype=dt, device=I.device)
    n = num_levels(H, W)
    sweeps = torch.zeros(max(1, n), dtype=torch.int32, device=I.device)
    need = _lib().fge_converge_workspace_bytes(H, W, ctypes.byref(p))
    ws = torch.empty(max(1, need), dtype=torch.uint8, device=I.device)
    _check(_lib().fge_estimate_foreground_converge(
        I.data_ptr(), alpha.data_ptr(), H, W, ctypes.byref(p), float(tol), int(max_sweeps),
        F.data_ptr(), B.data_ptr(), sweeps.data_ptr(), ws.data_ptr(), ws.numel(),
        _stream_ptr(stream)), "fge_estimate_foreground_converge")
    return F, B, sweeps[:n]


@_on_stream
def estimate_foreground_converge_passes(I, alpha, params: Params | None = None, tol: float = 1e-4,
                                        max_passes: int = 100, F=None, B=None, stream=None):
    """The "while not converged" level loop on the fused kernels, tested after every pass of two
    sweeps (fge_estimate_foreground_converge_passes).  Returns (F, B, passes), passes a list of the
    per-level pass counts.  Blocks until done."""
    import torch
    p = params if params is not None else default_params()
    dt = storage_dtype(p)
    _, H, W = I.shape
    for name, t in (("I", I), ("alpha", alpha)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor of dtype {dt}")
    if tuple(alpha.shape) != (H, W):
        raise ValueError("alpha must be (H, W) matching I")
    if F is None:
        F = torch.empty((3, H, W), dtype=dt, device=I.device)
    if B is None:
        B = torch.empty((3, H, W), dtype=dt, device=I.device)
    n = num_levels(H, W)
    passes = (ctypes.c_int32 * max(1, n))()
    need = _lib().fge_converge_passes_workspace_bytes(H, W, ctypes.byref(p))
    ws = torch.empty(max(1, need), dtype=torch.uint8, device=I.device)
    _check(_lib().fge_estimate_foreground_converge_passes(
        I.data_ptr(), alpha.data_ptr(), H, W, ctypes.byref(p), float(tol), int(max_passes),
        F.data_ptr(), B.data_ptr(), passes, ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
        "fge_estimate_foreground_converge_passes")
    return F, B, list(passes)[:n]


@_on_stream
def quality(F, G, alpha, sigma: float = 1.4, stream=None, out=None):
    """The paper's error measures of F against the reference G over the translucent pixels of
    `alpha`, weighted by alpha (fge_quality): a float64 CUDA tensor [SAD, MSE, GRAD, count]."""
    import torch
    if F.dim() != 3 or F.shape[0] != 3:
        raise ValueError("F must be (3, H, W)")
    _, H, W = F.shape
    for name, t, shp in (("F", F, (3, H, W)), ("G", G, (3, H, W)), ("alpha", alpha, (H, W))):
        if tuple(t.shape) != shp or t.dtype != F.dtype or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor {shp} of dtype {F.dtype}")
    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=F.device)
    ws = torch.empty(_lib().fge_quality_workspace_bytes(H, W), dtype=torch.uint8, device=F.device)
    _check(_lib().fge_quality(F.data_ptr(), G.data_ptr(), alpha.data_ptr(), H, W,
                              _dtype_code(F.dtype), float(sigma), out.data_ptr(), ws.data_ptr(),
                              ws.numel(), _stream_ptr(stream)), "fge_quality")
    return out


@_on_stream
def composite(F, alpha, B, stream=None):
    """alpha F + (1 - alpha) B on the device (fge_composite)."""
    import torch
    if F.dim() != 3 or F.shape[0] != 3:
        raise ValueError("F must be (3, H, W)")
    _, H, W = F.shape
    for name, t, shp in (("F", F, (3, H, W)), ("alpha", alpha, (H, W)), ("B", B, (3, H, W))):
        if tuple(t.shape) != shp or t.dtype != F.dtype or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor {shp} of dtype {F.dtype}")
    C = torch.empty_like(F)
    _check(_lib().fge_composite(F.data_ptr(), alpha.data_ptr(), B.data_ptr(), H, W,
                                _dtype_code(F.dtype), C.data_ptr(), _stream_ptr(stream)),
           "fge_composite")
    return C


def level_options(resize: str = "smooth", tol: float = -1.0, max_sweeps: int = 100,
                  passes: bool = False) -> LevelOptions:
    o = LevelOptions()
    o.size = ctypes.sizeof(LevelOptions)
    o.resize = {"nearest": RESIZE_NEAREST, "smooth": RESIZE_SMOOTH}[resize]
    o.tol = float(tol)
    o.max_sweeps = int(max_sweeps)
    o.passes = 1 if passes else 0
    return o


@_on_stream
def estimate_foreground_levels(I, alpha, params: Params | None = None, resize: str = "smooth",
                               tol: float = -1.0, max_sweeps: int = 100, F=None, B=None,
                               stream=None, passes: bool = False):
    """The level loop with a resize variant and, for tol >= 0, the convergence stop
    (fge_estimate_foreground_levels): tested after every sweep on per-level kernels, or with
    passes=True after every pass of two sweeps on the fused kernels (max_sweeps then caps the
    passes, and the call completes before it returns).  Returns (F, B, sweeps -- or passes -- per
    level; the counts are written in the convergence form only).  Does not synchronise otherwise."""
    import torch
    p = params if params is not None else default_params()
    o = level_options(resize, tol, max_sweeps, passes)
    dt = storage_dtype(p)
    _, H, W = I.shape
    for name, t in (("I", I), ("alpha", alpha)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor of dtype {dt}")
    if tuple(alpha.shape) != (H, W):
        raise ValueError("alpha must be (H, W) matching I")
    if F is None:
        F = torch.empty((3, H, W), dtype=dt, device=I.device)
    if B is None:
        B = torch.empty((3, H, W), dtype=dt, device=I.device)
    n = num_levels(H, W)
    sweeps = torch.zeros(max(1, n), dtype=torch.int32, device=I.device)
    need = _lib().fge_levels_workspace_bytes(H, W, ctypes.byref(p), ctypes.byref(o))
    ws = torch.empty(max(1, need), dtype=torch.uint8, device=I.device)
    _check(_lib().fge_estimate_foreground_levels(
        I.data_ptr(), alpha.data_ptr(), H, W, ctypes.byref(p), ctypes.byref(o), F.data_ptr(),
        B.data_ptr(), sweeps.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
        "fge_estimate_foreground_levels")
    return F, B, sweeps[:n]
