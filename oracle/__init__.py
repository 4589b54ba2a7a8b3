"""FP64 CPU oracle for multi-level foreground estimation (arXiv 2006.14970).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference that the GPU path is checked
against.  Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import it.
It shares no code with the product package and imports nothing from it.

The arithmetic lives in ``fge_oracle.c`` (plain C, IEEE double, built with gcc); this module only
builds that file and marshals numpy arrays to it.  Functions and the paper passages they follow:

* :func:`num_levels`, :func:`level_size`, :func:`level_plan` -- Algorithm 1's level count,
  level sizes and the 10/2 iteration rule of Section III-D.
* :func:`resize_nearest` -- Algorithm 1's ``resize`` under the nearest-neighbour reading.
* :func:`sweep` -- one pass of Algorithm 1's per-pixel loop (eq. 9 plus the output clamp) in
  raster, red-black or Jacobi order.
* :func:`ml` -- Algorithm 1 end to end.
* :func:`energy` -- the global quadratic energy whose stationarity conditions are eq. 9.

The module :mod:`oracle.closed_form` (NumPy / SciPy) is the minimiser of the global closed-form
cost of Section III-B (eq. 2, with the eps regulariser of Section III-C) by a sparse direct solve.

Layout everywhere: ``I``, ``F``, ``B`` are float64 arrays of shape (3, H, W) (planar RGB), the
matte is (H, W).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fge_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

ORDERS = {"raster": 0, "redblack": 1, "jacobi": 2}

_libs: dict[bool, ctypes.CDLL] = {}


def build(force: bool = True) -> str:
    """Compile ``fge_oracle.c`` with gcc (strict IEEE double, no FMA) twice: ``liboracle.so``
    (one thread) and ``liboracle_omp.so`` (OpenMP; red-black and Jacobi sweeps split their rows
    over threads, with bit-identical results)."""
    for path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.run(
                ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", *extra,
                 "-o", tmp, _SRC, "-lm"],
                check=True)
            os.replace(tmp, path)
    return _LIB


def threads(parallel: bool = True) -> int:
    """Threads one sweep of the chosen build uses (OMP_NUM_THREADS, else all cores)."""
    return _load(parallel).fgo_threads()


def _load(parallel: bool = False):
    if parallel in _libs:
        return _libs[parallel]
    path = _LIB_OMP if parallel else _LIB
    if not os.path.exists(path):
        build(force=False)
    lib = ctypes.CDLL(path)
    lib.fgo_threads.argtypes = []
    lib.fgo_threads.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    i32, f64 = ctypes.c_int, ctypes.c_double
    lib.fgo_num_levels.argtypes = [i32, i32]
    lib.fgo_num_levels.restype = i32
    lib.fgo_level_size.argtypes = [i32, i32, i32]
    lib.fgo_level_size.restype = i32
    lib.fgo_resize_nearest.argtypes = [dp, i32, i32, i32, dp, i32, i32]
    lib.fgo_resize_nearest.restype = None
    lib.fgo_sweep.argtypes = [dp, dp, dp, dp, i32, i32, f64, f64, i32]
    lib.fgo_sweep.restype = None
    lib.fgo_ml.argtypes = [dp, dp, i32, i32, f64, f64, i32, i32, i32, i32, dp, dp, dp, dp]
    lib.fgo_ml.restype = i32
    lib.fgo_energy.argtypes = [dp, dp, dp, dp, i32, i32, f64, f64]
    lib.fgo_energy.restype = f64
    ip = ctypes.POINTER(ctypes.c_int)
    lib.fgo_ml_schedule.argtypes = [dp, dp, i32, i32, f64, f64, i32, ip, dp, dp]
    lib.fgo_ml_schedule.restype = i32
    lib.fgo_ml_converge.argtypes = [dp, dp, i32, i32, f64, f64, i32, f64, i32, ip, dp, dp]
    lib.fgo_ml_converge.restype = i32
    lib.fgo_ml_converge_every.argtypes = [dp, dp, i32, i32, f64, f64, i32, i32, f64, i32, ip, dp,
                                          i32, dp, dp]
    lib.fgo_ml_converge_every.restype = i32
    lib.fgo_resize_area.argtypes = [dp, i32, i32, i32, dp, i32, i32]
    lib.fgo_resize_area.restype = None
    lib.fgo_resize_bilinear.argtypes = [dp, i32, i32, i32, dp, i32, i32]
    lib.fgo_resize_bilinear.restype = None
    lib.fgo_ml_resize.argtypes = [dp, dp, i32, i32, f64, f64, i32, i32, ip, dp, dp]
    lib.fgo_ml_resize.restype = i32
    _libs[parallel] = lib
    return lib


def _ptr(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64c(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def num_levels(w: int, h: int) -> int:
    """Algorithm 1: ceil(log2(max(w, h))), at least 1."""
    return _load().fgo_num_levels(int(w), int(h))


def level_size(full: int, level: int, n_levels: int) -> int:
    """Algorithm 1: round(full ** (level / n_levels))."""
    return _load().fgo_level_size(int(full), int(level), int(n_levels))


def level_plan(W: int, H: int, small_size: int = 32, iters_small: int = 10,
               iters_big: int = 2) -> list[tuple[int, int, int]]:
    """[(w_l, h_l, iterations)] for l = 1..n_l (Algorithm 1 and the iteration rule of III-D)."""
    n = num_levels(W, H)
    out = []
    for lv in range(1, n + 1):
        w, h = level_size(W, lv, n), level_size(H, lv, n)
        it = iters_small if (w <= small_size and h <= small_size) else iters_big
        out.append((w, h, it))
    return out


def resize_nearest(src: np.ndarray, wd: int, hd: int) -> np.ndarray:
    """Nearest resize of a (P, hs, ws) or (hs, ws) array to (P, hd, wd) / (hd, wd)."""
    s = _f64c(src)
    squeeze = s.ndim == 2
    if squeeze:
        s = s[None]
    p, hs, ws = s.shape
    d = np.empty((p, hd, wd), dtype=np.float64)
    _load().fgo_resize_nearest(_ptr(s), ws, hs, p, _ptr(d), wd, hd)
    return d[0] if squeeze else d


def sweep(F: np.ndarray, B: np.ndarray, I: np.ndarray, alpha: np.ndarray, omega: float = 0.1,
          eps: float = 5e-3, order: str = "redblack", n: int = 1) -> tuple[np.ndarray, np.ndarray]:
    """Run ``n`` sweeps of Algorithm 1's per-pixel loop at one level; returns new (F, B)."""
    F = _f64c(F).copy()
    B = _f64c(B).copy()
    I = _f64c(I)
    a = _f64c(alpha)
    _, h, w = I.shape
    lib = _load()
    for _ in range(n):
        lib.fgo_sweep(_ptr(F), _ptr(B), _ptr(I), _ptr(a), w, h, float(omega), float(eps),
                      ORDERS[order])
    return F, B


def ml(I: np.ndarray, alpha: np.ndarray, omega: float = 0.1, eps: float = 5e-3,
       small_size: int = 32, iters_small: int = 10, iters_big: int = 2,
       order: str = "redblack", init=None, parallel: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """Algorithm 1 (multi-level estimation) in FP64.  ``init`` = (f3, b3) overrides the zero
    1x1 start (used only by the constant-image fixed-point test).  ``parallel`` runs the OpenMP
    build (same bits; raster order stays sequential)."""
    I = _f64c(I)
    a = _f64c(alpha)
    _, H, W = I.shape
    assert a.shape == (H, W)
    F = np.empty((3, H, W), dtype=np.float64)
    B = np.empty((3, H, W), dtype=np.float64)
    if init is not None:
        f0, b0 = _f64c(init[0]), _f64c(init[1])
        pf, pb = _ptr(f0), _ptr(b0)
    else:
        pf = pb = None
    _load(parallel).fgo_ml(_ptr(I), _ptr(a), W, H, float(omega), float(eps), int(small_size),
                   int(iters_small), int(iters_big), ORDERS[order], pf, pb, _ptr(F), _ptr(B))
    return F, B


def energy(F: np.ndarray, B: np.ndarray, I: np.ndarray, alpha: np.ndarray, omega: float = 0.1,
           eps: float = 5e-3) -> float:
    """Global quadratic energy (data term plus each undirected 4-neighbour edge once)."""
    F, B, I, a = _f64c(F), _f64c(B), _f64c(I), _f64c(alpha)
    _, h, w = I.shape
    return _load().fgo_energy(_ptr(F), _ptr(B), _ptr(I), _ptr(a), w, h, float(omega), float(eps))


def ml_schedule(I: np.ndarray, alpha: np.ndarray, sweeps, omega: float = 0.1, eps: float = 5e-3,
                order: str = "redblack") -> tuple[np.ndarray, np.ndarray]:
    """Algorithm 1 with sweeps[l-1] sweeps at level l (replays a given schedule)."""
    I = _f64c(I)
    a = _f64c(alpha)
    _, H, W = I.shape
    n = num_levels(W, H)
    sw = (ctypes.c_int * n)(*[int(k) for k in sweeps])
    if len(sweeps) != n:
        raise ValueError(f"{n} levels, {len(sweeps)} sweep counts")
    F = np.empty((3, H, W), dtype=np.float64)
    B = np.empty((3, H, W), dtype=np.float64)
    _load().fgo_ml_schedule(_ptr(I), _ptr(a), W, H, float(omega), float(eps), ORDERS[order], sw,
                            _ptr(F), _ptr(B))
    return F, B


def ml_converge(I: np.ndarray, alpha: np.ndarray, tol: float, max_sweeps: int,
                omega: float = 0.1, eps: float = 5e-3, order: str = "redblack"):
    """Algorithm 1's "while not converged" form: per level, sweep until the level energy changes
    by at most tol (relative) or max_sweeps sweeps.  Returns (F, B, sweeps per level)."""
    I = _f64c(I)
    a = _f64c(alpha)
    _, H, W = I.shape
    n = num_levels(W, H)
    sw = (ctypes.c_int * n)()
    F = np.empty((3, H, W), dtype=np.float64)
    B = np.empty((3, H, W), dtype=np.float64)
    _load().fgo_ml_converge(_ptr(I), _ptr(a), W, H, float(omega), float(eps), ORDERS[order],
                            float(tol), int(max_sweeps), sw, _ptr(F), _ptr(B))
    return F, B, list(sw)


def ml_converge_every(I: np.ndarray, alpha: np.ndarray, m: int, tol: float, max_checks: int,
                      omega: float = 0.1, eps: float = 5e-3, order: str = "redblack",
                      rel_cap: int = 0):
    """The same loop condition tested every m sweeps: per level, groups of m sweeps until the
    level energy changes over a group by at most tol (relative) or max_checks groups.  Returns
    (F, B, groups per level) and, with rel_cap > 0, the relative energy change of each group
    (levels x rel_cap, NaN past a level's last group)."""
    I = _f64c(I)
    a = _f64c(alpha)
    _, H, W = I.shape
    n = num_levels(W, H)
    ch = (ctypes.c_int * n)()
    F = np.empty((3, H, W), dtype=np.float64)
    B = np.empty((3, H, W), dtype=np.float64)
    rel = np.full((n, max(rel_cap, 1)), np.nan)
    _load().fgo_ml_converge_every(_ptr(I), _ptr(a), W, H, float(omega), float(eps), ORDERS[order],
                                  int(m), float(tol), int(max_checks), ch,
                                  _ptr(rel) if rel_cap > 0 else None, int(rel_cap), _ptr(F), _ptr(B))
    if rel_cap > 0:
        return F, B, list(ch), rel
    return F, B, list(ch)


RESIZES = {"nearest": 0, "smooth": 1}


def _resize_with(fn, src, wd, hd):
    s = _f64c(src)
    squeeze = s.ndim == 2
    if squeeze:
        s = s[None]
    p, hs, ws = s.shape
    d = np.empty((p, hd, wd), dtype=np.float64)
    fn(_ptr(s), ws, hs, p, _ptr(d), wd, hd)
    return d[0] if squeeze else d


def resize_area(src: np.ndarray, wd: int, hd: int) -> np.ndarray:
    """Area (overlap-weighted mean) resize of a (P, hs, ws) or (hs, ws) array."""
    return _resize_with(_load().fgo_resize_area, src, wd, hd)


def resize_bilinear(src: np.ndarray, wd: int, hd: int) -> np.ndarray:
    """Bilinear resize with half-integer pixel centres, clamped at the borders."""
    return _resize_with(_load().fgo_resize_bilinear, src, wd, hd)


def ml_resize(I: np.ndarray, alpha: np.ndarray, resize: str = "smooth", sweeps=None,
              omega: float = 0.1, eps: float = 5e-3, order: str = "redblack"):
    """Algorithm 1 with the resize variant ("nearest" or "smooth": area for I and alpha, bilinear
    for F and B) and per-level sweep counts (default: the fixed 10 / 2 rule)."""
    I = _f64c(I)
    a = _f64c(alpha)
    _, H, W = I.shape
    if sweeps is None:
        sweeps = [it for _, _, it in level_plan(W, H)]
    n = num_levels(W, H)
    if len(sweeps) != n:
        raise ValueError(f"{n} levels, {len(sweeps)} sweep counts")
    sw = (ctypes.c_int * n)(*[int(k) for k in sweeps])
    F = np.empty((3, H, W), dtype=np.float64)
    B = np.empty((3, H, W), dtype=np.float64)
    _load().fgo_ml_resize(_ptr(I), _ptr(a), W, H, float(omega), float(eps), ORDERS[order],
                          RESIZES[resize], sw, _ptr(F), _ptr(B))
    return F, B
