"""GPU: the closed-form solve of eq. 2 (fge_closed_form, block-Jacobi PCG in float64 on the
device) against the oracle's sparse direct solve of the same normal equations
(oracle/closed_form.py), element by element, and against the paper's stopping measure, the
relative residual |b - A x| / |b| per channel (the remark after eq. 2 quotes 1e-6), recomputed by
the oracle from the returned F, B.

Tolerances.  A CG iterate with relative residual rho is within |A^-1| rho |b| of the minimiser;
the condition number of these systems grows with the image (the smallest eigenvalue is about
eps (pi / side)^2), so element-wise comparisons run at a tight tolerance (1e-12) where the
float64 solve error is below 1e-8, and the bars below are then set by the storage rounding:
float64 storage 1e-6, float32 storage 1e-5 (2^-24 of values up to ~1.5, plus the solve), float16
storage 2e-3 (2^-11 of the same, against the oracle on float16-rounded inputs).  At the paper's
1e-6 the result is checked by its residual, which the oracle computes from the float64 output.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from oracle import closed_form as cf
from paper_2006_14970_amd import synth

pytestmark = pytest.mark.gpu

_cache = {}


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need an MI355X"
    from paper_2006_14970_amd import fge
    fge.load()
    return torch, fge


def sample(kind, W, H):
    key = ("s", kind, W, H)
    if key not in _cache:
        if kind == "smooth":
            _cache[key] = synth.smooth(W, H, seed=900 + W + 7 * H)
        elif kind == "random":
            rng = np.random.default_rng(970 + W + 7 * H)
            _cache[key] = _random_sample(rng, W, H)
        elif kind == "strands":
            _cache[key] = synth.strands(W, H, seed=950 + W + 7 * H,
                                        n_strands=max(1, 200 * W * H // (1024 * 768)))
        else:   # config 2: the 1024x768 strand image
            _cache[key] = synth.config2()
    return _cache[key]


def _random_sample(rng, W, H):
    """Uniform random image and matte (tiny sizes, where the generators' mattes are constant)."""
    return SimpleNamespace(I=rng.random((3, H, W)), alpha=rng.random((H, W)))


def oracle_solve(kind, W, H, I=None, alpha=None, tag=""):
    key = ("o", kind, W, H, tag)
    if key not in _cache:
        s = sample(kind, W, H)
        _cache[key] = cf.solve(s.I if I is None else I, s.alpha if alpha is None else alpha,
                               1.0, 5e-3)
    return _cache[key]


def run(gpu, I, alpha, dt="f64", F0=None, B0=None, **kw):
    torch, fge = gpu
    storage = {"f64": fge.F64, "f32": fge.F32, "f16": fge.F16}[dt]
    tdt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}[dt]
    p = fge.cf_default_params(storage=storage, **kw)
    It = torch.from_numpy(np.ascontiguousarray(I)).to(tdt).cuda()
    at = torch.from_numpy(np.ascontiguousarray(alpha)).to(tdt).cuda()
    F = B = None
    if F0 is not None:
        F = torch.from_numpy(np.ascontiguousarray(F0)).to(tdt).cuda()
        B = torch.from_numpy(np.ascontiguousarray(B0)).to(tdt).cuda()
    F, B, info = fge.closed_form(It, at, p, F=F, B=B)
    torch.cuda.synchronize()
    return F.double().cpu().numpy(), B.double().cpu().numpy(), info


def maxabs(a, b):
    return float(np.abs(a - b).max())


SHAPES = [("smooth", 64, 64), ("strands", 256, 192), ("smooth", 97, 61), ("smooth", 700, 301),
          ("random", 2, 1), ("random", 1, 2), ("smooth", 1, 300), ("smooth", 300, 1),
          ("smooth", 63, 5), ("smooth", 125, 3)]


@pytest.mark.parametrize("kind,W,H", SHAPES)
def test_matches_direct_solve_float64(gpu, kind, W, H):
    """Tight tolerance, float64 storage: the iterate is the oracle's minimiser to 1e-6 max-abs
    (sizes span several spmv strips in x and y and ragged tails; 1 x N and N x 1 edge cases)."""
    s = sample(kind, W, H)
    Fo, Bo = oracle_solve(kind, W, H)
    F, B, info = run(gpu, s.I, s.alpha, "f64", tol=1e-12)
    err = max(maxabs(F, Fo), maxabs(B, Bo))
    print(f"{W}x{H}: {info['iterations']} iterations, max-abs vs direct solve {err:.2e}")
    assert info["converged"] and not info["breakdown"]
    assert err <= 1e-6, err
    assert max(info["rel_residual"]) <= 1e-11


@pytest.mark.parametrize("kind,W,H", [("smooth", 64, 64), ("strands", 256, 192),
                                      ("c2", 1024, 768)])
def test_paper_residual_criterion(gpu, kind, W, H):
    """At the paper's 1e-6 the stored (float64) result's relative residual per channel, recomputed
    by the oracle from the assembled matrix, is at most 1e-6 and equals the device's own figure."""
    s = sample(kind, W, H)
    F, B, info = run(gpu, s.I, s.alpha, "f64", tol=1e-6)
    res = cf.relative_residuals(s.I, s.alpha, F, B, 1.0, 5e-3)
    print(f"{W}x{H}: iterations {info['channel_iterations']}, residuals {res}")
    assert info["converged"]
    assert np.all(res <= 1e-6), res
    assert np.allclose(res, info["rel_residual"], rtol=1e-6, atol=0), (res, info["rel_residual"])
    # the recurrence's own residual stopped it; the recomputed one agrees to rounding
    assert np.allclose(info["recursive_rel_residual"], res, rtol=1e-3)


@pytest.mark.timeout(900)
def test_config2_matches_direct_solve(gpu):
    """The 1024 x 768 strand workload against the oracle's direct solve (about a minute of CPU),
    float64 storage (float32 storage is compared at 256 x 192 below)."""
    s = sample("c2", 1024, 768)
    Fo, Bo = oracle_solve("c2", 1024, 768)
    F, B, info = run(gpu, s.I, s.alpha, "f64", tol=1e-12)
    err = max(maxabs(F, Fo), maxabs(B, Bo))
    print(f"1024x768 f64: {info['iterations']} iterations, max-abs {err:.2e}")
    assert info["converged"] and err <= 1e-6, err


@pytest.mark.parametrize("kind,W,H", [("strands", 256, 192), ("smooth", 97, 61)])
def test_float32_and_float16_storage(gpu, kind, W, H):
    """Reduced storage: the inputs are read as stored, so the oracle solves on the rounded inputs;
    the bar is the rounding of the stored output."""
    s = sample(kind, W, H)
    for dt, np_dt, tol in (("f32", np.float32, 1e-5), ("f16", np.float16, 2e-3)):
        I = s.I.astype(np_dt).astype(np.float64)
        a = s.alpha.astype(np_dt).astype(np.float64)
        Fo, Bo = oracle_solve(kind, W, H, I, a, tag=dt)
        F, B, info = run(gpu, s.I, s.alpha, dt, tol=1e-12)
        err = max(maxabs(F, Fo), maxabs(B, Bo))
        print(f"{W}x{H} {dt}: max-abs vs direct solve on rounded inputs {err:.2e}")
        assert info["converged"] and err <= tol, (dt, err)


def test_constant_matte_singular_system(gpu):
    """A matte constant over the whole image leaves A singular (the direction orthogonal to
    (a, 1 - a), constant over the image, is in its null space); b is in A's range, so CG still
    reaches a minimiser: the residual is what is checked (the minimiser is not unique)."""
    rng = np.random.default_rng(11)
    for W, H in ((2, 1), (1, 2), (40, 30)):
        I = rng.random((3, H, W))
        a = np.full((H, W), 0.4)
        F, B, info = run(gpu, I, a, "f64", tol=1e-10)
        res = cf.relative_residuals(I, a, F, B, 1.0, 5e-3)
        assert info["converged"] and np.all(res <= 1e-10), (W, H, res)


def test_constant_image_and_complement(gpu):
    """A constant image is its own solution (F = B = c for any matte: U (U . c) = U c = b), and
    alpha -> 1 - alpha swaps F and B."""
    rng = np.random.default_rng(7)
    H, W = 70, 90
    c = np.array([0.2, 0.55, 0.9])
    I = np.broadcast_to(c[:, None, None], (3, H, W)).copy()
    a = rng.uniform(0, 1, (H, W))
    F, B, info = run(gpu, I, a, "f64", tol=1e-12)
    assert info["converged"]
    assert maxabs(F, I) <= 1e-10 and maxabs(B, I) <= 1e-10
    s = sample("smooth", 97, 61)
    F1, B1, _ = run(gpu, s.I, s.alpha, "f64", tol=1e-12)
    F2, B2, _ = run(gpu, s.I, 1.0 - s.alpha, "f64", tol=1e-12)
    assert maxabs(F1, B2) <= 1e-8 and maxabs(B1, F2) <= 1e-8


def test_warm_start_from_multilevel_estimate(gpu):
    """Starting from the multi-level estimate (Algorithm 1 on the GPU) reaches the same minimiser."""
    torch, fge = gpu
    s = sample("strands", 256, 192)
    Fo, Bo = oracle_solve("strands", 256, 192)
    It = torch.from_numpy(s.I).float().cuda()
    at = torch.from_numpy(s.alpha).float().cuda()
    Fm, Bm = fge.estimate_foreground(It, at, fge.default_params(omega=1.0))
    torch.cuda.synchronize()
    F0, B0 = Fm.double().cpu().numpy(), Bm.double().cpu().numpy()
    _, _, cold = run(gpu, s.I, s.alpha, "f64", tol=1e-6)
    F, B, warm = run(gpu, s.I, s.alpha, "f64", F0=F0, B0=B0, tol=1e-12, warm_start=1)
    print(f"iterations to 1e-6: cold {cold['iterations']}; warm start to 1e-12 {warm['iterations']}")
    assert warm["converged"]
    assert max(maxabs(F, Fo), maxabs(B, Bo)) <= 1e-6


def test_deterministic_and_iteration_cap(gpu):
    s = sample("strands", 256, 192)
    F1, B1, i1 = run(gpu, s.I, s.alpha, "f64", tol=1e-8)
    F2, B2, i2 = run(gpu, s.I, s.alpha, "f64", tol=1e-8)
    i1.pop("device_ms")
    i2.pop("device_ms")
    assert np.array_equal(F1, F2) and np.array_equal(B1, B2) and i1 == i2
    F, B, info = run(gpu, s.I, s.alpha, "f64", tol=1e-8, max_iter=5)
    assert not info["converged"] and info["iterations"] == 5
    res = cf.relative_residuals(s.I, s.alpha, F, B, 1.0, 5e-3)
    assert np.allclose(res, info["rel_residual"], rtol=1e-6)
