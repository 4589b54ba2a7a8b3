"""GPU tests of the smooth resize variant (area averaging of the image and matte, bilinear
resize of F and B) against the oracle's form of Algorithm 1 with the same variant.  With the
red-black order and fixed counts a level's sweeps run on the fused kernels (two sweeps per pass,
the tile kernel or, above 2^18 px, the streaming kernel; an odd count ends with one sweep on the
per-level kernels); otherwise on the per-level kernels."""
import numpy as np
import pytest

import oracle
from paper_2006_14970_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-4, "f16": 2e-3}


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need an MI355X"
    from paper_2006_14970_amd import fge
    fge.load()
    return torch, fge


def maxabs(x, y):
    return float(np.abs(x - y).max())


@pytest.mark.parametrize("order", ["redblack", "jacobi"])
@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("wh", [(1, 1), (5, 3), (64, 64), (300, 200), (257, 129), (1, 300), (1024, 768)])
def test_smooth_fixed_counts_match_oracle(gpu, order, storage, wh):
    torch, fge = gpu
    W, H = wh
    p = fge.default_params(storage=fge.F16 if storage == "f16" else fge.F32,
                           order=fge.JACOBI if order == "jacobi" else fge.REDBLACK)
    dt = fge.storage_dtype(p)
    s = synth.strands(W, H, seed=5 * W + H, n_strands=max(1, W * H // 4000))
    I = torch.from_numpy(s.I).to(dt).cuda()
    a = torch.from_numpy(s.alpha).to(dt).cuda()
    F, B, _ = fge.estimate_foreground_levels(I, a, p, resize="smooth")
    torch.cuda.synchronize()
    Fo, Bo = oracle.ml_resize(I.double().cpu().numpy(), a.double().cpu().numpy(), "smooth",
                              order=order)
    err = max(maxabs(F.double().cpu().numpy(), Fo), maxabs(B.double().cpu().numpy(), Bo))
    print(f"smooth {order} {storage} {W}x{H}: {err:.2e}")
    assert err <= TOL[storage]


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_smooth_converge_replays_in_oracle(gpu, storage):
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16 if storage == "f16" else fge.F32)
    dt = fge.storage_dtype(p)
    s = synth.strands(320, 240, seed=77, n_strands=20)
    I = torch.from_numpy(s.I).to(dt).cuda()
    a = torch.from_numpy(s.alpha).to(dt).cuda()
    F, B, sw = fge.estimate_foreground_levels(I, a, p, resize="smooth", tol=1e-4, max_sweeps=300)
    torch.cuda.synchronize()
    sw = sw.cpu().tolist()
    assert all(1 <= k <= 300 for k in sw)
    Fo, Bo = oracle.ml_resize(I.double().cpu().numpy(), a.double().cpu().numpy(), "smooth", sweeps=sw)
    err = max(maxabs(F.double().cpu().numpy(), Fo), maxabs(B.double().cpu().numpy(), Bo))
    print(f"smooth converge {storage}: sweeps {sw}, {err:.2e}")
    assert err <= TOL[storage]


def test_nearest_levels_equal_converge_path(gpu):
    torch, fge = gpu
    p = fge.default_params()
    s = synth.smooth(200, 150, seed=9)
    I = torch.from_numpy(s.I).float().cuda()
    a = torch.from_numpy(s.alpha).float().cuda()
    r1 = fge.estimate_foreground_levels(I, a, p, resize="nearest", tol=1e-4, max_sweeps=50)
    r2 = fge.estimate_foreground_converge(I, a, p, tol=1e-4, max_sweeps=50)
    torch.cuda.synchronize()
    assert torch.equal(r1[0], r2[0]) and torch.equal(r1[1], r2[1]) and torch.equal(r1[2], r2[2])


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("wh,strip_rows", [((300, 200), 0), ((1024, 768), 0), ((1024, 768), 11)])
def test_smooth_fused_passes_match_per_level_kernels(gpu, storage, wh, strip_rows):
    """The fused passes against the per-level kernels (kernel NAIVE) on the same input: the same
    sweeps in another rounding order, so equal to float32 rounding (in binary16 storage, up to
    one unit in the last place where a level's rounding differs), and both within the tolerance
    of the oracle."""
    torch, fge = gpu
    W, H = wh
    st = fge.F16 if storage == "f16" else fge.F32
    p = fge.default_params(storage=st, strip_rows=strip_rows)
    q = fge.default_params(storage=st, kernel=fge.KERNEL_NAIVE)
    dt = fge.storage_dtype(p)
    s = synth.strands(W, H, seed=7 * W + H, n_strands=max(1, W * H // 4000))
    I = torch.from_numpy(s.I).to(dt).cuda()
    a = torch.from_numpy(s.alpha).to(dt).cuda()
    F1, B1, _ = fge.estimate_foreground_levels(I, a, p, resize="smooth")
    F2, B2, _ = fge.estimate_foreground_levels(I, a, q, resize="smooth")
    torch.cuda.synchronize()
    d = max(float((F1.double() - F2.double()).abs().max()), float((B1.double() - B2.double()).abs().max()))
    print(f"fused vs per-level {storage} {W}x{H} rows {strip_rows}: {d:.2e}")
    assert d <= (1e-5 if storage == "f32" else 2e-3)
    Fo, Bo = oracle.ml_resize(I.double().cpu().numpy(), a.double().cpu().numpy(), "smooth")
    err = max(maxabs(F1.double().cpu().numpy(), Fo), maxabs(B1.double().cpu().numpy(), Bo))
    assert err <= TOL[storage]


@pytest.mark.parametrize("iters", [(3, 3), (10, 1), (4, 5)])
def test_smooth_fused_passes_any_sweep_count(gpu, iters):
    """Sweep counts other than 10 / 2: whole passes, then one per-level sweep for an odd count."""
    torch, fge = gpu
    W, H = 333, 211
    p = fge.default_params(iters_small=iters[0], iters_big=iters[1])
    s = synth.strands(W, H, seed=91, n_strands=20)
    I = torch.from_numpy(s.I).float().cuda()
    a = torch.from_numpy(s.alpha).float().cuda()
    F, B, _ = fge.estimate_foreground_levels(I, a, p, resize="smooth")
    torch.cuda.synchronize()
    sweeps = [k for _, _, k in oracle.level_plan(W, H, iters_small=iters[0], iters_big=iters[1])]
    Fo, Bo = oracle.ml_resize(I.double().cpu().numpy(), a.double().cpu().numpy(), "smooth",
                              sweeps=sweeps)
    err = max(maxabs(F.double().cpu().numpy(), Fo), maxabs(B.double().cpu().numpy(), Bo))
    print(f"smooth fused sweeps {iters}: {err:.2e}")
    assert err <= TOL["f32"]


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("wh", [(320, 240), (1024, 768), (1, 1), (97, 3)])
def test_smooth_converge_passes_replay_in_oracle(gpu, storage, wh):
    """The convergence form tested after every pass of two sweeps, on the fused kernels, with the
    smooth resize (passes=True): the result equals the oracle's smooth form run with the device's
    pass counts (two sweeps each), at 1024 x 768 with the streaming kernel on the last level."""
    torch, fge = gpu
    W, H = wh
    p = fge.default_params(storage=fge.F16 if storage == "f16" else fge.F32)
    dt = fge.storage_dtype(p)
    s = synth.strands(W, H, seed=11 * W + H, n_strands=max(1, W * H // 4000))
    I = torch.from_numpy(s.I).to(dt).cuda()
    a = torch.from_numpy(s.alpha).to(dt).cuda()
    F, B, ps = fge.estimate_foreground_levels(I, a, p, resize="smooth", tol=1e-4, max_sweeps=150,
                                              passes=True)
    ps = ps.cpu().tolist()
    assert len(ps) == fge.num_levels(H, W) and all(1 <= k <= 150 for k in ps)
    Fo, Bo = oracle.ml_resize(I.double().cpu().numpy(), a.double().cpu().numpy(), "smooth",
                              sweeps=[2 * k for k in ps])
    err = max(maxabs(F.double().cpu().numpy(), Fo), maxabs(B.double().cpu().numpy(), Bo))
    print(f"smooth converge passes {storage} {W}x{H}: passes {ps}, {err:.2e}")
    assert err <= TOL[storage]


def test_passes_option_limits_and_nearest(gpu):
    """passes=True: tol 1 stops every level after its first pass, tol 0 runs max_sweeps passes;
    with the nearest resize it is fge_estimate_foreground_converge_passes (same counts, same
    bits), in either order."""
    torch, fge = gpu
    p = fge.default_params()
    s = synth.smooth(200, 150, seed=12)
    I = torch.from_numpy(s.I).float().cuda()
    a = torch.from_numpy(s.alpha).float().cuda()
    n = fge.num_levels(150, 200)
    _, _, ps = fge.estimate_foreground_levels(I, a, p, resize="smooth", tol=1.0, max_sweeps=40,
                                              passes=True)
    assert ps.cpu().tolist() == [1] * n
    _, _, ps = fge.estimate_foreground_levels(I, a, p, resize="smooth", tol=0.0, max_sweeps=3,
                                              passes=True)
    assert ps.cpu().tolist() == [3] * n
    F1, B1, c1 = fge.estimate_foreground_levels(I, a, p, resize="nearest", tol=1e-4, max_sweeps=60,
                                                passes=True)
    F2, B2, c2 = fge.estimate_foreground_converge_passes(I, a, p, tol=1e-4, max_passes=60)
    torch.cuda.synchronize()
    assert c1.cpu().tolist() == list(c2) and torch.equal(F1, F2) and torch.equal(B1, B2)
    q = fge.default_params(order=fge.JACOBI)
    F1, B1, c1 = fge.estimate_foreground_levels(I, a, q, resize="nearest", tol=1e-4, max_sweeps=60,
                                                passes=True)
    F2, B2, c2 = fge.estimate_foreground_converge_passes(I, a, q, tol=1e-4, max_passes=60)
    torch.cuda.synchronize()
    assert c1.cpu().tolist() == list(c2) and torch.equal(F1, F2) and torch.equal(B1, B2)
