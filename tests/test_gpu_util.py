"""GPU tests of the reporting and layout kernels: the device energy against the oracle's FP64
energy, the residual statistics against a plain NumPy evaluation, and the layout conversions
bit-exact against NumPy's casts."""
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
    return torch, fge


@pytest.mark.parametrize("wh", [(1, 1), (7, 3), (300, 200), (1024, 768), (129, 1000)])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_energy_matches_oracle(gpu, wh, storage):
    torch, fge = gpu
    W, H = wh
    p = fge.default_params(storage=fge.F16 if storage == "f16" else fge.F32, omega=0.3, eps_r=0.01)
    dt = fge.storage_dtype(p)
    s = synth.strands(W, H, seed=W + H, n_strands=max(1, W * H // 4000))
    I = torch.from_numpy(s.I).to(dt).cuda()
    a = torch.from_numpy(s.alpha).to(dt).cuda()
    F, B = fge.estimate_foreground(I, a, p)
    out = fge.energy(I, a, F, B, p).cpu().numpy()
    I64, a64 = I.double().cpu().numpy(), a.double().cpu().numpy()
    F64, B64 = F.double().cpu().numpy(), B.double().cpu().numpy()
    e = oracle.energy(F64, B64, I64, a64, omega=float(np.float32(0.3)), eps=float(np.float32(0.01)))
    # The oracle adds its ~6 W H terms one after the other into one float64 accumulator; its own
    # rounding grows with the term count (~1e-12 relative at 1024x768).  A missing or doubled
    # edge moves E by 1e-8 relative or more.
    rel = max(1e-12, 2e-17 * 6 * W * H)
    assert abs(out[0] - e) <= rel * max(1.0, abs(e)), (out[0], e)
    assert abs(out[1] + out[2] - out[0]) <= 1e-12 * max(1.0, abs(e))
    r = np.abs(a64[None] * F64 + (1 - a64[None]) * B64 - I64)
    frac = (a64 > 0) & (a64 < 1)
    assert out[5] == frac.sum()
    if frac.any():
        rf = r[:, frac]
        assert abs(out[3] - rf.sum() / frac.sum()) <= 1e-12
        assert abs(out[4] - rf.max()) <= 1e-14   # the device may contract a*F + b*B into an FMA
    data = float(((a64[None] * F64 + (1 - a64[None]) * B64 - I64) ** 2).sum())
    assert abs(out[1] - data) <= rel * max(1.0, data)


def test_layout_conversions_bit_exact(gpu):
    torch, fge = gpu
    rng = np.random.default_rng(11)
    H, W = 37, 53
    u8 = rng.integers(0, 256, size=(H, W, 4), dtype=np.uint8)
    img = torch.from_numpy(u8).cuda()
    I, a = fge.hwc_to_planar(img, torch.float32)
    ref = u8.astype(np.float32) / np.float32(255.0)
    assert np.array_equal(I.cpu().numpy(), np.moveaxis(ref[..., :3], 2, 0))
    assert np.array_equal(a.cpu().numpy(), ref[..., 3])
    I16, a16 = fge.hwc_to_planar(img[..., :3].contiguous(), torch.float16)
    assert a16 is None
    assert np.array_equal(I16.cpu().numpy(), np.moveaxis(ref[..., :3], 2, 0).astype(np.float16))
    f = rng.uniform(-0.2, 1.2, size=(3, H, W)).astype(np.float32)
    ft = torch.from_numpy(f).cuda()
    back = fge.planar_to_hwc(ft).cpu().numpy()
    want = np.round(np.clip(np.moveaxis(f, 0, 2), 0, 1) * np.float32(255.0)).astype(np.uint8)
    assert np.array_equal(back, want)
    hf = fge.planar_to_hwc(ft, torch.float16).cpu().numpy()
    assert np.array_equal(hf, np.moveaxis(f, 0, 2).astype(np.float16))
    # the round trip of 8-bit values is exact
    rt = fge.planar_to_hwc(I).cpu().numpy()
    assert np.array_equal(rt, u8[..., :3])


@pytest.mark.parametrize("wh", [(1, 1), (3, 2), (19, 13), (300, 200), (1024, 768)])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_quality_matches_oracle(gpu, wh, storage):
    torch, fge = gpu
    from oracle import metrics
    W, H = wh
    dt = torch.float16 if storage == "f16" else torch.float32
    s = synth.strands(W, H, seed=W + 2 * H, n_strands=max(1, W * H // 4000))
    rng = np.random.default_rng(W * H)
    a = torch.from_numpy(np.clip(s.alpha + rng.uniform(-0.05, 0.05, s.alpha.shape), 0, 1)).to(dt).cuda()
    G = torch.from_numpy(s.F).to(dt).cuda()
    F = torch.from_numpy(np.clip(s.F + rng.normal(0, 0.05, s.F.shape), 0, 1)).to(dt).cuda()
    out = fge.quality(F, G, a).cpu().numpy()
    sad, mse, grad, n = metrics.quality(F.double().cpu().numpy(), G.double().cpu().numpy(),
                                        a.double().cpu().numpy())
    print(f"{W}x{H} {storage}: SAD {out[0]:.6g} MSE {out[1]:.6g} GRAD {out[2]:.6g} n {out[3]:.0f}")
    assert out[3] == n
    for got, want in ((out[0], sad), (out[1], mse), (out[2], grad)):
        assert abs(got - want) <= 1e-10 * max(1e-30, abs(want)), (got, want)


@pytest.mark.parametrize("sigma", [0.5, 1.9, 2.2, 3.5])
def test_quality_filter_radius(gpu, sigma):
    """Filter radii int(4 sigma + 0.5) of 2 and 8 (the tiled kernel's smallest and largest) and 9
    and 14 (the direct sum), on a size with ragged tiles (70 x 37) and one smaller than the
    radius (5 x 4, mirrored borders folding more than once)."""
    torch, fge = gpu
    from oracle import metrics
    for W, H in ((70, 37), (5, 4)):
        s = synth.strands(W, H, seed=5 * W + H, n_strands=2)
        rng = np.random.default_rng(W + H)
        a = torch.from_numpy(np.clip(s.alpha + rng.uniform(-0.05, 0.05, s.alpha.shape), 0, 1)).float().cuda()
        G = torch.from_numpy(s.F).float().cuda()
        F = torch.from_numpy(np.clip(s.F + rng.normal(0, 0.05, s.F.shape), 0, 1)).float().cuda()
        out = fge.quality(F, G, a, sigma=sigma).cpu().numpy()
        want = metrics.quality(F.double().cpu().numpy(), G.double().cpu().numpy(),
                               a.double().cpu().numpy(), sigma)
        assert out[3] == want[3]
        for got, w in zip(out[:3], want[:3]):
            assert abs(got - w) <= 1e-10 * max(1e-30, abs(w)), (sigma, W, H, got, w)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_composite_bit_exact(gpu, storage):
    torch, fge = gpu
    from oracle import metrics
    dt = torch.float16 if storage == "f16" else torch.float32
    rng = np.random.default_rng(12)
    H, W = 77, 131
    F = torch.from_numpy(rng.uniform(0, 1, (3, H, W))).to(dt).cuda()
    a = torch.from_numpy(rng.uniform(0, 1, (H, W))).to(dt).cuda()
    B = torch.from_numpy(rng.uniform(0, 1, (3, H, W))).to(dt).cuda()
    C = fge.composite(F, a, B).cpu().numpy()
    want = metrics.composite(F.double().cpu().numpy(), a.double().cpu().numpy(),
                             B.double().cpu().numpy()).astype(np.float16 if storage == "f16" else np.float32)
    assert np.array_equal(C, want)
