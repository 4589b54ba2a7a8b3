"""GPU parity: the HIP path through the C ABI against the FP64 oracle (red-black order).

Tolerances (max-abs over every F and B value in [0, 1]): 1e-4 with float32 storage, 2e-3 with
float16 storage.  The float16 comparison is against the oracle run on the original float64
inputs, so it covers input quantisation and the once-per-level rounding of F and B.
"""
import numpy as np
import pytest

import oracle
from paper_2006_14970_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-4, "f16": 2e-3}
_cache = {}


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need an MI355X"
    from paper_2006_14970_amd import fge
    fge.load()
    return torch, fge


def sample_of(name):
    if name not in _cache:
        s = {"c1": synth.config1, "c2": synth.config2, "c3": synth.config3}[name]()
        _cache[name] = s
    return _cache[name]


def oracle_of(name, order="redblack"):
    key = (name, order)
    if key not in _cache:
        s = sample_of(name)
        _cache[key] = oracle.ml(s.I, s.alpha, order=order)
    return _cache[key]


def run(gpu, I, alpha, **kw):
    torch, fge = gpu
    p = fge.default_params(**kw)
    dt = fge.storage_dtype(p)
    It = torch.from_numpy(np.ascontiguousarray(I)).to(dt).cuda()
    at = torch.from_numpy(np.ascontiguousarray(alpha)).to(dt).cuda()
    F, B = fge.estimate_foreground(It, at, p)
    torch.cuda.synchronize()
    return F.double().cpu().numpy(), B.double().cpu().numpy()


def maxabs(a, b):
    return float(np.abs(a - b).max())


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_configs_match_oracle(gpu, name, storage):
    torch, fge = gpu
    s = sample_of(name)
    Fo, Bo = oracle_of(name)
    F, B = run(gpu, s.I, s.alpha, storage=fge.F16 if storage == "f16" else fge.F32)
    err = max(maxabs(F, Fo), maxabs(B, Bo))
    print(f"{name} {storage}: max-abs vs FP64 oracle = {err:.3e}")
    assert err <= TOL[storage]
    assert F.min() >= 0 and F.max() <= 1 and B.min() >= 0 and B.max() <= 1
    if storage == "f32":
        e_gpu = oracle.energy(F, B, s.I, s.alpha)
        e_rb = oracle.energy(Fo, Bo, s.I, s.alpha)
        print(f"{name}: final energy GPU {e_gpu:.6f}, oracle red-black {e_rb:.6f}")
        assert abs(e_gpu - e_rb) <= 1e-4 * e_rb


def test_f16_against_rounded_inputs(gpu):
    """Separates input quantisation from kernel error: oracle on float16-rounded inputs."""
    torch, fge = gpu
    s = sample_of("c2")
    I16 = s.I.astype(np.float16).astype(np.float64)
    a16 = s.alpha.astype(np.float16).astype(np.float64)
    Fo, Bo = oracle.ml(I16, a16)
    F, B = run(gpu, s.I, s.alpha, storage=fge.F16)
    err = max(maxabs(F, Fo), maxabs(B, Bo))
    print(f"c2 f16 vs oracle on f16-rounded inputs: {err:.3e}")
    assert err <= TOL["f16"]


RAGGED = [(1, 1), (2, 1), (1, 2), (3, 5), (5, 3), (1, 300), (300, 1), (2, 700), (33, 33),
          (64, 65), (65, 64), (127, 40), (128, 40), (129, 41), (130, 9), (247, 130), (248, 131),
          (249, 132), (250, 3), (368, 101), (369, 77), (600, 401), (1001, 257), (257, 1003)]


@pytest.mark.parametrize("wh", RAGGED)
def test_ragged_sizes(gpu, wh):
    W, H = wh
    s = synth.smooth(W, H, seed=700 + W + 3 * H)
    Fo, Bo = oracle.ml(s.I, s.alpha)
    F, B = run(gpu, s.I, s.alpha)
    err = max(maxabs(F, Fo), maxabs(B, Bo))
    assert err <= TOL["f32"], (W, H, err)


@pytest.mark.parametrize("wh", [(700, 500), (129, 300), (40, 1000)])
def test_strands_sizes_f16(gpu, wh):
    torch, fge = gpu
    W, H = wh
    s = synth.strands(W, H, seed=900 + W, n_strands=W * H // 4000)
    Fo, Bo = oracle.ml(s.I, s.alpha)
    F, B = run(gpu, s.I, s.alpha, storage=fge.F16)
    assert max(maxabs(F, Fo), maxabs(B, Bo)) <= TOL["f16"]


def test_strip_rows_do_not_change_results(gpu):
    """Streaming kernel on every fine level: every stored pixel goes through the same arithmetic
    whatever the strip height, so the output is bit-identical across strip heights (only halo
    work differs), and it matches the oracle."""
    torch, fge = gpu
    s = sample_of("c2")
    Fo, Bo = oracle_of("c2")
    ref = run(gpu, s.I, s.alpha, strip_rows=0, tile_max_px=-1)
    assert max(maxabs(ref[0], Fo), maxabs(ref[1], Bo)) <= TOL["f32"]
    for rows in (1, 2, 3, 8, 13, 64, 400, 768):
        F, B = run(gpu, s.I, s.alpha, strip_rows=rows, tile_max_px=-1)
        assert np.array_equal(F, ref[0]) and np.array_equal(B, ref[1]), rows


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_fine_kernel_choices_match_oracle(gpu, storage):
    """Tile kernel on every fine level, streaming kernel on every fine level, and the default
    split, each against the oracle."""
    torch, fge = gpu
    st = fge.F16 if storage == "f16" else fge.F32
    s = sample_of("c2")
    Fo, Bo = oracle_of("c2")
    for kw in ({"tile_max_px": 1 << 30}, {"tile_max_px": -1}, {"tile_max_px": 0},
               {"tile_max_px": 100000}):
        F, B = run(gpu, s.I, s.alpha, storage=st, **kw)
        assert max(maxabs(F, Fo), maxabs(B, Bo)) <= TOL[storage], kw


@pytest.mark.parametrize("wh", [(33, 35), (65, 64), (100, 37), (129, 130), (300, 7), (7, 300),
                                (511, 259), (1001, 257)])
def test_tile_kernel_ragged(gpu, wh):
    W, H = wh
    s = synth.strands(W, H, seed=300 + W, n_strands=max(1, W * H // 3000))
    Fo, Bo = oracle.ml(s.I, s.alpha)
    for kw in ({"tile_max_px": 1 << 30}, {"tile_max_px": -1}):
        F, B = run(gpu, s.I, s.alpha, **kw)
        assert max(maxabs(F, Fo), maxabs(B, Bo)) <= TOL["f32"], (wh, kw)


def test_naive_path_matches_oracle(gpu):
    torch, fge = gpu
    for name in ("c1", "c2"):
        s = sample_of(name)
        Fo, Bo = oracle_of(name)
        F, B = run(gpu, s.I, s.alpha, kernel=fge.KERNEL_NAIVE)
        assert max(maxabs(F, Fo), maxabs(B, Bo)) <= TOL["f32"], name


def test_without_coarse_kernel(gpu):
    """Every level through the per-level kernels (coarse levels on the naive path)."""
    torch, fge = gpu
    s = sample_of("c2")
    Fo, Bo = oracle_of("c2")
    F, B = run(gpu, s.I, s.alpha, coarse_max_px=-1)
    assert max(maxabs(F, Fo), maxabs(B, Bo)) <= TOL["f32"]
    F2, B2 = run(gpu, s.I, s.alpha, coarse_max_px=256)
    assert max(maxabs(F2, Fo), maxabs(B2, Bo)) <= TOL["f32"]


def test_nondefault_parameters(gpu):
    s = synth.strands(300, 200, seed=31, n_strands=20)
    for kw in ({"omega": 0.0, "eps_r": 0.05}, {"omega": 1.0, "eps_r": 1e-3},
               {"iters_small": 3, "small_size": 64}):
        Fo, Bo = oracle.ml(s.I, s.alpha, omega=kw.get("omega", 0.1), eps=kw.get("eps_r", 5e-3),
                           small_size=kw.get("small_size", 32), iters_small=kw.get("iters_small", 10))
        F, B = run(gpu, s.I, s.alpha, **kw)
        assert max(maxabs(F, Fo), maxabs(B, Bo)) <= TOL["f32"], kw


def test_deterministic(gpu):
    s = sample_of("c2")
    a = run(gpu, s.I, s.alpha)
    b = run(gpu, s.I, s.alpha)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_alpha_complement_swaps(gpu):
    s = synth.smooth(333, 222, seed=41)
    F, B = run(gpu, s.I, s.alpha)
    F2, B2 = run(gpu, s.I, 1.0 - s.alpha)
    assert maxabs(F2, B) <= 1e-5 and maxabs(B2, F) <= 1e-5


def test_constant_image(gpu):
    rng = np.random.default_rng(3)
    H, W = 211, 307
    c = np.array([0.2, 0.55, 0.9])
    I = np.broadcast_to(c[:, None, None], (3, H, W)).copy()
    a = rng.uniform(0, 1, (H, W))
    Fo, Bo = oracle.ml(I, a)
    F, B = run(gpu, I, a)
    assert max(maxabs(F, Fo), maxabs(B, Bo)) <= TOL["f32"]


def test_orders_by_energy(gpu):
    """Red-black (GPU) and the paper's raster order reach close energies on the full image."""
    s = sample_of("c2")
    F, B = run(gpu, s.I, s.alpha)
    Fr, Br = oracle_of("c2", "raster")
    e_gpu = oracle.energy(F, B, s.I, s.alpha)
    e_raster = oracle.energy(Fr, Br, s.I, s.alpha)
    print(f"c2 final energy: GPU red-black {e_gpu:.6f}, oracle raster {e_raster:.6f}")
    assert abs(e_gpu - e_raster) <= 0.02 * e_raster


def test_runtime_errors(gpu):
    torch, fge = gpu
    s = synth.smooth(300, 200, seed=5)
    p = fge.default_params()
    I = torch.from_numpy(s.I).float().cuda()
    a = torch.from_numpy(s.alpha).float().cuda()
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(fge.FgeError) as e:
        fge.estimate_foreground(I, a, p, workspace=small)
    assert e.value.status == fge.FGE_EWORKSPACE
    with pytest.raises(ValueError):
        fge.estimate_foreground(I.half(), a.half(), p)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_paired_input_path(gpu, storage):
    """Streaming levels with an even width and the identity input map whose previous level is not
    exactly half as wide (1000 -> 501, 1920 -> 966, 1366 -> 709, 2000 -> 1002): paired loads of
    I and alpha and paired stores, per-pixel reads of the previous level."""
    torch, fge = gpu
    for k, (W, H) in enumerate(((1000, 600), (1920, 1080), (1366, 768), (2000, 300))):
        s = synth.strands(W, H, seed=1200 + k, n_strands=W * H // 4000)
        Fo, Bo = oracle.ml(s.I, s.alpha, parallel=True)
        F, B = run(gpu, s.I, s.alpha, storage=fge.F16 if storage == "f16" else fge.F32)
        err = max(maxabs(F, Fo), maxabs(B, Bo))
        assert err <= TOL[storage], (W, H, err)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_paired_input_path_odd_width(gpu, storage):
    """Odd widths on the paired paths: interior strips and the first strip pair their columns
    (the pair of an odd row then starts on an odd element), the last strip, which starts on an
    odd column, stays unpaired.  Widths with several interior strips, one interior strip and
    none (247 = two border strips only), heights odd and even; every finest level is above the
    tile kernel's 256K-pixel limit, so it streams."""
    torch, fge = gpu
    for k, (W, H) in enumerate(((1001, 600), (1921, 1081), (4001, 150), (247, 1201), (301, 1001))):
        s = synth.strands(W, H, seed=1300 + k, n_strands=max(1, W * H // 4000))
        Fo, Bo = oracle.ml(s.I, s.alpha, parallel=True)
        F, B = run(gpu, s.I, s.alpha, storage=fge.F16 if storage == "f16" else fge.F32)
        err = max(maxabs(F, Fo), maxabs(B, Bo))
        assert err <= TOL[storage], (W, H, err)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_raw_abi_non_square_height_first(gpu, storage):
    """The C symbol called through ctypes directly (not the Python wrapper), with a non-square
    image whose sizes are passed in the ABI's (H, W) order: 301 rows of 700 pixels.  A caller
    that swapped them would get a transposed plan; the result must match the oracle."""
    import ctypes
    torch, fge = gpu
    H, W = 301, 700
    s = synth.smooth(W, H, seed=4242)
    assert s.I.shape == (3, H, W)
    Fo, Bo = oracle.ml(s.I, s.alpha)
    p = fge.default_params(storage=fge.F16 if storage == "f16" else fge.F32)
    dt = fge.storage_dtype(p)
    It = torch.from_numpy(np.ascontiguousarray(s.I)).to(dt).cuda()
    at = torch.from_numpy(np.ascontiguousarray(s.alpha)).to(dt).cuda()
    F = torch.empty((3, H, W), dtype=dt, device="cuda")
    B = torch.empty_like(F)
    lib = ctypes.CDLL(fge.LIB_PATH)
    lib.fge_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    lib.fge_workspace_bytes.restype = ctypes.c_size_t
    lib.fge_estimate_foreground.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.c_void_p]
    lib.fge_estimate_foreground.restype = ctypes.c_int
    need = lib.fge_workspace_bytes(H, W, ctypes.addressof(p))
    ws = torch.empty(max(1, need), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.fge_estimate_foreground(It.data_ptr(), at.data_ptr(), H, W, ctypes.addressof(p),
                                     F.data_ptr(), B.data_ptr(), ws.data_ptr(), need, stream)
    assert st == 0, st
    torch.cuda.synchronize()
    err = max(maxabs(F.double().cpu().numpy(), Fo), maxabs(B.double().cpu().numpy(), Bo))
    print(f"raw ABI {H}x{W} {storage}: max-abs vs oracle {err:.3e}")
    assert err <= TOL[storage]


def test_side_stream_scratch_survives_default_stream_allocations(gpu):
    """estimate_foreground on a side stream with a library-allocated workspace: after the call
    returns, memory freed and reallocated on the default stream must not reuse the workspace
    while the side stream still runs (the binding marks it in use by that stream)."""
    torch, fge = gpu
    s = sample_of("c2")
    Fo, Bo = oracle_of("c2")
    p = fge.default_params()
    It = torch.from_numpy(np.ascontiguousarray(s.I)).float().cuda()
    at = torch.from_numpy(np.ascontiguousarray(s.alpha)).float().cuda()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    # keep the side stream busy first so the estimation is still queued when the scratch is freed
    with torch.cuda.stream(side):
        busy = torch.randn(1 << 24, device="cuda")
        for _ in range(20):
            busy = busy * 1.0000001 + 0.5
    F, B = fge.estimate_foreground(It, at, p, stream=side)
    junk = [torch.full((1 << 22,), 7.0, device="cuda") for _ in range(8)]   # default stream
    side.synchronize()
    torch.cuda.synchronize()
    err = max(maxabs(F.double().cpu().numpy(), Fo), maxabs(B.double().cpu().numpy(), Bo))
    assert err <= TOL["f32"], err
    del junk, busy
