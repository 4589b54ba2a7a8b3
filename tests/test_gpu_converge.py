"""GPU tests of the Jacobi order and of the convergence form of the level loop.

Jacobi with the fixed counts is compared element by element with the oracle's Jacobi order.  In
the convergence form the sweep count of a level is a decision taken on an energy computed from
float32 state on the device and from float64 state in the oracle, so near the threshold the two
can differ by one sweep: the test replays the device's counts in the oracle (a per-level schedule)
and compares the results element by element, and checks the counts against the oracle's own
decisions to within one sweep per level.
"""
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


def to_dev(torch, fge, p, s):
    dt = fge.storage_dtype(p)
    return (torch.from_numpy(s.I).to(dt).cuda(), torch.from_numpy(s.alpha).to(dt).cuda())


def inputs64(I, a):
    return I.double().cpu().numpy(), a.double().cpu().numpy()


def maxabs(x, y):
    return float(np.abs(x - y).max())


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("wh", [(64, 64), (1, 1), (5, 3), (300, 200), (257, 129), (1024, 768)])
def test_jacobi_fixed_counts_match_oracle(gpu, storage, wh):
    torch, fge = gpu
    W, H = wh
    p = fge.default_params(order=fge.JACOBI, storage=fge.F16 if storage == "f16" else fge.F32)
    s = synth.strands(W, H, seed=3 * W + H, n_strands=max(1, W * H // 4000))
    I, a = to_dev(torch, fge, p, s)
    F, B = fge.estimate_foreground(I, a, p)
    torch.cuda.synchronize()
    Fo, Bo = oracle.ml(*inputs64(I, a), order="jacobi")
    err = max(maxabs(F.double().cpu().numpy(), Fo), maxabs(B.double().cpu().numpy(), Bo))
    print(f"jacobi {W}x{H} {storage}: {err:.2e}")
    assert err <= TOL[storage]


@pytest.mark.parametrize("order", ["redblack", "jacobi"])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_converge_matches_oracle(gpu, order, storage):
    torch, fge = gpu
    p = fge.default_params(order=fge.JACOBI if order == "jacobi" else fge.REDBLACK,
                           storage=fge.F16 if storage == "f16" else fge.F32)
    s = synth.strands(300, 220, seed=41, n_strands=20)
    I, a = to_dev(torch, fge, p, s)
    tol = 1e-4
    F, B, sw = fge.estimate_foreground_converge(I, a, p, tol=tol, max_sweeps=300)
    torch.cuda.synchronize()
    sw = sw.cpu().tolist()
    I64, a64 = inputs64(I, a)
    Fo, Bo, swo = oracle.ml_converge(I64, a64, tol, 300, order=order)
    print(f"{order} {storage}: device sweeps {sw}, oracle sweeps {swo}")
    assert all(1 <= k <= 300 for k in sw)
    assert all(abs(x - y) <= 1 for x, y in zip(sw, swo))
    Fr, Br = oracle.ml_schedule(I64, a64, sw, order=order)
    err = max(maxabs(F.double().cpu().numpy(), Fr), maxabs(B.double().cpu().numpy(), Br))
    assert err <= TOL[storage], err
    if sw == swo:
        assert max(maxabs(F.double().cpu().numpy(), Fo), maxabs(B.double().cpu().numpy(), Bo)) <= TOL[storage]


def test_converge_limits_and_fixed_form(gpu):
    torch, fge = gpu
    p = fge.default_params()
    s = synth.smooth(200, 150, seed=5)
    I, a = to_dev(torch, fge, p, s)
    n = fge.num_levels(150, 200)
    F, B, sw = fge.estimate_foreground_converge(I, a, p, tol=1.0, max_sweeps=50)
    torch.cuda.synchronize()
    assert sw.cpu().tolist() == [1] * n
    Fr, Br = oracle.ml_schedule(*inputs64(I, a), [1] * n)
    assert max(maxabs(F.double().cpu().numpy(), Fr), maxabs(B.double().cpu().numpy(), Br)) <= 1e-4
    _, _, sw = fge.estimate_foreground_converge(I, a, p, tol=0.0, max_sweeps=3)
    torch.cuda.synchronize()
    assert sw.cpu().tolist() == [3] * n
    # tol < 0: the fixed counts, equal to the red-black oracle
    F, B, _ = fge.estimate_foreground_converge(I, a, p, tol=-1.0)
    torch.cuda.synchronize()
    Fo, Bo = oracle.ml(*inputs64(I, a))
    assert max(maxabs(F.double().cpu().numpy(), Fo), maxabs(B.double().cpu().numpy(), Bo)) <= 1e-4


def test_converge_is_asynchronous_and_repeatable(gpu):
    """Two back-to-back calls on one stream with no synchronisation in between give the same
    counts and bit-identical results (the stop flag is reset per level on the device)."""
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16)
    s = synth.smooth(333, 211, seed=6)
    I, a = to_dev(torch, fge, p, s)
    r1 = fge.estimate_foreground_converge(I, a, p, tol=1e-5, max_sweeps=100)
    r2 = fge.estimate_foreground_converge(I, a, p, tol=1e-5, max_sweeps=100)
    torch.cuda.synchronize()
    assert torch.equal(r1[2], r2[2]) and torch.equal(r1[0], r2[0]) and torch.equal(r1[1], r2[1])
