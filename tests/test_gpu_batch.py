"""GPU: batched uneven-size images (persistent kernels, per-step work queues, hipGraph).

Every batched image follows its own level plan through the same kernel bodies as the
single-image path, so its F and B must be bit-identical to fge_estimate_foreground's; a few are
also checked against the FP64 oracle.
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


def inputs(torch, fge, samples, params):
    dt = fge.storage_dtype(params)
    Is = [torch.from_numpy(s.I).to(dt).cuda() for s in samples]
    As = [torch.from_numpy(s.alpha).to(dt).cuda() for s in samples]
    return Is, As


def single(torch, fge, I, a, params):
    F, B = fge.estimate_foreground(I, a, params)
    return F, B


SIZES = [(1, 1), (3, 2), (37, 64), (64, 37), (129, 300), (300, 129), (257, 255), (700, 421),
         (1000, 77), (16, 900), (520, 520), (128, 128)]


# Single images whose run of tile levels is one pyramid launch: runs of 2 to 5 levels, regions
# near the 40x40 limit (level ratios well below 2 on one axis), and a run that ends at the
# finest level (images too small to stage their inputs in F).
PYRAMID_SIZES = [(65, 65), (300, 7000), (7000, 300), (517, 1029), (1001, 257), (640, 480),
                 (1920, 1080), (3001, 2999)]


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_pyramid_bit_identical_to_per_level_tiles(gpu, storage):
    """The single-image path runs its tile levels as one pyramid launch (lower levels recomputed
    in LDS per output tile); a batch of one image runs the same levels one launch each.  The
    stored results must be the same bits, and match the oracle."""
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16 if storage == "f16" else fge.F32)
    for k, (w, h) in enumerate(PYRAMID_SIZES):
        s = synth.smooth(w, h, seed=950 + k)
        Is, As = inputs(torch, fge, [s], p)
        F1, B1 = single(torch, fge, Is[0], As[0], p)
        b = fge.Batch([(h, w)], p)
        Fs, Bs = b.run(Is, As)
        torch.cuda.synchronize()
        assert torch.equal(Fs[0], F1) and torch.equal(Bs[0], B1), (w, h)
        b.close()
        if w * h <= 1 << 20:
            Fo, Bo = oracle.ml(s.I, s.alpha, parallel=True)
            err = max(float(np.abs(F1.cpu().numpy().astype(np.float64) - Fo).max()),
                      float(np.abs(B1.cpu().numpy().astype(np.float64) - Bo).max()))
            assert err <= TOL[storage], (w, h, err)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batch_bit_identical_to_single(gpu, storage):
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16 if storage == "f16" else fge.F32)
    samples = [synth.strands(w, h, seed=60 + i, n_strands=max(1, w * h // 3000))
               for i, (w, h) in enumerate(SIZES)]
    Is, As = inputs(torch, fge, samples, p)
    b = fge.Batch([(h, w) for w, h in SIZES], p)
    Fs, Bs = b.run(Is, As)
    torch.cuda.synchronize()
    for i in range(len(SIZES)):
        F1, B1 = single(torch, fge, Is[i], As[i], p)
        torch.cuda.synchronize()
        assert torch.equal(Fs[i], F1) and torch.equal(Bs[i], B1), SIZES[i]
    for i in (2, 5, 7):
        s = samples[i]
        Fo, Bo = oracle.ml(s.I, s.alpha)
        err = max(float((Fs[i].double().cpu() - torch.from_numpy(Fo)).abs().max()),
                  float((Bs[i].double().cpu() - torch.from_numpy(Bo)).abs().max()))
        assert err <= TOL[storage], (SIZES[i], err)
    b.close()


def test_batch_run_twice_reuses_plan(gpu):
    torch, fge = gpu
    p = fge.default_params()
    sizes = SIZES[:6]
    samples = [synth.smooth(w, h, seed=80 + i) for i, (w, h) in enumerate(sizes)]
    Is, As = inputs(torch, fge, samples, p)
    b = fge.Batch([(h, w) for w, h in sizes], p)
    Fs1, Bs1 = b.run(Is, As)
    Is2 = [I.flip(-1).contiguous() for I in Is]
    Fs2, Bs2 = b.run(Is2, As)
    torch.cuda.synchronize()
    for i in range(len(sizes)):
        F1, B1 = single(torch, fge, Is[i], As[i], p)
        F2, B2 = single(torch, fge, Is2[i], As[i], p)
        torch.cuda.synchronize()
        assert torch.equal(Fs1[i], F1) and torch.equal(Bs2[i], B2)
    b.close()


def test_batch_graph_replays(gpu):
    """Capture once, replay several times with eager work and synchronisations in between; every
    replay must reproduce the eager result (outputs are cleared before each replay)."""
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16)
    sizes = [(300, 200), (129, 300), (700, 421), (64, 37)]
    samples = [synth.smooth(w, h, seed=90 + i) for i, (w, h) in enumerate(sizes)]
    Is, As = inputs(torch, fge, samples, p)
    b = fge.Batch([(h, w) for w, h in sizes], p)
    ref = b.run(Is, As)
    torch.cuda.synchronize()
    ref = ([F.clone() for F in ref[0]], [B.clone() for B in ref[1]])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        Fs, Bs = b.capture(Is, As, stream=stream)
    torch.cuda.synchronize()
    for rep in range(4):
        for t in Fs + Bs:
            t.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work
        torch.cuda.synchronize()
        b.replay(stream)
        stream.synchronize()
        for i in range(len(sizes)):
            assert torch.equal(Fs[i], ref[0][i]) and torch.equal(Bs[i], ref[1][i]), (rep, i)
        del junk
    b.close()


def test_uneven_batch_workload_f16(gpu):
    """The 64-image uneven batch (W, H uniform on [256, 2048], float16 storage): a sample of
    images bit-identical to their single-image runs, and every image against the oracle (the
    OpenMP build, same bits as the one-thread oracle)."""
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16)
    sizes = synth.batch_sizes()
    samples = [synth.batch_image(i, w, h) for i, (w, h) in enumerate(sizes)]
    Is, As = inputs(torch, fge, samples, p)
    b = fge.Batch([(h, w) for w, h in sizes], p)
    Fs, Bs = b.run(Is, As)
    torch.cuda.synchronize()
    order = sorted(range(len(sizes)), key=lambda i: sizes[i][0] * sizes[i][1])
    for i in order[:3] + order[-3:] + [7, 31]:
        F1, B1 = single(torch, fge, Is[i], As[i], p)
        torch.cuda.synchronize()
        assert torch.equal(Fs[i], F1) and torch.equal(Bs[i], B1), (i, sizes[i])
    worst = 0.0
    for i in range(len(sizes)):
        s = samples[i]
        Fo, Bo = oracle.ml(s.I, s.alpha, parallel=True)
        err = max(float(np.abs(Fs[i].cpu().numpy().astype(np.float64) - Fo).max()),
                  float(np.abs(Bs[i].cpu().numpy().astype(np.float64) - Bo).max()))
        worst = max(worst, err)
        assert err <= TOL["f16"], (i, sizes[i], err)
    print(f"64 batch images: worst f16 max-abs vs oracle {worst:.2e}")
    b.close()


def test_batch_recapture_waits_for_queued_replays(gpu):
    """Capture, queue replays, re-capture the same plan with other buffers at once (the new
    capture refills the pinned table buffer the first graph's upload reads), replay the new
    graph: both graphs' results must be bit-identical to eager runs of their own inputs."""
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16)
    sizes = [(300, 200), (129, 300), (700, 421)]
    shapes = [(h, w) for w, h in sizes]
    sa = [synth.smooth(w, h, seed=300 + i) for i, (w, h) in enumerate(sizes)]
    sb = [synth.smooth(w, h, seed=400 + i) for i, (w, h) in enumerate(sizes)]
    Ia, Aa = inputs(torch, fge, sa, p)
    Ib, Ab = inputs(torch, fge, sb, p)
    b = fge.Batch(shapes, p)
    ws_a = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda")
    ws_b = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        Fa, Ba = b.capture(Ia, Aa, workspace=ws_a, stream=stream)
        for _ in range(3):
            b.replay(stream)
        Fb, Bb = b.capture(Ib, Ab, workspace=ws_b, stream=stream)
        b.replay(stream)
    stream.synchronize()
    for i in range(len(sizes)):
        F1, B1 = single(torch, fge, Ia[i], Aa[i], p)
        F2, B2 = single(torch, fge, Ib[i], Ab[i], p)
        torch.cuda.synchronize()
        assert torch.equal(Fa[i], F1) and torch.equal(Ba[i], B1), ("first graph", i)
        assert torch.equal(Fb[i], F2) and torch.equal(Bb[i], B2), ("second graph", i)
    b.close()
