"""GPU tests of the autotuner: every candidate runs, the chosen settings are among them, results
under the chosen settings match the oracle (single image) and the single-image path (batch),
and the JSON cache answers a repeated search."""
import json
import os

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


def test_autotune_single(gpu, tmp_path):
    torch, fge = gpu
    s = synth.strands(1024, 768, seed=2, n_strands=200)
    I = torch.from_numpy(s.I).float().cuda()
    a = torch.from_numpy(s.alpha).float().cuda()
    cache = str(tmp_path / "tune.json")
    best, ent = fge.autotune(I, a, reps=2, cache_path=cache)
    print([(e["strip_rows"], e["tile_max_px"], round(e["ms"], 4)) for e in ent])
    assert len(ent) == 21 and all(e["status"] == 0 and e["ms"] > 0 for e in ent)
    fastest = min(ent, key=lambda e: e["ms"])
    assert (best.strip_rows, best.tile_max_px) == (fastest["strip_rows"], fastest["tile_max_px"])
    F, B = fge.estimate_foreground(I, a, best)
    torch.cuda.synchronize()
    Fo, Bo = oracle.ml(s.I, s.alpha)
    err = max(float(np.abs(F.double().cpu().numpy() - Fo).max()),
              float(np.abs(B.double().cpu().numpy() - Bo).max()))
    assert err <= 1e-4
    assert len(json.load(open(cache))) == 1
    mtime = os.path.getmtime(cache)
    best2, _ = fge.autotune(I, a, reps=2, cache_path=cache)     # answered by the cache
    assert (best2.strip_rows, best2.tile_max_px) == (best.strip_rows, best.tile_max_px)
    assert os.path.getmtime(cache) == mtime


def test_autotune_batch_matches_single(gpu):
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16)
    sizes = [(1500, 900), (300, 2000), (700, 700), (256, 260), (2048, 1000), (64, 64)]
    imgs = [synth.smooth_device(w, h, 7000 + k, "cuda", dtype=torch.float16)
            for k, (w, h) in enumerate(sizes)]
    torch.cuda.synchronize()
    Is = [x[0] for x in imgs]
    As = [x[1] for x in imgs]
    best, ent = fge.autotune_batch([(h, w) for w, h in sizes], Is, As, p, reps=2)
    assert len(ent) == 21 and all(e["status"] == 0 for e in ent)
    b = fge.Batch([(h, w) for w, h in sizes], best)
    Fs, Bs = b.run(Is, As)
    torch.cuda.synchronize()
    for (I, a), F, B in zip(imgs, Fs, Bs):
        F1, B1 = fge.estimate_foreground(I, a, best)
        torch.cuda.synchronize()
        assert torch.equal(F, F1) and torch.equal(B, B1)
    b.close()
