"""The input generators (no estimation arithmetic here): the device form of the smooth generator
agrees with the NumPy form, and the serving stream has the stated size distribution."""
import math

import numpy as np
import pytest

from paper_2006_14970_amd import synth


@pytest.mark.parametrize("wh", [(64, 64), (301, 170), (17, 900)])
def test_smooth_device_matches_numpy_fields(wh):
    import torch
    W, H = wh
    s = synth.smooth(W, H, seed=77)
    I, a, F, B = synth.smooth_device(W, H, 77, "cpu", return_fields=True)
    assert tuple(I.shape) == (3, H, W) and tuple(a.shape) == (H, W)
    assert np.abs(F.double().numpy() - s.F).max() < 1e-5
    assert np.abs(B.double().numpy() - s.B).max() < 1e-5
    assert np.abs(a.double().numpy() - s.alpha).max() < 1e-5
    I64 = I.double().numpy()
    assert I64.min() >= 0.0 and I64.max() <= 1.0
    # the composite is the compositing equation plus N(0, 0.01^2) noise (clipped)
    resid = I64 - (a.double().numpy()[None] * F.double().numpy() +
                   (1 - a.double().numpy()[None]) * B.double().numpy())
    assert 0.007 < resid.std() < 0.0105
    I16, a16 = synth.smooth_device(W, H, 77, "cpu", dtype=torch.float16)
    assert I16.dtype == torch.float16 and torch.equal(I16, I.half())


def test_serving_stream_distribution():
    reqs = synth.serving_requests(n=2000, rate_per_s=1000.0)
    A = np.array([r.W * r.H for r in reqs]) / 1e6
    asp = np.array([r.W / r.H for r in reqs])
    assert A.min() > 0.24 and A.max() < 16.1
    # log-uniform on [0.25, 16]: mean (16 - 0.25) / ln 64 = 3.787 MP
    assert abs(A.mean() - 15.75 / math.log(64.0)) < 0.25
    assert asp.min() > 0.49 and asp.max() < 2.01
    t = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(t) > 0) and abs(t[-1] / 2000 - 1e-3) < 1e-4
    # sizes do not depend on the rate (arrival gaps only scale)
    again = synth.serving_requests(n=2000, rate_per_s=10.0)
    assert [(r.W, r.H) for r in again] == [(r.W, r.H) for r in reqs]
    assert abs(again[7].arrival_s - 100.0 * reqs[7].arrival_s) < 1e-9
