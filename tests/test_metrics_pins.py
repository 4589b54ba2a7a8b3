"""Pins of the quality-measure oracle (oracle/metrics.py) against closed forms and a derivative
kernel assembled here from its definition (sampled Gaussian, normalised, times -x / sigma^2,
radius int(4 sigma + 0.5), mirrored borders)."""
import math

import numpy as np
import pytest

from oracle import metrics

SIG = 1.4


def kernel(sigma=SIG):
    r = int(4.0 * sigma + 0.5)
    x = np.arange(-r, r + 1, dtype=np.float64)
    phi = np.exp(-0.5 * x * x / (sigma * sigma))
    phi /= phi.sum()
    return x, phi, -x / (sigma * sigma) * phi


def reflect(i, n):
    m = i % (2 * n)
    return m if m < n else 2 * n - 1 - m


def grad_by_hand(D, y, x, sigma=SIG):
    """gx, gy of one channel D at (y, x): out[i] = sum_j w(-j) D[i + j] along the derivative axis,
    with smoothing along the other (correlation with the mirrored kernel)."""
    h, w = D.shape
    xs, phi, der = kernel(sigma)
    r = len(xs) // 2
    gx = gy = 0.0
    for a in range(-r, r + 1):          # offset along y
        for b in range(-r, r + 1):      # offset along x
            v = D[reflect(y + a, h), reflect(x + b, w)]
            gx += phi[r + a] * der[r - b] * v
            gy += der[r - a] * phi[r + b] * v
    return gx, gy


def test_sad_mse_closed_form():
    a = np.array([[0.0, 0.5, 1.0], [0.25, 0.75, 0.5]])
    G = np.full((3, 2, 3), 0.4)
    F = G + 0.1
    sad, mse, grad, n = metrics.quality(F, G, a)
    assert n == 4
    assert abs(sad - 2.0 * 3 * 0.1) < 1e-12          # sum of translucent alphas = 2.0
    assert abs(mse - 2.0 * 3 * 0.01) < 1e-12
    assert abs(grad) < 1e-20                            # a constant difference has no gradient


def test_gradient_of_a_ramp():
    h, w, k = 40, 50, 0.013
    xs, phi, der = kernel()
    scale = float((xs * xs * phi).sum()) / (SIG * SIG)     # discrete second moment / sigma^2
    assert abs(scale - 1.0) < 1e-3
    D = np.broadcast_to(k * np.arange(w, dtype=np.float64)[None, None, :], (3, h, w)).copy()
    gx, gy = metrics.gradients(D)
    r = len(xs) // 2
    inner = (slice(None), slice(r, h - r), slice(r, w - r))
    np.testing.assert_allclose(gx[inner], k * scale, rtol=1e-12)
    np.testing.assert_allclose(gy[inner], 0.0, atol=1e-15)
    # transposed ramp: the roles swap
    gx2, gy2 = metrics.gradients(np.transpose(D[:, :40, :40], (0, 2, 1)))
    np.testing.assert_allclose(gy2[:, r:40 - r, r:40 - r], k * scale, rtol=1e-12)


@pytest.mark.parametrize("yx", [(0, 0), (0, 7), (5, 0), (12, 17), (1, 18), (12, 2)])
def test_gradient_by_hand_with_mirrored_borders(yx):
    rng = np.random.default_rng(5)
    D = rng.normal(size=(3, 13, 19))
    gx, gy = metrics.gradients(D)
    y, x = yx
    for c in range(3):
        hx, hy = grad_by_hand(D[c], y, x)
        assert abs(gx[c, y, x] - hx) < 1e-12 and abs(gy[c, y, x] - hy) < 1e-12


def test_grad_measure_weights():
    rng = np.random.default_rng(6)
    h, w = 16, 21
    a = rng.uniform(-0.3, 1.3, (h, w)).clip(0, 1)
    F = rng.uniform(0, 1, (3, h, w))
    G = rng.uniform(0, 1, (3, h, w))
    sad, mse, grad, n = metrics.quality(F, G, a)
    gx, gy = metrics.gradients(F - G)
    m = (a > 0) & (a < 1)
    want = sum(a[y, x] * sum(gx[c, y, x] ** 2 + gy[c, y, x] ** 2 for c in range(3))
               for y in range(h) for x in range(w) if m[y, x])
    assert n == m.sum() and math.isclose(grad, want, rel_tol=1e-12)
    want_sad = sum(a[y, x] * sum(abs(F[c, y, x] - G[c, y, x]) for c in range(3))
                   for y in range(h) for x in range(w) if m[y, x])
    assert math.isclose(sad, want_sad, rel_tol=1e-12)


def test_composite_special_cases():
    rng = np.random.default_rng(7)
    F = rng.uniform(0, 1, (3, 4, 5))
    B = rng.uniform(0, 1, (3, 4, 5))
    assert np.array_equal(metrics.composite(F, np.zeros((4, 5)), B), B)
    assert np.array_equal(metrics.composite(F, np.ones((4, 5)), B), F)
    np.testing.assert_allclose(metrics.composite(F, np.full((4, 5), 0.5), B), (F + B) / 2, atol=1e-16)
