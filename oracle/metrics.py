"""Quality measures of an estimated foreground, and compositing -- TEST INFRASTRUCTURE ONLY.

Plain float64 NumPy (plus SciPy's Gaussian derivative filter as a library step) following the
paper's error measures (Section IV, "Error Measures"): over the translucent pixels
0 < alpha_i < 1 of the reference matte, each weighted by alpha_i,

    SAD  = sum alpha_i |F_i - G_i|_1           (L1 over the colour channels)
    MSE  = sum alpha_i |F_i - G_i|_2^2
    GRAD = sum alpha_i |grad F_i - grad G_i|_2^2,

with F the estimate and G the reference foreground; the gradient images come from first-order
Gaussian derivative filters with sigma = 1.4, in x and in y, for every channel.  Readings where
the paper is silent: the derivative filter is SciPy's (`gaussian_filter` with order 1 along one
axis and order 0 along the other: the sampled Gaussian normalised to sum 1, times -x / sigma^2,
truncated at int(4 sigma + 0.5) pixels), and borders are mirrored ('reflect': d c b a | a b c d).

Compositing onto a new background is eq. 1 used forward: C = alpha F + (1 - alpha) B_new.
"""
from __future__ import annotations

import numpy as np

SIGMA = 1.4


def _f64(x):
    return np.asarray(x, dtype=np.float64)


def gradients(F: np.ndarray, sigma: float = SIGMA):
    """(gx, gy) of every channel of a (3, H, W) image."""
    from scipy.ndimage import gaussian_filter
    F = _f64(F)
    gx = np.stack([gaussian_filter(F[c], sigma, order=(0, 1), mode="reflect") for c in range(F.shape[0])])
    gy = np.stack([gaussian_filter(F[c], sigma, order=(1, 0), mode="reflect") for c in range(F.shape[0])])
    return gx, gy


def quality(F_est: np.ndarray, F_ref: np.ndarray, alpha: np.ndarray, sigma: float = SIGMA):
    """(SAD, MSE, GRAD, number of translucent pixels)."""
    F, G, a = _f64(F_est), _f64(F_ref), _f64(alpha)
    m = (a > 0.0) & (a < 1.0)
    d = F - G
    sad = float((a[m] * np.abs(d[:, m]).sum(axis=0)).sum())
    mse = float((a[m] * (d[:, m] ** 2).sum(axis=0)).sum())
    gx, gy = gradients(d, sigma)          # the filters are linear: grad F - grad G = grad (F - G)
    grad = float((a[m] * (gx[:, m] ** 2 + gy[:, m] ** 2).sum(axis=0)).sum())
    return sad, mse, grad, int(m.sum())


def composite(F: np.ndarray, alpha: np.ndarray, B_new: np.ndarray) -> np.ndarray:
    """alpha F + (1 - alpha) B_new in float64, products and sum each rounded once."""
    F, a, B = _f64(F), _f64(alpha), _f64(B_new)
    return a[None] * F + (1.0 - a[None]) * B
