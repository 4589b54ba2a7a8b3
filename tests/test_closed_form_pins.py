"""Pins of the closed-form oracle (Section III-B, eq. 2, with the eps regulariser of Section
III-C), each reaching the expected value by a route independent of oracle/closed_form.py:

* the gradient of the C oracle's energy (oracle.energy: data term plus every undirected
  4-neighbour edge once, weight eps + omega |a_i - a_j|) equals 2 (A x - b) for the assembled
  matrix and right-hand side, on random points (the energy is quadratic, so central differences
  are exact up to rounding): a wrong weight, a missing or doubled edge, a transposed or swapped
  block fails it;
* the solve equals a dense least-squares solve of the stacked residual rows of the cost (a row
  per pixel and channel for the data term, one per edge and unknown kind for the smoothness);
* with omega = 0.1 the minimiser is a fixed point of Algorithm 1's per-pixel solve (eq. 9) in
  every order, the unclamped stationarity the paper derives (the clamp is inactive there);
* a constant image is reproduced exactly; alpha -> 1 - alpha swaps F and B; transposing the
  inputs transposes the result.
"""
import numpy as np
import pytest

import oracle
from oracle import closed_form as cf
from paper_2006_14970_amd import synth


def _rand_inputs(H, W, seed):
    rng = np.random.default_rng(seed)
    I = rng.random((3, H, W))
    a = rng.random((H, W))
    return I, a


@pytest.mark.parametrize("omega,eps", [(1.0, 5e-3), (0.1, 5e-3), (1.0, 0.05)])
def test_matrix_is_the_energy_gradient(omega, eps):
    H, W = 4, 5
    I, a = _rand_inputs(H, W, 1)
    A = cf.system_matrix(a, omega, eps)
    rng = np.random.default_rng(2)
    F = rng.random((3, H, W))
    B = rng.random((3, H, W))
    h = 1e-3
    for c in range(3):
        g = 2.0 * (A @ cf.pack(F[c], B[c]) - cf.rhs(I[c], a))
        for k in range(2 * H * W):
            target = F if k % 2 == 0 else B
            y, x = divmod(k // 2, W)
            Fp, Bp = F.copy(), B.copy()
            Fm, Bm = F.copy(), B.copy()
            (Fp if target is F else Bp)[c, y, x] += h
            (Fm if target is F else Bm)[c, y, x] -= h
            d = (oracle.energy(Fp, Bp, I, a, omega, eps) - oracle.energy(Fm, Bm, I, a, omega, eps))
            assert abs(d / (2 * h) - g[k]) <= 1e-9, (c, k, d / (2 * h), g[k])


def _lstsq(I, a, omega, eps):
    """Minimiser by dense least squares over the residual rows of the cost."""
    _, H, W = I.shape
    n = H * W
    wx, wy = np.zeros((H, W - 1)), np.zeros((H - 1, W))
    for y in range(H):
        for x in range(W - 1):
            wx[y, x] = eps + omega * abs(a[y, x + 1] - a[y, x])
    for y in range(H - 1):
        for x in range(W):
            wy[y, x] = eps + omega * abs(a[y + 1, x] - a[y, x])
    F = np.empty((3, H, W))
    B = np.empty((3, H, W))
    for c in range(3):
        rows, vals = [], []
        for y in range(H):
            for x in range(W):
                r = np.zeros(2 * n)          # unknowns: F (n), then B (n)
                i = y * W + x
                r[i] = a[y, x]
                r[n + i] = 1 - a[y, x]
                rows.append(r)
                vals.append(I[c, y, x])
        edges = [((y, x), (y, x + 1), wx[y, x]) for y in range(H) for x in range(W - 1)]
        edges += [((y, x), (y + 1, x), wy[y, x]) for y in range(H - 1) for x in range(W)]
        for (y0, x0), (y1, x1), w in edges:
            for off in (0, n):
                r = np.zeros(2 * n)
                r[off + y0 * W + x0] = np.sqrt(w)
                r[off + y1 * W + x1] = -np.sqrt(w)
                rows.append(r)
                vals.append(0.0)
        sol = np.linalg.lstsq(np.array(rows), np.array(vals), rcond=None)[0]
        F[c] = sol[:n].reshape(H, W)
        B[c] = sol[n:].reshape(H, W)
    return F, B


@pytest.mark.parametrize("hw", [(2, 3), (4, 5), (5, 2), (3, 3), (1, 4)])
@pytest.mark.parametrize("omega,eps", [(1.0, 5e-3), (0.1, 0.02)])
def test_solve_matches_dense_least_squares(hw, omega, eps):
    H, W = hw
    I, a = _rand_inputs(H, W, 10 + H * 7 + W)
    F, B = cf.solve(I, a, omega, eps)
    Fl, Bl = _lstsq(I, a, omega, eps)
    assert np.abs(F - Fl).max() <= 1e-9 and np.abs(B - Bl).max() <= 1e-9
    assert cf.relative_residuals(I, a, F, B, omega, eps).max() <= 1e-12
    assert np.allclose(cf.relative_residuals(I, a, 0 * F, 0 * B, omega, eps), 1.0)


def test_fixed_point_of_algorithm1_sweeps():
    """omega = 0.1: the global minimiser satisfies every pixel's 2x2 system of eq. 9 (the
    per-pixel solve of Algorithm 1) with the clamp inactive, so one sweep in any order keeps it."""
    s = synth.smooth(40, 30, seed=5)
    # the solution map is linear and reproduces constants, so squeezing the image into
    # [0.25, 0.75] keeps the minimiser inside (0, 1), where the clamp does nothing
    I = 0.25 + 0.5 * s.I
    F, B = cf.solve(I, s.alpha, omega=0.1, eps=5e-3)
    assert F.min() > 0 and B.min() > 0 and F.max() < 1 and B.max() < 1
    for order in ("jacobi", "redblack", "raster"):
        F1, B1 = oracle.sweep(F, B, I, s.alpha, 0.1, 5e-3, order=order)
        assert np.abs(F1 - F).max() <= 1e-10 and np.abs(B1 - B).max() <= 1e-10, order


def test_constant_image_is_reproduced():
    H, W = 9, 7
    rng = np.random.default_rng(3)
    a = rng.random((H, W))
    c = np.array([0.2, 0.55, 0.9])
    I = np.broadcast_to(c[:, None, None], (3, H, W)).copy()
    F, B = cf.solve(I, a)
    assert np.abs(F - I).max() <= 1e-12 and np.abs(B - I).max() <= 1e-12


def test_alpha_complement_swaps_and_transpose():
    I, a = _rand_inputs(6, 8, 4)
    F, B = cf.solve(I, a)
    F2, B2 = cf.solve(I, 1.0 - a)
    assert np.abs(F2 - B).max() <= 1e-11 and np.abs(B2 - F).max() <= 1e-11
    Ft, Bt = cf.solve(I.transpose(0, 2, 1).copy(), a.T.copy())
    assert np.abs(Ft - F.transpose(0, 2, 1)).max() <= 1e-11
    assert np.abs(Bt - B.transpose(0, 2, 1)).max() <= 1e-11
