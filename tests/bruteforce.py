"""Independent brute-force formulations used to pin the oracle (tests only).

Nothing here shares code with the oracle or the GPU path.  Each helper reaches the paper's
quantities by a different route than the oracle does:

* level sizes by the exact integer criterion for round(w^(l/n)) (no floating point);
* the nearest resize map by an exact search over rationals;
* the per-pixel update by a least-squares solve of the stacked residuals of the local cost
  (eq. 3) with numpy.linalg.lstsq, instead of Cramer's rule on the normal equations (eq. 9);
* the minimiser of the global energy by assembling its normal equations as a sparse matrix and
  calling scipy.sparse.linalg.spsolve.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def num_levels_exact(w: int, h: int) -> int:
    """ceil(log2(max(w, h))) via bit length, at least 1."""
    m = max(w, h)
    return max(1, (m - 1).bit_length())


def level_size_exact(full: int, level: int, n: int) -> int:
    """The integer k with |k - full^(level/n)| < 1/2, by the exact criterion
    (2k - 1)^n <= 2^n full^level < (2k + 1)^n (ties cannot occur: left side even, odd powers)."""
    target = (2 ** n) * (full ** level)
    # integer n-th root of target, then adjust to the odd bracket
    lo, hi = 0, 1
    while hi ** n <= target:
        hi *= 2
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if mid ** n <= target:
            lo = mid
        else:
            hi = mid
    root = lo                      # floor(target^(1/n)) = floor(2 full^(level/n))
    k = (root + 1) // 2            # nearest integer to root / 2 on the odd grid
    assert (2 * k - 1) ** n <= target < (2 * k + 1) ** n or k == 0
    return k


def nearest_index(x: int, n_src: int, n_dst: int) -> int:
    """Nearest-resize reading: the last source pixel whose left edge i/n_src lies at or before the
    destination pixel's left edge x/n_dst, found by exhaustive search over exact rationals."""
    edge = Fraction(x, n_dst)
    best = 0
    for i in range(n_src):
        if Fraction(i, n_src) <= edge:
            best = i
    return best


def resize_bf(src: np.ndarray, wd: int, hd: int) -> np.ndarray:
    p, hs, ws = src.shape
    xs = [nearest_index(x, ws, wd) for x in range(wd)]
    ys = [nearest_index(y, hs, hd) for y in range(hd)]
    return src[:, ys][:, :, xs]


def area_matrix(n_src: int, n_dst: int) -> np.ndarray:
    """Area resize along one axis: row x holds the overlap of every source pixel [i, i+1) with
    the destination footprint [x n_src/n_dst, (x+1) n_src/n_dst), divided by the footprint
    length, computed in exact rationals."""
    M = np.zeros((n_dst, n_src))
    for x in range(n_dst):
        lo, hi = Fraction(x * n_src, n_dst), Fraction((x + 1) * n_src, n_dst)
        for i in range(n_src):
            ov = min(Fraction(i + 1), hi) - max(Fraction(i), lo)
            if ov > 0:
                M[x, i] = float(ov / (hi - lo))
    return M


def bilinear_matrix(n_src: int, n_dst: int) -> np.ndarray:
    """Bilinear resize along one axis with half-integer pixel centres, clamped at the borders."""
    M = np.zeros((n_dst, n_src))
    for x in range(n_dst):
        u = min(max(Fraction(2 * x + 1, 2) * n_src / n_dst - Fraction(1, 2), 0), n_src - 1)
        i0 = int(u)
        f = u - i0
        i1 = min(i0 + 1, n_src - 1)
        M[x, i0] += float(1 - f)
        M[x, i1] += float(f)
    return M


def resize_separable_bf(src: np.ndarray, wd: int, hd: int, matrix) -> np.ndarray:
    p, hs, ws = src.shape
    My, Mx = matrix(hs, hd), matrix(ws, wd)
    return np.stack([My @ src[c] @ Mx.T for c in range(p)])


def neighbours(x: int, y: int, w: int, h: int):
    """The four neighbours of Algorithm 1, clamped into the image."""
    out = []
    for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        out.append((min(max(x + dx, 0), w - 1), min(max(y + dy, 0), h - 1)))
    return out


def local_solve_lstsq(a, I3, nb, omega, eps):
    """Minimise the local cost of eq. 3 for one pixel and each channel as a linear least-squares
    problem.  nb = [(alpha_j, F_j[3], B_j[3]), ...].  Returns unclamped (F[3], B[3])."""
    F = np.zeros(3)
    B = np.zeros(3)
    for c in range(3):
        rows = [[a, 1.0 - a]]
        rhs = [I3[c]]
        for aj, Fj, Bj in nb:
            r = np.sqrt(eps + omega * abs(a - aj))
            rows.append([r, 0.0])
            rhs.append(r * Fj[c])
            rows.append([0.0, r])
            rhs.append(r * Bj[c])
        sol, *_ = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)
        F[c], B[c] = sol
    return F, B


def update_bf(F, B, I, a, x, y, omega, eps, src_F=None, src_B=None):
    """New clamped (F, B) of pixel (x, y); neighbour values read from src_* (default F, B)."""
    _, h, w = I.shape
    sF = F if src_F is None else src_F
    sB = B if src_B is None else src_B
    nb = [(a[yj, xj], sF[:, yj, xj].copy(), sB[:, yj, xj].copy())
          for xj, yj in neighbours(x, y, w, h)]
    f, b = local_solve_lstsq(a[y, x], I[:, y, x], nb, omega, eps)
    return np.clip(f, 0.0, 1.0), np.clip(b, 0.0, 1.0)


def sweep_bf(F, B, I, a, omega=0.1, eps=5e-3, order="redblack"):
    F = F.copy()
    B = B.copy()
    _, h, w = I.shape
    if order == "raster":
        for y in range(h):
            for x in range(w):
                F[:, y, x], B[:, y, x] = update_bf(F, B, I, a, x, y, omega, eps)
    elif order == "redblack":
        for colour in (0, 1):
            for y in range(h):
                for x in range(w):
                    if (x + y) % 2 == colour:
                        F[:, y, x], B[:, y, x] = update_bf(F, B, I, a, x, y, omega, eps)
    elif order == "jacobi":
        F0, B0 = F.copy(), B.copy()
        for y in range(h):
            for x in range(w):
                F[:, y, x], B[:, y, x] = update_bf(F, B, I, a, x, y, omega, eps, F0, B0)
    else:
        raise ValueError(order)
    return F, B


def ml_bf(I, a, omega=0.1, eps=5e-3, small=32, it_small=10, it_big=2, order="redblack",
          resize="nearest"):
    """Algorithm 1 assembled from the helpers above (tiny images only).  resize "smooth": area
    resize of I and alpha, bilinear resize of F and B."""
    _, H, W = I.shape
    n = num_levels_exact(W, H)
    F = np.zeros((3, 1, 1))
    B = np.zeros((3, 1, 1))
    if resize == "smooth":
        down = lambda x, w, h: resize_separable_bf(x, w, h, area_matrix)       # noqa: E731
        up = lambda x, w, h: resize_separable_bf(x, w, h, bilinear_matrix)     # noqa: E731
    else:
        down = up = resize_bf
    for lv in range(1, n + 1):
        w, h = level_size_exact(W, lv, n), level_size_exact(H, lv, n)
        Il = down(I, w, h)
        al = down(a[None], w, h)[0]
        F = up(F, w, h)
        B = up(B, w, h)
        iters = it_small if (w <= small and h <= small) else it_big
        for _ in range(iters):
            F, B = sweep_bf(F, B, Il, al, omega, eps, order)
    return F, B


def direct_minimiser(I, a, omega=0.1, eps=5e-3):
    """argmin of the global energy (data term + every undirected 4-neighbour edge once) by a
    sparse direct solve of its normal equations, channel by channel."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import spsolve

    _, h, w = I.shape
    n = w * h
    idx = np.arange(n).reshape(h, w)
    rows, cols, vals = [], [], []

    def add(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(v)

    af = a.reshape(-1)
    # data term: (a F + (1 - a) B - I)^2 -> Hessian/2 blocks
    for i in range(n):
        ai = af[i]
        add(i, i, ai * ai)
        add(i, n + i, ai * (1 - ai))
        add(n + i, i, ai * (1 - ai))
        add(n + i, n + i, (1 - ai) ** 2)
    # edges
    for y in range(h):
        for x in range(w):
            for xj, yj in ((x + 1, y), (x, y + 1)):
                if xj >= w or yj >= h:
                    continue
                i, j = idx[y, x], idx[yj, xj]
                s = eps + omega * abs(af[i] - af[j])
                for off in (0, n):
                    add(off + i, off + i, s)
                    add(off + j, off + j, s)
                    add(off + i, off + j, -s)
                    add(off + j, off + i, -s)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(2 * n, 2 * n))
    F = np.zeros((3, h, w))
    B = np.zeros((3, h, w))
    for c in range(3):
        Ic = I[c].reshape(-1)
        rhs = np.concatenate([af * Ic, (1 - af) * Ic])
        g = spsolve(A.tocsc(), rhs)
        F[c] = g[:n].reshape(h, w)
        B[c] = g[n:].reshape(h, w)
    return F, B
