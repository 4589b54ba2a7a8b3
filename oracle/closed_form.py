"""Closed-form foreground estimation (the global cost of Section III-B, eq. 2) -- TEST
INFRASTRUCTURE ONLY.

Only the test suite and the benchmark's CPU-baseline leg may import this module; the product
package never does, and nothing here imports the product package.

The cost (eq. 2, Levin et al.'s closed-form colour estimation) is, per colour channel c,

    E_c(F, B) = sum_i (a_i F_i + (1 - a_i) B_i - I_i)^2
              + sum_i |a_ix| (F_ix^2 + B_ix^2) + |a_iy| (F_iy^2 + B_iy^2),

with the image gradients read as forward differences to the right and lower neighbour (the
gradient of the last column / row is zero).  Every horizontal and vertical neighbour pair {i, j}
then appears once, with weight |a_i - a_j|.  Two readings, both parameters of the functions below:

* the weight of an edge is ``eps + omega |a_i - a_j|``.  eq. 2 as printed has omega = 1, eps = 0;
  but then F (where a = 0) and B (where a = 1) are unconstrained wherever the matte is locally
  constant -- the paper makes exactly this remark when it introduces its regulariser eps_r in
  Section III-C -- and the normal equations are singular.  The default eps is therefore the
  paper's eps_r = 5e-3.  With omega = 0.1 the cost is the global quadratic whose per-pixel
  stationarity conditions are the 2x2 systems of eq. 9, i.e. the fixed point of Algorithm 1's
  sweeps;
* no clamp: the minimiser of the quadratic, as the paper's conjugate-gradient remark solves it.

The minimiser solves the normal equations A x = b of the 2n x 2n system (n = H W) of one channel,
the same matrix for all three channels:

    A = blockdiag_i(U_i U_i^T) + L (x) Id_2,   b_i = U_i I_i,   U_i = [a_i, 1 - a_i]^T,

L the weighted graph Laplacian of the 4-neighbour grid.  The unknowns are ordered per pixel,
(F_i, B_i) at positions 2i and 2i + 1.  The solve is a sparse LU factorisation (SciPy's SuperLU
with a symmetric minimum-degree ordering and no pivoting, which is stable for this symmetric
positive definite matrix) used for the three right-hand sides.  The minimiser is unique when the
matte is not constant over the whole image; the functions do not check that.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def edge_weights(alpha: np.ndarray, omega: float = 1.0, eps: float = 5e-3):
    """Weights of the horizontal edges (H, W-1) -- pixel (y, x) to (y, x+1) -- and of the vertical
    edges (H-1, W) -- pixel (y, x) to (y+1, x)."""
    a = np.asarray(alpha, dtype=np.float64)
    wx = eps + omega * np.abs(a[:, 1:] - a[:, :-1])
    wy = eps + omega * np.abs(a[1:, :] - a[:-1, :])
    return wx, wy


def system_matrix(alpha: np.ndarray, omega: float = 1.0, eps: float = 5e-3) -> sp.csr_matrix:
    """The 2n x 2n matrix A of the normal equations (unknown 2i = F_i, 2i + 1 = B_i)."""
    a = np.asarray(alpha, dtype=np.float64)
    H, W = a.shape
    n = H * W
    wx, wy = edge_weights(a, omega, eps)
    idx = np.arange(n).reshape(H, W)
    ei = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    ej = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    ew = np.concatenate([wx.ravel(), wy.ravel()])
    # Laplacian: -w off the diagonal for every edge, the sum of the pixel's edge weights on it
    deg = np.bincount(ei, weights=ew, minlength=n) + np.bincount(ej, weights=ew, minlength=n)
    lap = sp.coo_matrix((np.concatenate([-ew, -ew, deg]),
                         (np.concatenate([ei, ej, np.arange(n)]),
                          np.concatenate([ej, ei, np.arange(n)]))), shape=(n, n))
    # the smoothness acts on F and on B alike
    A = sp.kron(lap, sp.identity(2), format="coo")
    af = a.ravel()
    p = np.arange(n)
    data = sp.coo_matrix((np.concatenate([af * af, af * (1 - af), af * (1 - af), (1 - af) ** 2]),
                          (np.concatenate([2 * p, 2 * p, 2 * p + 1, 2 * p + 1]),
                           np.concatenate([2 * p, 2 * p + 1, 2 * p, 2 * p + 1]))), shape=(2 * n, 2 * n))
    return (A + data).tocsr()


def rhs(I_c: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """b of one channel: (a_i I_i, (1 - a_i) I_i) per pixel."""
    a = np.asarray(alpha, dtype=np.float64).ravel()
    v = np.asarray(I_c, dtype=np.float64).ravel()
    b = np.empty(2 * a.size)
    b[0::2] = a * v
    b[1::2] = (1.0 - a) * v
    return b


def pack(F_c: np.ndarray, B_c: np.ndarray) -> np.ndarray:
    x = np.empty(2 * F_c.size)
    x[0::2] = np.asarray(F_c, dtype=np.float64).ravel()
    x[1::2] = np.asarray(B_c, dtype=np.float64).ravel()
    return x


def solve(I: np.ndarray, alpha: np.ndarray, omega: float = 1.0, eps: float = 5e-3):
    """The minimiser (F, B) of the cost above, each (3, H, W) float64."""
    I = np.asarray(I, dtype=np.float64)
    a = np.asarray(alpha, dtype=np.float64)
    _, H, W = I.shape
    A = system_matrix(a, omega, eps).tocsc()
    lu = spla.splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    F = np.empty((3, H, W))
    B = np.empty((3, H, W))
    for c in range(3):
        x = lu.solve(rhs(I[c], a))
        F[c] = x[0::2].reshape(H, W)
        B[c] = x[1::2].reshape(H, W)
    return F, B


def relative_residuals(I: np.ndarray, alpha: np.ndarray, F: np.ndarray, B: np.ndarray,
                       omega: float = 1.0, eps: float = 5e-3) -> np.ndarray:
    """||b - A x|| / ||b|| of each channel for a candidate (F, B): the stopping measure of the
    paper's conjugate-gradient remark."""
    A = system_matrix(alpha, omega, eps)
    out = np.empty(3)
    for c in range(3):
        b = rhs(I[c], alpha)
        out[c] = np.linalg.norm(b - A @ pack(F[c], B[c])) / np.linalg.norm(b)
    return out
