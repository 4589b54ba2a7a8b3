"""Seeded synthetic inputs for foreground estimation.

This module only *generates data*: known foreground/background fields, an alpha matte and the
composite image I = alpha F + (1 - alpha) B + noise (the compositing equation, eq. 1, used forward
as an image-formation model).  It contains none of the estimation method's arithmetic and is the
one module that both the GPU path's callers and the oracle's tests draw inputs from.

The paper evaluates on a photographic dataset that is not available here; these generators stand
in for it with the shapes and statistics the workloads call for:

* ``smooth``  -- F and B are sums of 8 random low-frequency sinusoids per channel, alpha is a radial
  ramp with a 12 px transition band (the 64x64 parity workload, also used for the batch and the
  serving streams).
* ``strands`` -- the same smooth fields plus 5% mid-frequency value noise; alpha is a union of
  random ellipses plus thin cubic-Bezier "hair" strands (1-3 px wide), Gaussian-blurred with
  sigma 1.5, giving roughly 30% fractional pixels (the 1024x768 and 4096x3072 workloads).

All arithmetic is float64 numpy with PCG64 generators seeded explicitly.  Arrays are planar:
images (3, H, W), the matte (H, W).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

NOISE_SIGMA = 0.01


@dataclass
class Sample:
    I: np.ndarray        # (3, H, W) composite, clipped to [0, 1]
    alpha: np.ndarray    # (H, W) in [0, 1]
    F: np.ndarray        # (3, H, W) ground-truth foreground
    B: np.ndarray        # (3, H, W) ground-truth background
    seed: int
    kind: str

    @property
    def shape(self):
        return self.alpha.shape

    def fractional_fraction(self) -> float:
        a = self.alpha
        return float(np.mean((a > 0.0) & (a < 1.0)))


def _sinusoid_field(rng: np.random.Generator, W: int, H: int, terms: int = 8) -> np.ndarray:
    """One channel: 0.05 + 0.9 * minmax(sum_k A_k sin(2 pi (fx x / W + fy y / H) + phi_k)).

    Evaluated separably, sin(a + b) = sin a cos b + cos a sin b, so the sum is one rank-2*terms
    matrix product."""
    x = np.arange(W, dtype=np.float64)
    y = np.arange(H, dtype=np.float64)
    left = np.empty((H, 2 * terms))
    right = np.empty((2 * terms, W))
    for k in range(terms):
        fx, fy = rng.uniform(-3.0, 3.0, size=2)
        amp = rng.uniform(0.5, 1.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        ax = 2.0 * math.pi * fx * x / W + phi
        by = 2.0 * math.pi * fy * y / H
        left[:, 2 * k] = amp * np.cos(by)
        left[:, 2 * k + 1] = amp * np.sin(by)
        right[2 * k] = np.sin(ax)
        right[2 * k + 1] = np.cos(ax)
    acc = left @ right
    lo, hi = acc.min(), acc.max()
    if hi - lo < 1e-12:
        return np.full((H, W), 0.5)
    return 0.05 + 0.9 * (acc - lo) / (hi - lo)


def _lerp_upsample(grid: np.ndarray, W: int, H: int, wavelength: float) -> np.ndarray:
    """Bilinear upsampling of a coarse random grid (value noise) to H x W."""
    gx = np.arange(W, dtype=np.float64) / wavelength
    gy = np.arange(H, dtype=np.float64) / wavelength
    ix = np.floor(gx).astype(np.int64)
    iy = np.floor(gy).astype(np.int64)
    fx = gx - ix
    fy = gy - iy
    rows = grid[:, ix] * (1.0 - fx) + grid[:, ix + 1] * fx          # (gh, W)
    return rows[iy, :] * (1.0 - fy)[:, None] + rows[iy + 1, :] * fy[:, None]


def _value_noise(rng: np.random.Generator, W: int, H: int) -> np.ndarray:
    """Mid-frequency texture in [-1, 1]: value noise at 16, 32 and 64 px wavelengths."""
    out = np.zeros((H, W), dtype=np.float64)
    total = 0.0
    for wl, weight in ((16.0, 0.25), (32.0, 0.35), (64.0, 0.4)):
        gw = int(math.ceil(W / wl)) + 2
        gh = int(math.ceil(H / wl)) + 2
        grid = rng.uniform(-1.0, 1.0, size=(gh, gw))
        out += weight * _lerp_upsample(grid, W, H, wl)
        total += weight
    return out / total


def _radial_ramp(W: int, H: int, band: float = 12.0) -> np.ndarray:
    """alpha = clip(0.5 + (R - r) / band), R = 0.3 min(W, H), centred."""
    R = 0.3 * min(W, H)
    x = np.arange(W, dtype=np.float64) - (W - 1) / 2.0
    y = np.arange(H, dtype=np.float64) - (H - 1) / 2.0
    r = np.sqrt(x[None, :] ** 2 + y[:, None] ** 2)
    return np.clip(0.5 + (R - r) / band, 0.0, 1.0)


def _ellipse_blob(rng: np.random.Generator, W: int, H: int, count: int = 6) -> np.ndarray:
    m = np.zeros((H, W), dtype=bool)
    x = np.arange(W, dtype=np.float64)
    y = np.arange(H, dtype=np.float64)
    s = min(W, H)
    for _ in range(count):
        cx = rng.uniform(0.3, 0.7) * W
        cy = rng.uniform(0.3, 0.7) * H
        rx = rng.uniform(0.1, 0.25) * s
        ry = rng.uniform(0.1, 0.25) * s
        th = rng.uniform(0.0, math.pi)
        c, si = math.cos(th), math.sin(th)
        dx = x[None, :] - cx
        dy = y[:, None] - cy
        u = (dx * c + dy * si) / rx
        v = (-dx * si + dy * c) / ry
        m |= (u * u + v * v) <= 1.0
    return m


def _strands(rng: np.random.Generator, W: int, H: int, count: int,
             length: float = 140.0) -> np.ndarray:
    """Rasterise `count` cubic Bezier strands 1-3 px wide (disk stamps every 0.4 px)."""
    m = np.zeros((H, W), dtype=bool)
    if count <= 0:
        return m
    p0 = np.stack([rng.uniform(0, W, count), rng.uniform(0, H, count)], axis=1)
    ang = rng.uniform(0, 2 * math.pi, count)
    ln = length * rng.uniform(0.6, 1.4, count)
    d = np.stack([np.cos(ang), np.sin(ang)], axis=1) * ln[:, None]
    bend = rng.normal(0.0, 0.35, size=(count, 2, 2)) * ln[:, None, None]
    p3 = p0 + d
    p1 = p0 + d / 3.0 + bend[:, 0]
    p2 = p0 + 2.0 * d / 3.0 + bend[:, 1]
    width = rng.uniform(1.0, 3.0, count)
    nsamp = int(math.ceil(2.5 * length / 0.4))
    t = np.linspace(0.0, 1.0, nsamp)[None, :, None]
    pts = ((1 - t) ** 3 * p0[:, None] + 3 * (1 - t) ** 2 * t * p1[:, None]
           + 3 * (1 - t) * t ** 2 * p2[:, None] + t ** 3 * p3[:, None])      # (count, nsamp, 2)
    rad = np.repeat(width / 2.0, nsamp)
    px = pts[..., 0].reshape(-1)
    py = pts[..., 1].reshape(-1)
    for oy in range(-2, 3):
        for ox in range(-2, 3):
            xx = np.floor(px).astype(np.int64) + ox
            yy = np.floor(py).astype(np.int64) + oy
            ok = (xx >= 0) & (xx < W) & (yy >= 0) & (yy < H)
            ok &= (xx + 0.5 - px) ** 2 + (yy + 0.5 - py) ** 2 <= rad ** 2
            m[yy[ok], xx[ok]] = True
    return m


def _compose(rng: np.random.Generator, F: np.ndarray, B: np.ndarray, alpha: np.ndarray,
             noise: float) -> np.ndarray:
    I = alpha[None] * F + (1.0 - alpha[None]) * B
    if noise > 0:
        I = I + rng.normal(0.0, noise, size=I.shape)
    return np.clip(I, 0.0, 1.0)


def smooth(W: int, H: int, seed: int, noise: float = NOISE_SIGMA) -> Sample:
    """Sinusoid F/B, radial-ramp alpha, composite with N(0, noise^2), all from one seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    F = np.stack([_sinusoid_field(rng, W, H) for _ in range(3)])
    B = np.stack([_sinusoid_field(rng, W, H) for _ in range(3)])
    alpha = _radial_ramp(W, H)
    I = _compose(rng, F, B, alpha, noise)
    return Sample(I=I, alpha=alpha, F=F, B=B, seed=seed, kind="smooth")


def strands(W: int, H: int, seed: int, n_strands: int, noise: float = NOISE_SIGMA,
            sigma: float = 1.5) -> Sample:
    """Textured F/B, blob plus hair-strand alpha blurred with sigma, composite with noise."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.Generator(np.random.PCG64(seed))
    F = np.stack([np.clip(_sinusoid_field(rng, W, H) + 0.05 * _value_noise(rng, W, H), 0, 1)
                  for _ in range(3)])
    B = np.stack([np.clip(_sinusoid_field(rng, W, H) + 0.05 * _value_noise(rng, W, H), 0, 1)
                  for _ in range(3)])
    hard = _ellipse_blob(rng, W, H) | _strands(rng, W, H, n_strands)
    alpha = np.clip(gaussian_filter(hard.astype(np.float64), sigma=sigma, mode="nearest"), 0, 1)
    # values within 1e-6 of 0 or 1 are snapped, so "fractional" means visibly fractional
    alpha[alpha < 1e-6] = 0.0
    alpha[alpha > 1.0 - 1e-6] = 1.0
    I = _compose(rng, F, B, alpha, noise)
    return Sample(I=I, alpha=alpha, F=F, B=B, seed=seed, kind="strands")


# --- the workloads -------------------------------------------------------------------------

def config1() -> Sample:
    """64x64, smooth generator, seed 1."""
    return smooth(64, 64, seed=1)


def config2() -> Sample:
    """1024x768, strand generator with 200 strands, seed 2."""
    return strands(1024, 768, seed=2, n_strands=200)


def config3() -> Sample:
    """4096x3072 (12.6 MP), strand generator with 16 x 200 strands, seed 3."""
    return strands(4096, 3072, seed=3, n_strands=3200)


def batch_sizes(n: int = 64, seed: int = 4, lo: int = 256, hi: int = 2048):
    """Uneven batch: W and H each uniform on the integers [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = rng.integers(lo, hi + 1, size=n)
    H = rng.integers(lo, hi + 1, size=n)
    return [(int(w), int(h)) for w, h in zip(W, H)]


def batch_image(i: int, W: int, H: int) -> Sample:
    """Image i of the uneven batch: smooth generator with seed 4000 + i."""
    return smooth(W, H, seed=4000 + i)


@dataclass
class Request:
    rid: int
    W: int
    H: int
    arrival_s: float


def serving_requests(n: int = 2000, rate_per_s: float = 100.0, seed: int = 5,
                     area_mp=(0.25, 16.0), aspect=(0.5, 2.0)) -> list[Request]:
    """Poisson arrivals; area log-uniform in area_mp megapixels, aspect uniform in `aspect`;
    W = round(sqrt(A r)), H = round(sqrt(A / r))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps)
    la, lb = math.log(area_mp[0]), math.log(area_mp[1])
    A = np.exp(rng.uniform(la, lb, size=n)) * 1e6
    r = rng.uniform(aspect[0], aspect[1], size=n)
    W = np.maximum(1, np.round(np.sqrt(A * r))).astype(int)
    H = np.maximum(1, np.round(np.sqrt(A / r))).astype(int)
    return [Request(i, int(W[i]), int(H[i]), float(t[i])) for i in range(n)]


def request_image(req: Request) -> Sample:
    """Image of a serving request: smooth generator with seed 5000 + request id."""
    return smooth(req.W, req.H, seed=5000 + req.rid)


# --- the smooth generator evaluated with torch on a device -------------------------------------

def _sinusoid_params(rng: np.random.Generator, terms: int = 8):
    """The draws of one _sinusoid_field call, in the same order."""
    out = []
    for _ in range(terms):
        fx, fy = rng.uniform(-3.0, 3.0, size=2)
        amp = rng.uniform(0.5, 1.0)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        out.append((fx, fy, amp, phi))
    return out


def smooth_device(W: int, H: int, seed: int, device, dtype=None, out_I=None, out_alpha=None,
                  noise: float = NOISE_SIGMA, return_fields: bool = False):
    """``smooth`` evaluated with torch in float32 on `device` (for workloads of thousands of
    megapixels, which NumPy would take minutes to draw).  The sinusoid parameters come from the
    same PCG64(seed) draws as ``smooth``, so F, B and alpha agree with it to float32 rounding;
    the noise is drawn from torch's generator seeded with `seed` (a different stream).  Writes
    I (3, H, W) and alpha (H, W), converted to `dtype`, into out_I / out_alpha when given."""
    import torch
    dtype = dtype or torch.float32
    rng = np.random.Generator(np.random.PCG64(seed))
    x = torch.arange(W, device=device, dtype=torch.float32)
    y = torch.arange(H, device=device, dtype=torch.float32)

    def field(params):
        fx, fy, amp, phi = (torch.tensor(v, device=device, dtype=torch.float32)
                            for v in zip(*params))
        ax = 2.0 * math.pi * fx[:, None] * x[None, :] / W + phi[:, None]       # (terms, W)
        by = 2.0 * math.pi * fy[:, None] * y[None, :] / H                      # (terms, H)
        left = torch.cat([amp[:, None] * torch.cos(by), amp[:, None] * torch.sin(by)]).T
        right = torch.cat([torch.sin(ax), torch.cos(ax)])
        acc = left @ right
        lo, hi = acc.min(), acc.max()
        return 0.05 + 0.9 * (acc - lo) / torch.clamp(hi - lo, min=1e-12)

    F = torch.stack([field(_sinusoid_params(rng)) for _ in range(3)])
    B = torch.stack([field(_sinusoid_params(rng)) for _ in range(3)])
    R = 0.3 * min(W, H)
    r = torch.sqrt((x[None, :] - (W - 1) / 2.0) ** 2 + (y[:, None] - (H - 1) / 2.0) ** 2)
    alpha = torch.clamp(0.5 + (R - r) / 12.0, 0.0, 1.0)
    I = alpha[None] * F + (1.0 - alpha[None]) * B
    if noise > 0:
        gen = torch.Generator(device=device)
        gen.manual_seed(seed)
        I = I + noise * torch.randn(I.shape, generator=gen, device=device, dtype=torch.float32)
    I = torch.clamp(I, 0.0, 1.0)
    if out_I is None:
        out_I = torch.empty((3, H, W), dtype=dtype, device=device)
    if out_alpha is None:
        out_alpha = torch.empty((H, W), dtype=dtype, device=device)
    out_I.copy_(I)
    out_alpha.copy_(alpha)
    if return_fields:
        return out_I, out_alpha, F, B
    return out_I, out_alpha
