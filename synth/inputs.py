"""Seeded synthetic image-restoration problems (FP64, host side).

The paper's experiments use toolbox test images and toolbox blur/noise
generators that are not available here (Section 4, Examples 1 and 2).  These
generators stand in for them with the same *shape* of workload: square
piecewise-constant images, defocus-like (rotated Gaussian) or shake-like
(line-segment) point spread functions, a zero or reflexive boundary, and white
Gaussian noise scaled to a relative level ``||e|| / ||b||`` (the NoiseLevel of
Section 4).

Conventions shared by every consumer:

* images and PSFs are row-major ``m x n`` float64 arrays, ``X[i, j]`` with ``i``
  the row; the PSF has the same orientation as the image;
* the PSF centre ``(l, q)`` is the 0-based index of the pixel that holds the
  PSF's peak;
* the observation is produced with the *exact* blur (the full convolution with
  the boundary condition), not with any Kronecker approximation, as the paper
  does when it builds its test problems (Section 4, Example 1).

The blur here is a data generator: a direct FFT convolution of the extended
image.  The restoration method never calls it.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from scipy.signal import fftconvolve

BC_ZERO = 0
BC_REFLEXIVE = 1

# Seed bases per configuration number c (image 1000+c, noise 2000+c,
# batch parameters 3000+c, power-iteration start 4000+c).
SEED_IMAGE = 1000
SEED_NOISE = 2000
SEED_BATCH = 3000
SEED_POWER = 4000


def make_image(m: int, n: int, seed: int, n_rect: int = 20) -> np.ndarray:
    """Sum of ``n_rect`` axis-aligned rectangles with U(0,1) intensities plus a
    smooth linear ramp, clipped to [0, 1]."""
    rng = np.random.default_rng(seed)
    x = np.zeros((m, n))
    hmin, hmax = max(1, math.ceil(m / 16)), max(1, math.ceil(m / 4))
    wmin, wmax = max(1, math.ceil(n / 16)), max(1, math.ceil(n / 4))
    for _ in range(n_rect):
        i0 = int(rng.integers(0, m))
        j0 = int(rng.integers(0, n))
        h = int(rng.integers(hmin, hmax + 1))
        w = int(rng.integers(wmin, wmax + 1))
        val = float(rng.uniform(0.0, 1.0))
        x[i0:min(m, i0 + h), j0:min(n, j0 + w)] += val
    ii = np.arange(m)[:, None] / max(1, m - 1)
    jj = np.arange(n)[None, :] / max(1, n - 1)
    x += 0.2 * ii + 0.1 * jj
    return np.clip(x, 0.0, 1.0)


def gaussian_psf(m: int, n: int, sigma=(2.0, 4.0), theta_deg: float = 30.0,
                 center: Optional[tuple] = None) -> np.ndarray:
    """Rotated anisotropic Gaussian, normalised to sum 1, peak at ``center``.

    With ``dx = j - q``, ``dy = i - l``: ``u = cos(t) dx + sin(t) dy`` and
    ``v = -sin(t) dx + cos(t) dy``; ``P ~ exp(-u^2/(2 s1^2) - v^2/(2 s2^2))``.
    ``theta_deg = 0`` (or 90) gives a separable (rank-one) PSF.
    """
    l, q = center if center is not None else (m // 2, n // 2)
    s1, s2 = float(sigma[0]), float(sigma[1])
    t = math.radians(theta_deg)
    dy = (np.arange(m) - l)[:, None].astype(np.float64)
    dx = (np.arange(n) - q)[None, :].astype(np.float64)
    u = math.cos(t) * dx + math.sin(t) * dy
    v = -math.sin(t) * dx + math.cos(t) * dy
    p = np.exp(-u * u / (2 * s1 * s1) - v * v / (2 * s2 * s2))
    return p / p.sum()


def motion_psf(m: int, n: int, length: float = 15.0, angle_deg: float = 30.0,
               center: Optional[tuple] = None) -> np.ndarray:
    """Straight-line motion blur: a segment of ``length`` pixels through the
    centre at ``angle_deg``, bilinearly splatted and normalised to sum 1."""
    l, q = center if center is not None else (m // 2, n // 2)
    t = math.radians(angle_deg)
    ns = max(2, int(math.ceil(length * 4)) + 1)
    s = np.linspace(-0.5 * length, 0.5 * length, ns)
    ys = l + s * math.sin(t)
    xs = q + s * math.cos(t)
    p = np.zeros((m, n))
    for y, x in zip(ys, xs):
        y0, x0 = int(math.floor(y)), int(math.floor(x))
        fy, fx = y - y0, x - x0
        for di, wy in ((0, 1 - fy), (1, fy)):
            for dj, wx in ((0, 1 - fx), (1, fx)):
                yy, xx = y0 + di, x0 + dj
                if 0 <= yy < m and 0 <= xx < n:
                    p[yy, xx] += wy * wx
    return p / p.sum()


def defocus_psf(m: int, n: int, radius: float = 4.0, center: Optional[tuple] = None) -> np.ndarray:
    """Out-of-focus blur: a uniform disk of ``radius`` pixels around the
    centre, each pixel weighted by the covered fraction (4 x 4 subsamples),
    normalised to sum 1."""
    l, q = center if center is not None else (m // 2, n // 2)
    sub = (np.arange(4) + 0.5) / 4.0 - 0.5
    dy = (np.arange(m) - l)[:, None, None, None] + sub[None, None, :, None]
    dx = (np.arange(n) - q)[None, :, None, None] + sub[None, None, None, :]
    p = ((dy * dy + dx * dx) <= radius * radius).mean(axis=(2, 3))
    return p / p.sum()


def blur(x: np.ndarray, psf: np.ndarray, center: tuple, bc: int) -> np.ndarray:
    """Exact spatially invariant blur of ``x`` (the data model ``b = A x``).

    ``out[i, j] = sum_{a,b} psf[a, b] * xe[i - (a - l), j - (b - q)]`` where
    ``xe`` extends ``x`` by zeros (``bc = 0``) or by half-sample symmetric
    reflection ``x[-1-t] = x[t]`` (``bc = 1``).  Implemented as a 'valid' FFT
    convolution of the extended image.
    """
    m, n = x.shape
    assert psf.shape == (m, n)
    l, q = center
    pads = ((m - 1 - l, l), (n - 1 - q, q))
    if bc == BC_ZERO:
        xe = np.pad(x, pads, mode="constant")
    elif bc == BC_REFLEXIVE:
        xe = np.pad(x, pads, mode="symmetric")
    else:
        raise ValueError("bc must be 0 (zero) or 1 (reflexive)")
    return fftconvolve(xe, psf, mode="valid")


def add_noise(b: np.ndarray, level: float, seed: int) -> np.ndarray:
    """``b + e`` with ``e = level * ||b|| * g / ||g||``, ``g`` white Gaussian."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(b.shape)
    return b + level * np.linalg.norm(b) * g / np.linalg.norm(g)


def power_start(m: int, n: int, seed: int) -> np.ndarray:
    """Random start matrix for the Lipschitz-constant power iteration."""
    return np.random.default_rng(seed).standard_normal((m, n))


@dataclasses.dataclass
class Problem:
    name: str
    x_true: np.ndarray
    psf: np.ndarray
    center: tuple
    bc: int
    r: int
    lam: float
    iters: int
    noise_level: float
    b: np.ndarray          # exact blurred image
    bobs: np.ndarray       # observed image b + e
    v0: np.ndarray         # power-iteration start
    precision: str

    @property
    def shape(self):
        return self.x_true.shape


def _problem(name, m, n, psf, bc, r, lam, iters, nl, c, precision, seed_shift=0):
    x = make_image(m, n, SEED_IMAGE + c + seed_shift)
    center = (m // 2, n // 2)
    b = blur(x, psf, center, bc)
    bobs = add_noise(b, nl, SEED_NOISE + c + seed_shift)
    v0 = power_start(m, n, SEED_POWER + c + seed_shift)
    return Problem(name, x, psf, center, bc, r, lam, iters, nl, b, bobs, v0, precision)


WORKLOADS = {   # the named single-image workloads, by number
    1: dict(name="fp64-64", n=64, sigma=(2.0, 4.0), theta=30.0, bc=BC_ZERO, r=3,
            nl=0.01, lam=0.02, iters=100, precision="fp64"),
    2: dict(name="fp32-512", n=512, sigma=(3.0, 8.0), theta=45.0, bc=BC_REFLEXIVE, r=5,
            nl=0.005, lam=0.01, iters=200, precision="fp32"),
    3: dict(name="bf16x3-2048", n=2048, sigma=(4.0, 12.0), theta=30.0, bc=BC_REFLEXIVE, r=5,
            nl=0.01, lam=0.02, iters=300, precision="bf16x3"),
}


def config(c: int, n: Optional[int] = None, iters: Optional[int] = None) -> Problem:
    """Problem of workload ``c``: 1 is the FP64 64^2 case (zero boundary,
    r = 3), 2 the FP32 512^2 case (reflexive, r = 5), 3 the BF16X3 2048^2
    precision study (reflexive, r = 5, 300 iterations).  ``n`` overrides the
    image size (same generator recipe, used for reduced-size test cases)."""
    cfg = WORKLOADS[c]
    size = cfg["n"] if n is None else n
    psf = gaussian_psf(size, size, cfg["sigma"], cfg["theta"])
    return _problem(cfg["name"], size, size, psf, cfg["bc"], cfg["r"], cfg["lam"],
                    cfg["iters"] if iters is None else iters, cfg["nl"], c,
                    cfg["precision"])


def batch_problems(count: int = 64, seed: int = SEED_BATCH + 4, sizes=None,
                   iters: int = 100) -> List[Problem]:
    """Uneven batch: square n in {128, 192, ..., 1024}, per-image rotated
    Gaussian or motion PSF, reflexive/zero boundary, rank r in {1..8},
    lambda log-uniform in [1e-3, 1e-1], 1% noise."""
    rng = np.random.default_rng(seed)
    choices = list(range(128, 1025, 64)) if sizes is None else list(sizes)
    out = []
    for t in range(count):
        n = int(rng.choice(choices))
        if rng.uniform() < 0.5:
            s1 = float(rng.uniform(1.0, 6.0))
            s2 = float(rng.uniform(s1, 4.0 * s1))
            psf = gaussian_psf(n, n, (s1, s2), float(rng.uniform(0.0, 180.0)))
        else:
            psf = motion_psf(n, n, float(rng.integers(5, 32)), float(rng.uniform(0.0, 180.0)))
        bc = int(rng.integers(0, 2))
        r = int(rng.integers(1, 9))
        lam = float(10.0 ** rng.uniform(-3.0, -1.0))
        out.append(_problem(f"batch-{t}", n, n, psf, bc, r, lam, iters, 0.01, 4,
                            "fp32", seed_shift=10 * t))
    return out


def diff_problems(count: int = 8, n: int = 512, r: int = 4, iters: int = 50) -> List[Problem]:
    """Differentiable-form batch: ``count`` images of size ``n``, each blurred
    by one shared rotated Gaussian PSF (sigma = (3, 8), theta = 45 deg,
    reflexive boundary), 1% noise, lambda = 0.01, rank ``r``; the images and
    the noise differ per item (seeds of configuration 5 shifted by 10 per
    item)."""
    psf = gaussian_psf(n, n, (3.0, 8.0), 45.0)
    return [_problem(f"diff-{t}", n, n, psf, BC_REFLEXIVE, r, 0.01, iters, 0.01, 5, "fp32", seed_shift=10 * t)
            for t in range(count)]


def paper_problems(n: int = 256, iters: int = 50, lam: float = 0.02):
    """Stand-ins for the paper's experiments (Section 4): an n x n image blurred
    with a defocus disk (radius n/64) and, separately, with a motion blur
    (length n/16 at 30 deg), reflexive boundary, 1% noise.  Returns a dict
    kind -> Problem with r left at 5 (the sweep sets its own rank)."""
    out = {}
    for t, (kind, psf) in enumerate((("defocus", defocus_psf(n, n, n / 64.0)),
                                     ("motion", motion_psf(n, n, n / 16.0, 30.0)))):
        out[kind] = _problem(f"paper-{kind}", n, n, psf, BC_REFLEXIVE, 5, lam, iters, 0.01, 6, "fp64",
                             seed_shift=10 * t)
    return out
