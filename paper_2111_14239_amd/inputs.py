"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the codec itself: it only draws images and
per-image parameters.  Images are separable first-order autoregressive (AR(1))
fields, the signal model the rounded KLT is designed for (§2.1, §4): the
paper's USC-SIPI photographs are not available, so these fields stand in.

Recipe (per image, numpy PCG64 ``default_rng(seed)``):
  e ~ N(0, 1) i.i.d., shape (H, W)
  row pass     Y[:, 0] = e[:, 0] / sqrt(1 - rho^2),  Y[:, j] = rho Y[:, j-1] + e[:, j]
  column pass  Z[0, :] = Y[0, :] / sqrt(1 - rho^2),  Z[i, :] = rho Z[i-1, :] + Y[i, :]
  z = Z (1 - rho^2)                      (unit variance, covariance rho^(|di| + |dj|))
  pixel = clip(floor(128 + 40 z + 1/2), 0, 255) as uint8
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.signal import lfilter

__all__ = ["ar1_image", "ImageSpec", "single_image", "fixed_batch", "uneven_batch",
           "large_block_batch", "serving_requests", "random_image"]


def _ar1_along(x: np.ndarray, rho: float, axis: int) -> np.ndarray:
    first = np.take(x, [0], axis=axis)
    zi = first * (1.0 / math.sqrt(1.0 - rho * rho) - 1.0)
    y, _ = lfilter([1.0], [1.0, -rho], x, axis=axis, zi=zi)
    return y


def ar1_image(H: int, W: int, rho: float, seed: int) -> np.ndarray:
    """One seeded H x W uint8 AR(1) field with correlation rho (recipe above)."""
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((H, W))
    Y = _ar1_along(e, rho, axis=1)
    Z = _ar1_along(Y, rho, axis=0)
    z = Z * (1.0 - rho * rho)
    return np.clip(np.floor(128.0 + 40.0 * z + 0.5), 0, 255).astype(np.uint8)


def random_image(H: int, W: int, seed: int) -> np.ndarray:
    """Uniform random uint8 pixels (worst case for coefficient magnitudes)."""
    return np.random.default_rng(seed).integers(0, 256, size=(H, W), dtype=np.uint8)


@dataclass
class ImageSpec:
    """One image of a workload and the parameters it is coded with."""
    H: int
    W: int
    rho: float
    alpha: float
    r: int
    seed: int
    N: int = 8
    ell: int = 128

    def image(self) -> np.ndarray:
        return ar1_image(self.H, self.W, self.rho, self.seed)


def single_image() -> ImageSpec:
    """512 x 512, rho = 0.95, N = 8, alpha = 2, level shift 128, r = 10."""
    return ImageSpec(512, 512, 0.95, 2.0, 10, seed=1000)


def fixed_batch(n: int = 256, side: int = 1024, seed0: int = 2000):
    """n images side x side; rho uniform over {0.1, 0.3, 0.5, 0.7, 0.9, 0.95},
    alpha uniform over {1, 2, 3}, and r sweeping 1..64 across the batch
    (image i gets r = 1 + i mod 64)."""
    rng = np.random.default_rng(seed0)
    rhos = rng.choice([0.1, 0.3, 0.5, 0.7, 0.9, 0.95], size=n)
    alphas = rng.choice([1.0, 2.0, 3.0], size=n)
    return [ImageSpec(side, side, float(rhos[i]), float(alphas[i]), 1 + i % 64, seed=seed0 + 1 + i)
            for i in range(n)]


def _side_multiple(x: float, N: int, lo: int) -> int:
    return max(lo, N * int(x // N))


def uneven_batch(n: int = 2000, seed0: int = 3000, lo: int = 64, hi: int = 4096):
    """n images whose long side is log-uniform in [lo, hi], aspect ratio uniform
    in [1, 4], sides multiples of 8 (at least lo), random orientation; rho
    uniform in [0.1, 0.95], r uniform in 1..64, alpha = 2."""
    rng = np.random.default_rng(seed0)
    out = []
    for i in range(n):
        L = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        a = rng.uniform(1.0, 4.0)
        long_side = _side_multiple(L, 8, lo)
        short_side = _side_multiple(L / a, 8, lo)
        H, W = (long_side, short_side) if rng.random() < 0.5 else (short_side, long_side)
        rho = float(rng.uniform(0.1, 0.95))
        r = int(rng.integers(1, 65))
        out.append(ImageSpec(H, W, rho, 2.0, r, seed=seed0 + 1 + i))
    return out


def large_block_batch(N: int, n: int = 64, side: int = 2048, seed0: int = 4000):
    """n images side x side, rho = 0.9, block length N; alpha is chosen by the
    caller from the KLT (largest entry mapped to 8); r keeps the same fraction
    of coefficients as r = 10 of 64."""
    r = max(1, math.ceil(10 * N * N / 64))
    return [ImageSpec(side, side, 0.9, float("nan"), r, seed=seed0 + 100 * N + i, N=N)
            for i in range(n)]


def serving_requests(rate: float, count: int, seed0: int = 5000, lo: int = 256, hi: int = 8192):
    """Open-loop Poisson arrivals: (arrival time in s, ImageSpec) with sides
    independently log-uniform in [lo, hi] (multiples of 8), rho uniform in
    [0.1, 0.95], r uniform in 1..64, N = 8, alpha = 2."""
    rng = np.random.default_rng(seed0 + int(rate))
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for i in range(count):
        H = _side_multiple(math.exp(rng.uniform(math.log(lo), math.log(hi))), 8, lo)
        W = _side_multiple(math.exp(rng.uniform(math.log(lo), math.log(hi))), 8, lo)
        out.append((float(t[i]), ImageSpec(H, W, float(rng.uniform(0.1, 0.95)), 2.0,
                                           int(rng.integers(1, 65)), seed=seed0 + 7919 * i)))
    return out
