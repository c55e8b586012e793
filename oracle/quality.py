"""Mean structural similarity (MSSIM), the paper's third image-quality
measure (§4.1, which takes it from Wang et al., "Image quality assessment:
from error visibility to structural similarity", 2004).

TEST INFRASTRUCTURE ONLY (same rules as ``oracle.rklt_oracle``): imported by
tests and by nothing in the product path.  Float64 numpy.

Definition (the paper gives no parameters; these are the cited work's
defaults, see the readings in the design notes):
  window   w = 11 x 11 Gaussian, standard deviation 1.5, normalised to sum 1;
  for every window position fully inside the image ("valid" positions,
  (H - 10) (W - 10) of them):
    mu_x = sum w x,  mu_y = sum w y,
    s_xx = sum w x^2 - mu_x^2,  s_yy = sum w y^2 - mu_y^2,
    s_xy = sum w x y - mu_x mu_y,
    SSIM = (2 mu_x mu_y + C1) (2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1) (s_xx + s_yy + C2)),
    C1 = (0.01 L)^2, C2 = (0.03 L)^2, L = 255;
  MSSIM = the mean of SSIM over those positions.
"""
from __future__ import annotations

import numpy as np

__all__ = ["WINDOW", "SIGMA", "K1", "K2", "L", "gaussian_window", "ssim_map", "mssim"]

WINDOW = 11
SIGMA = 1.5
K1, K2, L = 0.01, 0.03, 255.0


def gaussian_window(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """size x size weights exp(-(i^2 + j^2) / (2 sigma^2)) about the centre,
    normalised to sum 1."""
    c = (size - 1) / 2.0
    i = np.arange(size, dtype=np.float64) - c
    g = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def _window_means(a: np.ndarray, w: np.ndarray) -> np.ndarray:
    """sum w * a over every valid window position (no padding)."""
    win = np.lib.stride_tricks.sliding_window_view(a, w.shape)
    return np.einsum("ijkl,kl->ij", win, w)


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """SSIM of every valid window position, (H - 10) x (W - 10)."""
    if x.shape != y.shape or x.ndim != 2 or min(x.shape) < WINDOW:
        raise ValueError("ssim_map: two images of one shape, both sides at least 11")
    w = gaussian_window()
    xf = x.astype(np.float64)
    yf = y.astype(np.float64)
    mx = _window_means(xf, w)
    my = _window_means(yf, w)
    sxx = _window_means(xf * xf, w) - mx * mx
    syy = _window_means(yf * yf, w) - my * my
    sxy = _window_means(xf * yf, w) - mx * my
    C1 = (K1 * L) ** 2
    C2 = (K2 * L) ** 2
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def mssim(x: np.ndarray, y: np.ndarray) -> float:
    """Mean of ssim_map(x, y)."""
    return float(np.mean(ssim_map(x, y)))
