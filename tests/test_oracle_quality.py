"""Pins of the MSSIM oracle (the paper's third quality measure, §4.1, from
the SSIM of Wang et al. 2004): closed forms, invariants and a brute-force
evaluation that shares nothing with the oracle's vectorised one."""
import math

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import quality as q

C1 = (0.01 * 255) ** 2
C2 = (0.03 * 255) ** 2


def test_window_is_a_normalised_separable_gaussian():
    w = q.gaussian_window()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    g = np.array([math.exp(-(k - 5) ** 2 / (2 * 1.5 ** 2)) for k in range(11)])
    g /= g.sum()
    assert np.allclose(w, np.outer(g, g), rtol=0, atol=1e-16)
    assert np.array_equal(w, w.T) and np.array_equal(w, w[::-1, ::-1])


def test_identical_images_score_one():
    x = np.random.default_rng(1).integers(0, 256, (40, 37)).astype(np.uint8)
    m = q.ssim_map(x, x)
    assert m.shape == (30, 27)
    assert np.allclose(m, 1.0, rtol=0, atol=1e-12) and q.mssim(x, x) == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("a,b", [(0, 0), (0, 255), (100, 130), (255, 17)])
def test_constant_images_closed_form(a, b):
    # no variance anywhere: SSIM = (2ab + C1) / (a^2 + b^2 + C1)
    x = np.full((16, 20), a, np.uint8)
    y = np.full((16, 20), b, np.uint8)
    want = (2 * a * b + C1) / (a * a + b * b + C1)
    assert np.allclose(q.ssim_map(x, y), want, rtol=1e-12, atol=1e-12)


def test_brute_force_on_a_tiny_image():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 256, (12, 14))
    y = np.clip(x + rng.integers(-40, 41, x.shape), 0, 255)
    wts = [[math.exp(-((i - 5) ** 2 + (j - 5) ** 2) / 4.5) for j in range(11)] for i in range(11)]
    tot = sum(map(sum, wts))
    got = q.ssim_map(x.astype(np.uint8), y.astype(np.uint8))
    for r in range(2):
        for c in range(4):
            sx = sy = sxx = syy = sxy = 0.0
            for i in range(11):
                for j in range(11):
                    wt = wts[i][j] / tot
                    a, b = float(x[r + i, c + j]), float(y[r + i, c + j])
                    sx += wt * a
                    sy += wt * b
                    sxx += wt * a * a
                    syy += wt * b * b
                    sxy += wt * a * b
            vx, vy, cxy = sxx - sx * sx, syy - sy * sy, sxy - sx * sy
            want = (2 * sx * sy + C1) * (2 * cxy + C2) / ((sx * sx + sy * sy + C1) * (vx + vy + C2))
            assert got[r, c] == pytest.approx(want, rel=1e-12, abs=1e-12)


def test_mean_shift_keeps_structure_and_contrast():
    # y = x + c: the variances and the covariance equal s_xx, so SSIM reduces
    # to the luminance term, with window means from an independent routine
    rng = np.random.default_rng(9)
    x = rng.integers(0, 200, (30, 33))
    y = x + 30
    mx = correlate2d(x.astype(float), q.gaussian_window(), mode="valid")
    want = (2 * mx * (mx + 30) + C1) / (mx ** 2 + (mx + 30) ** 2 + C1)
    assert np.allclose(q.ssim_map(x.astype(np.uint8), y.astype(np.uint8)), want, rtol=1e-9, atol=1e-12)


def test_symmetry_range_and_inversion():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, (32, 32)).astype(np.uint8)
    y = np.clip(x.astype(int) + rng.integers(-60, 61, x.shape), 0, 255).astype(np.uint8)
    assert np.allclose(q.ssim_map(x, y), q.ssim_map(y, x), rtol=0, atol=1e-15)
    m = q.ssim_map(x, y)
    assert np.all(m <= 1.0 + 1e-12) and np.all(m >= -1.0 - 1e-12)
    assert 0.0 < q.mssim(x, y) < 1.0
    assert q.mssim(x, (255 - x).astype(np.uint8)) < 0.0  # inverted structure


def test_rejects_small_or_mismatched_images():
    with pytest.raises(ValueError):
        q.ssim_map(np.zeros((10, 20), np.uint8), np.zeros((10, 20), np.uint8))
    with pytest.raises(ValueError):
        q.ssim_map(np.zeros((20, 20), np.uint8), np.zeros((20, 21), np.uint8))
