"""Pins of the float-transform codec oracle (§4.1, the comparison arms of
Table 3: exact KLT and DCT).

Pins: quadruple loops on tiny images, perfect reconstruction at full
retention, Parseval for orthonormal M, the closed forms of a constant image
and of DC-only retention with the DCT, the DCT against scipy, and agreement
with the (separately pinned) exact rounded-KLT codec when the rounded
transform is orthogonal, where both arms compute the same rationals; an exact
tie (dyadic transform) pins the floor(x + 1/2) rounding.
"""
import math

import numpy as np
import pytest
import scipy.fft

from oracle import rklt_oracle as o
from oracle import metrics as m
from oracle.float_codec import codec_float
from paper_2111_14239_amd.inputs import ar1_image, random_image


def _loops(img, M, r, ell):
    """Forward, truncation and inverse as explicit sums, with M^-1 = M^T
    (M orthonormal)."""
    N = M.shape[0]
    H, W = img.shape
    keep = set(o.zigzag_order(N)[:r])
    out = np.empty((H, W))
    for by in range(0, H, N):
        for bx in range(0, W, N):
            X = [[float(img[by + a, bx + b]) - ell for b in range(N)] for a in range(N)]
            B = [[0.0] * N for _ in range(N)]
            for k in range(N):
                for l in range(N):
                    s = 0.0
                    for a in range(N):
                        for b in range(N):
                            s += M[k, a] * M[l, b] * X[a][b]
                    B[k][l] = s if (k, l) in keep else 0.0
            for a in range(N):
                for b in range(N):
                    s = 0.0
                    for k in range(N):
                        for l in range(N):
                            s += M[k, a] * M[l, b] * B[k][l]
                    out[by + a, bx + b] = s + ell
    return out


@pytest.mark.parametrize("kind", ["dct", "klt"])
@pytest.mark.parametrize("r", [1, 3, 10, 16])
def test_matches_quadruple_loops(kind, r):
    N = 4
    M = m.dct_matrix(N) if kind == "dct" else o.klt(N, 0.7)
    img = random_image(8, 12, seed=3 + r)
    got = codec_float(img, M, r, 128)
    want = _loops(img, M, r, 128)
    assert np.allclose(got["pre_round"], want, atol=1e-9)
    assert np.array_equal(got["recon"], np.clip(np.floor(want + 0.5), 0, 255).astype(np.uint8))


@pytest.mark.parametrize("N", [4, 8, 16, 32])
def test_full_retention_reconstructs(N):
    rng = np.random.default_rng(N)
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    img = random_image(2 * N, 3 * N, seed=N)
    for M in (Q, m.dct_matrix(N), o.klt(N, 0.95), np.diag(np.arange(1.0, N + 1)) @ m.dct_matrix(N)):
        res = codec_float(img, M, N * N, 128)
        assert np.allclose(res["pre_round"], img, atol=1e-8)
        assert np.array_equal(res["recon"], img) and res["sse"] == 0 and math.isinf(res["psnr"])


@pytest.mark.parametrize("N", [4, 8, 16])
def test_parseval(N):
    img = ar1_image(4 * N, 4 * N, 0.9, seed=N)
    for M in (m.dct_matrix(N), o.klt(N, 0.3)):
        B = codec_float(img, M, 1, 100)["B"]
        X = o.blocks_of(img.astype(np.float64), N) - 100.0
        assert np.allclose(np.sum(B * B, axis=(2, 3)), np.sum(X * X, axis=(2, 3)), rtol=1e-12)


@pytest.mark.parametrize("c,ell", [(0, 128), (200, 128), (77, 0), (255, 255)])
def test_constant_image_dct(c, ell):
    N = 8
    img = np.full((16, 24), c, dtype=np.uint8)
    res = codec_float(img, m.dct_matrix(N), 1, ell)
    B = res["B"]
    assert np.allclose(B[:, :, 0, 0], N * (c - ell), atol=1e-10)
    B0 = B.copy()
    B0[:, :, 0, 0] = 0
    assert np.allclose(B0, 0, atol=1e-10)
    assert np.array_equal(res["recon"], img)


def test_dc_only_dct_is_block_mean():
    N = 8
    img = random_image(32, 40, seed=5)
    res = codec_float(img, m.dct_matrix(N), 1, 128)
    means = o.blocks_of(img.astype(np.float64), N).mean(axis=(2, 3))
    want = np.repeat(np.repeat(means, N, axis=0), N, axis=1)
    assert np.allclose(res["pre_round"], want, atol=1e-10)


def test_dct_matrix_against_scipy():
    for N in (4, 8, 16, 32):
        assert np.allclose(m.dct_matrix(N), scipy.fft.dct(np.eye(N), norm="ortho", axis=0), atol=1e-14)


def test_orthogonal_rounded_transform_agrees_with_exact_arm():
    # When T T^T is diagonal, T_hat = S T is orthonormal and the rounded arm's
    # reconstruction T_hat^T (mask (.) B_hat) T_hat + ell is the float arm's
    # with M = T_hat.  The exact arm rounds the exact rationals; the float arm
    # must agree away from rounding ties.
    found = 0
    for rho in (0.1, 0.3, 0.5, 0.7, 0.9):
        for alpha in (2.0, 3.0):
            T = o.rounded_klt(8, rho, alpha)
            if not o.is_orthogonal(T):
                continue
            found += 1
            _, s = o.scaling(T)
            That = np.diag(s) @ T.astype(np.float64)
            img = ar1_image(32, 48, rho, seed=int(10 * rho))
            for r in (1, 6, 15, 40):
                exact = o.codec(img, 8, rho, alpha, r, 128)
                flt = codec_float(img, That, r, 128)
                assert np.allclose(flt["pre_round"], exact["pre_round"], atol=1e-9)
                frac = flt["pre_round"] - np.floor(flt["pre_round"])
                away = np.abs(frac - 0.5) > 1e-9
                assert np.array_equal(flt["recon"][away], exact["recon"][away])
    assert found >= 2


def test_klt_decorrelates_markov_model():
    # the KLT rows are the eigenvectors of the covariance: K R K^T is diagonal
    for N in (4, 8, 16):
        K = o.klt(N, 0.8)
        R = o.markov_covariance(N, 0.8)
        D = K @ R @ K.T
        assert np.allclose(D - np.diag(np.diag(D)), 0, atol=1e-10)
        assert np.allclose(K @ K.T, np.eye(N), atol=1e-12)


def test_rejects_bad_arguments():
    img = random_image(8, 8, seed=1)
    with pytest.raises(o.OracleError):
        codec_float(img, m.dct_matrix(8), 0)
    with pytest.raises(o.OracleError):
        codec_float(img.astype(np.int16), m.dct_matrix(8), 1)
    with pytest.raises(o.OracleError):
        codec_float(img, np.ones((8, 4)), 1)


def test_exact_tie_rounds_up():
    # an orthonormal transform with dyadic entries (Walsh-Hadamard / 2) keeps
    # every step exact, so a block mean of k + 1/2 is an exact tie under
    # DC-only retention: floor(x + 1/2) takes it up (round-half-even would
    # take 100.5 down)
    H = 0.5 * np.array([[1, 1, 1, 1], [1, 1, -1, -1], [1, -1, -1, 1], [1, -1, 1, -1]], dtype=np.float64)
    img = np.zeros((4, 8), dtype=np.uint8)
    img[:, :4] = 100
    img[:2, :2] = 101
    img[2:, 2:] = 101          # 8 of 16 pixels at 101: mean 100.5
    img[:, 4:] = 101
    img[:2, 4:6] = 102
    img[2:, 6:] = 102          # mean 101.5
    for ell in (0, 128, 200):
        res = codec_float(img, H, 1, ell)
        assert res["pre_round"][0, 0] == 100.5 and res["pre_round"][0, 4] == 101.5
        assert np.all(res["recon"][:, :4] == 101) and np.all(res["recon"][:, 4:] == 102)
