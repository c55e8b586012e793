"""Pins of the oracle's codec (§4.1, Appendix A): zig-zag, blockwise forward
transform, zonal truncation, inverse, reconstruction and PSNR.

Pins: brute-force quadruple loops on tiny images, the JPEG zig-zag table,
closed forms (full retention, constant-image leak), Parseval, linearity,
exact rationals against float64, and the MSE/PSNR pairs printed in Table 3.
"""
import math

import numpy as np
import pytest

from oracle import rklt_oracle as o
from golden_io import integers, matrices, table
from paper_2111_14239_amd.inputs import ar1_image, random_image


def _t(name):
    return matrices("table1_rklt.txt")[name]["rows"]


def _alpha8(N, rho=0.9):
    return 8.0 / float(np.max(np.abs(o.klt(N, rho))))


def test_zigzag_matches_jpeg_table():
    order = o.zigzag_order(8)
    assert [8 * i + j for i, j in order] == integers("jpeg_zigzag8.txt")


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32])
def test_zigzag_is_a_diagonal_walk(N):
    order = o.zigzag_order(N)
    assert sorted(order) == [(i, j) for i in range(N) for j in range(N)]
    for (i0, j0), (i1, j1) in zip(order, order[1:]):
        assert max(abs(i1 - i0), abs(j1 - j0)) == 1  # neighbouring cells
        assert i1 + j1 >= i0 + j0  # anti-diagonals never go back
    # on anti-diagonal k the row index rises when k is odd, falls when k is even
    for k in range(1, 2 * N - 1):
        rows = [i for i, j in order if i + j == k]
        assert rows == (sorted(rows) if k % 2 else sorted(rows, reverse=True))


def test_zigzag_mask_counts():
    for r in (1, 10, 15, 64):
        mk = o.zigzag_mask(8, r)
        assert mk.sum() == r
    # r = 15 keeps exactly the anti-diagonals i + j <= 4 and compresses ~77 % (§4.2)
    mk = o.zigzag_mask(8, 15)
    i, j = np.indices((8, 8))
    assert np.array_equal(mk, (i + j <= 4).astype(np.int64))
    assert round(100 * (1 - 15 / 64)) == 77


def _brute_forward(img, T, ell):
    T = [[int(v) for v in row] for row in T]
    N = len(T)
    H, W = img.shape
    out = np.zeros((H // N, W // N, N, N), dtype=np.int64)
    for by in range(H // N):
        for bx in range(W // N):
            for i in range(N):
                for j in range(N):
                    acc = 0
                    for mm in range(N):
                        for nn in range(N):
                            acc += T[i][mm] * (int(img[by * N + mm, bx * N + nn]) - ell) * T[j][nn]
                    out[by, bx, i, j] = acc
    return out


@pytest.mark.parametrize("shape", [(8, 8), (16, 24), (40, 8)])
@pytest.mark.parametrize("tname", ["T1", "T2", "T3", "T4"])
def test_forward_matches_brute_force(shape, tname):
    img = random_image(*shape, seed=100 * shape[0] + shape[1] + int(tname[1]))
    T = _t(tname)
    for ell in (0, 128, 37):
        assert np.array_equal(o.forward_blocks(img, T, ell), _brute_forward(img, T, ell))


@pytest.mark.parametrize("N", [4, 16])
def test_forward_brute_force_large_entries(N):
    T = o.rounded_klt(N, 0.9, _alpha8(N))
    img = random_image(2 * N, N, seed=N)
    assert np.array_equal(o.forward_blocks(img, T, 128), _brute_forward(img, T, 128))


def test_blocks_round_trip_and_rejects_ragged():
    img = random_image(24, 40, seed=3)
    assert np.array_equal(o.image_of(o.blocks_of(img, 8)), img)
    b = o.blocks_of(img, 8)
    assert np.array_equal(b[1, 2], img[8:16, 16:24])
    with pytest.raises(o.OracleError):
        o.blocks_of(random_image(20, 16, seed=1), 8)


def test_exact_inverse_is_an_inverse():
    for T in [_t(n) for n in ("T1", "T2", "T3", "T4")] + [
            o.rounded_klt(8, 0.3896, 2.0), o.rounded_klt(8, 0.5, 3.0),
            o.rounded_klt(4, 0.9, _alpha8(4)), o.rounded_klt(16, 0.9, _alpha8(16))]:
        adj, det = o.exact_inverse(T)
        P = np.array(adj, dtype=object) @ np.asarray(T, dtype=object)
        assert det > 0
        assert np.array_equal(P, det * np.eye(T.shape[0], dtype=np.int64).astype(object))


@pytest.mark.parametrize("tname", ["T1", "T2", "T3", "T4"])
def test_full_retention_reconstructs_exactly(tname):
    rho = {"T1": 0.2, "T2": 0.5, "T3": 0.7, "T4": 0.9}[tname]
    img = ar1_image(32, 48, rho, seed=7)
    res = o.codec(img, 8, rho, 2.0, 64, 128)
    assert np.array_equal(res["T"], _t(tname))
    assert np.array_equal(res["recon"], img)
    assert np.array_equal(res["recon_f64"], img)
    assert res["sse"] == 0 and res["psnr"] == math.inf


@pytest.mark.parametrize("N", [4, 16])
def test_full_retention_large_blocks(N):
    img = random_image(2 * N, 2 * N, seed=N)
    res = o.codec(img, N, 0.9, _alpha8(N), N * N, 128)
    assert np.array_equal(res["recon"], img) and np.array_equal(res["recon_f64"], img)


def test_constant_image_leak_closed_form():
    # Constant image c with no level shift: B = c sigma sigma^T with sigma = T 1.
    # For T_1 (T T^T = 6 I) the zig-zag r = 15 mask drops the energy
    # c^2 (sum sigma^2)^2 - c^2 sum_kept sigma_i^2 sigma_j^2 = 416 c^2, and the
    # unrounded error energy per pixel is that / (36 * 64).
    c = 128
    img = np.full((16, 16), c, np.uint8)
    res = o.codec(img, 8, 0.3, 2.0, 15, ell=0)
    sigma = _t("T1").sum(axis=1)
    assert list(sigma) == [6, 0, 2, 0, 2, 0, 2, 0]
    pre_mse = float(np.mean((res["pre_round"] - c) ** 2))
    assert pre_mse == pytest.approx(c * c * 416 / 2304, rel=1e-12)
    assert res["mse"] == pytest.approx(2965.4375, abs=1e-9)
    # T_2..T_4 only have row sums on rows 0 and 2, kept at r = 15: exact
    for rho in (0.5, 0.7, 0.9):
        assert o.codec(img, 8, rho, 2.0, 15, ell=0)["sse"] == 0
    # with the level shift of 128 every block is zero and nothing leaks
    assert o.codec(img, 8, 0.3, 2.0, 15, ell=128)["sse"] == 0


@pytest.mark.parametrize("rho", [0.2, 0.9])
def test_parseval_for_orthogonal_t(rho):
    img = ar1_image(32, 32, rho, seed=11)
    res = o.codec(img, 8, rho, 2.0, 10, 128)
    X = o.blocks_of(img.astype(np.int64), 8) - 128
    assert np.allclose(np.sum(res["B_hat"] ** 2, axis=(2, 3)), np.sum(X * X, axis=(2, 3)), rtol=1e-12)


def test_forward_is_linear_in_shifted_pixels():
    T = _t("T3")
    a, b = random_image(16, 16, 1), random_image(16, 16, 2)
    Ba, Bb = o.forward_blocks(a, T, 0), o.forward_blocks(b, T, 0)
    # B(a) + B(b) = T (a + b) T^T, with a + b formed on int64 blocks
    X = o.blocks_of(a.astype(np.int64), 8) + o.blocks_of(b.astype(np.int64), 8)
    assert np.array_equal(Ba + Bb, np.matmul(np.matmul(T, X), T.T))
    # shifting by ell subtracts ell * sigma sigma^T per block
    sig = T.sum(axis=1)
    assert np.array_equal(o.forward_blocks(a, T, 128), Ba - 128 * np.outer(sig, sig))


def test_scaled_coefficients_are_t_hat_products():
    img = random_image(16, 8, 5)
    T = _t("T2")
    d, s = o.scaling(T)
    Th = np.diag(s) @ T
    X = o.blocks_of(img.astype(np.float64), 8) - 128
    ref = np.matmul(np.matmul(Th, X), Th.T)
    assert np.allclose(o.scaled_coefficients(o.forward_blocks(img, T, 128), s), ref, rtol=0, atol=1e-9)


@pytest.mark.parametrize("rho", [0.2, 0.5, 0.7, 0.9])
@pytest.mark.parametrize("r", [1, 10, 37])
def test_exact_and_float_reconstruction_differ_only_at_ties(rho, r):
    img = ar1_image(64, 64, rho, seed=21)
    res = o.codec(img, 8, rho, 2.0, r, 128)
    diff = res["recon"].astype(int) - res["recon_f64"].astype(int)
    assert np.max(np.abs(diff)) <= 1
    frac = res["pre_round"] - np.floor(res["pre_round"])
    near_tie = np.abs(frac - 0.5) < 1e-9
    assert np.all(near_tie[diff != 0])


def test_unrounded_error_non_increasing_in_r_for_orthogonal_t():
    img = ar1_image(64, 64, 0.9, seed=5)
    prev = math.inf
    for r in range(1, 65):
        res = o.codec(img, 8, 0.9, 2.0, r, 128, exact=False)
        e = float(np.sum((res["pre_round"] - img) ** 2))
        assert e <= prev + 1e-6
        prev = e
    assert prev < 1e-12


def test_psnr_matches_table3_pairs():
    for row in table("table3_mse_psnr.txt"):
        vals = [float(v) for v in row[1:]]
        for mse, psnr in zip(vals[0::2], vals[1::2]):
            assert round(o.psnr_from_mse(mse), 3) == pytest.approx(psnr, abs=1.5e-3), row[0]
    assert o.psnr_from_mse(0) == math.inf


def test_codec_rejects_bad_input():
    img = random_image(16, 16, 1)
    with pytest.raises(o.OracleError):
        o.codec(img, 8, 0.0, 2.0, 10)
    with pytest.raises(o.OracleError):
        o.codec(img, 8, 0.5, 1.0, 10)  # round(K) = 0: singular
    with pytest.raises(o.OracleError):
        o.codec(random_image(12, 16, 1), 8, 0.5, 2.0, 10)
    with pytest.raises(o.OracleError):
        o.codec(img.astype(np.int16), 8, 0.5, 2.0, 10)
