"""Pins of the oracle's transform design (§2, §3): KLT, rounded KLT, scaling,
Algorithm 1, the §3.1 figures of merit and the §3.2 factorizations.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden/), library eigen-solvers, the DCT from scipy, or
mathematical identities that a wrong index, sign or dropped term would break.
"""
import math

import numpy as np
import pytest
import scipy.fft

from oracle import rklt_oracle as o
from oracle import metrics as m
from golden_io import matrices, table

NS = (2, 3, 4, 5, 8, 16, 32)
RHOS = (0.01, 0.1, 0.3, 0.5, 0.8, 0.95, 0.99)


@pytest.mark.parametrize("N", NS)
@pytest.mark.parametrize("rho", RHOS)
def test_omega_roots_bracketed_and_distinct(N, rho):
    w = o.omega_roots(N, rho)
    for k in range(N):
        assert k * math.pi / N < w[k] < (k + 1) * math.pi / N
    # each root solves tan(N w) = -(1-rho^2) sin w / ((1+rho^2) cos w - 2 rho)
    # in the angle sense: the two sides are the same line through the origin
    for wk in w:
        lhs = (math.sin(N * wk), math.cos(N * wk))
        rhs = (-(1 - rho ** 2) * math.sin(wk), (1 + rho ** 2) * math.cos(wk) - 2 * rho)
        cross = lhs[0] * rhs[1] - lhs[1] * rhs[0]
        assert abs(cross) <= 1e-12 * math.hypot(*rhs)


@pytest.mark.parametrize("N", NS)
@pytest.mark.parametrize("rho", RHOS)
def test_klt_is_orthonormal_eigenbasis_of_markov_covariance(N, rho):
    K = o.klt(N, rho)
    R = o.markov_covariance(N, rho)
    lam = o.klt_eigenvalues(N, rho)
    assert np.allclose(K @ K.T, np.eye(N), atol=1e-12)
    scale = float(np.max(lam))
    assert np.allclose(K @ R @ K.T, np.diag(lam), atol=1e-12 * scale * N)
    # the eigenvalues from the closed form equal a library eigen-solver's
    ref = np.linalg.eigvalsh(R)[::-1]
    assert np.allclose(np.sort(lam)[::-1], ref, atol=1e-12 * scale * N)
    # ... and decrease with k (row 0 is the most energetic basis vector)
    assert np.all(np.diff(lam) < 0)
    # rows match the library's eigenvectors up to sign
    vals, vecs = np.linalg.eigh(R)
    vecs = vecs[:, ::-1].T
    for k in range(N):
        assert abs(abs(float(np.dot(K[k], vecs[k]))) - 1.0) < 1e-9


def test_klt_rows_alternate_symmetric_antisymmetric():
    # row k has parity (-1)^k under n -> N-1-n; this is what makes the
    # butterfly A_1 of §3.2 factor every rounded KLT
    for N in (4, 8, 16, 32):
        for rho in RHOS:
            K = o.klt(N, rho)
            for k in range(N):
                assert np.allclose(K[k][::-1], (-1) ** k * K[k], atol=1e-12)


def test_table1_rounded_klt_matrices_and_scaling():
    gold = matrices("table1_rklt.txt")
    for name in ("T1", "T2", "T3", "T4"):
        g = gold[name]
        for rho in g["rho"]:
            T = o.rounded_klt(8, rho, 2.0)
            assert np.array_equal(T, g["rows"]), (name, rho)
            d, s = o.scaling(T)
            assert list(d) == g["d"]
            assert np.allclose(s, 1 / np.sqrt(np.array(g["d"], dtype=float)))
    # T_4 is the RDCT; rho = 0.95 (outside the 0.1 grid) also gives T_4
    assert np.array_equal(o.rounded_klt(8, 0.95, 2.0), gold["T4"]["rows"])
    assert np.array_equal(o.rounded_klt(8, 0.99, 2.0), gold["T4"]["rows"])


def test_orthogonality_of_table1_matrices():
    gold = matrices("table1_rklt.txt")
    assert o.is_orthogonal(gold["T1"]["rows"]) and o.is_orthogonal(gold["T4"]["rows"])
    assert not o.is_orthogonal(gold["T2"]["rows"]) and not o.is_orthogonal(gold["T3"]["rows"])


def test_algorithm1_finds_the_four_table1_matrices():
    gold = matrices("table1_rklt.txt")
    found = m.derive_matrices(8, 2.0, 0.1)
    assert [round(r, 6) for r, _ in found] == [0.1, 0.4, 0.7, 0.8]
    for (rho, T), name in zip(found, ("T1", "T2", "T3", "T4")):
        assert np.array_equal(T, gold[name]["rows"])


def test_rho_between_grid_points_gives_unlisted_matrix():
    # Between the printed intervals' 0.1-grid samples there is a narrow range
    # (about 0.38906 < rho < 0.39024) where round(2K) is T_1 with T_2's row 6.
    gold = matrices("table1_rklt.txt")
    T = o.rounded_klt(8, 0.3896, 2.0)
    expect = gold["T1"]["rows"].copy()
    expect[6] = gold["T2"]["rows"][6]
    assert np.array_equal(T, expect)
    assert not o.is_orthogonal(T)
    o.scaling(T)  # non-singular


def test_alpha_one_is_degenerate_at_n8():
    # the largest |K_ij| is below 1/2 for every rho, so round(K) = 0 (§2.3)
    for rho in (0.05, 0.1, 0.3, 0.5, 0.7, 0.9, 0.95, 0.99):
        K = o.klt(8, rho)
        assert np.max(np.abs(K)) < 0.5
        T = o.rounded_klt(8, rho, 1.0)
        assert not T.any()
        with pytest.raises(o.OracleError):
            o.scaling(T)


def test_alpha_range_bound():
    # alpha in [0, 3/(2 gamma)] keeps entries in {0, +-1}; about [0, 3.07] at N = 8 (§3)
    for rho in (0.1, 0.5, 0.9):
        gamma = np.max(np.abs(o.klt(8, rho)))
        amax = 3 / (2 * gamma)
        assert 3.0 < amax < 3.25
        T = o.rounded_klt(8, rho, amax * 0.999)
        assert set(np.unique(T)) <= {-1, 0, 1}


def test_table2_coding_and_similarity_measures():
    rows = {r[0]: r for r in table("table2_measures.txt")}
    for i, rho in ((1, 0.3), (2, 0.4), (3, 0.7), (4, 0.8)):
        K = o.klt(8, rho)
        R = o.markov_covariance(8, rho)
        kr = rows[f"K{rho}"]
        assert round(m.coding_gain(K, R), 4) == pytest.approx(float(kr[2]), abs=1e-4)
        assert m.transform_efficiency(K, R) == pytest.approx(100.0, abs=1e-9)
        T = o.rounded_klt(8, rho, 2.0)
        d, s = o.scaling(T)
        Th = np.diag(s) @ T
        tr = rows[f"That{i}"]
        assert m.total_error_energy(K, Th) == pytest.approx(float(tr[4]), abs=1e-4)
        assert m.mse_vs_klt(K, Th, R) == pytest.approx(float(tr[5]), abs=1e-4)
        if i in (1, 4):
            # orthogonal T: T_hat^-1 = T_hat^T, so both readings coincide
            assert m.coding_gain(Th, R) == pytest.approx(float(tr[2]), abs=1e-4)
            assert m.transform_efficiency(Th, R) == pytest.approx(float(tr[3]), abs=1e-4)
        else:
            # non-orthogonal T: the printed Cg is reproduced with T_hat^T in B_k
            assert m.coding_gain(Th, R, Th.T) == pytest.approx(float(tr[2]), abs=1e-4)


def test_rdct_vs_dct_reference_values():
    rows = {r[0]: r for r in table("table2_measures.txt")}
    C = m.dct_matrix(8)
    # the DCT matrix is the library's orthonormal DCT-II
    assert np.allclose(C, scipy.fft.dct(np.eye(8), norm="ortho", axis=0), atol=1e-14)
    T4 = o.rounded_klt(8, 0.95, 2.0)
    d, s = o.scaling(T4)
    Th = np.diag(s) @ T4
    R = o.markov_covariance(8, 0.95)
    ref = rows["RDCTvsDCT"]
    assert m.total_error_energy(C, Th) == pytest.approx(float(ref[4]), abs=1e-4)
    assert m.mse_vs_klt(C, Th, R) == pytest.approx(float(ref[5]), abs=1e-4)
    # the KLT tends to the DCT as rho -> 1 (§1)
    K = o.klt(8, 0.999)
    assert np.max(np.abs(np.abs(K) - np.abs(C))) < 0.02


def _adds(M):
    return int(sum(max(int(np.count_nonzero(row)) - 1, 0) for row in M))


def test_fast_algorithm_factorizations_and_addition_counts():
    g = matrices("fast_algorithm.txt")
    gold = matrices("table1_rklt.txt")
    I4, J4 = np.eye(4, dtype=np.int64), np.eye(4, dtype=np.int64)[::-1]
    A1 = np.block([[I4, J4], [J4, -I4]])
    B2 = g["B2"]["rows"]
    B2i = {
        1: [g["B21"]["rows"]],
        2: [g["B22"]["rows"]],
        3: [g["B23_F1"]["rows"], g["B23_F2"]["rows"]],
        4: [g["B24_F1"]["rows"], g["B24_F2"]["rows"]],
    }
    P = {1: g["P1"]["rows"], 2: g["P2"]["rows"], 3: g["P3"]["rows"], 4: g["P3"]["rows"]}
    Z = np.zeros((4, 4), dtype=np.int64)
    for i in (1, 2, 3, 4):
        Bi = B2i[i][0] if len(B2i[i]) == 1 else B2i[i][0] @ B2i[i][1]
        A2 = np.block([[Bi, Z], [Z, B2]])
        assert np.array_equal(P[i] @ A2 @ A1, gold[f"T{i}"]["rows"]), i
        adds = _adds(A1) + sum(_adds(F) for F in B2i[i]) + _adds(B2)
        assert adds == g["_adds"][f"T{i}"]
    # the direct form needs (nonzeros - rows) additions: 40/40/42/40
    assert [_adds(gold[f"T{i}"]["rows"]) for i in (1, 2, 3, 4)] == [40, 40, 42, 40]


def test_large_block_alpha_for_entries_up_to_eight():
    # alpha = 8 / gamma maps the largest |K_ij| to exactly 8, so |T_ij| <= 8
    for N in (4, 16, 32):
        K = o.klt(N, 0.9)
        gamma = np.max(np.abs(K))
        T = o.rounded_klt(N, 0.9, 8.0 / gamma)
        assert np.max(np.abs(T)) == 8
        o.scaling(T)
    assert o.is_orthogonal(o.rounded_klt(4, 0.9, 8.0 / np.max(np.abs(o.klt(4, 0.9)))))


def test_invalid_parameters_raise():
    with pytest.raises(o.OracleError):
        o.omega_roots(8, 0.0)
    with pytest.raises(o.OracleError):
        o.omega_roots(8, 1.0)
    with pytest.raises(o.OracleError):
        o.rounded_klt(8, 0.5, 0.0)
    with pytest.raises(o.OracleError):
        o.zigzag_mask(8, 0)
    with pytest.raises(o.OracleError):
        o.zigzag_mask(8, 65)
