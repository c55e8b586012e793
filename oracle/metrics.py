"""Figures of merit of §3.1 and the design procedure of Algorithm 1 (§3).

TEST INFRASTRUCTURE ONLY (same rules as ``oracle.rklt_oracle``): imported by
tests and by nothing in the product path.  Float64 numpy, written from the
definitions in §3.1.1-§3.1.4.
"""
from __future__ import annotations

import math

import numpy as np

from .rklt_oracle import markov_covariance, rounded_klt

__all__ = ["coding_gain", "transform_efficiency", "mse_vs_klt", "total_error_energy",
           "derive_matrices", "dct_matrix"]


def coding_gain(That: np.ndarray, R: np.ndarray, inverse: np.ndarray | None = None) -> float:
    """Unified coding gain (§3.1.1):
        Cg = 10 log10 prod_k (A_k B_k)^(-1/N),
        A_k = su((h_k^T h_k) (.) R),  h_k the k-th row of T_hat,
        B_k = ||g_k||^2,              g_k the k-th row of the inverse.
    ``inverse`` defaults to T_hat^-1.  Table 2's values for the
    non-orthogonal T_hat_2, T_hat_3 are reproduced with T_hat^T in its place
    (see the tests)."""
    N = That.shape[0]
    G = np.linalg.inv(That) if inverse is None else inverse
    total = 0.0
    for k in range(N):
        h = That[k][None, :]
        A = float(np.sum((h.T @ h) * R))
        Bk = float(np.sum(G[k] * G[k]))
        total += math.log10(A * Bk) / N
    return -10.0 * total


def transform_efficiency(That: np.ndarray, R: np.ndarray) -> float:
    """eta = 100 sum_i |r_ii| / sum_ij |r_ij| with r = T_hat R T_hat^T (§3.1.2)."""
    C = That @ R @ That.T
    return 100.0 * float(np.sum(np.abs(np.diag(C)))) / float(np.sum(np.abs(C)))


def mse_vs_klt(K: np.ndarray, That: np.ndarray, R: np.ndarray) -> float:
    """MSE = (1/N) tr{(K - T_hat) R (K - T_hat)^T} (§3.1.3)."""
    D = K - That
    return float(np.trace(D @ R @ D.T)) / K.shape[0]


def total_error_energy(K: np.ndarray, That: np.ndarray) -> float:
    """epsilon = pi ||K - T_hat||_F^2 (§3.1.4)."""
    return math.pi * float(np.sum((K - That) ** 2))


def derive_matrices(N: int, alpha: float, step: float):
    """Algorithm 1: sweep rho over step, 2 step, ..., 1 - step and collect each
    T' = round(alpha K^rho) that differs from the previous one.  Returns a list
    of (first rho, T)."""
    out = []
    prev = np.zeros((N, N), dtype=np.int64)
    count = int(round(1.0 / step)) - 1
    for i in range(1, count + 1):
        rho = i * step
        Tp = rounded_klt(N, rho, alpha)
        if not np.array_equal(Tp, prev):
            out.append((rho, Tp))
            prev = Tp
    return out


def dct_matrix(N: int) -> np.ndarray:
    """Orthonormal DCT-II matrix, C[k][n] = c_k cos(pi (2n+1) k / (2N))."""
    C = np.empty((N, N))
    for k in range(N):
        ck = math.sqrt(1.0 / N) if k == 0 else math.sqrt(2.0 / N)
        for n in range(N):
            C[k, n] = ck * math.cos(math.pi * (2 * n + 1) * k / (2 * N))
    return C


def covariance(N: int, rho: float) -> np.ndarray:
    return markov_covariance(N, rho)
