"""Oracle for the rounded-KLT (RKLT) block codec.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference that the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product library and its Python binding never do, and this module
imports nothing from them.

Source: Radünz, Bayer, Cintra, "Low-complexity Rounded KLT Approximation for
Image Compression" (arXiv 2111.14239).  Everything here is float64 or exact
integer arithmetic (numpy int64 / Python ints / fractions), written step by step
in the paper's notation:

  N      block length (the paper studies N = 8)
  rho    correlation coefficient of the first-order Markov model, 0 < rho < 1
  alpha  expansion factor of the rounded KLT
  K      exact KLT of the Markov-1 model (§2.1)
  T      rounded KLT, T = round(alpha K) with round(x) = floor(x + 1/2)  (Eq. 2, §2.3)
  d, s   d = diag(T T^T), s = d^(-1/2); S = diag(s); T_hat = S T        (Eq. 1, §2.2)
  r      number of zig-zag coefficients kept per block                  (§4.1)
  ell    level shift subtracted from pixels before the forward transform

Readings where the paper is garbled or silent (each pinned by a test):
  * §2.1 prints k_ij with the index of omega and of the phase swapped; the
    orthonormal reading used here is K[k][n] = sqrt(2/(N+lambda_k)) *
    sin(omega_k (n - (N-1)/2) + (k+1) pi/2), k the basis index, n the sample.
  * omega_k is the root of the §2.1 equation in (k pi/N, (k+1) pi/N).
  * §4.1 writes the 2D transform as K A K^-1; for a non-orthogonal T the
    separable form B = T A T^T with the exact inverse T_hat^-1 is used
    (Appendix A gives T_hat A T_hat^T for the orthogonal case).
  * Reconstructed pixels are rounded with the same floor(x + 1/2) rule as T,
    clipped to [0, 255] and stored as uint8 before MSE is taken.
  * Zig-zag order is the JPEG one: (0,0), (0,1), (1,0), (2,0), (1,1), (0,2), ...
    with i the row (vertical frequency) of B.

Parity pins: every function here is pinned by ``tests/test_oracle_*.py``
against values the paper prints (tests/golden/), closed forms, library
routines and brute force.  The transform-efficiency metric for non-orthogonal
T_hat (Table 2, rows T_hat_2 and T_hat_3) is "parity unpinned": no reading
tried reproduces the printed eta.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

__all__ = [
    "OracleError",
    "markov_covariance",
    "omega_roots",
    "klt_eigenvalues",
    "klt",
    "rounded_klt",
    "scaling",
    "is_orthogonal",
    "exact_inverse",
    "zigzag_order",
    "zigzag_mask",
    "blocks_of",
    "image_of",
    "forward_blocks",
    "scaled_coefficients",
    "reconstruct_exact",
    "reconstruct_float",
    "psnr_from_mse",
    "codec",
]


class OracleError(ValueError):
    """Invalid parameters or a singular rounded transform."""


# --------------------------------------------------------------------------
# §2.1  KLT of a first-order Markov signal
# --------------------------------------------------------------------------

def markov_covariance(N: int, rho: float) -> np.ndarray:
    """R_x[i][j] = rho^|i-j|: unit-variance first-order Markov covariance (§1, §3.1.1)."""
    idx = np.arange(N)
    return np.power(float(rho), np.abs(idx[:, None] - idx[None, :]).astype(np.float64))


def _omega_equation(w: float, N: int, rho: float) -> float:
    """The §2.1 equation tan(N w) = -(1-rho^2) sin w / ((1+rho^2) cos w - 2 rho)
    with the denominators cleared:
        g(w) = sin(N w) ((1+rho^2) cos w - 2 rho) + (1-rho^2) sin w cos(N w).
    """
    return (math.sin(N * w) * ((1.0 + rho * rho) * math.cos(w) - 2.0 * rho)
            + (1.0 - rho * rho) * math.sin(w) * math.cos(N * w))


def omega_roots(N: int, rho: float) -> np.ndarray:
    """The N roots omega_0 < ... < omega_{N-1} of the §2.1 equation in (0, pi).

    Root k lies in the open interval (k pi / N, (k+1) pi / N); it is found by
    plain bisection on g.  g(0) = g(pi) = 0 are trivial roots, so the outer
    interval ends are moved inside by a tiny margin.
    """
    if not (0.0 < rho < 1.0):
        raise OracleError("rho must lie in (0, 1)")
    roots = np.empty(N, dtype=np.float64)
    margin = 1e-9 * math.pi / N
    for k in range(N):
        a = k * math.pi / N
        b = (k + 1) * math.pi / N
        if k == 0:
            a += margin
        if k == N - 1:
            b -= margin
        ga, gb = _omega_equation(a, N, rho), _omega_equation(b, N, rho)
        if ga == 0.0:
            roots[k] = a
            continue
        if gb == 0.0:
            roots[k] = b
            continue
        if (ga > 0) == (gb > 0):
            raise OracleError(f"no sign change for root {k} (N={N}, rho={rho})")
        for _ in range(200):
            m = 0.5 * (a + b)
            if m <= a or m >= b:
                break
            gm = _omega_equation(m, N, rho)
            if gm == 0.0:
                a = b = m
                break
            if (gm > 0) == (ga > 0):
                a, ga = m, gm
            else:
                b = m
        roots[k] = 0.5 * (a + b)
    return roots


def klt_eigenvalues(N: int, rho: float, omega: np.ndarray | None = None) -> np.ndarray:
    """lambda_k = (1 - rho^2) / (1 + rho^2 - 2 rho cos omega_k)  (§2.1)."""
    if omega is None:
        omega = omega_roots(N, rho)
    return (1.0 - rho * rho) / (1.0 + rho * rho - 2.0 * rho * np.cos(omega))


def klt(N: int, rho: float) -> np.ndarray:
    """Exact KLT K_N^rho (§2.1), row k = k-th basis vector, column n = sample n:
        K[k][n] = sqrt(2 / (N + lambda_k)) * sin(omega_k (n - (N-1)/2) + (k+1) pi / 2).
    """
    w = omega_roots(N, rho)
    lam = klt_eigenvalues(N, rho, w)
    K = np.empty((N, N), dtype=np.float64)
    for k in range(N):
        for n in range(N):
            K[k, n] = math.sqrt(2.0 / (N + lam[k])) * math.sin(
                w[k] * (n - (N - 1) / 2.0) + (k + 1) * math.pi / 2.0)
    return K


# --------------------------------------------------------------------------
# §2.3  Rounded KLT (Eq. 2) and §2.2 scaling (Eq. 1)
# --------------------------------------------------------------------------

def rounded_klt(N: int, rho: float, alpha: float) -> np.ndarray:
    """T = round(alpha * K_N^rho), round(x) = floor(x + 1/2) element-wise (Eq. 2)."""
    if alpha <= 0:
        raise OracleError("alpha must be positive")
    K = klt(N, rho)
    return np.floor(alpha * K + 0.5).astype(np.int64)


def _exact_det(T: np.ndarray) -> Fraction:
    M = [[Fraction(int(v)) for v in row] for row in T]
    n = len(M)
    det = Fraction(1)
    for c in range(n):
        p = next((i for i in range(c, n) if M[i][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            M[c], M[p] = M[p], M[c]
            det = -det
        det *= M[c][c]
        for i in range(c + 1, n):
            f = M[i][c] / M[c][c]
            if f:
                for j in range(c, n):
                    M[i][j] -= f * M[c][j]
    return det


def scaling(T: np.ndarray):
    """d = diag(T T^T) (integers) and s = d^(-1/2), so S = diag(s), T_hat = S T.

    Eq. (1) gives S = sqrt((T T^T)^-1) for orthogonal T and
    sqrt(diag(T T^T)^-1) otherwise; both equal diag(s) because T T^T is
    diagonal when T is orthogonal.  A zero row or det T = 0 is rejected.
    """
    T = np.asarray(T, dtype=np.int64)
    d = np.array([int(np.dot(T[i], T[i])) for i in range(T.shape[0])], dtype=np.int64)
    if np.any(d == 0) or _exact_det(T) == 0:
        raise OracleError("singular rounded transform")
    s = 1.0 / np.sqrt(d.astype(np.float64))
    return d, s


def is_orthogonal(T: np.ndarray) -> bool:
    """True when the rows of T are mutually orthogonal (T T^T diagonal)."""
    T = np.asarray(T, dtype=np.int64)
    G = T @ T.T
    return bool(np.all(G == np.diag(np.diag(G))))


def exact_inverse(T: np.ndarray):
    """Exact inverse of an integer matrix: returns (adj, det) with
    T^-1 = adj / det, adj an integer (Python int) matrix, det > 0.
    Gauss-Jordan elimination over the rationals."""
    n = T.shape[0]
    M = [[Fraction(int(T[i][j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)]
         for i in range(n)]
    for c in range(n):
        p = next((i for i in range(c, n) if M[i][c] != 0), None)
        if p is None:
            raise OracleError("singular rounded transform")
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for i in range(n):
            if i != c and M[i][c] != 0:
                f = M[i][c]
                M[i] = [a - f * b for a, b in zip(M[i], M[c])]
    inv = [row[n:] for row in M]
    den = 1
    for row in inv:
        for v in row:
            den = den * v.denominator // math.gcd(den, v.denominator)
    adj = [[int(v * den) for v in row] for row in inv]
    return adj, den


# --------------------------------------------------------------------------
# §4.1  zig-zag zonal selection
# --------------------------------------------------------------------------

def zigzag_order(N: int):
    """The standard zig-zag scan of an N x N coefficient block (§4.1), as a list
    of (i, j) with i the row of B.  Walk: start at (0,0), step right, then run
    down-left to the border, step down (or right at the bottom), run up-right
    to the border, step right (or down at the right edge), and repeat."""
    order = [(0, 0)]
    i, j = 0, 0
    down_left = False  # direction of the next diagonal run
    while len(order) < N * N:
        if not down_left:
            # step at the top/right border before a down-left run
            if j + 1 < N:
                j += 1
            else:
                i += 1
            order.append((i, j))
            while i + 1 < N and j - 1 >= 0:
                i, j = i + 1, j - 1
                order.append((i, j))
            down_left = True
        else:
            # step at the left/bottom border before an up-right run
            if i + 1 < N:
                i += 1
            else:
                j += 1
            order.append((i, j))
            while i - 1 >= 0 and j + 1 < N:
                i, j = i - 1, j + 1
                order.append((i, j))
            down_left = False
    return order


def zigzag_mask(N: int, r: int) -> np.ndarray:
    """0/1 matrix keeping the first r zig-zag positions (§4.1)."""
    if not (1 <= r <= N * N):
        raise OracleError("r must lie in [1, N^2]")
    m = np.zeros((N, N), dtype=np.int64)
    for (i, j) in zigzag_order(N)[:r]:
        m[i, j] = 1
    return m


# --------------------------------------------------------------------------
# §4.1  blockwise 2D transform, truncation, inverse, and quality measures
# --------------------------------------------------------------------------

def blocks_of(img: np.ndarray, N: int) -> np.ndarray:
    """Split an H x W image into disjoint N x N sub-blocks: shape (H/N, W/N, N, N)."""
    H, W = img.shape
    if H % N or W % N:
        raise OracleError("image sides must be multiples of N")
    return img.reshape(H // N, N, W // N, N).transpose(0, 2, 1, 3)


def image_of(blocks: np.ndarray) -> np.ndarray:
    """Inverse of blocks_of: rearrange sub-blocks into the image (§4.1)."""
    bh, bw, N, _ = blocks.shape
    return blocks.transpose(0, 2, 1, 3).reshape(bh * N, bw * N)


def forward_blocks(img: np.ndarray, T: np.ndarray, ell: int) -> np.ndarray:
    """B = T (A - ell) T^T for every N x N sub-block A, exact int64 (§4.1, Appendix A)."""
    T = np.asarray(T, dtype=np.int64)
    N = T.shape[0]
    X = blocks_of(np.asarray(img, dtype=np.int64), N) - int(ell)
    return np.matmul(np.matmul(T, X), T.T)


def scaled_coefficients(B: np.ndarray, s: np.ndarray) -> np.ndarray:
    """B_hat = T_hat (A - ell) T_hat^T = (s s^T) (.) B in float64 (Appendix A, Eq. 3)."""
    return np.outer(s, s)[None, None, :, :] * B.astype(np.float64)


def _round_half_up_div(Z, D):
    """floor(Z / D + 1/2) for integers (D > 0), exactly."""
    return (2 * Z + D) // (2 * D)


def reconstruct_exact(B: np.ndarray, mask: np.ndarray, T: np.ndarray, ell: int) -> np.ndarray:
    """Exact reconstruction (§4.1): keep the masked coefficients, apply the
    exact inverse and round.  The scaling cancels:
        T_hat^-1 (mask (.) B_hat) T_hat^-T = T^-1 (mask (.) B) T^-T
                                          = adj (mask (.) B) adj^T / det^2,
    so each pixel is the rational ell + Z / det^2, rounded as floor(x + 1/2)
    and clipped to [0, 255].  Uses int64 when the worst-case magnitude fits,
    Python integers otherwise."""
    adj, det = exact_inverse(np.asarray(T))
    Y = B * mask[None, None, :, :]
    D = det * det
    N = len(adj)
    amax = max(abs(v) for row in adj for v in row)
    ymax = int(np.max(np.abs(Y))) if Y.size else 0
    bound = N * N * amax * amax * max(ymax, 1) * 2 + D
    if bound < 2 ** 62 and D < 2 ** 62:
        A = np.array(adj, dtype=np.int64)
        Z = np.matmul(np.matmul(A, Y.astype(np.int64)), A.T)
        q = _round_half_up_div(Z, np.int64(D))
    else:
        A = np.array(adj, dtype=object)
        Z = np.matmul(np.matmul(A, Y.astype(object)), A.T)
        q = _round_half_up_div(Z, D).astype(np.int64)
    rec = np.clip(q + int(ell), 0, 255).astype(np.uint8)
    return image_of(rec)


def reconstruct_float(B: np.ndarray, mask: np.ndarray, T: np.ndarray, s: np.ndarray, ell: int):
    """Float64 reconstruction (§4.1): A' = ell + G (mask (.) B_hat) G^T with
    G = T_hat^-1 = (S T)^-1.  Returns (uint8 image, unrounded float64 image)."""
    That = np.diag(s) @ np.asarray(T, dtype=np.float64)
    G = np.linalg.inv(That)
    Bh = scaled_coefficients(B, s) * mask[None, None, :, :]
    Ap = np.matmul(np.matmul(G, Bh), G.T) + float(ell)
    rec = np.clip(np.floor(Ap + 0.5), 0, 255).astype(np.uint8)
    return image_of(rec), image_of(Ap)


def psnr_from_mse(mse: float) -> float:
    """PSNR = 10 log10(255^2 / MSE) in dB, +inf when MSE = 0 (§4.1, Table 3)."""
    if mse == 0:
        return math.inf
    return 10.0 * math.log10(255.0 * 255.0 / mse)


def codec(img: np.ndarray, N: int, rho: float, alpha: float, r: int, ell: int = 128,
          exact: bool = True) -> dict:
    """The JPEG-like compression experiment of §4.1 on one uint8 image:
    N x N blocks -> B = T (A-ell) T^T -> keep the first r zig-zag
    coefficients -> inverse -> reassemble -> SSE, MSE, PSNR.

    Returns a dict with T, d, s, B (int64 blocks), B_hat (float64 blocks),
    recon (uint8; exact rationals when ``exact`` else float64), recon_f64
    (float64-rounded uint8), pre-rounding float64 image, and sse/mse/psnr
    of ``recon``.
    """
    img = np.asarray(img)
    if img.dtype != np.uint8 or img.ndim != 2:
        raise OracleError("image must be a 2D uint8 array")
    if not (0.0 < rho < 1.0):
        raise OracleError("rho must lie in (0, 1)")
    T = rounded_klt(N, rho, alpha)
    d, s = scaling(T)
    mask = zigzag_mask(N, r)
    B = forward_blocks(img, T, ell)
    Bh = scaled_coefficients(B, s)
    rec_f, Ap = reconstruct_float(B, mask, T, s, ell)
    rec = reconstruct_exact(B, mask, T, ell) if exact else rec_f
    diff = img.astype(np.int64) - rec.astype(np.int64)
    sse = int(np.sum(diff * diff))
    mse = sse / img.size
    return {
        "T": T, "d": d, "s": s, "mask": mask, "B": B, "B_hat": Bh,
        "recon": rec, "recon_f64": rec_f, "pre_round": Ap,
        "sse": sse, "mse": mse, "psnr": psnr_from_mse(mse),
    }
