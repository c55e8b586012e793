"""The quantisation step of Appendix A for the rounded KLT: the scaling
matrix S folded into a JPEG-style quantisation matrix.

TEST INFRASTRUCTURE ONLY (same rules as ``oracle.rklt_oracle``): imported by
tests and by nothing in the product path.

Appendix A: with R = s s^T (s = diag S, T orthogonal) the scaled
coefficients are T_hat A T_hat^T = R (.) B, B = T A T^T the exact integer
transform, and quantising them with Q,
    B_bar = round((R (.) B) / Q) = round(B / Q~),   Q~ = Q / R,
needs no multiplication by S: the scaling lives in Q~.  The decoder
multiplies the codes by Q (the dequantised scaled coefficients) and applies
T_hat^-1 on both sides, as the zonal codec of §4.1 does with its kept
coefficients.

Readings (the Appendix gives neither a decoder nor a precision):
  * round(x) = floor(x + 1/2), the paper's rounding of Eq. (2);
  * the division by Q~ is a decision that floating point takes, so it is
    evaluated in the precision of the device, FP32: t = fl32(B * q) with
    q = fl32((s_i s_j) / Q_ij) computed in FP64 from s_i = 1 / sqrt(d_i),
    and the code is floor(t + 1/2) taken exactly on that FP32 value;
    ``codes_f64`` gives the FP64 definition round(B s_i s_j / Q_ij), which
    the tests pin these codes to away from rounding ties;
  * the zonal mask of §4.1 still applies first (r = N^2 keeps every
    coefficient, the plain JPEG-style quantiser);
  * the dequantised coefficient is fl32(Q_ij) * c in FP32 (exact for the
    integer Q of the tests), the inverse and the pixel rounding are the
    zonal codec's: A' = T_hat^-1 (Q (.) c) T_hat^-T + ell in FP64,
    recon = clip(floor(A' + 1/2), 0, 255).
"""
from __future__ import annotations

import numpy as np

from .rklt_oracle import OracleError, forward_blocks, image_of, psnr_from_mse, rounded_klt, scaling, zigzag_mask

__all__ = ["quantizer_reciprocal", "quantize", "codes_f64", "codec_quantized"]


def quantizer_reciprocal(s: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """q_ij = fl32((s_i s_j) / Q_ij): the FP32 reciprocal of Q~ = Q / R."""
    Q = np.asarray(Q, dtype=np.float64)
    return ((s[:, None] * s[None, :]) / Q).astype(np.float32)


def quantize(B: np.ndarray, q: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Codes of the integer coefficient blocks B (shape (..., N, N)):
    floor(fl32(B q) + 1/2) on the kept positions, 0 elsewhere (int64)."""
    t = B.astype(np.float32) * q            # one FP32 rounding per product
    c = np.floor(t.astype(np.float64) + 0.5)  # exact on an FP32 value
    return (c * mask).astype(np.int64)


def codes_f64(B: np.ndarray, s: np.ndarray, Q: np.ndarray, mask: np.ndarray):
    """The FP64 definition round(B / Q~) and the unrounded quotients."""
    x = B.astype(np.float64) * (s[:, None] * s[None, :]) / np.asarray(Q, dtype=np.float64)
    return (np.floor(x + 0.5) * mask).astype(np.int64), x


def codec_quantized(img: np.ndarray, N: int, rho: float, alpha: float, Q: np.ndarray, r: int | None = None,
                    ell: int = 128) -> dict:
    """Code one uint8 image with T = round(alpha K_rho) and quantiser Q.
    Returns T, s, B (int64 blocks), codes, dequantised coefficients (FP64 of
    the FP32 products), recon (uint8), pre_round, sse, mse, psnr."""
    img = np.asarray(img)
    if img.dtype != np.uint8 or img.ndim != 2:
        raise OracleError("image must be a 2D uint8 array")
    Q = np.asarray(Q, dtype=np.float64)
    if Q.shape != (N, N) or not np.all((Q > 0) & (Q <= 1e6)):
        raise OracleError("Q must be N x N with entries in (0, 1e6]")
    r = N * N if r is None else r
    T = rounded_klt(N, rho, alpha)
    _, s = scaling(T)
    mask = zigzag_mask(N, r)
    B = forward_blocks(img, T, ell)
    codes = quantize(B, quantizer_reciprocal(s, Q), mask)
    deq = (Q.astype(np.float32) * codes.astype(np.float32)).astype(np.float64)
    That = np.diag(s) @ T.astype(np.float64)
    G = np.linalg.inv(That)
    Ap = np.matmul(np.matmul(G, deq), G.T) + float(ell)
    rec = np.clip(np.floor(Ap + 0.5), 0, 255).astype(np.uint8)
    recon = image_of(rec)
    diff = img.astype(np.int64) - recon.astype(np.int64)
    sse = int(np.sum(diff * diff))
    mse = sse / img.size
    return {"T": T, "s": s, "mask": mask, "B": B, "codes": codes, "deq": deq, "recon": recon,
            "pre_round": image_of(Ap), "sse": sse, "mse": mse, "psnr": psnr_from_mse(mse)}
