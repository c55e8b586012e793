"""The compression experiment of §4.1 with a float transform: the paper's
comparison arms (the exact KLT K_rho for several rho, and the DCT; Table 3).

TEST INFRASTRUCTURE ONLY (same rules as ``oracle.rklt_oracle``): imported by
tests and by nothing in the product path.  Float64 numpy.

For an N x N transform M (row k the k-th basis vector) and every disjoint
N x N sub-block A of an 8-bit image:
  B   = M (A - ell) M^T                      2D forward transform (§4.1)
  keep the first r coefficients of the zig-zag scan, zero the rest (§4.1)
  A'  = M^-1 (masked B) M^-T + ell           inverse (M^-1 = M^T when M is
                                             orthonormal, as K_rho and the DCT are)
  recon = clip(floor(A' + 1/2), 0, 255)      the same pixel rounding as the
                                             rounded-KLT arm
  SSE, MSE = SSE / (H W), PSNR = 10 log10(255^2 / MSE).
No scaling stage: M is already orthonormal (the rounded arm's S makes T_hat so).
"""
from __future__ import annotations

import numpy as np

from .rklt_oracle import OracleError, blocks_of, image_of, psnr_from_mse, zigzag_mask

__all__ = ["codec_float"]


def codec_float(img: np.ndarray, M: np.ndarray, r: int, ell: int = 128) -> dict:
    """Code one uint8 image with the float transform M, keeping r zig-zag
    coefficients per block.  Returns B (float64 blocks, every coefficient),
    mask, recon (uint8), pre_round (float64 image A'), sse, mse, psnr."""
    img = np.asarray(img)
    if img.dtype != np.uint8 or img.ndim != 2:
        raise OracleError("image must be a 2D uint8 array")
    M = np.asarray(M, dtype=np.float64)
    N = M.shape[0]
    if M.shape != (N, N):
        raise OracleError("M must be square")
    if not (1 <= r <= N * N):
        raise OracleError("r outside 1..N*N")
    X = blocks_of(img.astype(np.float64), N) - float(ell)
    B = np.matmul(np.matmul(M, X), M.T)
    mask = zigzag_mask(N, r)
    G = np.linalg.inv(M)
    Ap = np.matmul(np.matmul(G, B * mask[None, None, :, :]), G.T) + float(ell)
    rec = np.clip(np.floor(Ap + 0.5), 0, 255).astype(np.uint8)
    recon = image_of(rec)
    diff = img.astype(np.int64) - recon.astype(np.int64)
    sse = int(np.sum(diff * diff))
    mse = sse / img.size
    return {"B": B, "mask": mask, "recon": recon, "pre_round": image_of(Ap),
            "sse": sse, "mse": mse, "psnr": psnr_from_mse(mse)}
