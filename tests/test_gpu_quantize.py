"""GPU parity of the Appendix A quantiser (S folded into Q~ = Q / R) against
the oracle, through the C ABI.

Bars:
  * integer coefficients B (coef_out): bit-exact;
  * quantised, dequantised coefficients Q c (scaled_out): bit-exact (the
    codes are the same FP32 steps on both sides);
  * reconstructed pixels: at most 1 LSB from the oracle (FP64 inverse of the
    same dequantised coefficients), and only where the oracle's value lies
    within TIE_BAND of a rounding tie (the device inverse is FP32 on the
    panel kernel, two-part fp16 products with FP32 sums on the region
    kernel; images with a dump take the panel kernel, the others the region
    kernel within its bounds);
  * SSE: exactly sum((img - recon)^2) of the returned reconstruction; PSNR
    within the tie tolerance of the oracle's.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import rklt_oracle as o
from oracle.quantize import codec_quantized, quantize, quantizer_reciprocal
from paper_2111_14239_amd import rklt
from paper_2111_14239_amd.inputs import ar1_image, random_image

pytestmark = pytest.mark.gpu

TIE_BAND = {4: 2e-3, 8: 2e-3, 16: 5e-3, 32: 1e-2}
PSNR_TOL = 1e-3


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = rklt.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def ramp(N, q0, step):
    i = np.arange(N)
    return q0 + step * (i[:, None] + i[None, :]).astype(np.float64)


def unit_q(N, rho, alpha):
    _, s = o.scaling(o.rounded_klt(N, rho, alpha))
    return s[:, None] * s[None, :]


def run_plain(ctx, img, qid, r, ell, dump):
    x = torch.from_numpy(img).cuda()
    dst = torch.empty_like(x)
    coef = torch.empty(x.numel(), dtype=torch.int32, device="cuda") if dump else None
    scaled = torch.empty(x.numel(), dtype=torch.float32, device="cuda") if dump else None
    res = rklt.new_results(1)
    ctx.codec(rklt.image_desc(x, qid, r, dst=dst, level_shift=ell, coef_out=coef, scaled_out=scaled),
              int(res.data_ptr()))
    torch.cuda.synchronize()
    out = rklt.read_results(res)[0]
    out["recon"] = dst.cpu().numpy()
    out["coef"] = coef.cpu().numpy() if dump else None
    out["scaled"] = scaled.cpu().numpy() if dump else None
    return out


def check(img, N, rho, alpha, Q, r, ell, got):
    ref = codec_quantized(img, N, rho, alpha, Q, r=r, ell=ell)
    nb = (img.shape[0] // N) * (img.shape[1] // N)
    if got["coef"] is not None:
        assert np.array_equal(got["coef"].reshape(nb, N * N), ref["B"].reshape(nb, N * N))
        # the quantiser's output for every coefficient, before the zonal mask
        allc = quantize(ref["B"], quantizer_reciprocal(ref["s"], Q), np.ones((N, N), dtype=np.int64))
        want = np.float32(Q).astype(np.float32)[None, None] * allc.astype(np.float32)
        assert np.array_equal(got["scaled"].reshape(nb, N * N), want.reshape(nb, N * N))
    diff = got["recon"].astype(np.int64) - ref["recon"].astype(np.int64)
    assert np.max(np.abs(diff)) <= 1
    if np.any(diff):
        frac = ref["pre_round"] - np.floor(ref["pre_round"])
        near = np.abs(frac - 0.5) <= TIE_BAND[N]
        assert np.all(near[diff != 0]), "a pixel away from a rounding tie differs"
    e = img.astype(np.int64) - got["recon"].astype(np.int64)
    assert got["sse"] == int(np.sum(e * e))
    if ref["sse"] == 0:
        assert got["sse"] == 0 and math.isinf(got["psnr_db"])
    else:
        frac = ref["pre_round"] - np.floor(ref["pre_round"])
        near = np.abs(frac - 0.5) <= TIE_BAND[N]
        ee = np.abs(img.astype(np.int64) - ref["recon"].astype(np.int64))[near]
        dsse = int(np.sum(2 * ee + 1))
        tol = PSNR_TOL if dsse == 0 else max(PSNR_TOL, 10 * math.log10((ref["sse"] + dsse) / max(ref["sse"] - dsse, 1)))
        assert got["psnr_db"] == pytest.approx(ref["psnr"], abs=tol)
    return ref


CASES = [(8, 0.9, 2.0), (8, 0.5, 3.0), (8, 0.1, 2.0), (4, 0.7, 4.0), (16, 0.9, 6.0), (32, 0.9, 8.0)]


@pytest.mark.parametrize("N,rho,alpha", CASES)
def test_quantised_codec_matches_oracle(ctx, N, rho, alpha):
    tid = ctx.transform_id(N, rho, alpha)
    H, W = (6 * N if N < 32 else 3 * N), 2 * 128 + (3 * N if N >= 8 else 4 * N)  # ragged panel tail
    img = ar1_image(H, W, rho, seed=N)
    qs = [ramp(N, 1.0, 1.5), np.full((N, N), 3.0), ramp(N, 0.37, 0.11), unit_q(N, rho, alpha)]
    for k, Q in enumerate(qs):
        qid = ctx.add_quantizer(tid, Q)
        for r, ell, dump in ((N * N, 128, True), (max(1, N * N // 4), 0, False), (N * N, 37, False)):
            check(img, N, rho, alpha, Q, r, ell, run_plain(ctx, img, qid, r, ell, dump))


def test_limits_fine_and_coarse(ctx):
    img = random_image(64, 136, seed=3)
    tid = ctx.transform_id(8, 0.9, 2.0)
    fine = run_plain(ctx, img, ctx.add_quantizer(tid, np.full((8, 8), 1e-3)), 64, 128, False)
    assert np.array_equal(fine["recon"], img) and fine["sse"] == 0
    coarse = run_plain(ctx, img, ctx.add_quantizer(tid, np.full((8, 8), 1e6)), 64, 200, True)
    assert np.all(coarse["recon"] == 200) and not np.any(coarse["scaled"])


def test_mixed_plan_and_full_size_sample(ctx):
    # quantised and zonal images in one plan (region kernel with the
    # quantiser and the N = 8 matrix-core kernel), then 1024 x 1024 images
    # checked on strips of block rows
    tid = ctx.transform_id(8, 0.9, 2.0)
    Q = ramp(8, 2.0, 1.0)
    qid = ctx.add_quantizer(tid, Q)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    xs = [torch.randint(0, 256, (1024, 1024), dtype=torch.uint8, device="cuda", generator=gen) for _ in range(3)]
    small = ar1_image(72, 200, 0.9, seed=4)
    xs.append(torch.from_numpy(small).cuda())
    ds = [rklt.empty_pitched(x.shape[0], x.shape[1]) for x in xs]
    ids = [qid, tid, qid, qid]
    plan = ctx.plan([rklt.image_desc(x, i, 64 if i == qid else 15, dst=d) for x, d, i in zip(xs, ds, ids)])
    assert plan.images_per_class[5] == 3 and plan.images_per_class[2] == 1
    res = rklt.new_results(len(xs))
    plan.run(int(res.data_ptr()))
    torch.cuda.synchronize()
    out = rklt.read_results(res)
    for x, d, i, got in zip(xs, ds, ids, out):
        img = x.cpu().numpy()
        rec = d.cpu().numpy()
        e = img.astype(np.int64) - rec.astype(np.int64)
        assert got["sse"] == int(np.sum(e * e))
        for y0 in (0, img.shape[0] - 8):
            strip = img[y0:y0 + 8]
            ref = (codec_quantized(strip, 8, 0.9, 2.0, Q) if i == qid else o.codec(strip, 8, 0.9, 2.0, 15))
            diff = rec[y0:y0 + 8].astype(np.int64) - ref["recon"].astype(np.int64)
            assert np.max(np.abs(diff)) <= 1
            frac = ref["pre_round"] - np.floor(ref["pre_round"])
            assert np.all((np.abs(frac - 0.5) <= TIE_BAND[8])[diff != 0])
    plan.close()


def test_quantizer_registration(ctx):
    tid = ctx.transform_id(8, 0.9, 2.0)
    Q = ramp(8, 1.0, 1.0)
    a = ctx.add_quantizer(tid, Q)
    assert ctx.add_quantizer(tid, Q) == a and a != tid
    assert ctx.add_quantizer(tid, 2 * Q) != a
    assert ctx.mfma_form(a, 64) == 0 and ctx.transform_exact(a) == (False, 0)
    for bad in (np.zeros((8, 8)), np.full((8, 8), np.nan), np.full((8, 8), 2e6), -Q):
        with pytest.raises(rklt.RkltError) as e:
            ctx.add_quantizer(tid, bad)
        assert e.value.status == rklt.E_INVAL
    for bad_id in (a, ctx.float_transform_id("dct", 8), 9999, -1):
        with pytest.raises(rklt.RkltError) as e:
            ctx.add_quantizer(bad_id, Q)
        assert e.value.status == rklt.E_INVAL
