"""GPU parity of the float comparison transforms (§4.1, Table 3: the exact
KLT K_rho and the DCT) against the oracle, through the C ABI.

Bars (the device codes in FP32 on the panel kernel, which takes images with a
coefficient dump, and with two-part fp16 operands and FP32 sums on the region
matrix-core kernel, which takes the others; the oracle in FP64):
  * FP32 coefficients B (scaled_out dump): |gpu - oracle| <= BTOL[N], a bound
    of FP32 accumulation over N terms twice, 128 N^2 2^-22;
  * reconstructed pixels: at most 1 LSB from the oracle, and only where the
    oracle's value lies within TIE_BAND of a rounding tie (x.5);
  * SSE: exactly sum((img - recon)^2) of the returned reconstruction;
    PSNR within the tie tolerance of the oracle's.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import metrics as m
from oracle import quality as q
from oracle import rklt_oracle as o
from oracle.float_codec import codec_float
from paper_2111_14239_amd import rklt
from paper_2111_14239_amd.inputs import ar1_image, random_image

pytestmark = pytest.mark.gpu

TIE_BAND = {4: 2e-3, 8: 2e-3, 16: 5e-3, 32: 1e-2}
PSNR_TOL = 1e-3


def btol(N):
    return 128.0 * N * N * 2.0 ** -22


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = rklt.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def oracle_matrix(kind, N):
    return m.dct_matrix(N) if kind == "dct" else o.klt(N, float(kind[1:]))


def gpu_id(ctx, kind, N):
    return ctx.float_transform_id("dct", N) if kind == "dct" else ctx.float_transform_id("klt", N, float(kind[1:]))


def run_plain(ctx, img, tid, r, ell, dump=True):
    x = torch.from_numpy(img).cuda()
    dst = torch.empty_like(x)
    scaled = torch.empty(x.numel(), dtype=torch.float32, device="cuda") if dump else None
    res = rklt.new_results(1)
    ctx.codec(rklt.image_desc(x, tid, r, dst=dst, level_shift=ell, scaled_out=scaled), int(res.data_ptr()))
    torch.cuda.synchronize()
    out = rklt.read_results(res)[0]
    out["recon"] = dst.cpu().numpy()
    out["scaled"] = scaled.cpu().numpy() if dump else None
    return out


def tie_tol(img, ref, N):
    frac = ref["pre_round"] - np.floor(ref["pre_round"])
    near = np.abs(frac - 0.5) <= TIE_BAND[N]
    e = np.abs(img.astype(np.int64) - ref["recon"].astype(np.int64))[near]
    dsse = int(np.sum(2 * e + 1))
    if dsse == 0 or ref["sse"] == 0:
        return PSNR_TOL
    lo = max(ref["sse"] - dsse, 1)
    return max(PSNR_TOL, 10 * math.log10((ref["sse"] + dsse) / lo))


def check(img, M, r, ell, got, N):
    ref = codec_float(img, M, r, ell)
    if got.get("scaled") is not None:
        nb = (img.shape[0] // N) * (img.shape[1] // N)
        err = np.abs(got["scaled"].reshape(nb, N * N).astype(np.float64) - ref["B"].reshape(nb, N * N))
        assert err.max() <= btol(N), float(err.max())
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
        assert got["psnr_db"] == pytest.approx(ref["psnr"], abs=tie_tol(img, ref, N))
    return ref, int(np.count_nonzero(diff))


KINDS = ["dct", "k0.3", "k0.4", "k0.7", "k0.8"]


@pytest.mark.parametrize("dump", [True, False])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("r", [1, 15, 40, 64])
def test_n8_arms_of_table3(ctx, kind, r, dump):
    # the paper's comparison arms at N = 8 on both kernels (panel with the
    # dump, region without); several panels and regions, ragged tails
    img = ar1_image(88, 424, 0.9, seed=r)
    tid = gpu_id(ctx, kind, 8)
    check(img, oracle_matrix(kind, 8), r, 128, run_plain(ctx, img, tid, r, 128, dump=dump), 8)


@pytest.mark.parametrize("N", [4, 16, 32])
@pytest.mark.parametrize("kind", ["dct", "k0.8"])
def test_other_block_sizes(ctx, N, kind):
    tid = gpu_id(ctx, kind, N)
    M = oracle_matrix(kind, N)
    img = random_image(3 * N + (N if N < 32 else 0), 5 * 64 + 2 * N, seed=N)
    for r in sorted({1, 3, N * N // 4, N * N}):
        for ell in (128, 0):
            check(img, M, r, ell, run_plain(ctx, img, tid, r, ell, dump=(r == N * N // 4)), N)


@pytest.mark.parametrize("dump", [True, False])
def test_full_retention_and_constant_images(ctx, dump):
    tid = gpu_id(ctx, "dct", 8)
    img = random_image(64, 192, seed=3)
    got = run_plain(ctx, img, tid, 64, 128, dump=dump)
    assert np.array_equal(got["recon"], img) and got["sse"] == 0 and math.isinf(got["psnr_db"])
    for c in (0, 17, 128, 255):
        flat = np.full((32, 136), c, dtype=np.uint8)
        got = run_plain(ctx, flat, tid, 1, 128, dump=dump)
        assert np.array_equal(got["recon"], flat) and got["sse"] == 0


def test_mixed_plan_with_rounded_and_float_transforms(ctx):
    # one plan: N = 8 matrix-core (rounded, ell 128), region kernel (rounded,
    # ell 0, and the float images: DCT, K_0.8, K_0.3)
    specs = [("rklt", 0.9, 2.0, 15, 128), ("dct", None, None, 15, 128), ("k0.8", None, None, 10, 0),
             ("rklt", 0.5, 3.0, 6, 0), ("dct", None, None, 1, 77), ("k0.3", None, None, 64, 128)]
    imgs, xs, dsts, descs = [], [], [], []
    for k, (kind, rho, alpha, r, ell) in enumerate(specs):
        img = ar1_image(64 + 8 * k, 136 + 16 * k, 0.9, seed=40 + k)
        x = torch.from_numpy(img).cuda()
        d = torch.empty_like(x)
        tid = ctx.transform_id(8, rho, alpha) if kind == "rklt" else gpu_id(ctx, kind, 8)
        imgs.append(img)
        xs.append(x)
        dsts.append(d)
        descs.append(rklt.image_desc(x, tid, r, dst=d, level_shift=ell))
    plan = ctx.plan(descs)
    assert plan.images_per_class[6] == 4 and plan.launches >= 3
    res = rklt.new_results(len(specs))
    ms = torch.zeros(len(specs), dtype=torch.float64, device="cuda")
    plan.run(int(res.data_ptr()))
    plan.mssim(int(ms.data_ptr()))
    torch.cuda.synchronize()
    out = rklt.read_results(res)
    mss = ms.cpu().numpy()
    for (kind, rho, alpha, r, ell), img, d, got, g in zip(specs, imgs, dsts, out, mss):
        got["recon"] = d.cpu().numpy()
        if kind == "rklt":
            ref = o.codec(img, 8, rho, alpha, r, ell)
            assert np.max(np.abs(got["recon"].astype(int) - ref["recon"].astype(int))) <= 1
        else:
            check(img, oracle_matrix(kind, 8), r, ell, got, 8)
        assert abs(g - q.mssim(img, got["recon"])) <= 2e-5
    plan.close()


def test_full_size_batch_sampled(ctx):
    # 1024 x 1024 images coded with the DCT and K_0.8 at r = 15 (the paper's
    # figure setting) in one plan; each image checked on two strips of block
    # rows against the oracle, and its SSE against the returned reconstruction
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    kinds = ["dct", "k0.8", "dct", "k0.4"]
    xs = [torch.randint(0, 256, (1024, 1024), dtype=torch.uint8, device="cuda", generator=gen) for _ in kinds]
    ds = [rklt.empty_pitched(1024, 1024) for _ in kinds]
    plan = ctx.plan([rklt.image_desc(x, gpu_id(ctx, k, 8), 15, dst=d) for x, d, k in zip(xs, ds, kinds)])
    res = rklt.new_results(len(kinds))
    plan.run(int(res.data_ptr()))
    torch.cuda.synchronize()
    out = rklt.read_results(res)
    for k, x, d, got in zip(kinds, xs, ds, out):
        img = x.cpu().numpy()
        rec = d.cpu().numpy()
        e = img.astype(np.int64) - rec.astype(np.int64)
        assert got["sse"] == int(np.sum(e * e))
        for y0 in (0, 1016):
            strip = img[y0:y0 + 8]
            ref = codec_float(strip, oracle_matrix(k, 8), 15, 128)
            diff = rec[y0:y0 + 8].astype(np.int64) - ref["recon"].astype(np.int64)
            assert np.max(np.abs(diff)) <= 1
            frac = ref["pre_round"] - np.floor(ref["pre_round"])
            assert np.all((np.abs(frac - 0.5) <= TIE_BAND[8])[diff != 0])
    plan.close()


def test_float_transform_registration(ctx):
    C = rklt.dct_matrix(8)
    a = ctx.add_float_transform(C)
    assert ctx.add_float_transform(C) == a            # identical M: same id
    assert ctx.add_float_transform(2.0 * C) != a      # a scaled M is another transform
    assert ctx.mfma_form(a, 15) == 0 and ctx.transform_exact(a) == (False, 0)
    with pytest.raises(rklt.RkltError) as e:
        ctx.add_float_transform(np.ones((8, 8)))
    assert e.value.status == rklt.E_SINGULAR
    bad = C.copy()
    bad[3, 3] = np.nan
    with pytest.raises(rklt.RkltError) as e:
        ctx.add_float_transform(bad)
    assert e.value.status == rklt.E_INVAL
    with pytest.raises(rklt.RkltError) as e:
        ctx.add_float_transform(rklt.dct_matrix(2))
    assert e.value.status == rklt.E_INVAL
    # integer coefficient dumps do not exist for a float transform
    x = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    coef = torch.empty(64, dtype=torch.int32, device="cuda")
    res = rklt.new_results(1)
    with pytest.raises(rklt.RkltError) as e:
        ctx.codec(rklt.image_desc(x, a, 1, dst=torch.empty_like(x), coef_out=coef), int(res.data_ptr()))
    assert e.value.status == rklt.E_INVAL and "float" in str(e.value)
    # a rounded transform with the same N keeps its own id
    assert ctx.transform_id(8, 0.9, 2.0) != a
