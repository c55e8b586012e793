"""GPU parity of the region matrix-core kernel (32 x 32 regions of
(32 / N)^2 blocks, N in {4, 8, 16, 32}, any level shift within its bounds)
against the oracle, through the C ABI.

Bars: the forward transform is exact int32 inside the kernel and the inverse
FP32, so reconstructed pixels are at most 1 LSB from the oracle's
exact-rational reconstruction and differ only where the oracle's value lies
within TIE_BAND of a rounding tie; SSE equals the returned reconstruction's;
PSNR within the tie tolerance.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import rklt_oracle as o
from paper_2111_14239_amd import rklt
from paper_2111_14239_amd.inputs import ar1_image, random_image

pytestmark = pytest.mark.gpu

TIE_BAND = {4: 2e-3, 8: 2e-3, 16: 5e-3, 32: 1e-2}


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = rklt.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def alpha8(N, rho):
    return 8.0 / float(np.max(np.abs(o.klt(N, rho))))


def check(img, N, rho, alpha, r, got_rec, got, ell=128):
    ref = o.codec(img, N, rho, alpha, r, ell)
    diff = got_rec.astype(np.int64) - ref["recon"].astype(np.int64)
    assert np.max(np.abs(diff)) <= 1
    if np.any(diff):
        frac = ref["pre_round"] - np.floor(ref["pre_round"])
        near = np.abs(frac - 0.5) <= TIE_BAND[N]
        assert np.all(near[diff != 0]), "a pixel away from a rounding tie differs"
    e = img.astype(np.int64) - got_rec.astype(np.int64)
    assert got["sse"] == int(np.sum(e * e))
    if ref["sse"] == 0:
        assert got["sse"] == 0 and math.isinf(got["psnr_db"])
    else:
        assert got["psnr_db"] == pytest.approx(o.psnr_from_mse(got["sse"] / img.size), abs=1e-4)
        frac = ref["pre_round"] - np.floor(ref["pre_round"])
        near = np.abs(frac - 0.5) <= TIE_BAND[N]
        ee = np.abs(img.astype(np.int64) - ref["recon"].astype(np.int64))[near]
        dsse = int(np.sum(2 * ee + 1))
        tol = 1e-3 if dsse == 0 else max(1e-3, 10 * math.log10((ref["sse"] + dsse) / max(ref["sse"] - dsse, 1)))
        assert got["psnr_db"] == pytest.approx(ref["psnr"], abs=tol)
    return int(np.count_nonzero(diff))


def run_plan(ctx, imgs, tids, rs, ells=None):
    ells = ells or [128] * len(imgs)
    xs = [torch.from_numpy(im).cuda() for im in imgs]
    ds = [rklt.empty_pitched(im.shape[0], im.shape[1]) for im in imgs]
    plan = ctx.plan([rklt.image_desc(x, t, r, dst=d, level_shift=l) for x, d, t, r, l in zip(xs, ds, tids, rs, ells)])
    res = rklt.new_results(len(imgs))
    plan.run(int(res.data_ptr()))
    torch.cuda.synchronize()
    out = rklt.read_results(res)
    recs = [d.cpu().numpy() for d in ds]
    per = plan.images_per_class
    plan.close()
    return recs, out, per


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("rho", [0.9, 0.5])
def test_region_kernel_matches_oracle(ctx, N, rho):
    alphas = [alpha8(N, rho)] + ([4.0] if N == 16 else [12.0])
    # several regions with a ragged region row and column (N = 16: sides
    # that are not multiples of 32)
    H, W = (80, 208) if N == 16 else (96, 160)
    img = ar1_image(H, W, rho, seed=N)
    for alpha in alphas:
        tid = ctx.transform_id(N, rho, alpha)
        rs = sorted({1, 3, N * N // 4, math.ceil(10 * N * N / 64), N * N})
        recs, out, per = run_plan(ctx, [img] * len(rs), [tid] * len(rs), rs)
        assert per[4] == len(rs), per
        for r, rec, got in zip(rs, recs, out):
            check(img, N, rho, alpha, r, rec, got)


@pytest.mark.parametrize("N", [4, 8, 16, 32])
def test_region_kernel_level_shifts(ctx, N):
    # any level shift (N = 8 with ell = 128 stays on the N = 8 matrix-core
    # kernel); region rows and columns cut by the image edge (N < 32)
    rho = 0.9
    alpha = alpha8(N, rho) if N != 8 else 2.0
    tid = ctx.transform_id(N, rho, alpha)
    H = 40 if N <= 8 else (48 if N == 16 else 64)
    W = 200 if N <= 8 else (208 if N == 16 else 96)
    img = ar1_image(H, W, rho, seed=60 + N)
    ells = [0, 37, 255] + ([128] if N != 8 else [])
    rs = [1, max(1, N * N // 4), N * N]
    cases = [(r, e) for r in rs for e in ells]
    recs, out, per = run_plan(ctx, [img] * len(cases), [tid] * len(cases), [r for r, _ in cases],
                              [e for _, e in cases])
    # the kernel takes a level shift while 128 L1 + |128 - ell| max|sig| <=
    # 32640 (its row sums split into two signed bytes); the rest goes to the
    # panel kernel
    T = o.rounded_klt(N, rho, alpha)
    L1, msig = int(np.abs(T).sum(1).max()), int(np.abs(T.sum(1)).max())
    fits = [128 * L1 + abs(128 - e) * msig <= 32640 for _, e in cases]
    assert per[4] == sum(fits) and per[0] == len(cases) - sum(fits), per
    assert N == 32 or all(fits)
    for (r, e), rec, got in zip(cases, recs, out):
        check(img, N, rho, alpha, r, rec, got, e)


def test_plain_path_and_random_pixels(ctx):
    for N in (16, 32):
        tid = ctx.transform_id(N, 0.9, alpha8(N, 0.9))
        img = random_image(3 * N, 5 * N, seed=N + 1)
        x = torch.from_numpy(img).cuda()
        d = torch.empty_like(x)
        res = rklt.new_results(1)
        for r in (1, N * N // 2, N * N):
            ctx.codec(rklt.image_desc(x, tid, r, dst=d), int(res.data_ptr()))
            torch.cuda.synchronize()
            check(img, N, 0.9, alpha8(N, 0.9), r, d.cpu().numpy(), rklt.read_results(res)[0])


def test_mixed_classes_in_one_plan(ctx):
    # N = 16: level shifts 128 and 0 on the region kernel, a transform
    # beyond its bounds (alpha 100: row sums of |T| beyond 255) on the panel
    # kernel
    N = 16
    a8 = alpha8(N, 0.9)
    t8 = ctx.transform_id(N, 0.9, a8)
    tbig = ctx.transform_id(N, 0.9, 100.0)
    imgs = [ar1_image(64, 96, 0.9, seed=3), ar1_image(48, 112, 0.7, seed=4), ar1_image(32, 48, 0.9, seed=5)]
    recs, out, per = run_plan(ctx, imgs, [t8, t8, tbig], [40, 64, 40], [128, 0, 128])
    assert per[4] == 2 and per[0] == 1, per
    for (img, al, r, ell), rec, got in zip(zip(imgs, [a8, a8, 100.0], [40, 64, 40], [128, 0, 128]), recs, out):
        check(img, N, 0.9, al, r, rec, got, ell)


def test_full_size_sampled(ctx):
    # 2048 x 2048 images (the block-size workload), each checked on strips of
    # block rows at the top and bottom against the oracle, SSE in full
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    for N, r in ((16, 40), (32, 1024)):
        alpha = alpha8(N, 0.9)
        tid = ctx.transform_id(N, 0.9, alpha)
        xs = [torch.randint(0, 256, (2048, 2048), dtype=torch.uint8, device="cuda", generator=gen) for _ in range(2)]
        ds = [torch.empty_like(x) for x in xs]
        plan = ctx.plan([rklt.image_desc(x, tid, r, dst=d) for x, d in zip(xs, ds)])
        assert plan.images_per_class[4] == 2
        res = rklt.new_results(2)
        plan.run(int(res.data_ptr()))
        torch.cuda.synchronize()
        out = rklt.read_results(res)
        for x, d, got in zip(xs, ds, out):
            img, rec = x.cpu().numpy(), d.cpu().numpy()
            e = img.astype(np.int64) - rec.astype(np.int64)
            assert got["sse"] == int(np.sum(e * e))
            for y0 in (0, 2048 - N):
                ref = o.codec(img[y0:y0 + N], N, 0.9, alpha, r, 128)
                diff = rec[y0:y0 + N].astype(np.int64) - ref["recon"].astype(np.int64)
                assert np.max(np.abs(diff)) <= 1
                frac = ref["pre_round"] - np.floor(ref["pre_round"])
                assert np.all((np.abs(frac - 0.5) <= TIE_BAND[N])[diff != 0])
        plan.close()


@pytest.mark.parametrize("N", [16, 32])
def test_precision_of_the_region_inverse(ctx, N):
    # the two-part fp16 inverse against the oracle's exact rational
    # reconstruction on 256 x 256 AR(1) images: every differing pixel lies
    # within the tie band, few differ, and the figures are printed (-s)
    rho = 0.9
    a = alpha8(N, rho)
    tid = ctx.transform_id(N, rho, a)
    stats = []
    for r in sorted({1, math.ceil(10 * N * N / 64), N * N // 4, N * N}):
        img = ar1_image(256, 256, rho, seed=700 + N + r)
        recs, out, per = run_plan(ctx, [img], [tid], [r])
        assert per[4] == 1
        ref = o.codec(img, N, rho, a, r, 128)
        check(img, N, rho, a, r, recs[0], out[0])
        diff = recs[0].astype(np.int64) - ref["recon"].astype(np.int64)
        frac = ref["pre_round"] - np.floor(ref["pre_round"])
        off = int(np.count_nonzero(diff))
        stats.append((r, off / diff.size, float(np.max(np.abs(frac - 0.5)[diff != 0], initial=0.0)),
                      abs(out[0]["psnr_db"] - ref["psnr"])))
        assert off / diff.size <= 2e-3
    print(f"\nN={N} region kernel: (r, share of pixels off by one, largest |x - tie| among them, |dPSNR| dB)",
          [(r, f"{s:.2e}", f"{t:.1e}", f"{p:.1e}") for r, s, t, p in stats])


def test_region_tiles_grow_for_the_largest_images(ctx):
    # 32768 x 32800 pixels at N = 16: 1,049,600 regions, more than 65535
    # tiles of the default 16 regions, so the library widens this image's
    # tiles (plain path and plan); SSE against the reconstruction (summed on
    # the device in int64) and sampled regions against the oracle
    N, rho = 16, 0.9
    a = alpha8(N, rho)
    tid = ctx.transform_id(N, rho, a)
    H, W = 32768, 32800
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9)
    x = torch.randint(0, 256, (H, W), dtype=torch.uint8, device="cuda", generator=gen)
    d = torch.empty_like(x)
    res = rklt.new_results(1)
    ctx.codec(rklt.image_desc(x, tid, 40, dst=d), int(res.data_ptr()))
    torch.cuda.synchronize()
    g = rklt.read_results(res)[0]
    assert 0 < g["tiles"] <= 65535
    sse = int(((x.to(torch.int64) - d.to(torch.int64)) ** 2).sum().item())
    assert g["sse"] == sse
    rng = np.random.default_rng(2)
    for ry, rx in rng.integers(0, [H // 32, W // 32 - 1], size=(6, 2)):
        img = x[32 * ry:32 * ry + 32, 32 * rx:32 * rx + 32].cpu().numpy()
        rec = d[32 * ry:32 * ry + 32, 32 * rx:32 * rx + 32].cpu().numpy()
        ref = o.codec(img, N, rho, a, 40, 128)
        diff = rec.astype(np.int64) - ref["recon"].astype(np.int64)
        assert np.max(np.abs(diff)) <= 1
        frac = ref["pre_round"] - np.floor(ref["pre_round"])
        assert np.all((np.abs(frac - 0.5) <= TIE_BAND[N])[diff != 0])
    # the right edge: W = 32800 leaves a half region (16 columns) per region row
    img = x[:32, W - 48:].cpu().numpy()
    rec = d[:32, W - 48:].cpu().numpy()
    ref = o.codec(img, N, rho, a, 40, 128)
    assert np.max(np.abs(rec.astype(np.int64) - ref["recon"].astype(np.int64))) <= 1
    del x, d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("N,ell", [(4, 0), (8, 0), (8, 200), (4, 128)])
def test_region_plain_path_small_blocks(ctx, N, ell):
    # one image on the plain path at N = 4 and 8 (N = 8 only with ell != 128,
    # which the N = 8 kernels do not take), sides that cut regions
    rho = 0.7
    alpha = alpha8(N, rho) if N == 4 else 2.0
    tid = ctx.transform_id(N, rho, alpha)
    img = random_image(72, 104, seed=N + ell)
    x = torch.from_numpy(img).cuda()
    d = torch.empty_like(x)
    res = rklt.new_results(1)
    for r in (1, N * N // 2, N * N):
        ctx.codec(rklt.image_desc(x, tid, r, dst=d, level_shift=ell), int(res.data_ptr()))
        torch.cuda.synchronize()
        check(img, N, rho, alpha, r, d.cpu().numpy(), rklt.read_results(res)[0], ell)


@pytest.mark.parametrize("ell", [128, 0, 77])
def test_exact_ties_round_up_on_a_dyadic_transform(ctx, ell):
    # N = 4, alpha = 2 gives the Walsh matrix (T T^T = 4 I): every product of
    # the region kernel is then exact and A' - ell has denominator 16, so a
    # share of the pixels sits exactly on a tie x + 1/2, which the paper's
    # rounding floor(A' + 1/2) takes up; the device must agree bit for bit
    T = o.rounded_klt(4, 0.9, 2.0)
    assert np.array_equal(T @ T.T, 4 * np.eye(4, dtype=T.dtype))
    tid = ctx.transform_id(4, 0.9, 2.0)
    imgs = [ar1_image(64, 96, 0.9, seed=11), random_image(40, 136, seed=12)]
    ties = 0
    for r in (1, 2, 3, 6, 10, 16):
        recs, out, per = run_plan(ctx, imgs, [tid] * 2, [r] * 2, [ell] * 2)
        assert per[4] == 2
        for img, rec, got in zip(imgs, recs, out):
            ref = o.codec(img, 4, 0.9, 2.0, r, ell)
            frac = ref["pre_round"] - np.floor(ref["pre_round"])
            ties += int(np.count_nonzero(frac == 0.5))
            assert np.array_equal(rec, ref["recon"]), (r, ell)
            assert got["sse"] == ref["sse"]
    assert ties > 100
