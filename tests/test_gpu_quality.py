"""GPU parity of the MSSIM kernels (rklt_plan_mssim) against the FP64 oracle.

Bar: |MSSIM_gpu - MSSIM_oracle| <= 2e-5.  The window sums run in FP32 on
pixels minus 128, so the second moments (at most 128^2) carry an absolute
error of a few 1e-3 against C2 = 58.5 in the denominator; one window's SSIM
can move by ~5e-5 at worst and the mean over thousands of windows far less.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import quality as q
from paper_2111_14239_amd import rklt
from paper_2111_14239_amd.inputs import ar1_image

pytestmark = pytest.mark.gpu
TOL = 2e-5


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = rklt.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _run(ctx, specs, pitched=False):
    xs, dsts, descs = [], [], []
    for (H, W, rho, alpha, r, seed, with_dst) in specs:
        img = ar1_image(H, W, rho, seed)
        x = rklt.to_pitched(img) if pitched else torch.from_numpy(img).cuda()
        d = (rklt.empty_pitched(H, W) if pitched else torch.empty_like(x)) if with_dst else None
        xs.append((img, x))
        dsts.append(d)
        descs.append(rklt.image_desc(x, ctx.transform_id(8, rho, alpha), r, dst=d))
    plan = ctx.plan(descs)
    res = rklt.new_results(len(specs))
    out = torch.full((len(specs),), -7.0, dtype=torch.float64, device="cuda")
    plan.run(int(res.data_ptr()))
    plan.mssim(int(out.data_ptr()))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    plan.close()
    return xs, dsts, got


SPECS = [(64, 72, 0.9, 2.0, 10, 1, True), (8, 8, 0.95, 2.0, 64, 2, True), (136, 264, 0.5, 2.0, 3, 3, True),
         (16, 16, 0.3, 3.0, 20, 4, True), (264, 520, 0.7, 2.0, 37, 5, True), (40, 48, 0.5, 2.0, 5, 6, False),
         (1024, 1024, 0.95, 2.0, 10, 7, True), (520, 64, 0.9, 3.0, 1, 8, True)]


@pytest.mark.parametrize("pitched", [False, True])
def test_mssim_matches_oracle(ctx, pitched):
    xs, dsts, got = _run(ctx, SPECS, pitched)
    for (img, _), d, g, spec in zip(xs, dsts, got, SPECS):
        H, W = spec[:2]
        if d is None or min(H, W) < 11:
            assert math.isnan(g), spec
            continue
        want = q.mssim(img, d.cpu().numpy())
        assert abs(g - want) <= TOL, (spec, g, want)
    # deterministic: the same plan twice gives the same bits
    _, _, again = _run(ctx, SPECS, pitched)
    assert np.array_equal(np.nan_to_num(got, nan=-1), np.nan_to_num(again, nan=-1))


def test_mssim_of_identical_and_constant_images(ctx):
    # full retention reconstructs exactly: MSSIM = 1; a constant image codes
    # to itself at r = 1 with level shift 128 when its value is 128
    specs = [(128, 136, 0.9, 2.0, 64, 11, True)]
    xs, dsts, got = _run(ctx, specs)
    assert abs(got[0] - 1.0) <= 1e-6
    x = torch.full((64, 64), 128, dtype=torch.uint8, device="cuda")
    d = torch.empty_like(x)
    plan = ctx.plan([rklt.image_desc(x, ctx.transform_id(8, 0.9, 2.0), 1, dst=d)])
    res = rklt.new_results(1)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.run(int(res.data_ptr()))
    plan.mssim(int(out.data_ptr()))
    torch.cuda.synchronize()
    assert torch.equal(d, x) and abs(out.item() - 1.0) <= 1e-6
    plan.close()


def test_mssim_uneven_batch_sample(ctx):
    # a 300-image slice of the uneven batch (random pixels, coded), each
    # image's MSSIM against the oracle
    from paper_2111_14239_amd.inputs import uneven_batch
    specs = [s for s in uneven_batch(2000) if s.H * s.W <= 1 << 20][:300]
    g = torch.Generator(device="cuda")
    g.manual_seed(31)
    xs = [torch.randint(0, 256, (s.H, s.W), dtype=torch.uint8, device="cuda", generator=g) for s in specs]
    ds = [torch.empty_like(x) for x in xs]
    plan = ctx.plan([rklt.image_desc(x, ctx.transform_id(8, s.rho, s.alpha), s.r, dst=d)
                     for x, d, s in zip(xs, ds, specs)])
    res = rklt.new_results(len(specs))
    out = torch.zeros(len(specs), dtype=torch.float64, device="cuda")
    plan.run(int(res.data_ptr()))
    plan.mssim(int(out.data_ptr()))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for k in range(0, len(specs), 15):
        want = q.mssim(xs[k].cpu().numpy(), ds[k].cpu().numpy())
        assert abs(got[k] - want) <= TOL, (k, got[k], want)
    plan.close()
