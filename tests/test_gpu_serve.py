"""GPU tests of plan reuse and of the continuous-batching server: every
request served in a mixed batch gives the same reconstruction, SSE and PSNR
as the same image coded alone with the plain path (bit-exact), whatever the
batch it landed in, the stream slot or the arena offset."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2111_14239_amd import rklt
from paper_2111_14239_amd.inputs import ar1_image, serving_requests
from paper_2111_14239_amd.serve import Server, pool_requests

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = rklt.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def plain(ctx, x, rho, alpha, r, ell=128):
    dst, res, _, _ = rklt.codec_image(ctx, x, rho, alpha, r, level_shift=ell)
    torch.cuda.synchronize()
    return dst.cpu().numpy(), rklt.read_results(res)[0]


SETS = [
    [(64, 72, 0.2, 2.0, 1, 11), (8, 8, 0.95, 2.0, 64, 12), (136, 264, 0.5, 2.0, 10, 13)],
    [(264, 520, 0.7, 2.0, 37, 14), (72, 1024, 0.3896, 2.0, 15, 15), (520, 64, 0.9, 3.0, 28, 16),
     (16, 16, 0.3, 3.0, 50, 17), (200, 200, 0.95, 2.0, 63, 18), (32, 8, 0.5, 3.0, 5, 19)],
    [(1024, 1024, 0.95, 2.0, 10, 20)],
]


def test_plan_update_reuses_one_plan(ctx):
    stream = torch.cuda.Stream()
    plan = None
    res = rklt.new_results(8)
    for specs in SETS:
        xs, dsts, descs = [], [], []
        for (H, W, rho, alpha, r, seed) in specs:
            x = torch.from_numpy(ar1_image(H, W, rho, seed)).cuda()
            d = torch.zeros_like(x)
            xs.append(x)
            dsts.append(d)
            descs.append(rklt.image_desc(x, ctx.transform_id(8, rho, alpha), r, dst=d))
        torch.cuda.synchronize()
        if plan is None:
            plan = ctx.plan(descs)
        else:
            plan.update(descs, stream)
        assert plan.n == len(specs)
        assert plan.pixels == sum(H * W for (H, W, *_) in specs)
        plan.run(int(res.data_ptr()), stream)
        stream.synchronize()
        got = rklt.read_results(res[:len(specs) * rklt.RESULT_BYTES])
        for x, d, g, (H, W, rho, alpha, r, seed) in zip(xs, dsts, got, specs):
            rec, alone = plain(ctx, x, rho, alpha, r)
            assert np.array_equal(d.cpu().numpy(), rec), (H, W, rho)
            assert (g["sse"], g["psnr_db"]) == (alone["sse"], alone["psnr_db"]), (H, W, rho)
    # an empty update leaves a plan that refuses to run
    with pytest.raises(rklt.RkltError):
        plan.update([], stream)
    with pytest.raises(rklt.RkltError):
        plan.run(int(res.data_ptr()), stream)
    plan.close()


def _pool(side=512):
    rhos = [0.1, 0.3, 0.5, 0.7, 0.9, 0.95]
    return [torch.from_numpy(ar1_image(side, side, r, 900 + k)).cuda() for k, r in enumerate(rhos)], rhos


@pytest.mark.parametrize("streams,arena_kib,burst", [(2, 4096, True), (2, 4096, False), (3, 600, False),
                                                     (1, 300, True)])
def test_server_results_match_plain_path(ctx, streams, arena_kib, burst):
    pool, rhos = _pool()
    items = serving_requests(rate=20000.0, count=80, seed0=6100 + streams, lo=8, hi=512)
    if burst:  # everything arrives at once: batches must form
        items = [(0.0, spec) for _, spec in items]
    reqs = pool_requests(items, pool, rhos)
    out = {}

    def keep(req, dst):
        out[id(req)] = dst.clone()

    srv = Server(ctx, arena_kib * 1024, streams=streams, max_batch=16)
    summary = srv.serve(reqs, on_done=keep)
    torch.cuda.synchronize()
    assert summary["served"] == len(reqs) and summary["rejected"] == 0
    if burst:
        assert summary["batches"] < len(reqs) // 4  # requests were batched together
    assert srv.arena.in_use == 0
    for q in reqs:
        rec, alone = plain(ctx, q.src, q.rho, q.alpha, q.r)
        assert np.array_equal(out[id(q)].cpu().numpy(), rec), (q.src.shape, q.rho, q.r)
        assert (q.result["sse"], q.result["psnr_db"]) == (alone["sse"], alone["psnr_db"])
        assert q.arrival <= q.admitted <= q.launched <= q.done


def test_server_rejects_requests_larger_than_the_arena(ctx):
    pool, rhos = _pool()
    items = serving_requests(rate=5000.0, count=12, seed0=6200, lo=8, hi=64)
    reqs = pool_requests(items, pool, rhos)
    big = pool_requests([(reqs[3].arrival, items[3][1])], [pool[0]], [0.5])[0]
    big.src = pool[0]  # 512 x 512 = 256 KiB > the 128 KiB arena
    reqs[3] = big
    srv = Server(ctx, 128 * 1024, streams=2, max_batch=4)
    summary = srv.serve(reqs)
    assert summary["rejected"] == 1 and big.rejected and not big.result
    assert summary["served"] == len(reqs) - 1
    for q in reqs:
        if q is not big:
            _, alone = plain(ctx, q.src, q.rho, q.alpha, q.r)
            assert q.result["sse"] == alone["sse"]


def test_convenience_codec_and_codec_batch(ctx):
    imgs = [torch.from_numpy(ar1_image(H, W, 0.9, 70 + k)).cuda() for k, (H, W) in enumerate([(64, 64), (136, 264)])]
    rec, sse, psnr = rklt.codec(imgs[0], 0.9, 2.0, 10, ctx=ctx)
    d, res, _, _ = rklt.codec_image(ctx, imgs[0], 0.9, 2.0, 10)
    torch.cuda.synchronize()
    assert torch.equal(rec, d) and sse == rklt.read_results(res)[0]["sse"]
    recs, results = rklt.codec_batch(imgs, [(0.9, 2.0, 10), (0.5, 3.0, 33, 128, 8)], ctx=ctx)
    assert torch.equal(recs[0], rec) and results[0]["sse"] == sse and results[0]["psnr_db"] == psnr
    d1, res1, _, _ = rklt.codec_image(ctx, imgs[1], 0.5, 3.0, 33)
    torch.cuda.synchronize()
    assert torch.equal(recs[1], d1) and results[1]["sse"] == rklt.read_results(res1)[0]["sse"]
