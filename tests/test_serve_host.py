"""Host logic of the continuous-batching server (no GPU): the arena's
first-fit allocator and the latency summary."""
import numpy as np

from paper_2111_14239_amd.serve import Arena, Request, summarize


def test_arena_never_overlaps_and_coalesces():
    rng = np.random.default_rng(7)
    a = Arena(1 << 20)
    live = {}
    for step in range(4000):
        if live and rng.random() < 0.45:
            off = list(live)[int(rng.integers(len(live)))]
            a.free(off)
            del live[off]
        else:
            n = int(rng.integers(1, 40000))
            off = a.alloc(n)
            if off is None:
                # first fit fails only if no free range is large enough
                need = (n + 255) // 256 * 256
                assert all(size < need for _, size in a._free)
                continue
            assert off % 256 == 0 and off + n <= a.nbytes
            live[off] = n
        spans = sorted((o, o + (n + 255) // 256 * 256) for o, n in live.items())
        assert all(e0 <= s1 for (_, e0), (s1, _) in zip(spans, spans[1:])), step
        assert a.in_use == sum(e - s for s, e in spans)
        free = sorted(a._free)
        # free ranges are disjoint, never adjacent (merged) and cover the rest
        assert all(o0 + n0 < o1 for (o0, n0), (o1, _) in zip(free, free[1:]))
        assert sum(n for _, n in free) + a.in_use == a.nbytes
    for off in list(live):
        a.free(off)
    assert a._free == [(0, 1 << 20)] and a.in_use == 0


def test_arena_first_fit_and_exact_fill():
    a = Arena(4096)
    x = a.alloc(1024)
    y = a.alloc(1024)
    z = a.alloc(2048)
    assert (x, y, z) == (0, 1024, 2048) and a.alloc(1) is None
    a.free(y)
    assert a.alloc(1000) == 1024  # the hole is reused
    a.free(x)
    a.free(z)
    assert a.alloc(2049) is None  # 1024 + 2048 free but not contiguous
    a.free(1024)
    assert a.alloc(4096) == 0


def test_summary_percentiles():
    class Src:
        shape = (8, 8)
    reqs = []
    for k in range(100):
        q = Request(arrival=k * 1e-3, src=Src(), rho=0.5, alpha=2.0, r=1)
        q.done = q.arrival + (k + 1) * 1e-3  # latencies 1..100 ms
        reqs.append(q)
    rej = Request(arrival=0.0, src=Src(), rho=0.5, alpha=2.0, r=1)
    rej.rejected, rej.done = True, 0.0
    s = summarize(reqs + [rej], wall=1.0, batches=10)
    assert s["served"] == 100 and s["rejected"] == 1
    assert abs(s["p50_ms"] - 50.5) < 1e-9 and abs(s["p99_ms"] - 99.01) < 1e-9
    span = reqs[-1].done - reqs[0].arrival
    assert abs(s["throughput_mpix_s"] - 100 * 64 / span / 1e6) < 1e-12
