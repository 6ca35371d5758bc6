"""Serving form: every request's result is the same alone and in the mix, and the
admitted device footprint never exceeds the budget."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def pools():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_09087_amd import synth
    p2 = synth.quantize_u16(synth.grf((512, 512), seed=16), 4096)
    p3 = synth.quantize_u16(synth.grf((64, 64, 64), seed=17), 4096)
    d2, d3 = torch.from_numpy(p2.view(np.int16)).cuda(), torch.from_numpy(p3.view(np.int16)).cuda()
    torch.cuda.synchronize()
    return p2, p3, d2, d3


def _requests(pools, rate, n, seed):
    from paper_2203_09087_amd import synth
    p2, p3, d2, d3 = pools
    reqs = synth.serving_requests(rate, n, seed=seed, side2d=(16, 512), side3d=(4, 64))
    views = []
    for q in reqs:
        o, s = q["offset"], q["shape"]
        if len(s) == 2:
            views.append((d2[o[0]:o[0] + s[0], o[1]:o[1] + s[1]], p2[o[0]:o[0] + s[0], o[1]:o[1] + s[1]]))
        else:
            views.append((d3[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]],
                          p3[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]]))
    return [q["t"] for q in reqs], views


@pytest.mark.parametrize("budget", [1 << 30, 600_000])
def test_mix_equals_alone(pools, oracle_mod, budget):
    from paper_2203_09087_amd import ecc, serve
    arrivals, views = _requests(pools, rate=20000.0, n=120, seed=21)
    say(f"case: serving 120 requests, budget {budget}")
    srv = serve.Server(budget_bytes=budget, max_batch=16, lanes=2)
    done = srv.run_open_loop(arrivals, lambda i: serve.Request(source=views[i][0], nbins=4096,
                                                               value_range=(0, 4095)))
    torch.cuda.synchronize()
    import gc
    assert gc.isenabled()             # the loop pauses the collector and restores it
    assert len(done) == len(views)
    assert srv.peak_held <= budget
    alone = ecc.Context(0, "vertex")
    by_source = {id(v[0]): v for v in views}
    for r in done:
        dev, host = by_source[id(r.source)]
        ref = alone.compute(dev.contiguous(), 4096, value_range=(0, 4095))
        torch.cuda.synchronize()
        assert np.array_equal(r.out.cpu().numpy(), ref.cpu().numpy())
    for r in done[:12]:
        dev, host = by_source[id(r.source)]
        want = oracle_mod.ecc(np.ascontiguousarray(host), 4096, "vertex", value_range=(0, 4095))
        assert np.array_equal(r.out.cpu().numpy(), want)
    alone.close()
    srv.close()
    assert srv.batches < len(views)   # requests were batched together


@pytest.mark.timeout(600)
def test_full_size_mix_equals_alone(oracle_mod):
    """The serving configuration the benchmark times: crops of a 4096^2 and a
    384^3 uint16 GRF pool (2D sides 128..4096, 3D sides 32..384, log-uniform),
    4096 bins, an 8 GiB admission budget, batches of up to 64 on two lanes, at
    5000 requests/s.  Every result equals the request computed alone; every
    25th equals the oracle."""
    from paper_2203_09087_amd import ecc, serve, synth
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("case: full-size serving pools (seeds 61, 62)")
    p2 = synth.quantize_u16(synth.grf((4096, 4096), seed=61), 4096)
    p3 = synth.quantize_u16(synth.grf((384, 384, 384), seed=62), 4096)
    d2, d3 = torch.from_numpy(p2.view(np.int16)).cuda(), torch.from_numpy(p3.view(np.int16)).cuda()
    reqs = synth.serving_requests(5000.0, 400, seed=6)
    views = []
    for q in reqs:
        o, s = q["offset"], q["shape"]
        sl = tuple(slice(a, a + b) for a, b in zip(o, s))
        views.append((d2[sl], p2[sl]) if len(s) == 2 else (d3[sl], p3[sl]))
    budget = 8 << 30
    say(f"case: serving {len(views)} full-size requests at 5000/s, budget {budget}")
    srv = serve.Server(budget_bytes=budget, max_batch=64, lanes=2)
    alone = ecc.Context(0, "vertex")
    try:
        done = srv.run_open_loop([q["t"] for q in reqs],
                                 lambda i: serve.Request(source=views[i][0], nbins=4096, value_range=(0, 4095)))
        torch.cuda.synchronize()
        assert len(done) == len(views)
        assert srv.peak_held <= budget
        by_source = {id(v[0]): v for v in views}
        for k, r in enumerate(done):
            dev, host = by_source[id(r.source)]
            got = r.out.cpu().numpy()
            ref = alone.compute(dev.contiguous(), 4096, value_range=(0, 4095))
            torch.cuda.synchronize()
            assert np.array_equal(got, ref.cpu().numpy()), (k, host.shape)
            if k % 25 == 0:
                want = oracle_mod.ecc(np.ascontiguousarray(host), 4096, "vertex", value_range=(0, 4095),
                                      threads=16)
                assert np.array_equal(got, want), (k, host.shape)
    finally:
        alone.close()
        srv.close()


def test_sources_written_on_another_stream(oracle_mod):
    """Sources still being written on a side stream when they are submitted (no
    host synchronization in between): every lane waits for the submitting
    stream before it reads them.  A long run of matrix products ahead of the
    writes on that stream would make a lane that did not wait read zeros."""
    from paper_2203_09087_amd import serve, synth
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import time
    say("case: serving sources written on a side stream")
    host = [synth.quantize_u16(synth.grf((256, 256) if i % 2 else (24, 40, 32), seed=100 + i), 4096)
            for i in range(12)]
    pinned = [torch.from_numpy(h.view(np.int16)).pin_memory() for h in host]
    srv = serve.Server(budget_bytes=1 << 30, max_batch=4, lanes=2)
    side = torch.cuda.Stream()
    reqs = []
    try:
        with torch.cuda.stream(side):
            m = torch.randn(2048, 2048, device="cuda")
            for _ in range(30):
                m = torch.tanh(m @ m)
            for i, p in enumerate(pinned):
                src = torch.zeros(p.shape, dtype=torch.int16, device="cuda")
                src.copy_(p, non_blocking=True)
                if i % 3 == 0:
                    src = src.transpose(0, 1)   # a strided source: the lane makes the copy
                r = serve.Request(source=src, nbins=4096, value_range=(0, 4095))
                r.t_arrival = time.perf_counter()
                srv.submit(r)
                reqs.append((r, i))
                del src
            srv.drain()
        torch.cuda.synchronize()
        assert len(reqs) == len(host)
        for r, i in reqs:
            assert r.done is not None and r.batch_size >= 1 and r.device_ms > 0.0
            h = np.swapaxes(host[i], 0, 1) if i % 3 == 0 else host[i]
            want = oracle_mod.ecc(np.ascontiguousarray(h), 4096, "vertex", value_range=(0, 4095))
            assert np.array_equal(r.out.cpu().numpy(), want), i
    finally:
        srv.close()


def test_bad_requests_are_refused_at_submit(oracle_mod):
    """A request the batch call would refuse (a 5D image, nbins out of range) is
    refused when submitted, so it cannot fail the batch it would have joined;
    a 4D request is served like the others."""
    from paper_2203_09087_amd import serve
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import time
    say("case: serving refuses bad requests, serves a 4D one")
    srv = serve.Server(budget_bytes=1 << 28, max_batch=4, lanes=1)
    try:
        five = torch.zeros((2, 2, 3, 4, 5), dtype=torch.uint8, device="cuda")
        with pytest.raises(ValueError):
            srv.submit(serve.Request(source=five, nbins=16))
        one = torch.zeros((7,), dtype=torch.uint8, device="cuda")
        with pytest.raises(ValueError):
            srv.submit(serve.Request(source=one, nbins=16))
        with pytest.raises(ValueError):
            srv.submit(serve.Request(source=torch.zeros((4, 4), dtype=torch.uint8, device="cuda"), nbins=0))
        rng = np.random.default_rng(9)
        img = rng.integers(0, 256, size=(3, 5, 6, 70)).astype(np.uint8)
        r = serve.Request(source=torch.from_numpy(img).cuda(), nbins=256)
        r.t_arrival = time.perf_counter()
        srv.submit(r)
        srv.drain()
        torch.cuda.synchronize()
        assert np.array_equal(r.out.cpu().numpy(), oracle_mod.ecc(img, 256, "vertex"))
    finally:
        srv.close()
