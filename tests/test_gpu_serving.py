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
