"""GPU parity of the full uneven batch: 512 uint8 images (384 2D with sides
log-uniform in [64, 2048], 128 3D with sides log-uniform in [32, 256], smoothed
noise, about 5.8e8 voxels), 256 bins, in the launch configurations the benchmark
times: one ecc_compute_batch call, and the planned batch with its launch shape
tuned and replayed from a captured HIP graph.

Every output of the vertex batch is compared with the oracle; the top batch on
every eighth image (the oracle's cost), and the planned and replayed outputs
with the eager batch, all bit for bit.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*args):
    print(*args, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_09087_amd import synth
    say("case: generating the 512-image batch (seed 5)")
    imgs = synth.batch_images(count=512, seed=5)
    dev = [torch.from_numpy(a).cuda() for a in imgs]
    yield imgs, dev
    del dev


@pytest.mark.timeout(600)
@pytest.mark.parametrize("cons", ("vertex", "top"))
def test_full_batch_matches_oracle(batch, oracle_mod, cons):
    from paper_2203_09087_amd import ecc
    imgs, dev = batch
    ctx = ecc.Context(0, cons)
    try:
        say(f"case: full batch, {cons}, ecc_compute_batch")
        outs = [o.cpu().numpy() for o in ctx.compute_batch(dev, 256)]
        torch.cuda.synchronize()
        picks = range(len(imgs)) if cons == "vertex" else range(0, len(imgs), 8)
        for i in picks:
            want = oracle_mod.ecc(imgs[i], 256, cons, threads=16)
            assert np.array_equal(outs[i], want), (i, imgs[i].shape)

        say(f"case: full batch, {cons}, planned, tuned, graph replay")
        plan = ctx.plan_batch(dev, 256)
        try:
            plan.autotune(reps=1)
            for o, w in zip(plan.outs, outs):
                assert np.array_equal(o.cpu().numpy(), w)
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                plan.launch(stream=s)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                plan.launch(stream=s)
            for k in range(2):
                for o in plan.outs:
                    o.fill_(-1)
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                for i, (o, w) in enumerate(zip(plan.outs, outs)):
                    assert np.array_equal(o.cpu().numpy(), w), (k, i)
        finally:
            plan.close()
    finally:
        ctx.close()
