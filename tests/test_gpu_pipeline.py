"""The smoothing + ECC pipeline (Sec. 5, "Pipeline"): the device smoothing equals
the oracle's bit for bit, and every iteration's ECC equals the oracle's ECC of
the oracle-smoothed image."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def gauss_taps(sigma=2.0):
    t = np.exp(-0.5 * (np.arange(13) - 6.0) ** 2 / sigma ** 2)
    return (t / t.sum()).astype(np.float32)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_09087_amd import ecc
    c = ecc.Context(0, "vertex")
    yield c
    c.close()


@pytest.mark.parametrize("shape", [(1, 1), (1, 300), (300, 1), (13, 14), (257, 300), (600, 513)])
def test_smoothing_matches_oracle(ctx, oracle_mod, shape):
    rng = np.random.default_rng(70)
    img = rng.standard_normal(shape).astype(np.float32)
    taps = gauss_taps()
    say(f"case: smooth13 {shape}")
    got = ctx.smooth13(torch.from_numpy(img).cuda(), taps)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle_mod.smooth13(img, taps))


def test_smoothing_in_place_and_asymmetric_taps(ctx, oracle_mod):
    rng = np.random.default_rng(71)
    img = rng.standard_normal((90, 270)).astype(np.float32)
    taps = rng.uniform(-1, 1, 13).astype(np.float32)
    say("case: smooth13 in place, asymmetric taps")
    d = torch.from_numpy(img).cuda()
    ctx.smooth13(d, taps, out=d)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), oracle_mod.smooth13(img, taps))


@pytest.mark.parametrize("cons", ["vertex", "top"])
def test_pipeline_iterations_match_oracle(oracle_mod, cons):
    from paper_2203_09087_amd import ecc, synth
    img = synth.grf((256, 256), seed=72)
    taps = gauss_taps()
    c = ecc.Context(0, cons)
    try:
        d = torch.from_numpy(img).cuda()
        host = img.copy()
        for it in range(6):
            say(f"case: pipeline {cons} iteration {it}")
            got = c.compute(d, 1024, value_range="auto")
            c.smooth13(d, taps, out=d)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), oracle_mod.ecc(host, 1024, cons, value_range="auto"))
            host = oracle_mod.smooth13(host, taps)
            assert np.array_equal(d.cpu().numpy(), host)
    finally:
        c.close()
