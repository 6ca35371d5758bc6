"""Streaming of host-resident images in slabs of the first axis (Sec. 4.4): the
result equals the oracle and the in-device call for every slab size, dtype,
filtration and range mode, with pinned and pageable host memory."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CONS = ("vertex", "top")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def ctxs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_09087_amd import ecc
    c = {k: ecc.Context(0, k) for k in CONS}
    yield c
    for v in c.values():
        v.close()


def _host(a, pinned):
    t = torch.from_numpy(np.ascontiguousarray(a).view(np.int16) if a.dtype == np.uint16 else np.ascontiguousarray(a))
    return t.pin_memory() if pinned else t


def _image(rng, shape, dtype):
    if dtype == np.float32:
        return rng.standard_normal(shape).astype(np.float32)
    if dtype == np.uint16:
        return rng.integers(0, 300, shape).astype(np.uint16)
    return rng.integers(0, 40, shape).astype(np.uint8)


@pytest.mark.parametrize("cons", CONS)
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
def test_streamed_matches_oracle(ctxs, oracle_mod, cons, dtype):
    rng = np.random.default_rng(60)
    img = _image(rng, (11, 37, 70), dtype)
    rng_modes = [None, "auto"] if dtype != np.float32 else ["auto", (-1.0, 1.5)]
    for r in rng_modes:
        want = oracle_mod.ecc(img, 300, cons, value_range=r)
        for slab in (0, 1, 2, 3, 10, 11, 50):
            for pinned in (True, False):
                say(f"case: streamed {cons} {img.shape} {np.dtype(dtype).name} range={r} slab={slab} pinned={pinned}")
                h = _host(img, pinned)
                got = ctxs[cons].compute_streamed(h, 300, value_range=r, slab_planes=slab)
                torch.cuda.synchronize()
                assert np.array_equal(got.cpu().numpy(), want)


@pytest.mark.parametrize("cons", CONS)
def test_streamed_wide_histogram_and_2d(ctxs, oracle_mod, cons):
    rng = np.random.default_rng(61)
    img = rng.integers(0, 9000, (9, 20, 130)).astype(np.uint16)
    want = oracle_mod.ecc(img, 9000, cons, value_range=(0, 8999))
    say(f"case: streamed {cons} 9000 bins, slabs of 2")
    got = ctxs[cons].compute_streamed(_host(img, True), 9000, value_range=(0, 8999), slab_planes=2)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    img2 = rng.standard_normal((45, 300)).astype(np.float32)
    say(f"case: streamed {cons} 2D f32")
    got = ctxs[cons].compute_streamed(_host(img2, True), 64, value_range="auto")
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle_mod.ecc(img2, 64, cons, value_range="auto"))


def test_streamed_equals_device_call_on_a_large_volume(ctxs):
    from paper_2203_09087_amd import synth
    vol = synth.grf((160, 256, 256), seed=62)
    lo, hi = float(vol.min()), float(vol.max())
    ctx = ctxs["vertex"]
    say("case: streamed 160x256x256 f32 GRF vs device call, slabs of 16")
    dev = ctx.compute(torch.from_numpy(vol).cuda(), 4096, value_range=(lo, hi))
    got = ctx.compute_streamed(_host(vol, True), 4096, value_range=(lo, hi), slab_planes=16)
    got_auto = ctx.compute_streamed(_host(vol, True), 4096, value_range="auto", slab_planes=40)
    dev_auto = ctx.compute(torch.from_numpy(vol).cuda(), 4096, value_range="auto")
    torch.cuda.synchronize()
    assert torch.equal(got, dev) and torch.equal(got_auto, dev_auto)


@pytest.mark.parametrize("cons", CONS)
def test_streamed_many_slabs_matches_oracle(ctxs, oracle_mod, cons):
    """A 640 x 256 x 256 uint8 volume (40 MiB, smoothed noise) streamed in 320 slabs
    of 2 planes and in 13 slabs of 50, so the two slab buffers and their events
    are reused hundreds of times: equal to the oracle."""
    from paper_2203_09087_amd import synth
    vol = np.concatenate([synth.smoothed_noise_u8((64, 256, 256), sigma=2.0, seed=70 + k) for k in range(10)])
    want = oracle_mod.ecc(vol, 256, cons, value_range=(0, 255), threads=16)
    for slab in (2, 50):
        say(f"case: streamed {cons} {vol.shape} uint8, slabs of {slab}")
        got = ctxs[cons].compute_streamed(_host(vol, True), 256, value_range=(0, 255), slab_planes=slab)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want), slab


def test_streamed_rejects_device_tensors_and_bad_slabs(ctxs):
    from paper_2203_09087_amd import ecc
    ctx = ctxs["vertex"]
    with pytest.raises(ValueError):
        ctx.compute_streamed(torch.zeros((2, 3, 4), dtype=torch.uint8, device="cuda"), 8)
    with pytest.raises(ecc.EccError):
        ctx.compute_streamed(torch.zeros((2, 3, 4), dtype=torch.uint8), 8, slab_planes=-1)
