"""GPU parity in four dimensions: the HIP library's 4D path (signed 3D passes
over hyperplanes and over the max/min of adjacent hyperplanes) against the
oracle's direct enumeration of the 4D cubical complex, bit for bit.

Cases: every dtype and both filtrations, default / AUTO / explicit ranges, a
single hyperplane (equal to the 3D result), size-1 axes, rows wider than one
wave (ragged tails), float specials, a histogram wider than one LDS window, and a
4M-voxel image.
"""
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


def to_dev(a):
    if a.dtype == np.uint16:
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(ctx, oracle_mod, img, nbins, cons, rng=None, threads=8):
    print(f"case: 4d {cons} shape={img.shape} dtype={img.dtype} nbins={nbins} range={rng}", flush=True,
          file=sys.stderr)
    got = ctx.compute(to_dev(img), nbins, value_range=rng)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    want = oracle_mod.ecc(img, nbins, cons, value_range=rng, threads=threads)
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"{cons} {img.shape} {img.dtype} nbins={nbins} range={rng}: "
                             f"{bad.size} bins differ, first {bad[0]}: {got[bad[0]]} != {want[bad[0]]}")


SHAPES = [(1, 1, 1, 1), (2, 1, 1, 5), (3, 4, 5, 6), (1, 6, 9, 70), (4, 3, 10, 130), (5, 2, 17, 63),
          (2, 9, 1, 200), (6, 5, 4, 3)]


@pytest.mark.parametrize("cons", CONS)
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_4d_matches_oracle(ctxs, oracle_mod, cons, dtype):
    rng = np.random.default_rng(91 + CONS.index(cons))
    for shape in SHAPES:
        if dtype == "u8":
            img = rng.integers(0, 7, size=shape).astype(np.uint8)   # many ties
            check(ctxs[cons], oracle_mod, img, 256, cons)
            check(ctxs[cons], oracle_mod, img, 5, cons, rng=(1, 5))
        elif dtype == "u16":
            img = rng.integers(0, 3000, size=shape).astype(np.uint16)
            check(ctxs[cons], oracle_mod, img, 4096, cons, rng="auto")
            check(ctxs[cons], oracle_mod, img, 100, cons, rng=(200, 2800))
        else:
            img = rng.standard_normal(size=shape).astype(np.float32)
            check(ctxs[cons], oracle_mod, img, 1024, cons, rng="auto")
            check(ctxs[cons], oracle_mod, img, 64, cons, rng=(-1.0, 1.5))


@pytest.mark.parametrize("cons", CONS)
def test_4d_single_hyperplane_is_3d(ctxs, oracle_mod, cons):
    rng = np.random.default_rng(95)
    vol = rng.integers(0, 40, size=(7, 12, 90)).astype(np.uint8)
    got4 = ctxs[cons].compute(to_dev(vol[None]), 64, value_range=(0, 63))
    got3 = ctxs[cons].compute(to_dev(vol), 64, value_range=(0, 63))
    torch.cuda.synchronize()
    assert np.array_equal(got4.cpu().numpy(), got3.cpu().numpy())


@pytest.mark.parametrize("cons", CONS)
def test_4d_float_specials_and_wide_histogram(ctxs, oracle_mod, cons):
    rng = np.random.default_rng(96)
    img = rng.standard_normal(size=(3, 5, 6, 75)).astype(np.float32)
    flat = img.reshape(-1)
    idx = rng.choice(flat.size, size=40, replace=False)
    flat[idx[:15]] = np.nan
    flat[idx[15:25]] = np.inf
    flat[idx[25:]] = -np.inf
    check(ctxs[cons], oracle_mod, img, 512, cons, rng="auto")
    check(ctxs[cons], oracle_mod, img, 300, cons, rng=(-2.0, 2.0))
    wide = rng.integers(0, 65536, size=(3, 4, 7, 80)).astype(np.uint16)
    check(ctxs[cons], oracle_mod, wide, 9000, cons, rng=(0, 65535))


@pytest.mark.parametrize("cons", CONS)
def test_4d_larger_image(ctxs, oracle_mod, cons):
    from paper_2203_09087_amd import synth
    field = synth.grf((16, 32, 64, 128), seed=97)
    check(ctxs[cons], oracle_mod, field, 4096, cons, rng="auto")


@pytest.mark.parametrize("cons", CONS)
def test_4d_benchmark_field(ctxs, oracle_mod, cons):
    """The 4D workload the benchmark times: an 8 x 256^3 float32 GRF (k^-3 in four
    dimensions, seed 9), 4096 bins over its [min, max]."""
    from paper_2203_09087_amd import synth
    field = synth.grf((8, 256, 256, 256), seed=9)
    check(ctxs[cons], oracle_mod, field, 4096, cons, rng=(float(field.min()), float(field.max())), threads=16)


@pytest.mark.parametrize("cons", CONS)
def test_4d_in_batch_and_plan(ctxs, oracle_mod, cons):
    """4D images in a batch, between 2D and 3D images of every dtype, with every
    range mode: each result equals the oracle and the image computed alone, in a
    plain batch call and in a planned batch."""
    rng = np.random.default_rng(98 + CONS.index(cons))
    imgs = [rng.integers(0, 9, size=(3, 4, 5, 70)).astype(np.uint8),
            rng.standard_normal(size=(40, 130)).astype(np.float32),
            rng.standard_normal(size=(5, 6, 7, 64)).astype(np.float32),
            rng.integers(0, 3000, size=(9, 10, 11)).astype(np.uint16),
            rng.integers(0, 3000, size=(1, 5, 6, 200)).astype(np.uint16),
            rng.integers(0, 200, size=(2, 1, 1, 5)).astype(np.uint8),
            rng.standard_normal(size=(4, 3, 10, 130)).astype(np.float32)]
    ranges = [None, "auto", "auto", (100, 2900), "auto", (0, 199), (-1.0, 1.5)]
    nbins = 512
    ctx = ctxs[cons]
    print(f"case: 4d batch {cons} shapes={[a.shape for a in imgs]}", flush=True, file=sys.stderr)
    devs = [to_dev(a) for a in imgs]
    outs = ctx.compute_batch(devs, nbins, value_ranges=ranges)
    pouts = [torch.empty(nbins, dtype=torch.int64, device="cuda") for _ in imgs]
    plan = ctx.plan_batch(devs, nbins, value_ranges=ranges, outs=pouts)
    plan.launch()
    torch.cuda.synchronize()
    for i, (a, d, r) in enumerate(zip(imgs, devs, ranges)):
        want = oracle_mod.ecc(a, nbins, cons, value_range=r)
        alone = ctx.compute(d, nbins, value_range=r)
        torch.cuda.synchronize()
        assert np.array_equal(outs[i].cpu().numpy(), want), (i, a.shape)
        assert np.array_equal(pouts[i].cpu().numpy(), want), (i, a.shape)
        assert np.array_equal(alone.cpu().numpy(), want), (i, a.shape)
    plan.close()


@pytest.mark.parametrize("cons", CONS)
def test_4d_in_batch_wide_histogram(ctxs, oracle_mod, cons):
    """A 4D image in a batch whose histogram spans several LDS windows."""
    rng = np.random.default_rng(99)
    imgs = [rng.integers(0, 65536, size=(3, 4, 7, 80)).astype(np.uint16),
            rng.integers(0, 65536, size=(30, 90)).astype(np.uint16)]
    print(f"case: 4d batch {cons} 9000 bins", flush=True, file=sys.stderr)
    outs = ctxs[cons].compute_batch([to_dev(a) for a in imgs], 9000, value_ranges=[(0, 65535)] * 2)
    torch.cuda.synchronize()
    for o, a in zip(outs, imgs):
        assert np.array_equal(o.cpu().numpy(), oracle_mod.ecc(a, 9000, cons, value_range=(0, 65535)))


@pytest.mark.parametrize("cons", CONS)
def test_4d_benchmark_field_in_batch(ctxs, oracle_mod, cons):
    """The 8 x 256^3 float32 field as a batch of one (its 15 or 13 passes in one
    launch) equals the oracle."""
    from paper_2203_09087_amd import synth
    field = synth.grf((8, 256, 256, 256), seed=9)
    rng = (float(field.min()), float(field.max()))
    print(f"case: 4d benchmark field in a batch, {cons}", flush=True, file=sys.stderr)
    out = ctxs[cons].compute_batch([to_dev(field)], 4096, value_ranges=[rng])[0]
    torch.cuda.synchronize()
    want = oracle_mod.ecc(field, 4096, cons, value_range=rng, threads=16)
    assert np.array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("cons", CONS)
def test_4d_streamed_from_host(ctxs, oracle_mod, cons):
    """A 4D image in host memory streamed in slabs of 1, 2 and 3 hyperplanes (and
    the default): each slab counts the terms of its own hyperplanes, the one
    after them completing the last pair; every dtype, AUTO and explicit ranges,
    single-hyperplane and two-hyperplane images (the top filtration's last slab
    then owns no term)."""
    rng = np.random.default_rng(123 + CONS.index(cons))
    cases = [((5, 6, 9, 70), np.float32, "auto", 300), ((4, 3, 5, 130), np.uint16, "auto", 5000),
             ((2, 4, 6, 40), np.uint8, None, 256), ((1, 5, 5, 66), np.float32, (-1.0, 1.0), 64),
             ((7, 2, 3, 20), np.uint8, (3, 200), 17)]
    for shape, dt, rngv, nbins in cases:
        img = (rng.standard_normal(size=shape).astype(np.float32) if dt == np.float32
               else rng.integers(0, 6000 if dt == np.uint16 else 256, size=shape).astype(dt))
        host = torch.from_numpy(img.view(np.int16) if dt == np.uint16 else img).pin_memory()
        want = oracle_mod.ecc(img, nbins, cons, value_range=rngv, threads=8)
        for slab in (1, 2, 3, 0):
            say(f"case: 4d streamed {cons} shape={shape} {img.dtype} nbins={nbins} slab={slab}")
            got = ctxs[cons].compute_streamed(host, nbins, value_range=rngv, slab_planes=slab)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), (cons, shape, slab)


def test_5d_streaming_is_refused(ctxs):
    from paper_2203_09087_amd import ecc
    img = torch.zeros((2, 2, 3, 4, 5), dtype=torch.uint8)
    with pytest.raises(ecc.EccError) as e:
        ctxs["vertex"].compute_streamed(img, 16)
    assert e.value.status == ecc.ECC_ERR_UNSUPPORTED


@pytest.mark.parametrize("cons", CONS)
def test_4d_autotune_and_pinned_shapes_keep_results(oracle_mod, cons):
    """Tuning a 4D image (the shape of its 3D passes) and pinning shapes for it
    change only the time: every shape gives the oracle's ECC."""
    from paper_2203_09087_amd import ecc
    rng = np.random.default_rng(97)
    img = rng.standard_normal(size=(5, 12, 30, 140)).astype(np.float32)
    want = oracle_mod.ecc(img, 1024, cons, value_range=(-2.0, 2.0))
    ctx = ecc.Context(0, cons)
    try:
        d = to_dev(img)
        say(f"case: 4d autotune {cons}")
        ctx.autotune(d, 1024, value_range=(-2.0, 2.0), reps=1)
        got = ctx.compute(d, 1024, value_range=(-2.0, 2.0))
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want)
        for waves, wgs, depth, window in ((1, 1, 2, 0), (3, 4, 5, 300), (0, 0, 0, 0)):
            ctx.set_launch_shape(d, 1024, waves=waves, wgs_per_cu=wgs, depth=depth, window=window)
            got = ctx.compute(d, 1024, value_range=(-2.0, 2.0))
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), (waves, wgs, depth, window)
    finally:
        ctx.close()
