"""GPU parity: the HIP library against the oracle, bit for bit.

Everything here is exact integer work (bins are decided in the same IEEE double
arithmetic on both sides), so the bar is equality of every output value.  The
cases span several tiles with ragged tails, size-1 axes, images with few
distinct values (many ties, which exercise the tie-break), every dtype, both
filtrations, AUTO and explicit ranges, bin counts from 1 to 65535 (several LDS
bin windows), float specials, and the full-size workloads.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CONS = ("vertex", "top")


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


def say(*args):
    print(*args, flush=True, file=sys.stderr)


def check(ctx, oracle_mod, img, nbins, cons, rng=None, threads=8):
    say(f"case: {cons} shape={img.shape} dtype={img.dtype} nbins={nbins} range={rng}")
    got = ctx.compute(to_dev(img), nbins, value_range=rng)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    want = oracle_mod.ecc(img, nbins, cons, value_range=rng, threads=threads)
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"{cons} {img.shape} {img.dtype} nbins={nbins} range={rng}: "
                             f"{bad.size} bins differ, first {bad[0]}: {got[bad[0]]} != {want[bad[0]]}")


SHAPES = [(1, 1), (1, 7), (7, 1), (5, 5), (33, 65), (64, 64), (65, 63), (97, 130),
          (1, 1, 1), (1, 1, 5), (3, 1, 4), (9, 8, 33), (10, 9, 31), (17, 17, 17), (8, 8, 64),
          (2, 40, 70)]


def _image(rng, shape, dtype, levels):
    if dtype == np.float32:
        return (rng.integers(0, levels, size=shape) * 0.37 - 3.0).astype(np.float32)
    top = 256 if dtype == np.uint8 else 65536
    return rng.integers(0, min(levels, top), size=shape).astype(dtype)


@pytest.mark.parametrize("cons", CONS)
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
def test_shapes_dtypes(ctxs, oracle_mod, cons, dtype):
    rng = np.random.default_rng(100 + int(np.dtype(dtype).itemsize) + (7 if cons == "top" else 0))
    for shape in SHAPES:
        for levels in (3, 1000):
            img = _image(rng, shape, dtype, levels)
            if dtype == np.uint8:
                check(ctxs[cons], oracle_mod, img, 256, cons)
                check(ctxs[cons], oracle_mod, img, 7, cons, rng=(0, 255))
            elif dtype == np.uint16:
                check(ctxs[cons], oracle_mod, img, 4096, cons, rng="auto")
                check(ctxs[cons], oracle_mod, img, 100, cons, rng=(5, 700))
            else:
                check(ctxs[cons], oracle_mod, img, 4096, cons, rng="auto")
                check(ctxs[cons], oracle_mod, img, 100, cons, rng=(-2.0, 30.0))


@pytest.mark.parametrize("cons", CONS)
def test_bin_counts(ctxs, oracle_mod, cons):
    rng = np.random.default_rng(200)
    img2 = rng.integers(0, 65536, size=(70, 90)).astype(np.uint16)
    img3 = rng.integers(0, 65536, size=(12, 20, 40)).astype(np.uint16)
    for nbins in (1, 2, 255, 256, 4096, 8192, 8193, 20000, 65535):
        check(ctxs[cons], oracle_mod, img2, nbins, cons, rng="auto")
        check(ctxs[cons], oracle_mod, img3, nbins, cons, rng=(0, 65535))


@pytest.mark.parametrize("cons", CONS)
def test_float_specials(ctxs, oracle_mod, cons):
    rng = np.random.default_rng(300)
    img = rng.standard_normal((30, 41)).astype(np.float32)
    img.flat[rng.choice(img.size, 40, replace=False)] = np.nan
    img.flat[rng.choice(img.size, 10, replace=False)] = np.inf
    img.flat[rng.choice(img.size, 10, replace=False)] = -np.inf
    img.flat[rng.choice(img.size, 10, replace=False)] = -0.0
    img.flat[rng.choice(img.size, 10, replace=False)] = 0.0
    for r in ("auto", (-1.0, 1.0), (0.5, 0.5)):
        check(ctxs[cons], oracle_mod, img, 64, cons, rng=r)
    allnan = np.full((5, 6, 7), np.nan, dtype=np.float32)
    check(ctxs[cons], oracle_mod, allnan, 16, cons, rng="auto")
    flat = np.full((9, 3), 2.5, dtype=np.float32)
    check(ctxs[cons], oracle_mod, flat, 16, cons, rng="auto")


@pytest.mark.parametrize("cons", CONS)
def test_flat_ranges(ctxs, oracle_mod, cons):
    """hi == lo: values <= lo go to bin 0, values above it and NaN to the last bin,
    including lo = 0 (whose next double is subnormal), negative lo, and an
    explicit lo that no float equals."""
    tiny = np.float32(1e-45)             # smallest positive subnormal float
    vals = np.array([0.0, -0.0, tiny, -tiny, 1.0, -1.0, np.nan, np.inf, -np.inf,
                     0.1, np.nextafter(np.float32(0.1), np.float32(1)), -2.5,
                     np.nextafter(np.float32(-2.5), np.float32(0)), np.float32(3.4e38)],
                    dtype=np.float32)
    rng = np.random.default_rng(301)
    img = rng.choice(vals, size=(23, 70)).astype(np.float32)
    for lo in (0.0, -2.5, 0.1, float(np.float32(0.1)), 3.4e38):
        check(ctxs[cons], oracle_mod, img, 8, cons, rng=(lo, lo))


@pytest.mark.parametrize("cons", CONS)
def test_workload_small_2d(ctxs, oracle_mod, cons):
    """256 x 256 uint8 uniform noise, 256 bins (one per gray level)."""
    from paper_2203_09087_amd import synth
    check(ctxs[cons], oracle_mod, synth.uniform_u8((256, 256), seed=1), 256, cons)


@pytest.mark.parametrize("cons", CONS)
def test_workload_smoothed_3d(ctxs, oracle_mod, cons):
    """256^3 uint8 smoothed noise (sigma 2), 256 bins."""
    from paper_2203_09087_amd import synth
    img = synth.smoothed_noise_u8((256, 256, 256), sigma=2.0, seed=2)
    check(ctxs[cons], oracle_mod, img, 256, cons, threads=16)


def _tail(xpos, waves):
    """Positions left after the full x-chunks of 63 * waves positions."""
    return xpos - (xpos // (63 * waves)) * 63 * waves


@pytest.mark.parametrize("cons", CONS)
def test_packed_row_tails(oracle_mod, cons):
    """Rows whose positions leave a narrow tail (1 to 31 positions) after the
    full x-chunks of a 3D launch: the tail of every strip inside the image runs
    packed (t + 1 lanes per strip, several strips per wave), the strips at the
    image's first and last rows as ordinary bricks.  Widths, heights (one to a few
    strips, partial ones at either end) and forced wave counts cover tails of 1,
    2, 7, 8, 15, 16 and 31 positions, after one full chunk or in an image
    narrower than a chunk; every case gives the oracle's ECC."""
    from paper_2203_09087_amd import ecc
    rng = np.random.default_rng(78)
    extra = 1 if cons == "top" else 0   # the top filtration has n + 1 positions
    ctx = ecc.Context(0, cons)
    try:
        # one full chunk and a tail, or (chunks = 0) an image narrower than a chunk
        for waves, chunks in ((1, 1), (2, 1), (4, 1), (8, 1), (1, 0), (3, 0)):
            for t in (1, 2, 7, 8, 15, 16, 31):
                n2 = 63 * waves * chunks + t - extra
                if n2 < 1:
                    continue
                assert _tail(n2 + extra, waves) == t
                for n1 in (1, 3, 4, 5, 8, 26):
                    shape = (3, n1, n2)
                    img = (rng.standard_normal(size=shape).astype(np.float32) if (t + n1) % 2
                           else rng.integers(0, 9, size=shape).astype(np.uint8))
                    nbins = 300 if img.dtype == np.float32 else 9
                    rngv = "auto" if img.dtype == np.float32 else (0, 8)
                    dev = to_dev(img)
                    ctx.set_launch_shape(dev, nbins, waves=waves, depth=2, wgs_per_cu=1)
                    say(f"case: packed tail {cons} waves={waves} t={t} shape={shape} {img.dtype}")
                    got = ctx.compute(dev, nbins, value_range=rngv)
                    torch.cuda.synchronize()
                    want = oracle_mod.ecc(img, nbins, cons, value_range=rngv, threads=8)
                    assert np.array_equal(got.cpu().numpy(), want), (cons, waves, t, shape)
    finally:
        ctx.close()


def test_random_shapes_and_launch_shapes(oracle_mod):
    """Seeded random 3D and 4D images (widths around every tail length, few to
    many rows and planes, every dtype, both filtrations, narrow and windowed
    histograms) at random forced launch shapes (waves, workgroups per CU,
    depth, histogram copies) against the oracle."""
    from paper_2203_09087_amd import ecc
    rng = np.random.default_rng(2024)
    ctxs_ = {c: ecc.Context(0, c) for c in CONS}
    try:
        for case in range(144):
            cons = CONS[case % 2]
            ndim = 4 if case % 6 == 5 else 3
            n2 = int(rng.integers(1, 600))
            n1 = int(rng.integers(1, 40))
            n0 = int(rng.integers(1, 7))
            shape = ((int(rng.integers(1, 4)),) if ndim == 4 else ()) + (n0, n1, n2)
            kind = int(rng.integers(0, 3))
            if kind == 0:
                img = rng.integers(0, 256, size=shape).astype(np.uint8)
            elif kind == 1:
                img = rng.integers(0, 5000, size=shape).astype(np.uint16)
            else:
                img = rng.standard_normal(size=shape).astype(np.float32)
            nbins = int(rng.choice([1, 7, 256, 4096, 5000]))
            rngv = None if kind == 0 else "auto"
            waves = int(rng.integers(1, 10))
            wgs = int(rng.integers(1, 5))
            depth = int(rng.choice([1, 2, 5, 16]))
            copies = int(rng.choice([0, 2, 4, 8])) if nbins <= 1024 else 0
            ctx = ctxs_[cons]
            dev = to_dev(img)
            ctx.set_launch_shape(dev, nbins, waves=waves, wgs_per_cu=wgs, depth=depth, copies=copies)
            say(f"case {case}: {cons} shape={shape} {img.dtype} nbins={nbins} shape=({waves},{wgs},{depth},{copies})")
            got = ctx.compute(dev, nbins, value_range=rngv)
            torch.cuda.synchronize()
            want = oracle_mod.ecc(img, nbins, cons, value_range=rngv, threads=8)
            assert np.array_equal(got.cpu().numpy(), want), (case, cons, shape, img.dtype, nbins, waves, wgs, depth)
    finally:
        for c in ctxs_.values():
            c.close()


@pytest.fixture(scope="module")
def grf3d():
    from paper_2203_09087_amd import synth
    return synth.grf((512, 512, 512), seed=3)


@pytest.mark.parametrize("cons", CONS)
def test_workload_grf_512_cubed(ctxs, oracle_mod, grf3d, cons):
    """512^3 float32 GRF (k^-3), 4096 bins over [min, max], explicit and AUTO."""
    lo, hi = float(grf3d.min()), float(grf3d.max())
    check(ctxs[cons], oracle_mod, grf3d, 4096, cons, rng=(lo, hi), threads=16)
    check(ctxs[cons], oracle_mod, grf3d, 4096, cons, rng="auto", threads=16)


@pytest.fixture(scope="module")
def grf2d_u16():
    from paper_2203_09087_amd import synth
    return synth.quantize_u16(synth.grf((16384, 16384), seed=4), 4096)


@pytest.mark.parametrize("cons", CONS)
def test_workload_grf_16384_squared(ctxs, oracle_mod, grf2d_u16, cons):
    """16384^2 uint16 GRF quantized to 4096 levels, 4096 bins over [min, max]
    (AUTO), and over the explicit range [0, 4095]."""
    check(ctxs[cons], oracle_mod, grf2d_u16, 4096, cons, rng="auto", threads=16)
    check(ctxs[cons], oracle_mod, grf2d_u16, 4096, cons, rng=(0, 4095), threads=16)


@pytest.mark.parametrize("cons", CONS)
def test_compute_entry_point(ctxs, oracle_mod, cons):
    """ecc_compute itself (default range: [0, 255] for u8, AUTO otherwise), called
    through the C ABI on a 2D u8, a 3D u16 and a 4D f32 image."""
    from paper_2203_09087_amd import ecc, synth
    rng = np.random.default_rng(321 if cons == "vertex" else 322)
    cases = [
        (synth.uniform_u8((300, 517), seed=13), ecc.ECC_U8, 256),
        (rng.integers(0, 3000, size=(37, 70, 129)).astype(np.uint16), ecc.ECC_U16, 4096),
        (synth.grf((5, 20, 33, 70), seed=14), ecc.ECC_F32, 1000),
    ]
    for img, code, nbins in cases:
        say(f"case: ecc_compute {cons} {img.shape} {img.dtype} nbins={nbins}")
        dev = to_dev(img)
        out = torch.full((nbins,), -5, dtype=torch.int64, device="cuda")
        st = ecc.ecc_compute(ctxs[cons].handle, dev.data_ptr(), img.ndim, img.shape, code, nbins, out.data_ptr(), 0)
        assert st == ecc.ECC_OK, ecc.ecc_last_error(ctxs[cons].handle)
        torch.cuda.synchronize()
        rng_mode = None if code == ecc.ECC_U8 else "auto"
        want = oracle_mod.ecc(img, nbins, cons, value_range=rng_mode, threads=8)
        got = out.cpu().numpy()
        assert np.array_equal(got, want), (img.shape, np.nonzero(got != want)[0][:5])


@pytest.mark.parametrize("cons", CONS)
def test_batch_matches_single_and_oracle(ctxs, oracle_mod, cons):
    rng = np.random.default_rng(400)
    imgs, ranges = [], []
    for i in range(24):
        d = 2 if i % 3 else 3
        shape = tuple(int(s) for s in rng.integers(1, 90 if d == 2 else 24, size=d))
        kind = i % 4
        if kind == 0:
            imgs.append(rng.integers(0, 256, size=shape).astype(np.uint8)); ranges.append(None)
        elif kind == 1:
            imgs.append(rng.integers(0, 300, size=shape).astype(np.uint16)); ranges.append("auto")
        elif kind == 2:
            imgs.append(rng.standard_normal(shape).astype(np.float32)); ranges.append((-1.5, 1.5))
        else:
            imgs.append(rng.standard_normal(shape).astype(np.float32)); ranges.append("auto")
    say(f"case: batch of {len(imgs)} ({cons})")
    dev = [to_dev(a) for a in imgs]
    outs = ctxs[cons].compute_batch(dev, 512, value_ranges=ranges)
    torch.cuda.synchronize()
    for a, d, r, o in zip(imgs, dev, ranges, outs):
        single = ctxs[cons].compute(d, 512, value_range=r)
        torch.cuda.synchronize()
        want = oracle_mod.ecc(a, 512, cons, value_range=r)
        assert np.array_equal(o.cpu().numpy(), want), (a.shape, a.dtype, r)
        assert np.array_equal(single.cpu().numpy(), want), (a.shape, a.dtype, r)
    assert ctxs[cons].compute_batch([], 512) == []


@pytest.mark.parametrize("nbins", [4097, 20000])
def test_batch_wide_histograms(ctxs, oracle_mod, nbins):
    """Batches whose histograms need several LDS windows (merge per window, the
    scan after the last), with an image spread over many workgroups (more
    partial rows than the merge loads at once, and a ragged last round)."""
    rng = np.random.default_rng(410 + nbins)
    imgs = [rng.integers(0, 65536, size=(700, 900)).astype(np.uint16),
            rng.integers(0, 65536, size=(9, 30, 77)).astype(np.uint16),
            rng.standard_normal((3, 200)).astype(np.float32),
            rng.integers(0, 256, size=(1, 1)).astype(np.uint8)]
    ranges = [(0, 65535), "auto", "auto", None]
    for cons in CONS:
        say(f"case: batch with {nbins} bins ({cons})")
        dev = [to_dev(a) for a in imgs]
        outs = ctxs[cons].compute_batch(dev, nbins, value_ranges=ranges)
        torch.cuda.synchronize()
        for a, r, o in zip(imgs, ranges, outs):
            want = oracle_mod.ecc(a, nbins, cons, value_range=r, threads=8)
            assert np.array_equal(o.cpu().numpy(), want), (cons, a.shape, a.dtype, r)


@pytest.mark.parametrize("cons", CONS)
def test_unaligned_base_pointers(ctxs, oracle_mod, cons):
    """Images whose first element is not 16-byte aligned (a view into a larger
    buffer at an element offset): every dtype, AUTO and explicit ranges, alone
    and as a batch of one."""
    rng = np.random.default_rng(430)
    for dtype, shape, nb, rg in ((np.uint8, (37, 91), 256, None), (np.uint16, (9, 13, 70), 4096, "auto"),
                                 (np.float32, (5, 29, 33), 1000, "auto"), (np.float32, (61, 47), 300, (-1.0, 1.0))):
        n = int(np.prod(shape))
        for off in (1, 2, 3):
            full = (rng.standard_normal(n + 4).astype(np.float32) if dtype == np.float32
                    else rng.integers(0, 256 if dtype == np.uint8 else 65536, size=n + 4).astype(dtype))
            base = to_dev(full)
            view = base[off:off + n].view(shape)
            assert view.data_ptr() % 16 != 0
            host = full[off:off + n].reshape(shape)
            say(f"case: unaligned {np.dtype(dtype).name} {shape} offset {off} elements ({cons})")
            want = oracle_mod.ecc(host, nb, cons, value_range=rg)
            got = ctxs[cons].compute(view, nb, value_range=rg)
            one = ctxs[cons].compute_batch([view], nb, value_ranges=[rg])
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), (dtype, shape, off)
            assert np.array_equal(one[0].cpu().numpy(), want), (dtype, shape, off)


def test_repeat_runs_are_identical(ctxs):
    from paper_2203_09087_amd import synth
    img = to_dev(synth.grf((64, 80, 96), seed=9))
    say("case: determinism 64x80x96 f32")
    ref = ctxs["vertex"].compute(img, 4096, value_range="auto").cpu().numpy()
    for _ in range(20):
        got = ctxs["vertex"].compute(img, 4096, value_range="auto").cpu().numpy()
        assert np.array_equal(got, ref)


def test_non_default_stream(ctxs, oracle_mod):
    from paper_2203_09087_amd import synth
    a = synth.uniform_u8((300, 200), seed=12)
    say("case: side stream")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d = to_dev(a)
        out = ctxs["top"].compute(d, 256)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle_mod.ecc(a, 256, "top"))


def test_invalid_arguments_enqueue_nothing(ctxs):
    """Every bad argument returns ECC_ERR_INVALID_ARG and leaves the output untouched."""
    from paper_2203_09087_amd import ecc
    h = ctxs["vertex"].handle
    img = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    out = torch.full((16,), -7, dtype=torch.int64, device="cuda")
    good = ecc.make_image(img, out)

    def variant(**kw):
        im = ecc.make_image(img, out)
        for k, v in kw.items():
            if k == "dims":
                for i, x in enumerate(v):
                    im.dims[i] = x
            else:
                setattr(im, k, v)
        return im

    bad = [variant(data=None), variant(out=None), variant(ndim=1), variant(ndim=9),
           variant(dtype=7), variant(range_mode=9), variant(reserved=1), variant(dims=(0, 8)),
           variant(dims=(8, -1)), variant(range_mode=ecc.ECC_RANGE_EXPLICIT, lo=3.0, hi=2.0),
           variant(range_mode=ecc.ECC_RANGE_EXPLICIT, lo=0.5, hi=2.0),
           variant(range_mode=ecc.ECC_RANGE_EXPLICIT, lo=0.0, hi=256.0)]
    for im in bad:
        assert ecc.ecc_compute_ex(h, im, 16) == ecc.ECC_ERR_INVALID_ARG
        assert ecc.ecc_last_error(h)
    for nb in (0, -1, 65536):
        assert ecc.ecc_compute_ex(h, good, nb) == ecc.ECC_ERR_INVALID_ARG
    assert ecc.ecc_compute(h, img.data_ptr(), 2, (8, 8), 0, 16, 0) == ecc.ECC_ERR_INVALID_ARG
    assert ecc.ecc_compute(h, img.data_ptr(), 9, (8, 8), 0, 16, out.data_ptr()) == ecc.ECC_ERR_INVALID_ARG
    f = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    fim = ecc.make_image(f, out, (0.0, float("inf")))
    assert ecc.ecc_compute_ex(h, fim, 16) == ecc.ECC_ERR_INVALID_ARG
    # batch: the bad descriptor is named and nothing runs for the good ones either
    st = ecc.ecc_compute_batch(h, [good, variant(ndim=9)], 16)
    assert st == ecc.ECC_ERR_INVALID_ARG and "image 1" in ecc.ecc_last_error(h)
    torch.cuda.synchronize()
    assert (out.cpu() == -7).all()
    assert ecc.ecc_compute_ex(h, good, 16) == ecc.ECC_OK
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [1] * 16


def test_kernel_timing_counts_launches_and_changes_nothing(ctxs):
    """The timing hook counts one histogram launch per call and bin window, one per
    dtype group and window of a batch, and leaves results untouched."""
    from paper_2203_09087_amd import synth
    ctx = ctxs["vertex"]
    say("case: kernel timing, 64^3 u8 and a 3-image batch, 256 and 9000 bins")
    img = to_dev(synth.smoothed_noise_u8((64, 64, 64), 2.0, 12))
    plain = ctx.compute(img, 256)
    wide = ctx.compute(img, 9000, value_range=(0, 255))
    torch.cuda.synchronize()
    ctx.set_kernel_timing(True)
    try:
        for _ in range(3):
            got = ctx.compute(img, 256)
        got_wide = ctx.compute(img, 9000, value_range=(0, 255))   # 3 windows of 4096 bins
        f = torch.rand(20, 30, device="cuda", dtype=torch.float32)
        outs = ctx.compute_batch([img, img[:5].contiguous(), f], 256)   # u8 and f32 groups
        ms, n = ctx.kernel_time()
        assert n == 3 + 3 + 2 and ms > 0.0
        assert np.array_equal(got.cpu().numpy(), plain.cpu().numpy())
        assert np.array_equal(got_wide.cpu().numpy(), wide.cpu().numpy())
        assert np.array_equal(outs[0].cpu().numpy(), plain.cpu().numpy())
        assert ctx.kernel_time() == (0.0, 0)
    finally:
        ctx.set_kernel_timing(False)
    ctx.compute(img, 256, out=got)
    ms, n = ctx.kernel_time()
    assert n == 0


def _plan_inputs(seed):
    from paper_2203_09087_amd import synth
    rng = np.random.default_rng(seed)
    imgs = [synth.smoothed_noise_u8((70, 90), 1.5, seed), synth.smoothed_noise_u8((12, 30, 41), 1.5, seed + 1),
            rng.integers(0, 4096, (33, 600)).astype(np.uint16), rng.standard_normal((5, 9, 700)).astype(np.float32),
            synth.smoothed_noise_u8((1, 1), 1.0, seed + 2)]
    ranges = [None, (0, 255), "auto", "auto", None]
    return imgs, ranges


@pytest.mark.parametrize("cons", CONS)
def test_batch_plan_matches_batch_and_oracle(ctxs, oracle_mod, cons):
    """A planned batch gives the ECCs of ecc_compute_batch, launch after launch,
    and follows changes of the image contents (AUTO ranges recomputed)."""
    ctx = ctxs[cons]
    imgs, ranges = _plan_inputs(40)
    say(f"case: batch plan, {cons}, {len(imgs)} mixed images, 512 bins")
    dev = [to_dev(a) for a in imgs]
    plan = ctx.plan_batch(dev, 512, value_ranges=ranges)
    try:
        want_batch = [o.cpu().numpy() for o in ctx.compute_batch(dev, 512, value_ranges=ranges)]
        for _ in range(3):
            got = [o.cpu().numpy() for o in plan.launch()]
            torch.cuda.synchronize()
            for g, w in zip(got, want_batch):
                assert np.array_equal(g, w)
        for a, r, g in zip(imgs, ranges, got):
            assert np.array_equal(g, oracle_mod.ecc(a, 512, cons, value_range=r))
        # new contents in the same buffers
        imgs2, _ = _plan_inputs(41)
        for d, a in zip(dev, imgs2):
            d.copy_(to_dev(a))
        got2 = [o.cpu().numpy() for o in plan.launch()]
        torch.cuda.synchronize()
        for a, r, g in zip(imgs2, ranges, got2):
            assert np.array_equal(g, oracle_mod.ecc(a, 512, cons, value_range=r))
    finally:
        plan.close()


@pytest.mark.parametrize("cons", CONS)
def test_batch_plan_autotune_keeps_results(ctxs, oracle_mod, cons):
    """The plan's tuner picks one of its candidate shapes; the outputs after tuning
    and every later launch with the chosen shape equal the oracle."""
    ctx = ctxs[cons]
    imgs, ranges = _plan_inputs(42)
    say(f"case: batch plan autotune, {cons}, {len(imgs)} mixed images, 300 bins")
    dev = [to_dev(a) for a in imgs]
    plan = ctx.plan_batch(dev, 300, value_ranges=ranges)
    try:
        shape = plan.autotune(reps=1)
        assert shape["depth3"] in (4, 8, 16) and shape["depth2"] in (32, 64, 128)
        assert 1 <= shape["wgs_per_cu"] <= 4 and shape["ms"] > 0
        want = [oracle_mod.ecc(a, 300, cons, value_range=r) for a, r in zip(imgs, ranges)]
        for g, w in zip(plan.outs, want):
            assert np.array_equal(g.cpu().numpy(), w)
        for o in plan.outs:
            o.fill_(-5)
        got = [o.cpu().numpy() for o in plan.launch()]
        torch.cuda.synchronize()
        for g, w in zip(got, want):
            assert np.array_equal(g, w)
    finally:
        plan.close()


def test_batch_plan_graph_replay(ctxs, oracle_mod):
    """A planned batch captured into a HIP graph: every replay, with eager work
    and synchronisation between replays, equals the eager result."""
    ctx = ctxs["vertex"]
    imgs, ranges = _plan_inputs(42)
    say("case: batch plan captured in a graph, 4 replays")
    dev = [to_dev(a) for a in imgs]
    plan = ctx.plan_batch(dev, 512, value_ranges=ranges)
    try:
        eager = [o.clone() for o in plan.launch()]
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.launch(stream=s)          # warm-up on the capture stream
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            plan.launch(stream=s)
        for k in range(4):
            for o in plan.outs:
                o.fill_(-1)
            ctx.compute(dev[0], 64)            # unrelated eager work in between
            g.replay()
            torch.cuda.synchronize()
            for o, e in zip(plan.outs, eager):
                assert torch.equal(o, e), f"replay {k}"
        for a, r, o in zip(imgs, ranges, plan.outs):
            assert np.array_equal(o.cpu().numpy(), oracle_mod.ecc(a, 512, "vertex", value_range=r))
    finally:
        plan.close()


def test_set_launch_shape(oracle_mod):
    """A pinned launch shape (as a profiled run uses) gives the oracle's ECC;
    out-of-range fields are rejected without changing later calls."""
    from paper_2203_09087_amd import ecc
    rng = np.random.default_rng(51)
    img = rng.standard_normal((20, 70, 300)).astype(np.float32)
    want = oracle_mod.ecc(img, 4096, "vertex", value_range=(-2.0, 2.0))
    ctx = ecc.Context(0, "vertex")
    try:
        d = to_dev(img)
        for waves, wgs, depth in ((9, 4, 64), (2, 1, 3), (5, 3, 0), (0, 0, 0)):
            say(f"case: launch shape waves={waves} wgs_per_cu={wgs} depth={depth}")
            ctx.set_launch_shape(d, 4096, waves=waves, wgs_per_cu=wgs, depth=depth)
            got = ctx.compute(d, 4096, value_range=(-2.0, 2.0))
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), (waves, wgs, depth)
        for bad in ({"waves": 10}, {"wgs_per_cu": 17}, {"depth": 4097}, {"window": 4097}, {"copies": 3},
                    {"copies": 16}):
            with pytest.raises(ecc.EccError):
                ctx.set_launch_shape(d, 4096, **bad)
        got = ctx.compute(d, 4096, value_range=(-2.0, 2.0))
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want)
    finally:
        ctx.close()


@pytest.mark.parametrize("cons", CONS)
def test_bins_per_pass_split(oracle_mod, cons):
    """A launch shape whose window holds fewer bins than the histogram (several
    passes over the image, each with a smaller LDS histogram) gives the oracle's
    ECC, in 2D and 3D, for the default and the fused single-launch merge."""
    from paper_2203_09087_amd import ecc
    rng = np.random.default_rng(52)
    cases = [(rng.standard_normal((20, 70, 300)).astype(np.float32), 4096, (-2.0, 2.0), (2048, 1000, 4096, 1)),
             (rng.integers(0, 60000, size=(300, 700)).astype(np.uint16), 2500, (0, 59999), (1000, 2048, 64)),
             (rng.integers(0, 256, size=(9, 40, 50)).astype(np.uint8), 256, (0, 255), (100, 255, 256))]
    ctx = ecc.Context(0, cons)
    try:
        for img, nbins, r, windows in cases:
            want = oracle_mod.ecc(img, nbins, cons, value_range=r)
            d = to_dev(img)
            for w in windows:
                say(f"case: {cons} window={w} nbins={nbins} shape={img.shape}")
                ctx.set_launch_shape(d, nbins, window=w)
                got = ctx.compute(d, nbins, value_range=r)
                torch.cuda.synchronize()
                assert np.array_equal(got.cpu().numpy(), want), (img.shape, nbins, w)
    finally:
        ctx.close()


def test_reserve_then_calls_fit(oracle_mod):
    """ecc_reserve grows the scratch and table buffers ahead of the calls (which
    then give the oracle's ECC as before); sizes beyond its limits are refused
    and leave the context usable."""
    from paper_2203_09087_amd import ecc
    rng = np.random.default_rng(55)
    imgs = [rng.integers(0, 256, size=s).astype(np.uint8) for s in ((40, 50), (6, 30, 70), (300, 200))]
    ctx = ecc.Context(0, "vertex")
    try:
        scratch, tables = ecc.batch_reserve_bytes(len(imgs), sum(a.size for a in imgs), 256, 256)
        ctx.reserve(scratch, tables)
        with pytest.raises(ecc.EccError):
            ctx.reserve(1 << 41, 0)
        with pytest.raises(ecc.EccError):
            ctx.reserve(0, 1 << 31)
        outs = ctx.compute_batch([to_dev(a) for a in imgs], 256)
        torch.cuda.synchronize()
        for a, o in zip(imgs, outs):
            assert np.array_equal(o.cpu().numpy(), oracle_mod.ecc(a, 256, "vertex", value_range=(0, 255)))
    finally:
        ctx.close()


@pytest.mark.parametrize("cons", CONS)
def test_histogram_copies(oracle_mod, cons):
    """2, 4 or 8 copies of the LDS histogram (lane l adds to copy l mod copies),
    one window or several, smooth data with many equal neighbours: the oracle's
    ECC every time."""
    from paper_2203_09087_amd import ecc, synth
    vol = synth.smoothed_noise_u8((30, 70, 140), sigma=2.0, seed=53)
    img2 = synth.smoothed_noise_u8((200, 330), sigma=2.0, seed=54)
    ctx = ecc.Context(0, cons)
    try:
        for img, nbins in ((vol, 256), (img2, 256), (vol, 1000), (img2, 100)):
            d = to_dev(img)
            want = oracle_mod.ecc(img, nbins, cons, value_range=(0, 255))
            for copies in (2, 4, 8, 0):
                for window in (0, 64):
                    say(f"case: {cons} copies={copies} window={window} nbins={nbins} shape={img.shape}")
                    ctx.set_launch_shape(d, nbins, copies=copies, window=window)
                    got = ctx.compute(d, nbins, value_range=(0, 255))
                    torch.cuda.synchronize()
                    assert np.array_equal(got.cpu().numpy(), want), (img.shape, nbins, copies, window)
    finally:
        ctx.close()


@pytest.mark.parametrize("shape,dtype", [((40, 70, 300), np.float32), ((300, 2000), np.uint16)])
def test_autotune_keeps_results(oracle_mod, shape, dtype):
    """ecc_autotune picks a launch shape for the image shape; every later call
    on that shape (using it) gives the same ECC as before and as the oracle."""
    from paper_2203_09087_amd import ecc
    say(f"case: autotune {shape} {np.dtype(dtype).name}")
    rng = np.random.default_rng(50)
    img = (rng.standard_normal(shape).astype(np.float32) if dtype == np.float32
           else rng.integers(0, 4096, shape).astype(np.uint16))
    rng_arg = "auto"
    ctx = ecc.Context(0, "vertex")
    try:
        d = to_dev(img)
        before = ctx.compute(d, 1000, value_range=rng_arg).cpu().numpy()
        shape_chosen = ctx.autotune(d, 1000, value_range=rng_arg, reps=2)
        assert shape_chosen["ms"] > 0 and shape_chosen["waves"] >= 1 and shape_chosen["depth"] >= 1
        after = ctx.compute(d, 1000, value_range=rng_arg).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(before, after)
        assert np.array_equal(after, oracle_mod.ecc(img, 1000, "vertex", value_range=rng_arg))
    finally:
        ctx.close()
