"""GPU parity in five to eight dimensions: the HIP library's reduction of an
image one axis at a time (each hyperplane of the axis and the elementwise max
or min of each adjacent pair, with their signs, down to 4D and its signed 3D
passes) against the oracle's direct enumeration of the d-dimensional cubical
complex, bit for bit.

Cases: every dtype and both filtrations, default / AUTO / explicit ranges,
size-1 axes, rows wider than one wave, float specials (NaN must win the max and
lose the min of a pair, as the binning puts it in the last bin), a histogram
wider than one LDS window, the default-range entry point, tuned launch shapes,
and the entry points that do not take these images.
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


def check(ctx, oracle_mod, img, nbins, cons, rng=None):
    print(f"case: {img.ndim}d {cons} shape={img.shape} dtype={img.dtype} nbins={nbins} range={rng}", flush=True,
          file=sys.stderr)
    got = ctx.compute(to_dev(img), nbins, value_range=rng)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    want = oracle_mod.ecc(img, nbins, cons, value_range=rng, threads=16)
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"{cons} {img.shape} {img.dtype} nbins={nbins} range={rng}: "
                             f"{bad.size} bins differ, first {bad[0]}: {got[bad[0]]} != {want[bad[0]]}")


SHAPES = [(1, 1, 1, 1, 1), (2, 1, 3, 1, 5), (3, 2, 4, 5, 6), (2, 3, 2, 9, 70), (1, 4, 3, 6, 130),
          (2, 2, 3, 2, 3, 40), (3, 1, 2, 2, 2, 2, 65), (2, 2, 2, 2, 2, 2, 2, 3)]


@pytest.mark.parametrize("cons", CONS)
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_nd_matches_oracle(ctxs, oracle_mod, cons, dtype):
    rng = np.random.default_rng(101 + CONS.index(cons))
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
def test_nd_float_specials(ctxs, oracle_mod, cons):
    """NaN, infinities and signed zeros spread over every axis, so that pairs of
    hyperplanes combine NaN with numbers, with infinities and with NaN."""
    rng = np.random.default_rng(107)
    img = rng.standard_normal(size=(3, 3, 4, 5, 66)).astype(np.float32)
    flat = img.reshape(-1)
    idx = rng.permutation(flat.size)
    flat[idx[:400]] = np.nan
    flat[idx[400:500]] = np.inf
    flat[idx[500:600]] = -np.inf
    flat[idx[600:700]] = -0.0
    flat[idx[700:800]] = 0.0
    check(ctxs[cons], oracle_mod, img, 300, cons, rng="auto")
    check(ctxs[cons], oracle_mod, img, 50, cons, rng=(-0.5, 0.5))


@pytest.mark.parametrize("cons", CONS)
def test_nd_wide_histogram_and_larger_image(ctxs, oracle_mod, cons):
    """More bins than one LDS window (a merge per pass, adding into the output
    across the 4D parts) and a 1.3M-voxel 5D image of 5 x 4 parts."""
    rng = np.random.default_rng(109)
    img = rng.integers(0, 60000, size=(2, 3, 5, 12, 140)).astype(np.uint16)
    check(ctxs[cons], oracle_mod, img, 9000, cons, rng="auto")
    big = rng.standard_normal(size=(3, 4, 8, 60, 180)).astype(np.float32)
    check(ctxs[cons], oracle_mod, big, 4096, cons, rng="auto")


def test_nd_default_range_entry_point(ctxs, oracle_mod):
    """ecc_compute itself (default range: [0, 255] for u8, AUTO for u16) in 5D."""
    from paper_2203_09087_amd import ecc
    rng = np.random.default_rng(111)
    for cons in CONS:
        for img, code in ((rng.integers(0, 256, size=(2, 3, 4, 7, 90)).astype(np.uint8), ecc.ECC_U8),
                          (rng.integers(0, 9000, size=(3, 2, 3, 8, 33)).astype(np.uint16), ecc.ECC_U16)):
            print(f"case: ecc_compute {cons} {img.shape} {img.dtype}", flush=True, file=sys.stderr)
            dev = to_dev(img)
            out = torch.empty(512, dtype=torch.int64, device="cuda")
            st = ecc.ecc_compute(ctxs[cons].handle, dev.data_ptr(), img.ndim, img.shape, code, 512,
                                 out.data_ptr(), 0)
            assert st == ecc.ECC_OK, ecc.ecc_last_error(ctxs[cons].handle)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), oracle_mod.ecc(img, 512, cons, threads=16))


def test_nd_tuned_and_pinned_shapes_keep_results(oracle_mod):
    """Tuning a 5D image (the shape of its 3D passes) and pinning shapes for it
    leave the result unchanged."""
    from paper_2203_09087_amd import ecc
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(113)
    img = rng.standard_normal(size=(2, 3, 6, 40, 100)).astype(np.float32)
    for cons in CONS:
        want = oracle_mod.ecc(img, 1000, cons, value_range="auto", threads=16)
        ctx = ecc.Context(0, cons)
        try:
            dev = to_dev(img)
            ctx.autotune(dev, 1000, value_range="auto", reps=1)
            got = ctx.compute(dev, 1000, value_range="auto")
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want)
            for waves, depth, wgs in ((1, 1, 1), (2, 8, 3)):
                ctx.set_launch_shape(dev, 1000, waves=waves, depth=depth, wgs_per_cu=wgs)
                got = ctx.compute(dev, 1000, value_range="auto")
                torch.cuda.synchronize()
                assert np.array_equal(got.cpu().numpy(), want), (cons, waves, depth, wgs)
        finally:
            ctx.close()


def test_nd_is_refused_where_unsupported(ctxs):
    """Batches, plans, the fixed-scratch call and streaming do not take images of
    more than 4 (streaming: 3) dimensions; nothing runs and the output keeps its
    contents."""
    from paper_2203_09087_amd import ecc
    h = ctxs["vertex"].handle
    img = torch.zeros((2, 2, 3, 4, 5), dtype=torch.uint8, device="cuda")
    out = torch.full((16,), -7, dtype=torch.int64, device="cuda")
    im = ecc.make_image(img, out)
    assert ecc.ecc_compute_batch(h, [im], 16) == ecc.ECC_ERR_UNSUPPORTED
    assert "more than 4 dimensions" in ecc.ecc_last_error(h)
    assert ecc.ecc_compute_noalloc(h, im, 16) == ecc.ECC_ERR_UNSUPPORTED
    with pytest.raises(ecc.EccError) as e:
        ctxs["vertex"].compute_streamed(img.cpu(), 16)
    assert e.value.status == ecc.ECC_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert (out.cpu() == -7).all()
    assert ctxs["vertex"].compute(img, 16).cpu().tolist() == [1] * 16
