"""GPU: the entry point that allocates nothing (ecc_compute_noalloc) against
ecc_compute_ex, bit for bit, through the C ABI.

Every case makes two calls in a row on one context, the second with a smaller
image, so that the second call runs on the fixed scratch as the first one left
it.  The cases cover 2D, 3D and 4D images, both filtrations, AUTO and explicit
ranges, several LDS bin windows (nbins above 4096), and a 4D image whose passes
share one merge.  A last check makes sure an image too large for the fixed
scratch is refused before anything is enqueued.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*args):
    print(*args, flush=True, file=sys.stderr)


def to_dev(a):
    if a.dtype == np.uint16:
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def ecc_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_09087_amd import ecc
    return ecc


def _images(rng, shapes, dtype):
    out = []
    for sh in shapes:
        if dtype == np.float32:
            out.append(rng.standard_normal(sh).astype(np.float32))
        elif dtype == np.uint16:
            out.append(rng.integers(0, 4096, size=sh).astype(np.uint16))
        else:
            out.append(rng.integers(0, 256, size=sh).astype(np.uint8))
    return out


def _pair(ecc, ctx, img, nbins, value_range):
    """(noalloc result, compute_ex result) of one image, both through the C ABI."""
    dev = to_dev(img)
    out_n = torch.full((nbins,), -7, dtype=torch.int64, device="cuda")
    out_e = torch.full((nbins,), -9, dtype=torch.int64, device="cuda")
    st = ecc.ecc_compute_noalloc(ctx.handle, ecc.make_image(dev, out_n, value_range), nbins, 0)
    assert st == ecc.ECC_OK, ecc.ecc_last_error(ctx.handle)
    st = ecc.ecc_compute_ex(ctx.handle, ecc.make_image(dev, out_e, value_range), nbins, 0)
    assert st == ecc.ECC_OK, ecc.ecc_last_error(ctx.handle)
    torch.cuda.synchronize()
    return out_n.cpu().numpy(), out_e.cpu().numpy()


CASES = [
    # (construction, dtype, [first shape, smaller second shape], nbins, range)
    ("vertex", np.float32, [(96, 80, 72), (33, 17, 40)], 4096, "auto"),
    ("top", np.float32, [(70, 90, 65), (9, 10, 11)], 1000, (-2.5, 2.5)),
    ("vertex", np.uint16, [(700, 900), (65, 130)], 4096, (0, 4095)),
    ("top", np.uint16, [(600, 513), (1, 300)], 5000, "auto"),
    ("vertex", np.uint8, [(40, 50, 60), (2, 3, 4)], 256, None),
    ("vertex", np.float32, [(5, 24, 30, 40), (3, 8, 9, 10)], 4096, "auto"),
    ("top", np.uint8, [(4, 20, 21, 22), (2, 5, 6, 7)], 9000, (0, 255)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_equals_compute_ex(ecc_mod, case):
    cons, dtype, shapes, nbins, rng_mode = CASES[case]
    ctx = ecc_mod.Context(0, cons)
    try:
        rng = np.random.default_rng(700 + case)
        for k, img in enumerate(_images(rng, shapes, dtype)):
            say(f"noalloc case {case} call {k}: {cons} {img.shape} {img.dtype} nbins={nbins} range={rng_mode}")
            got, want = _pair(ecc_mod, ctx, img, nbins, rng_mode)
            if not np.array_equal(got, want):
                bad = np.nonzero(got != want)[0]
                raise AssertionError(f"call {k} {img.shape}: {bad.size} bins differ, first {bad[0]}: "
                                     f"{got[bad[0]]} != {want[bad[0]]}")
            assert got[-1] == 1
    finally:
        ctx.close()


def test_noalloc_two_contexts_share_scratch_in_turn(ecc_mod, oracle_mod):
    """Two contexts use the device's one fixed array one after the other; each
    result equals the oracle."""
    rng = np.random.default_rng(750)
    a = rng.standard_normal((64, 64, 64)).astype(np.float32)
    b = rng.integers(0, 256, size=(300, 200)).astype(np.uint8)
    cv, ct = ecc_mod.Context(0, "vertex"), ecc_mod.Context(0, "top")
    try:
        oa = torch.empty(4096, dtype=torch.int64, device="cuda")
        ob = torch.empty(256, dtype=torch.int64, device="cuda")
        cv.compute_noalloc(to_dev(a), 4096, oa, value_range="auto")
        torch.cuda.synchronize()
        ct.compute_noalloc(to_dev(b), 256, ob)
        torch.cuda.synchronize()
        assert np.array_equal(oa.cpu().numpy(), oracle_mod.ecc(a, 4096, "vertex", value_range="auto", threads=8))
        assert np.array_equal(ob.cpu().numpy(), oracle_mod.ecc(b, 256, "top", threads=8))
    finally:
        cv.close()
        ct.close()


def test_noalloc_refuses_an_image_beyond_the_fixed_scratch(ecc_mod):
    """2^40 u8 voxels with 4096 bins need 8193 workgroup rows of 16 KiB (each
    workgroup takes at most 2^27 voxels), far more than the fixed array holds:
    the call is refused on the host, so the data pointer (a small real buffer,
    not the claimed size) is never read."""
    ctx = ecc_mod.Context(0, "vertex")
    try:
        small = torch.zeros(16, dtype=torch.uint8, device="cuda")
        out = torch.zeros(4096, dtype=torch.int64, device="cuda")
        im = ecc_mod.ecc_image()
        im.data = small.data_ptr()
        im.ndim = 3
        im.dtype = ecc_mod.ECC_U8
        im.dims[0], im.dims[1], im.dims[2] = 1024, 1024, 1 << 20
        im.range_mode = ecc_mod.ECC_RANGE_EXPLICIT
        im.lo, im.hi = 0.0, 255.0
        im.out = out.data_ptr()
        st = ecc_mod.ecc_compute_noalloc(ctx.handle, im, 4096, 0)
        assert st == ecc_mod.ECC_ERR_UNSUPPORTED
        assert "fixed scratch" in ecc_mod.ecc_last_error(ctx.handle)
        torch.cuda.synchronize()
    finally:
        ctx.close()
