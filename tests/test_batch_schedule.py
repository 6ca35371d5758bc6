"""Host-side checks of how a batch is split over workgroups (no GPU needed).

Each segment of a batch is counted into one int32 workgroup histogram and one
int32 partial row (the block-shared counters of Sec. 4.3).  A voxel position adds
at most 8 in absolute value, so a segment must cover at most 2^27 voxels.  The schedule is computed by the library's own
host code through ``ecc_batch_schedule``; the descriptors point nowhere (the
diagnostic reads no image memory).
"""
import os

import pytest

from paper_2203_09087_amd import ecc

CAP = 1 << 27
FAKE = 0x1000   # never dereferenced: the schedule is host-only


def _img(dims, dtype=ecc.ECC_U8):
    im = ecc.ecc_image()
    im.data = FAKE
    im.out = FAKE
    im.ndim = len(dims)
    im.dtype = dtype
    for i, d in enumerate(dims):
        im.dims[i] = d
    im.range_mode = ecc.ECC_RANGE_DEFAULT
    return im


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not os.path.exists(ecc.LIB_PATH):
        pytest.skip("libecc_hip.so not built")
    ecc.load_library()


@pytest.mark.parametrize("wgs", [1, 2, 4])
@pytest.mark.parametrize("shape3", [4, 8, 16])
@pytest.mark.parametrize("cus", [8, 256])
def test_one_large_image_is_cut_below_the_counter_bound(wgs, shape3, cus):
    # one 4096^3 volume alone in a batch (6.9e10 voxels): an even split over
    # cus * wgs workgroups gives each 2^36 / (cus * wgs) voxels, 2^33 .. 2^26, far
    # above 2^27 for the small counts; the cap cuts those runs into more segments
    shape = ecc.ecc_batch_shape(shape3, 64, wgs, 0, 0.0)
    n = 4096
    st, segs, mx, ib, cb = ecc.ecc_batch_schedule([_img((n, n, n))], 256, shape, cu_count=cus)
    assert st == ecc.ECC_OK, ecc.ecc_last_error(None)
    assert 0 < mx <= CAP
    assert ib == cb
    if n ** 3 // (cus * wgs) > CAP:
        assert segs > cus * wgs   # runs were split


@pytest.mark.parametrize("cons", [ecc.ECC_VERTEX, ecc.ECC_TOP])
def test_large_2d_image_and_a_mix(cons):
    imgs = [_img((40000, 40000), ecc.ECC_U16), _img((64, 64)), _img((300, 200, 100), ecc.ECC_F32), _img((7, 9))]
    for wgs in (1, 3):
        shape = ecc.ecc_batch_shape(8, 128, wgs, 0, 0.0)
        st, segs, mx, ib, cb = ecc.ecc_batch_schedule(imgs, 4096, shape, cu_count=256, construction=cons)
        assert st == ecc.ECC_OK, ecc.ecc_last_error(None)
        assert mx <= CAP and ib == cb and all(b > 0 for b in ib)


def test_top_filtration_counts_the_extra_lattice_points():
    # the top filtration has one more position per type axis (the lattice point
    # before voxel 0): 24 rows (a whole number of row blocks) need one row block
    # more there
    im = [_img((2, 24, 10))]
    shape = ecc.ecc_batch_shape(8, 16, 1, 0, 0.0)
    _, _, _, ib_v, _ = ecc.ecc_batch_schedule(im, 256, shape, construction=ecc.ECC_VERTEX)
    _, _, _, ib_t, _ = ecc.ecc_batch_schedule(im, 256, shape, construction=ecc.ECC_TOP)
    assert ib_t[0] == ib_v[0] + 1


def test_schedule_rejects_an_unknown_construction():
    assert ecc.ecc_batch_schedule([_img((5, 5))], 256, construction=7)[0] == ecc.ECC_ERR_INVALID_ARG


def test_small_batches_keep_one_segment_per_image_per_workgroup():
    # the cap never splits small images: each image's bricks go to contiguous runs
    imgs = [_img((100, 120)), _img((33, 17, 50))]
    st, segs, mx, ib, cb = ecc.ecc_batch_schedule(imgs, 256, None, cu_count=256)
    assert st == ecc.ECC_OK
    assert ib == cb and segs == sum(ib)   # more workgroups than bricks: one brick each


def test_schedule_rejects_bad_descriptors():
    bad = _img((0, 5))
    st = ecc.ecc_batch_schedule([bad], 256)[0]
    assert st == ecc.ECC_ERR_INVALID_ARG and "dims" in ecc.ecc_last_error(None)
    nine = _img((2, 3, 4, 5))
    nine.ndim = 9
    st = ecc.ecc_batch_schedule([nine], 256)[0]
    assert st == ecc.ECC_ERR_INVALID_ARG
    # five dimensions are valid, but not taken by batches
    st = ecc.ecc_batch_schedule([_img((2, 3, 4, 5, 6))], 256)[0]
    assert st == ecc.ECC_ERR_UNSUPPORTED and "more than 4 dimensions" in ecc.ecc_last_error(None)


@pytest.mark.parametrize("nw", [1, 2, 5])
def test_4d_image_is_scheduled_as_its_signed_3d_passes(nw):
    """A 4D image in a batch is counted as 3D volumes: the vertex filtration's nw
    hyperplanes and nw - 1 adjacent pairs; the top filtration's pairs and only its
    interior hyperplanes (the coefficient -1 + [first] + [last] of an end
    hyperplane is 0), or the one hyperplane when nw is 1.  Every brick of them is
    covered, next to 2D and 3D images in the same batch."""
    hyper = (7, 9, 70)
    for cons in (ecc.ECC_VERTEX, ecc.ECC_TOP):
        st, _, _, ib3, _ = ecc.ecc_batch_schedule([_img(hyper)], 256, None, construction=cons)
        assert st == ecc.ECC_OK
        passes = 2 * nw - 1 if cons == ecc.ECC_VERTEX else (1 if nw == 1 else 2 * nw - 3)
        imgs = [_img((40, 50)), _img((nw,) + hyper, ecc.ECC_F32), _img((6, 5, 4), ecc.ECC_U16)]
        st, segs, mx, ib, cb = ecc.ecc_batch_schedule(imgs, 256, None, construction=cons)
        assert st == ecc.ECC_OK, ecc.ecc_last_error(None)
        assert ib == cb
        assert ib[1] == passes * ib3[0]
        assert 0 < mx <= CAP


@pytest.mark.parametrize("cons", [ecc.ECC_VERTEX, ecc.ECC_TOP])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_segment_count_within_the_reserve_bound(cons, seed):
    """The segment bound that ecc_reserve documents (and batch_reserve_bytes
    sizes a serving lane's scratch with), S <= 2 n + 6 C + V / 2^25 + 3, holds for
    mixed batches of every dtype, from tiny images to ones the 2^27 cap splits."""
    import numpy as np
    rng = np.random.default_rng(seed)
    for cus in (8, 256):
        for count in (1, 5, 64, 300):
            imgs = []
            nvox = 0
            for _ in range(count):
                if rng.random() < 0.5:
                    dims = tuple(int(v) for v in rng.integers(1, 3000, size=2))
                else:
                    dims = tuple(int(v) for v in rng.integers(1, 400, size=3))
                if rng.random() < 0.02:
                    dims = (1200, 1100, 1000)
                imgs.append(_img(dims, int(rng.integers(0, 3))))
                nvox += int(np.prod(dims))
            st, segs, mx, ib, cb = ecc.ecc_batch_schedule(imgs, 4096, None, cu_count=cus, construction=cons)
            assert st == ecc.ECC_OK, ecc.ecc_last_error(None)
            assert ib == cb
            assert segs <= 2 * count + 6 * cus + nvox // (1 << 25) + 3, (cus, count, segs, nvox)
            scratch, tables = ecc.batch_reserve_bytes(count, nvox, 4096, cus)
            assert scratch >= 1024 + tables + 4 * 4096 * segs
