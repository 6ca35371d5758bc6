"""Host-side checks of the brick layout of 3D images (no GPU needed).

A 3D brick is an x-chunk of 63 * waves position columns x 3 rows (a strip) x
`depth` planes, each wave on 63 columns of the chunk (its 64th lane supplies the
right neighbour of the 63rd).  A narrow tail of t < 32 positions left after the
full chunks is packed instead: t + 1 lanes per strip (t owning a position, one
supplying the right neighbour), 64 // (t + 1) strips per wave, for the strips
whose rows (three, and the row after them) all lie in the image; the tails of the
other strips run as ordinary bricks.

The rule is written out below independently of the library.  It must cover every
(strip, position) once, touch only rows inside the image in packed bricks, and
give the same brick count as the library's own host code, read through
``ecc_batch_schedule`` (which lists the bricks of a batch's volumes).
"""
import math
import os

import numpy as np
import pytest

from paper_2203_09087_amd import ecc

FAKE = 0x1000   # never dereferenced: the schedule is host-only
LANE_COLS, ROWS = 63, 3


def layout(n1, n2, top, waves):
    """(ordinary chunks per strip, strips, tail, strips per wave, first and end
    packed strip, packed bricks per plane block, bricks per plane block)."""
    org = -1 if top else 0
    xpos, ypos = n2 + top, n1 + top
    nyb = -(-ypos // ROWS)
    nxc, t = divmod(xpos, LANE_COLS * waves)
    sa = 1 if top else 0
    last = n1 - ROWS - 1 - org   # strip s is whole when org + 3 s + 3 <= n1 - 1
    sb = min(last // ROWS + 1, nyb) if last >= 0 else 0
    group = t + 1
    if t > 0 and group <= 32 and sb > sa and (ROWS * (64 // group) + 1) * n2 * 4 < 2 ** 31:
        spw = 64 // group
        npk = -(-(sb - sa) // (spw * waves))
        return dict(nxc=nxc, nyb=nyb, t=t, spw=spw, sa=sa, sb=sb, npk=npk,
                    per_z=nxc * nyb + npk + nyb - (sb - sa))
    nxc += 1 if t else 0
    return dict(nxc=nxc, nyb=nyb, t=0, spw=0, sa=0, sb=0, npk=0, per_z=nxc * nyb)


def cover(n1, n2, top, waves):
    """Counts of every (strip, position) over all bricks of one plane block."""
    Y = layout(n1, n2, top, waves)
    org = -1 if top else 0
    seen = {}
    main = Y["nxc"] * Y["nyb"]
    for r in range(Y["per_z"]):
        if r < main or r - main >= Y["npk"]:
            if r < main:
                xc, yb = r % Y["nxc"], r // Y["nxc"]
            else:
                e = r - main - Y["npk"]
                xc, yb = Y["nxc"], (e if e < Y["sa"] else Y["sb"] + e - Y["sa"])
            for w in range(waves):
                first = org + xc * LANE_COLS * waves + w * LANE_COLS
                for x in range(first, min(first + LANE_COLS, n2)):
                    seen[(yb, x)] = seen.get((yb, x), 0) + 1
        else:
            g = Y["t"] + 1
            for w in range(waves):
                s0 = Y["sa"] + ((r - main) * waves + w) * Y["spw"]
                for lane in range(64):
                    q, j = divmod(lane, g)
                    s = s0 + q
                    if q >= Y["spw"] or s >= Y["sb"]:
                        continue
                    rows = [org + ROWS * s + k for k in range(ROWS + 1)]
                    assert all(0 <= y < n1 for y in rows), (n1, n2, top, waves, s)
                    x = org + Y["nxc"] * LANE_COLS * waves + j
                    if j < Y["t"]:
                        seen[(s, x)] = seen.get((s, x), 0) + 1
                    else:
                        assert not 0 <= x < n2   # the neighbour lane past the row
    return Y, seen


def _cases(seed, count):
    rng = np.random.default_rng(seed)
    fixed = [(512, 512), (256, 256), (4, 8), (3, 100), (5, 70), (40, 505), (26, 127), (1, 1)]
    for n1, n2 in fixed:
        yield n1, n2
    for _ in range(count):
        yield int(rng.integers(1, 120)), int(rng.integers(1, 700))


@pytest.mark.parametrize("top", [0, 1])
def test_layout_covers_every_position_once(top):
    packed = 0
    for n1, n2 in _cases(5 + top, 120):
        for waves in (1, 2, 4, 8, 9):
            Y, seen = cover(n1, n2, top, waves)
            org = -1 if top else 0
            want = {(yb, x) for yb in range(Y["nyb"]) for x in range(org, n2)}
            assert set(seen) == want and set(seen.values()) == {1}, (n1, n2, top, waves)
            packed += Y["spw"] > 0
    assert packed > 100   # the packed path is exercised, not only the fallback


def _wpb(xpos, waves=9):
    """Waves per brick of a batch volume: the most lanes busy, the wider on ties."""
    cols = -(-xpos // LANE_COLS)
    best, best_eff = 1, -1.0
    for w in range(min(cols, waves), 0, -1):
        nx = -(-cols // w)
        eff = cols / (nx * w) * ((waves // w) * w) / waves
        if eff > best_eff + 1e-9:
            best, best_eff = w, eff
    return best


@pytest.mark.parametrize("top", [0, 1])
def test_library_counts_the_same_bricks(top):
    if not os.path.exists(ecc.LIB_PATH):
        pytest.skip("libecc_hip.so not built")
    ecc.load_library()
    depth = 8   # the default plane depth of an unplanned batch
    imgs, want = [], []
    for k, (n1, n2) in enumerate(_cases(11 + top, 60)):
        n0 = 1 + k % 20
        im = ecc.ecc_image()
        im.data = im.out = FAKE
        im.ndim, im.dtype = 3, ecc.ECC_U8
        im.dims[0], im.dims[1], im.dims[2] = n0, n1, n2
        imgs.append(im)
        Y = layout(n1, n2, top, _wpb(n2 + top))
        want.append(Y["per_z"] * math.ceil(n0 / depth))
    cons = ecc.ECC_TOP if top else ecc.ECC_VERTEX
    st, _, _, image_bricks, covered = ecc.ecc_batch_schedule(imgs, 256, None, construction=cons)
    assert st == ecc.ECC_OK, ecc.ecc_last_error(None)
    assert image_bricks == want
    assert covered == image_bricks
