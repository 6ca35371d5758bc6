"""Pins for the oracle: facts fixed by the paper's definitions and by mathematics.

Every check here reaches its expected value without the oracle's code: the naive
recount of Sec. 2.3 on complexes built cell by cell (``pins.complex_at``), Betti
numbers (Euler-Poincare, Eq. (1)) from GF(2) ranks and from connected-component
labelling, closed forms derived by counting cells of small images, invariances of
the Euler characteristic, and the Alexander-duality identity between the two
filtrations.
"""
import itertools
import math

import numpy as np
import pytest

import pins

CONS = ("vertex", "top")


def _ecc_bins(oracle_mod, b, nbins, cons):
    return oracle_mod.prefix(oracle_mod.vcec_from_bins(b, nbins, cons))


def _random_cases(seed, count, max_side, dims=(1, 2, 3), max_bins=6):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        d = int(rng.choice(dims))
        side = max_side if d < 3 else min(max_side, 5)
        shape = tuple(int(s) for s in rng.integers(1, side + 1, size=d))
        nb = int(rng.integers(1, max_bins + 1))
        yield rng.integers(0, nb, size=shape).astype(np.int32), nb


@pytest.mark.parametrize("cons", CONS)
def test_naive_recount_matches(oracle_mod, cons):
    """ECC_i equals chi of K_{<=t_i} rebuilt from scratch at every threshold (Sec. 2.3)."""
    for b, nb in _random_cases(11 if cons == "vertex" else 12, 120, 6):
        got = _ecc_bins(oracle_mod, b, nb, cons)
        want = pins.brute_ecc(b, nb, cons)
        assert np.array_equal(got, want), (b.shape, nb, got, want)


@pytest.mark.parametrize("cons", CONS)
def test_euler_poincare_2d_by_labelling(oracle_mod, cons):
    """2D: chi = beta_0 - beta_1 with both Betti numbers counted by labelling."""
    rng = np.random.default_rng(21)
    for _ in range(150):
        shape = tuple(int(s) for s in rng.integers(1, 9, size=2))
        nb = int(rng.integers(2, 6))
        b = rng.integers(0, nb, size=shape).astype(np.int32)
        got = _ecc_bins(oracle_mod, b, nb, cons)
        for t in range(nb):
            b0, b1 = pins.betti_labels(b, t, cons)
            assert got[t] == b0 - b1, (shape, t, got[t], b0, b1)


@pytest.mark.parametrize("cons", CONS)
def test_euler_poincare_3d_gf2(oracle_mod, cons):
    """3D: chi = b0 - b1 + b2 from GF(2) ranks; b0 and b2 also agree with labelling."""
    rng = np.random.default_rng(31 if cons == "vertex" else 32)
    for _ in range(25):
        shape = tuple(int(s) for s in rng.integers(1, 5, size=3))
        nb = int(rng.integers(2, 5))
        b = rng.integers(0, nb, size=shape).astype(np.int32)
        got = _ecc_bins(oracle_mod, b, nb, cons)
        for t in range(nb):
            cells = pins.complex_at(b, t, cons)
            betti = pins.betti_gf2(cells, 3)
            lab0, lab2 = pins.betti_labels(b, t, cons)
            assert betti[0] == lab0 and betti[2] == lab2, (shape, t, betti, lab0, lab2)
            assert got[t] == betti[0] - betti[1] + betti[2] - betti[3]


@pytest.mark.parametrize("cons", CONS)
def test_constant_image_steps_to_one(oracle_mod, cons):
    """A constant image is one contractible block: ECC = 0 below its level, 1 from it on."""
    for shape in [(1,), (5,), (1, 1), (1, 7), (4, 3), (1, 1, 1), (1, 4, 1), (3, 4, 5)]:
        for c in (0, 3, 7):
            b = np.full(shape, c, dtype=np.int32)
            got = _ecc_bins(oracle_mod, b, 8, cons)
            assert np.array_equal(got, (np.arange(8) >= c).astype(np.int64)), (shape, c, got)


@pytest.mark.parametrize("cons", CONS)
def test_last_value_is_one(oracle_mod, cons):
    """At the top threshold the complex is the whole box, which is contractible."""
    rng = np.random.default_rng(41)
    for shape in [(1000,), (37, 23), (64, 1), (9, 10, 11), (2, 31, 3)]:
        nb = 50
        b = rng.integers(0, nb, size=shape).astype(np.int32)
        assert _ecc_bins(oracle_mod, b, nb, cons)[-1] == 1


def _checker(shape):
    return (np.indices(shape).sum(axis=0) % 2).astype(np.int32)


def test_checkerboard_closed_forms(oracle_mod):
    """Checkerboards (0 at the origin, bins 0/1), ECC at level 0.

    vertex: the level-0 voxels have no face-neighbours at level 0, so the complex
            is ceil(N/2) isolated vertices.
    top (2D, n x n): the level-0 closed squares touch at corners; counting cells,
            V = (n+1)^2 - 2 (n even: the two corners of level-1 squares are missing)
            or (n+1)^2 (n odd), E = 4 * #squares (no shared edges), F = #squares."""
    for n in range(1, 9):
        for shape in [(n, n), (n, n + 1), (n, n, n)]:
            b = _checker(shape)
            got = _ecc_bins(oracle_mod, b, 2, "vertex")
            assert got[0] == math.ceil(b.size / 2) and got[1] == 1
        b = _checker((n, n))
        sq = (n * n + 1) // 2
        verts = (n + 1) ** 2 - (2 if n % 2 == 0 else 0)
        want = verts - 4 * sq + sq
        got = _ecc_bins(oracle_mod, b, 2, "top")
        assert got[0] == want and got[1] == 1, (n, got, want)


@pytest.mark.parametrize("cons", CONS)
def test_spike_and_pit(oracle_mod, cons):
    """One voxel above (spike) or below (pit) a constant background.

    Below the spike's level the complex is the box minus one voxel: a 2D interior
    spike leaves a hole (chi 0), a 3D interior spike a cavity (chi 2); at the image
    boundary nothing is enclosed (chi 1).  A pit is a point that grows into the box."""
    bg, hi, lo = 2, 5, 1
    for shape in [(7, 6), (5, 5, 6)]:
        d = len(shape)
        for pos in itertools.product(*[(0, 1, s // 2, s - 1) for s in shape]):
            interior = all(0 < p < s - 1 for p, s in zip(pos, shape))
            b = np.full(shape, bg, dtype=np.int32)
            b[pos] = hi
            got = _ecc_bins(oracle_mod, b, 7, cons)
            mid = (2 if d == 3 else 0) if interior else 1
            want = np.array([0, 0, mid, mid, mid, 1, 1])
            assert np.array_equal(got, want), (shape, pos, got)
            b[pos] = lo
            got = _ecc_bins(oracle_mod, b, 7, cons)
            assert np.array_equal(got, np.array([0, 1, 1, 1, 1, 1, 1])), (shape, pos, got)


@pytest.mark.parametrize("cons", CONS)
def test_invariances(oracle_mod, cons):
    """chi is invariant under flips and axis permutations (the tie-break changes,
    the complex does not), under adding a size-1 axis, and under doubling a layer."""
    rng = np.random.default_rng(51)
    for _ in range(20):
        d = int(rng.integers(1, 4))
        shape = tuple(int(s) for s in rng.integers(1, 9, size=d))
        nb = int(rng.integers(1, 9))
        b = rng.integers(0, nb, size=shape).astype(np.int32)
        ref = _ecc_bins(oracle_mod, b, nb, cons)
        for ax in range(d):
            assert np.array_equal(_ecc_bins(oracle_mod, np.flip(b, ax), nb, cons), ref)
        for perm in itertools.permutations(range(d)):
            assert np.array_equal(_ecc_bins(oracle_mod, np.transpose(b, perm), nb, cons), ref)
        if d < 3:
            for ax in range(d + 1):
                assert np.array_equal(_ecc_bins(oracle_mod, np.expand_dims(b, ax), nb, cons), ref)
            assert np.array_equal(_ecc_bins(oracle_mod, np.stack([b, b]), nb, cons), ref)
        threaded = oracle_mod.prefix(oracle_mod.vcec_from_bins(b, nb, cons, threads=4))
        assert np.array_equal(threaded, ref)


def test_duality_between_constructions(oracle_mod):
    """Alexander duality: with g = -f on the image and a collar below everything,
    chi_top(f <= t) = 1 - (-1)^d (chi_vertex(g <= -t-1) - 1 + (-1)^d).
    In bins: g = nbins - f inside, 0 on the collar, and g <= nbins-1-t <=> f > t."""
    rng = np.random.default_rng(61)
    for _ in range(150):
        d = int(rng.integers(1, 4))
        shape = tuple(int(s) for s in rng.integers(1, 7, size=d))
        nb = int(rng.integers(1, 7))
        f = rng.integers(0, nb, size=shape).astype(np.int32)
        top = _ecc_bins(oracle_mod, f, nb, "top")
        g = np.zeros(tuple(s + 2 for s in shape), dtype=np.int32)
        g[tuple(slice(1, -1) for _ in shape)] = nb - f
        ver = _ecc_bins(oracle_mod, g, nb + 1, "vertex")
        sgn = (-1) ** d
        for t in range(nb):
            assert top[t] == 1 - sgn * (ver[nb - 1 - t] - 1 + sgn), (shape, nb, t)


def test_vcec_is_difference_of_ecc(oracle_mod):
    """VCEC_0 = ECC_0 and VCEC_i = ECC_i - ECC_{i-1} (Sec. 2.3)."""
    rng = np.random.default_rng(71)
    b = rng.integers(0, 40, size=(13, 17, 5)).astype(np.int32)
    for cons in CONS:
        v = oracle_mod.vcec_from_bins(b, 40, cons)
        e = oracle_mod.prefix(v)
        assert np.array_equal(np.diff(e, prepend=0), v)
