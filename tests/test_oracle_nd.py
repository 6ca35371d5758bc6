"""Pins for the oracle in five to eight dimensions (the definitions of Sec. 2.1
and the VCEC of Sec. 2.3 are the same in every dimension).

Each check reaches its expected value without the oracle's code: the naive
recount on complexes built cell by cell in doubled coordinates
(``pins.brute_ecc``), the embedding of a lower-dimensional image as a single
hyperplane or as a doubled one, invariance of the Euler characteristic under
flips and axis permutations, the Alexander-duality identity between the two
filtrations, and closed forms: a constant image, an interior spike (below the
spike the complex is a d-box minus an open vertex star, homotopy equivalent to
the (d-1)-sphere: chi = 1 + (-1)^(d-1)) and a pit.
"""
import itertools

import numpy as np
import pytest

import pins

CONS = ("vertex", "top")


def _ecc(oracle_mod, b, nbins, cons, threads=1):
    return oracle_mod.prefix(oracle_mod.vcec_from_bins(b, nbins, cons, threads=threads))


@pytest.mark.parametrize("cons", CONS)
@pytest.mark.parametrize("d", [5, 6])
def test_naive_recount_nd(oracle_mod, cons, d):
    rng = np.random.default_rng(91 + d + (cons == "top"))
    for _ in range(6 if d == 5 else 3):
        shape = tuple(int(s) for s in rng.integers(1, 3 if d == 6 else 4, size=d))
        nb = int(rng.integers(1, 4))
        b = rng.integers(0, nb, size=shape).astype(np.int32)
        assert np.array_equal(_ecc(oracle_mod, b, nb, cons), pins.brute_ecc(b, nb, cons)), (shape, nb)


@pytest.mark.parametrize("cons", CONS)
def test_embedding_of_lower_images(oracle_mod, cons):
    """A 4D image as one hyperplane of a 5D one, at any axis, or as two equal
    hyperplanes; a 5D image likewise inside 6D."""
    rng = np.random.default_rng(97)
    for d in (4, 5):
        for _ in range(3):
            shape = tuple(int(s) for s in rng.integers(1, 4, size=d))
            nb = int(rng.integers(1, 6))
            b = rng.integers(0, nb, size=shape).astype(np.int32)
            ref = _ecc(oracle_mod, b, nb, cons)
            for ax in range(d + 1):
                assert np.array_equal(_ecc(oracle_mod, np.expand_dims(b, ax), nb, cons), ref)
            assert np.array_equal(_ecc(oracle_mod, np.ascontiguousarray(np.stack([b, b])), nb, cons), ref)


@pytest.mark.parametrize("cons", CONS)
def test_invariances_5d(oracle_mod, cons):
    rng = np.random.default_rng(98)
    shape = (2, 3, 2, 3, 2)
    nb = 4
    b = rng.integers(0, nb, size=shape).astype(np.int32)
    ref = _ecc(oracle_mod, b, nb, cons)
    for ax in range(5):
        assert np.array_equal(_ecc(oracle_mod, np.ascontiguousarray(np.flip(b, ax)), nb, cons), ref)
    for perm in itertools.permutations(range(5)):
        assert np.array_equal(_ecc(oracle_mod, np.ascontiguousarray(np.transpose(b, perm)), nb, cons), ref)
    assert np.array_equal(_ecc(oracle_mod, b, nb, cons, threads=2), ref)


def test_duality_5d(oracle_mod):
    """chi_top(f <= t) = 1 - (-1)^d (chi_vertex(g <= -t-1) - 1 + (-1)^d) with d = 5,
    g = nbins - f inside a collar of 0 (g <= nbins-1-t <=> f > t)."""
    rng = np.random.default_rng(99)
    for _ in range(6):
        shape = tuple(int(s) for s in rng.integers(1, 3, size=5))
        nb = int(rng.integers(1, 5))
        f = rng.integers(0, nb, size=shape).astype(np.int32)
        top = _ecc(oracle_mod, f, nb, "top")
        g = np.zeros(tuple(s + 2 for s in shape), dtype=np.int32)
        g[tuple(slice(1, -1) for _ in shape)] = nb - f
        ver = _ecc(oracle_mod, g, nb + 1, "vertex")
        for t in range(nb):
            assert top[t] == 1 + (ver[nb - 1 - t] - 1 - 1), (shape, nb, t)


@pytest.mark.parametrize("cons", CONS)
@pytest.mark.parametrize("d", [5, 6])
def test_closed_forms_nd(oracle_mod, cons, d):
    # constant image: empty below its bin, contractible from it on
    b = np.full((2, 3) + (2,) * (d - 2), 5, dtype=np.int32)
    assert np.array_equal(_ecc(oracle_mod, b, 8, cons), np.array([0] * 5 + [1] * 3))
    # interior spike s = 6 over background a = 2: a (d-1)-sphere on [a, s)
    b = np.full((3,) * d, 2, dtype=np.int32)
    b[(1,) * d] = 6
    sphere = 1 + (-1) ** (d - 1)
    assert np.array_equal(_ecc(oracle_mod, b, 8, cons), np.array([0, 0] + [sphere] * 4 + [1, 1]))
    # pit p = 1 below background a = 4: one component from p on, contractible
    b = np.full((3, 2) + (2,) * (d - 2), 4, dtype=np.int32)
    b[(2, 1) + (0,) * (d - 2)] = 1
    assert np.array_equal(_ecc(oracle_mod, b, 6, cons), np.array([0, 1, 1, 1, 1, 1]))


@pytest.mark.parametrize("cons", CONS)
def test_naive_recount_7d(oracle_mod, cons):
    """Seven dimensions, five of them two voxels long."""
    rng = np.random.default_rng(96 + (cons == "top"))
    b = rng.integers(0, 2, size=(2, 2, 1, 2, 1, 2, 2)).astype(np.int32)
    assert np.array_equal(_ecc(oracle_mod, b, 2, cons), pins.brute_ecc(b, 2, cons))


def test_largest_dimension_and_beyond(oracle_mod):
    """8 dimensions are taken (a 2^8 constant block is contractible), 9 are not."""
    b = np.zeros((2,) * 8, dtype=np.int32)
    for cons in CONS:
        assert np.array_equal(_ecc(oracle_mod, b, 2, cons), np.array([1, 1]))
    with pytest.raises(ValueError):
        oracle_mod.vcec_from_bins(np.zeros((1,) * 9, dtype=np.int32), 2)
