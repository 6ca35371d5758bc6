"""Pins for the oracle in four dimensions (the definitions of Sec. 2.1 and the
VCEC of Sec. 2.3 do not depend on the dimension).

Each check reaches its expected value without the oracle's code: the naive
recount on complexes built cell by cell in doubled coordinates
(``pins.brute_ecc``), the embedding of a 3D image as a single hyperplane or as a
doubled one, invariance of the Euler characteristic under flips and axis
permutations, the Alexander-duality identity between the two filtrations, and
closed forms for a constant image, an interior spike (the complex below the spike
is a 4-box minus an open vertex star, a homotopy 3-sphere: chi = 0) and a pit.
"""
import itertools

import numpy as np
import pytest

import pins

CONS = ("vertex", "top")


def _ecc(oracle_mod, b, nbins, cons, threads=1):
    return oracle_mod.prefix(oracle_mod.vcec_from_bins(b, nbins, cons, threads=threads))


@pytest.mark.parametrize("cons", CONS)
def test_naive_recount_4d(oracle_mod, cons):
    rng = np.random.default_rng(81 if cons == "vertex" else 82)
    for _ in range(25):
        shape = tuple(int(s) for s in rng.integers(1, 4, size=4))
        nb = int(rng.integers(1, 5))
        b = rng.integers(0, nb, size=shape).astype(np.int32)
        assert np.array_equal(_ecc(oracle_mod, b, nb, cons), pins.brute_ecc(b, nb, cons)), (shape, nb)


@pytest.mark.parametrize("cons", CONS)
def test_embedding_of_3d_images(oracle_mod, cons):
    """A 3D image as one hyperplane, at any axis, or as two equal hyperplanes."""
    rng = np.random.default_rng(83)
    for _ in range(10):
        shape = tuple(int(s) for s in rng.integers(1, 7, size=3))
        nb = int(rng.integers(1, 9))
        b = rng.integers(0, nb, size=shape).astype(np.int32)
        ref = _ecc(oracle_mod, b, nb, cons)
        for ax in range(4):
            assert np.array_equal(_ecc(oracle_mod, np.expand_dims(b, ax), nb, cons), ref)
        assert np.array_equal(_ecc(oracle_mod, np.ascontiguousarray(np.stack([b, b])), nb, cons), ref)


@pytest.mark.parametrize("cons", CONS)
def test_invariances_4d(oracle_mod, cons):
    rng = np.random.default_rng(84)
    for _ in range(4):
        shape = tuple(int(s) for s in rng.integers(1, 5, size=4))
        nb = int(rng.integers(2, 7))
        b = rng.integers(0, nb, size=shape).astype(np.int32)
        ref = _ecc(oracle_mod, b, nb, cons)
        for ax in range(4):
            assert np.array_equal(_ecc(oracle_mod, np.ascontiguousarray(np.flip(b, ax)), nb, cons), ref)
        for perm in itertools.permutations(range(4)):
            assert np.array_equal(_ecc(oracle_mod, np.ascontiguousarray(np.transpose(b, perm)), nb, cons), ref)
        assert np.array_equal(_ecc(oracle_mod, b, nb, cons, threads=3), ref)


def test_duality_4d(oracle_mod):
    """chi_top(f <= t) = 1 - (-1)^d (chi_vertex(g <= -t-1) - 1 + (-1)^d) with d = 4,
    g = nbins - f inside a collar of 0 (g <= nbins-1-t <=> f > t)."""
    rng = np.random.default_rng(85)
    for _ in range(20):
        shape = tuple(int(s) for s in rng.integers(1, 4, size=4))
        nb = int(rng.integers(1, 6))
        f = rng.integers(0, nb, size=shape).astype(np.int32)
        top = _ecc(oracle_mod, f, nb, "top")
        g = np.zeros(tuple(s + 2 for s in shape), dtype=np.int32)
        g[tuple(slice(1, -1) for _ in shape)] = nb - f
        ver = _ecc(oracle_mod, g, nb + 1, "vertex")
        for t in range(nb):
            assert top[t] == 1 - (ver[nb - 1 - t] - 1 + 1), (shape, nb, t)


@pytest.mark.parametrize("cons", CONS)
def test_closed_forms_4d(oracle_mod, cons):
    # constant image: empty below its bin, contractible from it on
    b = np.full((3, 2, 4, 3), 5, dtype=np.int32)
    assert np.array_equal(_ecc(oracle_mod, b, 8, cons), np.array([0] * 5 + [1] * 3))
    # interior spike s = 6 over background a = 2: a 3-sphere (chi 0) on [a, s)
    b = np.full((3, 3, 3, 3), 2, dtype=np.int32)
    b[1, 1, 1, 1] = 6
    assert np.array_equal(_ecc(oracle_mod, b, 8, cons), np.array([0, 0, 0, 0, 0, 0, 1, 1]))
    # pit p = 1 below background a = 4: one component from p on, contractible
    b = np.full((3, 4, 3, 3), 4, dtype=np.int32)
    b[2, 1, 0, 2] = 1
    assert np.array_equal(_ecc(oracle_mod, b, 6, cons), np.array([0, 1, 1, 1, 1, 1]))
