"""The golden curves under tests/golden/ (written by make_golden.py from the
oracle) still match the oracle, so an accidental change to its arithmetic shows
up here; the GPU parity tests compare the library against the same files."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name, cons):
    with open(os.path.join(GOLDEN, f"{name}_{cons}.txt")) as f:
        return np.array([int(l) for l in f if l.strip() and not l.startswith("#")], dtype=np.int64)


def golden_cases():
    import sys
    sys.path.insert(0, GOLDEN)
    import make_golden
    return make_golden.CASES


@pytest.mark.parametrize("cons", ["vertex", "top"])
def test_oracle_reproduces_golden(oracle_mod, cons):
    for name, (desc, make, nbins, rng) in golden_cases().items():
        want = load_golden(name, cons)
        got = oracle_mod.ecc(make(), nbins, cons, value_range=rng, threads=4)
        assert np.array_equal(got, want), name
        assert want[-1] == 1


@pytest.mark.gpu
@pytest.mark.parametrize("cons", ["vertex", "top"])
def test_library_matches_golden(cons):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_09087_amd import ecc
    ctx = ecc.Context(0, cons)
    for name, (desc, make, nbins, rng) in golden_cases().items():
        got = ctx.compute(torch.from_numpy(make()).cuda(), nbins, value_range=rng)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), load_golden(name, cons)), name
    ctx.close()
