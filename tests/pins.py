"""Independent checks ("pins") for the oracle, written without any of its code.

The oracle enumerates cells by (anchor, shape) and gives each its filtration
value.  The helpers here reach the same numbers by other routes:

* ``complex_at``  - builds the complex K_{<=t} itself, in doubled coordinates
  (a cell of the cubical grid is a point of Z^d whose odd coordinates are its
  non-degenerate intervals, as in the book of Kaczynski, Mischaikow and Mrozek
  that the paper follows in Sec. 2.1), by testing each cell's voxels against the
  threshold - the naive O(mn) recount of Sec. 2.3;
* ``betti_gf2``   - Betti numbers of that complex from ranks of its boundary
  matrices over GF(2) (Euler-Poincare, Eq. (1));
* ``betti_labels`` - beta_0 and beta_{d-1} from connected-component labelling of
  the thresholded voxel set and of its padded complement (scipy.ndimage), using
  the connectivity each construction induces.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy import ndimage


def _voxels_of_cell(c, shape, construction):
    """Voxels whose values decide cell ``c`` (doubled coordinates)."""
    per_axis = []
    for ci, ni in zip(c, shape):
        if construction == "vertex":
            # even: vertex at voxel ci/2 ; odd: edge between voxels (ci-1)/2 and (ci+1)/2
            per_axis.append((ci // 2,) if ci % 2 == 0 else (ci // 2, ci // 2 + 1))
        else:
            # odd: interval of voxel (ci-1)/2 ; even: lattice point between voxels ci/2-1 and ci/2
            if ci % 2 == 1:
                per_axis.append(((ci - 1) // 2,))
            else:
                per_axis.append(tuple(k for k in (ci // 2 - 1, ci // 2) if 0 <= k < ni))
    return itertools.product(*per_axis)


def complex_at(bins: np.ndarray, t: int, construction: str):
    """All cells (doubled coordinates) of K_{<=t}.

    vertex: a cell is present iff every one of its vertices (voxels) is <= t;
    top:    a cell is present iff some voxel containing it is <= t (the complex
            is the union of the closed voxels below the threshold)."""
    shape = bins.shape
    if construction == "vertex":
        ranges = [range(2 * n - 1) for n in shape]
        test = all
    else:
        ranges = [range(2 * n + 1) for n in shape]
        test = any
    cells = []
    for c in itertools.product(*ranges):
        if test(bins[v] <= t for v in _voxels_of_cell(c, shape, construction)):
            cells.append(c)
    return cells


def dim_of(c) -> int:
    return sum(ci % 2 for ci in c)


def euler_char(cells) -> int:
    return sum(-1 if dim_of(c) % 2 else 1 for c in cells)


def brute_ecc(bins: np.ndarray, nbins: int, construction: str) -> np.ndarray:
    """chi(K_{<=t}) for every t, each complex built from scratch."""
    return np.array([euler_char(complex_at(bins, t, construction)) for t in range(nbins)],
                    dtype=np.int64)


def _rank_gf2(rows) -> int:
    """Rank over GF(2) of a list of rows given as Python int bitsets."""
    rank = 0
    pivots = {}
    for r in rows:
        while r:
            top = r.bit_length() - 1
            if top in pivots:
                r ^= pivots[top]
            else:
                pivots[top] = r
                rank += 1
                break
    return rank


def betti_gf2(cells, d: int):
    """Betti numbers beta_0..beta_d of a cubical complex over GF(2)."""
    by_dim = [[] for _ in range(d + 1)]
    for c in cells:
        by_dim[dim_of(c)].append(c)
    index = [{c: i for i, c in enumerate(cs)} for cs in by_dim]
    ranks = [0] * (d + 2)          # ranks[k] = rank of boundary C_k -> C_{k-1}
    for k in range(1, d + 1):
        rows = []
        for c in by_dim[k]:
            r = 0
            for ax, ci in enumerate(c):
                if ci % 2:
                    for dc in (-1, 1):
                        f = list(c)
                        f[ax] = ci + dc
                        r |= 1 << index[k - 1][tuple(f)]   # KeyError = complex not closed
            rows.append(r)
        ranks[k] = _rank_gf2(rows)
    return [len(by_dim[k]) - ranks[k] - ranks[k + 1] for k in range(d + 1)]


def betti_labels(bins: np.ndarray, t: int, construction: str):
    """(beta_0, beta_{d-1}) by labelling.

    vertex: the complex joins face-adjacent voxels, so the voxel set is taken
            with face connectivity and the complement with full connectivity;
    top:    closed voxels touching at a corner are joined, so the connectivities
            are swapped.  beta_{d-1} counts bounded complement components."""
    d = bins.ndim
    fg = bins <= t
    face = ndimage.generate_binary_structure(d, 1)
    full = ndimage.generate_binary_structure(d, d)
    fg_conn, bg_conn = (face, full) if construction == "vertex" else (full, face)
    _, b0 = ndimage.label(fg, structure=fg_conn)
    bg = np.pad(~fg, 1, constant_values=True)
    _, nbg = ndimage.label(bg, structure=bg_conn)
    return b0, nbg - 1
