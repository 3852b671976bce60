"""Pins of the neighbourhood selection of Sec. 3.1.2 (the N kept cells with
the nearest centres to each boundary cell are subdivided too).

* The worked example of Figure 5, stored with its citation in
  tests/golden/neighbours_5x5.txt.
* Brute force with exact rational centres on dyadic mixed-level coverings
  (where the oracle's FP64 distances are exact): for every boundary cell the
  N nearest kept cells by (distance, cell id).
* A grid of non-square cells, where the nearest centres are known in closed
  form (the neighbours across the narrower width come first).
* N = 0 selects exactly the boundary cells; N >= the kept count selects every
  kept cell once any boundary cell exists.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2202_06111_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "neighbours_5x5.txt")


def _golden():
    out = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, tail = line.split(":")
            N, b = (int(v) for v in head.split())
            out.append((N, b, sorted(int(v) for v in tail.split())))
    return out


@pytest.mark.parametrize("N,b,want", _golden(), ids=[f"N{c[0]}" for c in _golden()])
def test_worked_example_figure5(oracle_lib, N, b, want):
    grid = W.Grid((5, 5), (0.0, 0.0), (5.0, 5.0))
    level, idx = oracle.coarse_cells(grid)       # row-major: B_k is cell k-1
    kept = np.ones(25, dtype=np.uint8)
    kept[24] = 0                                 # B25 removed (Figure 4)
    bnd = np.zeros(25, dtype=np.uint8)
    bnd[b - 1] = 1
    sel = oracle.neighbours(grid, level, idx, kept, bnd, N)
    got = sorted((np.nonzero(sel)[0] + 1).tolist())
    assert got == sorted([b] + want)


def _random_covering(rng, n0, splits):
    """A mixed-level covering of a dyadic grid: coarse cells, some split into
    their 2^n children (up to two levels), in canonical order."""
    n = len(n0)
    cells = {(0,) + tuple(int(v) for v in k) for k in np.ndindex(*n0)}
    for _ in range(splits):
        c = sorted(cells)[rng.integers(0, len(cells))]
        if c[0] >= 2:
            continue
        cells.remove(c)
        for ch in np.ndindex(*([2] * n)):
            cells.add((c[0] + 1,) + tuple(2 * c[1 + d] + ch[d] for d in range(n)))
    cells = sorted(cells)
    level = np.array([c[0] for c in cells], dtype=np.uint8)
    idx = np.array([c[1:] for c in cells], dtype=np.int32).reshape(len(cells), n)
    return level, idx


def _centre(grid, level, idx, c):
    w0 = [Fraction(grid.hi[d] - grid.lo[d]) / grid.n0[d] for d in range(grid.n)]
    L = int(level[c])
    return [Fraction(grid.lo[d]) + (2 * int(idx[c, d]) + 1) * w0[d] / 2 ** (L + 1)
            for d in range(grid.n)]


def _brute(grid, level, idx, kept, bnd, N):
    n_cells = level.shape[0]
    sel = np.zeros(n_cells, dtype=np.uint8)
    cen = [_centre(grid, level, idx, c) for c in range(n_cells)]
    for b in range(n_cells):
        if not (kept[b] and bnd[b]):
            continue
        sel[b] = 1
        cand = sorted((sum((x - y) ** 2 for x, y in zip(cen[b], cen[j])), j)
                      for j in range(n_cells) if j != b and kept[j])
        for _, j in cand[:N]:
            sel[j] = 1
    return sel


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("n", [2, 3])
def test_brute_force_dyadic(oracle_lib, seed, n):
    rng = np.random.Generator(np.random.PCG64(seed + 10 * n))
    n0 = (4, 3) if n == 2 else (3, 2, 3)
    grid = W.Grid(n0, tuple([0.0] * n), tuple(float(k) for k in n0))  # unit coarse cells
    level, idx = _random_covering(rng, n0, splits=6)
    kept = (rng.random(level.shape[0]) < 0.85).astype(np.uint8)
    bnd = ((rng.random(level.shape[0]) < 0.25) & (kept == 1)).astype(np.uint8)
    for N in (1, 3, 7, 12):
        got = oracle.neighbours(grid, level, idx, kept, bnd, N)
        np.testing.assert_array_equal(got, _brute(grid, level, idx, kept, bnd, N),
                                      err_msg=f"N={N}")


def test_non_square_cells(oracle_lib):
    """Cells 5/8 wide along x1 and 6/8 along x2: the two x1-neighbours of an
    interior cell are nearest, then the two x2-neighbours (the one with the
    smaller id first), then the diagonals."""
    grid = W.Grid((8, 8), (-2.5, -3.0), (2.5, 3.0))
    level, idx = oracle.coarse_cells(grid)
    kept = np.ones(64, dtype=np.uint8)
    bnd = np.zeros(64, dtype=np.uint8)
    c = 3 * 8 + 4                                     # cell (3, 4)
    bnd[c] = 1
    ids = lambda *ks: sorted(8 * a + b for a, b in ks)
    want = {2: ids((2, 4), (4, 4)),                   # across x1 (width 5/8)
            3: ids((2, 4), (4, 4), (3, 3)),           # then the lower-id x2 neighbour
            4: ids((2, 4), (4, 4), (3, 3), (3, 5))}
    for N, w in want.items():
        sel = oracle.neighbours(grid, level, idx, kept, bnd, N)
        assert sorted(np.nonzero(sel)[0].tolist()) == sorted([c] + w), N


def test_limits(oracle_lib):
    rng = np.random.Generator(np.random.PCG64(3))
    grid = W.Grid((4, 4), (0.0, 0.0), (4.0, 4.0))
    level, idx = _random_covering(rng, (4, 4), splits=4)
    kept = (rng.random(level.shape[0]) < 0.8).astype(np.uint8)
    bnd = ((rng.random(level.shape[0]) < 0.3) & (kept == 1)).astype(np.uint8)
    bnd[np.nonzero(kept)[0][0]] = 1
    np.testing.assert_array_equal(oracle.neighbours(grid, level, idx, kept, bnd, 0), bnd)
    allk = oracle.neighbours(grid, level, idx, kept, bnd, int(kept.sum()))
    np.testing.assert_array_equal(allk, kept)


def test_solve_with_neighbourhood_grows_the_refinement(oracle_lib):
    """A larger N subdivides a superset of the cells (the union of the kept
    region is unchanged by subdivision, Sec. 2.1)."""
    wl = W.Workload("nn", W.vdp(), W.Grid((12, 12), *W.VDP_BOX), W.evenly_spaced(-1, 1, 5),
                    W.LATTICE3, 1, "fp64", analysis="nonleaving")
    counts = []
    for N in (0, 3, 7):
        res = oracle.solve(wl.system, wl.grid, wl.samples, wl.u, 1, analysis=wl.analysis, nn=N)
        st = res["stats"][0]
        assert st["n_selected"] >= st["n_boundary"]
        counts.append(st["n_selected"])
    assert counts[0] < counts[1] < counts[2]
