"""Pins of the standard algorithm's subdivision (Sec. 2.1): every kept cell
of a level-0 covering is halved across one dimension, the dimension cycling
from one iteration to the next.

* Hand-worked small cases (tests/golden/bisect_small.txt, cited there).
* Exact geometry: with rational arithmetic, the two halves of every kept
  cell are exactly its lower and upper half across the cut dimension and
  nothing else is produced.
* The loop with nothing removed (a contracting linear field keeps every
  cell): after r iterations the covering is the full uniform grid whose cell
  counts were doubled along dimensions 0, 1, ..., (r - 1) mod n, and the last
  graph equals the graph built directly on that grid.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2202_06111_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bisect_small.txt")


def _cells(text):
    return [tuple(int(v) for v in c.split(",")) for c in text.split()]


def _golden():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            dim, n0, kept, n0_after, halves = [p.strip() for p in line.split("|")]
            cases.append((int(dim), tuple(int(v) for v in n0.split()), _cells(kept),
                          tuple(int(v) for v in n0_after.split()), _cells(halves)))
    return cases


@pytest.mark.parametrize("case", _golden(), ids=lambda c: f"dim{c[0]}-{'x'.join(map(str, c[1]))}")
def test_bisect_worked_cases(oracle_lib, case):
    dim, n0, kept_cells, n0_after, want = case
    n = len(n0)
    grid = W.Grid(n0, (0.0,) * n, (1.0,) * n)
    _, idx = oracle.coarse_cells(grid)
    kept = np.array([tuple(c) in kept_cells for c in idx.tolist()], dtype=np.uint8)
    g2, level, out = oracle.bisect(grid, idx, kept, dim)
    assert tuple(g2.n0) == n0_after
    assert not level.any()
    assert [tuple(c) for c in out.tolist()] == want


def _box(grid, cell):
    """Exact box of a level-0 cell: [lo + i w, lo + (i + 1) w], w = (hi - lo) / n0."""
    out = []
    for d, i in enumerate(cell):
        lo, hi = Fraction(grid.lo[d]), Fraction(grid.hi[d])
        w = (hi - lo) / grid.n0[d]
        out.append((lo + i * w, lo + (i + 1) * w))
    return tuple(out)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bisect_halves_exactly(oracle_lib, n, seed):
    rng = np.random.default_rng(100 * n + seed)
    n0 = tuple(int(v) for v in rng.integers(1, 5 if n < 4 else 3, size=n))
    grid = W.Grid(n0, tuple(rng.uniform(-3, 0, n)), tuple(rng.uniform(0.5, 3, n)))
    _, idx = oracle.coarse_cells(grid)
    kept = (rng.random(idx.shape[0]) < 0.6).astype(np.uint8)
    for dim in range(n):
        g2, _, out = oracle.bisect(grid, idx, kept, dim)
        got = [tuple(c) for c in out.tolist()]
        assert got == sorted(set(got)), "canonical order, no duplicates"
        assert len(got) == 2 * int(kept.sum())
        want = []
        for c in idx[kept.astype(bool)].tolist():
            box = _box(grid, c)
            a, b = box[dim]
            mid = (a + b) / 2
            for half in ((a, mid), (mid, b)):
                want.append(tuple(box[:dim]) + (half,) + tuple(box[dim + 1:]))
        assert sorted(_box(g2, c) for c in got) == sorted(want)


@pytest.mark.parametrize("n,rounds", [(1, 3), (2, 3), (3, 4)])
def test_loop_without_removals_is_the_uniform_grid(oracle_lib, n, rounds):
    system = W.linear(-0.5 * np.eye(n), np.zeros((n, 1)), 0.1, 2)
    n0 = (3, 2, 2)[:n]
    grid = W.Grid(n0, (-1.0,) * n, (1.0,) * n)
    u = np.zeros((1, 1))
    for analysis in ("controlled", "nonleaving"):
        res = oracle.solve(system, grid, W.LATTICE3, u, rounds, analysis=analysis,
                           subdivision="bisect", keep_graphs=True)
        assert len(res["stats"]) == rounds + 1
        want_n0 = list(n0)
        for r, st in enumerate(res["stats"]):
            if r > 0:
                want_n0[(r - 1) % n] *= 2
            assert st["n0"] == tuple(want_n0)
            assert st["n_cells"] == st["n_kept"] == int(np.prod(want_n0))
        fine = W.Grid(tuple(want_n0), grid.lo, grid.hi)
        assert tuple(res["grid"].n0) == tuple(want_n0)
        lv, ix = oracle.coarse_cells(fine)
        np.testing.assert_array_equal(res["idx"], ix)
        direct = oracle.build_graph(system, fine, W.LATTICE3, lv, ix, u)
        for k in ("row_ptr", "col", "out"):
            np.testing.assert_array_equal(res["graphs"][-1][k], direct[k])
