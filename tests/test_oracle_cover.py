"""Pins of the oracle's covering step: which cells a bounding box meets
(Definition 1 with closed cells, Sec. 2.1) and the OUT flag.

Everything here runs on dyadic grids and dyadic boxes, where the oracle's
floating-point positions are exact, so the expected values come from exact
rational arithmetic over every cell (brute force), not from the oracle's own
index formulas.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest

import oracle
from paper_2202_06111_amd import workloads as W


def _cells_meeting(lo, h, N, a, b, open_box):
    out = []
    for j in range(N):
        cl, ch = lo + j * h, lo + (j + 1) * h
        if open_box:
            if cl < b and a < ch:
                out.append(j)
        elif cl <= b and a <= ch:
            out.append(j)
    return out


@pytest.mark.parametrize("n", [1, 2, 3])
def test_cover_ranges_against_exact_brute_force(oracle_lib, n):
    rng = np.random.Generator(np.random.PCG64(11 + n))
    grid = W.Grid(tuple([8] * n), tuple([-2.5] * n), tuple([2.5] * n))
    for Lstar in (0, 1, 2):
        N = 8 << Lstar
        h = Fraction(5, 8) / 2 ** Lstar
        lo = Fraction(-5, 2)
        for trial in range(60):
            # multiples of h/4 so exact faces, outside points and degenerate boxes all occur
            q = rng.integers(-6, 4 * N + 6, size=(n, 2))
            q.sort(axis=1)
            if trial % 7 == 0:
                q[:, 1] = q[:, 0]  # degenerate box (a point in that dimension)
            a = [lo + int(q[d, 0]) * h / 4 for d in range(n)]
            b = [lo + int(q[d, 1]) * h / 4 for d in range(n)]
            R, Ri, outx = oracle.cover(grid, Lstar, np.array([float(v) for v in a]),
                                       np.array([float(v) for v in b]))
            want_out = any(a[d] < lo or b[d] > -lo for d in range(n))
            assert outx == want_out
            for d in range(n):
                closed = _cells_meeting(lo, h, N, a[d], b[d], open_box=False)
                interior = _cells_meeting(lo, h, N, a[d], b[d], open_box=True) or closed
                if closed:
                    assert (R[d, 0], R[d, 1]) == (closed[0], closed[-1])
                else:
                    assert R[d, 0] > R[d, 1]
                if interior:
                    assert (Ri[d, 0], Ri[d, 1]) == (interior[0], interior[-1])
                else:
                    assert Ri[d, 0] > Ri[d, 1]


def _identity(n):
    return W.linear(np.zeros((n, n)), np.zeros((n, 1)), dt=0.1, nsub=1)


@pytest.mark.parametrize("n,samples", [(1, W.LATTICE3), (2, W.LATTICE3), (3, W.CORNERS_CENTER)])
def test_identity_map_stencil(oracle_lib, n, samples):
    """With a zero field each image box is the cell itself; touching counts, so
    every cell is joined to itself and to its 3^n - 1 neighbours, clipped at
    the border of X; nothing is OUT and every cell is kept."""
    side = 6
    grid = W.Grid(tuple([side] * n), tuple([-1.5] * n), tuple([1.5] * n))
    level, idx = oracle.coarse_cells(grid)
    u = np.zeros((2, 1))
    g = oracle.build_graph(_identity(n), grid, samples, level, idx, u)
    assert g["out"].sum() == 0
    lin = {tuple(v): i for i, v in enumerate(idx.tolist())}
    for c in range(level.shape[0]):
        want = sorted(lin[tuple(np.add(idx[c], off))]
                      for off in itertools.product((-1, 0, 1), repeat=n)
                      if all(0 <= idx[c][d] + off[d] < side for d in range(n)))
        for j in range(2):
            r = c * 2 + j
            assert g["col"][g["row_ptr"][r]:g["row_ptr"][r + 1]].tolist() == want
    for analysis in ("controlled", "nonleaving"):
        kept, mask, _ = oracle.prune(g["row_ptr"], g["col"], g["out"], level.shape[0], 2, analysis)
        assert kept.all() and (mask[:, 0] == 3).all()


def _random_covering(rng, n0, splits):
    """A random adaptive covering: start from the coarse grid, split random
    cells into 2^n children `splits` times, and drop a few cells (holes)."""
    n = len(n0)
    cells = {(0,) + c for c in itertools.product(*[range(k) for k in n0])}
    for _ in range(splits):
        c = sorted(cells)[rng.integers(0, len(cells))]
        cells.remove(c)
        for ch in itertools.product((0, 1), repeat=n):
            cells.add((c[0] + 1,) + tuple(2 * c[1 + d] + ch[d] for d in range(n)))
    cells = sorted(cells)
    drop = set(rng.choice(len(cells), size=max(1, len(cells) // 10), replace=False).tolist())
    cells = [c for i, c in enumerate(cells) if i not in drop]
    level = np.array([c[0] for c in cells], dtype=np.uint8)
    idx = np.array([c[1:] for c in cells], dtype=np.int32).reshape(len(cells), n)
    return level, idx


@pytest.mark.parametrize("n", [1, 2])
def test_build_against_exact_box_overlap(oracle_lib, n):
    """Edges = cells whose closed box meets the closed image box; OUT = the box
    leaves X or its interior meets a part of X covered by no cell.  Checked
    with exact rationals against every cell of random adaptive coverings."""
    rng = np.random.Generator(np.random.PCG64(21 + n))
    n0 = (4,) * n
    grid = W.Grid(n0, (-2.0,) * n, (2.0,) * n)
    A = rng.uniform(-1.5, 1.5, size=(n, n))
    system = W.linear(A, np.ones((n, 1)), dt=0.25, nsub=2)
    u = np.array([[-0.5], [0.0], [0.75]])
    n_hole_out = 0
    for trial in range(4):
        level, idx = _random_covering(rng, n0, splits=6)
        g = oracle.build_graph(system, grid, W.LATTICE3, level, idx, u)
        rows = np.arange(level.shape[0] * 3)
        a, b, fin = oracle.bboxes(system, grid, W.LATTICE3, level, idx, u, rows)
        Lstar = int(level.max())
        hs = Fraction(1) / 2 ** Lstar
        Nf = 4 << Lstar
        boxes = []
        for c in range(level.shape[0]):
            w = Fraction(1) / 2 ** int(level[c])
            boxes.append([(Fraction(-2) + int(idx[c, d]) * w, Fraction(-2) + (int(idx[c, d]) + 1) * w)
                          for d in range(n)])
        for r in rows:
            A_ = [Fraction(float(v)) for v in a[r]]
            B_ = [Fraction(float(v)) for v in b[r]]
            # cell widths are powers of two, so the oracle's grid positions are
            # exact up to the one rounding of (a - lo); the random boxes here
            # never fall within that rounding of a face
            want = [c for c in range(level.shape[0])
                    if all(boxes[c][d][0] <= B_[d] and A_[d] <= boxes[c][d][1] for d in range(n))]
            got = g["col"][g["row_ptr"][r]:g["row_ptr"][r + 1]].tolist()
            assert got == want, (trial, r)
            outside = any(A_[d] < -2 or B_[d] > 2 for d in range(n))
            hole = False
            for k in itertools.product(range(Nf), repeat=n):
                fl = [Fraction(-2) + k[d] * hs for d in range(n)]
                meets = all((fl[d] < B_[d] and A_[d] < fl[d] + hs) if A_[d] < B_[d]
                            else (fl[d] <= B_[d] <= fl[d] + hs) for d in range(n))
                if not meets:
                    continue
                covered = any(all(boxes[c][d][0] <= fl[d] and fl[d] + hs <= boxes[c][d][1]
                                  for d in range(n)) for c in range(level.shape[0]))
                if not covered:
                    hole = True
                    break
            assert bool(g["out"][r]) == (outside or hole), (trial, r)
            n_hole_out += int(hole and not outside)
    assert n_hole_out > 0  # the hole rule was exercised
