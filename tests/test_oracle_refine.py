"""Pins of boundary selection, subdivision, the iteration loop and queries.

* The 5x5 worked example of Sec. 3.1.1 (Figure 4 and Remark 1), stored with
  its citation in tests/golden/boundary_5x5.txt.
* Subdivision preserves the union of the kept cells (Sec. 2.1: the covered
  set does not change, only the cell diameters).
* The kept region never grows across rounds and the cell count obeys
  n_{r+1} <= |K*_r| + (2^n - 1) |boundary_r|.
* Point queries against brute-force point location over the cell boxes.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2202_06111_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "boundary_5x5.txt")


def _golden_cases():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, tail = line.split(":")
            parts = head.split()
            cases.append((parts[0], parts[1], [int(v) for v in parts[2:]],
                          sorted(int(v) for v in tail.split())))
    return cases


@pytest.mark.parametrize("case,rule,removed,want", _golden_cases(),
                         ids=[f"{c[0]}-{c[1]}" for c in _golden_cases()])
def test_worked_example_5x5(oracle_lib, case, rule, removed, want):
    grid = W.Grid((5, 5), (0.0, 0.0), (5.0, 5.0))
    level, idx = oracle.coarse_cells(grid)       # row-major: B_k is cell k-1
    kept = np.ones(25, dtype=np.uint8)
    for b in removed:
        kept[b - 1] = 0
    bnd = oracle.boundary(grid, level, idx, kept, rule)
    assert sorted((np.nonzero(bnd)[0] + 1).tolist()) == want


def _region(grid, level, idx, sel, Lf):
    """Finest-level occupancy of the selected cells at level Lf."""
    n = grid.n
    occ = np.zeros(tuple(k << Lf for k in grid.n0), dtype=bool)
    for c in np.nonzero(sel)[0]:
        sh = Lf - int(level[c])
        sl = tuple(slice(int(idx[c, d]) << sh, (int(idx[c, d]) + 1) << sh) for d in range(n))
        occ[sl] = True
    return occ


@pytest.mark.parametrize("analysis", ["controlled", "nonleaving"])
def test_rounds_preserve_union_and_shrink(oracle_lib, analysis):
    wl = W.vdp_adaptive_32()
    if analysis == "controlled":  # coarse 32x32 keeps nothing under this analysis
        wl = W.Workload(wl.name, wl.system, W.Grid((48, 48), *W.VDP_BOX), wl.u, wl.samples, 3,
                        wl.precision)
    u = wl.u
    level, idx = oracle.coarse_cells(wl.grid)
    Lf = wl.rounds + 1
    prev_region = None
    for r in range(4):
        g = oracle.build_graph(wl.system, wl.grid, wl.samples, level, idx, u)
        kept, _, _ = oracle.prune(g["row_ptr"], g["col"], g["out"], level.shape[0], wl.K, analysis)
        region = _region(wl.grid, level, idx, kept, Lf)
        if prev_region is not None:
            assert not (region & ~prev_region).any()
        prev_region = region
        bnd = oracle.boundary(wl.grid, level, idx, kept, "shell")
        nl, ni = oracle.subdivide(wl.grid, level, idx, kept, bnd)
        assert nl.shape[0] == int(kept.sum()) + (2 ** wl.grid.n - 1) * int(bnd.sum())
        new_region = _region(wl.grid, nl, ni, np.ones(nl.shape[0], bool), Lf)
        np.testing.assert_array_equal(new_region, region)
        # canonical order: level, then row-major index
        key = [(int(nl[c]),) + tuple(int(v) for v in ni[c]) for c in range(nl.shape[0])]
        assert key == sorted(key) and len(set(key)) == len(key)
        level, idx = nl, ni
    assert prev_region.sum() > 0


def test_boundary_cells_are_exactly_those_touching_the_outside(oracle_lib):
    """Shell rule on a random kept pattern of a uniform grid: a kept cell is a
    boundary cell iff one of its 8 neighbours is dropped or outside the grid."""
    rng = np.random.Generator(np.random.PCG64(41))
    grid = W.Grid((9, 7), (0.0, 0.0), (9.0, 7.0))
    level, idx = oracle.coarse_cells(grid)
    kept = (rng.random(63) < 0.7).astype(np.uint8)
    bnd = oracle.boundary(grid, level, idx, kept, "shell")
    K2 = kept.reshape(9, 7)
    for c in range(63):
        i, j = divmod(c, 7)
        want = False
        if K2[i, j]:
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    a, b = i + di, j + dj
                    if (di or dj) and not (0 <= a < 9 and 0 <= b < 7 and K2[a, b]):
                        want = True
        assert bool(bnd[c]) == want


def test_query_against_point_location(oracle_lib):
    rng = np.random.Generator(np.random.PCG64(42))
    grid = W.Grid((4, 4), (-2.0, -2.0), (2.0, 2.0))
    level, idx = oracle.coarse_cells(grid)
    kept = np.ones(16, np.uint8)
    for _ in range(2):  # two refinement rounds with random keeps
        kept = (rng.random(level.shape[0]) < 0.8).astype(np.uint8)
        bnd = oracle.boundary(grid, level, idx, kept, "shell")
        level, idx = oracle.subdivide(grid, level, idx, kept, bnd)
    kept = (rng.random(level.shape[0]) < 0.8).astype(np.uint8)
    mask = rng.integers(0, 2 ** 63, size=(level.shape[0], 1), dtype=np.uint64) * kept[:, None]
    # dyadic query states, including faces, corners, the upper border and outside points
    q = rng.integers(-3, 4 * 16 + 4, size=(3000, 2))
    states = -2.0 + q / 16.0
    member, adm = oracle.query(grid, level, idx, kept, mask, states)
    for s in range(states.shape[0]):
        x = [Fraction(float(v)) for v in states[s]]
        inside = all(-2 <= v <= 2 for v in x)
        owner = None
        if inside:
            # half-open cells [lo, lo + w), the last cell of each axis closed at hi
            for c in range(level.shape[0]):
                w = Fraction(1, 2 ** int(level[c]))
                ok = True
                for d in range(2):
                    a = -2 + int(idx[c, d]) * w
                    b = a + w
                    if not (a <= x[d] < b or (x[d] == 2 and b == 2)):
                        ok = False
                if ok:
                    owner = c
                    break
        want_member = owner is not None and bool(kept[owner])
        assert bool(member[s]) == want_member, s
        assert int(adm[s, 0]) == (int(mask[owner, 0]) if want_member else 0)


def _random_mixed_covering(rng, n0, splits):
    """A covering with cells of several levels, made without the oracle: start
    from the coarse grid and, `splits` times, replace a random third of the
    cells by their 2^n children.  Returned in canonical order."""
    n = len(n0)
    cells = [(0,) + c for c in itertools.product(*[range(k) for k in n0])]
    for _ in range(splits):
        nxt = []
        for c in cells:
            if rng.random() < 0.35:
                L, ix = c[0], c[1:]
                for ch in itertools.product((0, 1), repeat=n):
                    nxt.append((L + 1,) + tuple(2 * ix[d] + ch[d] for d in range(n)))
            else:
                nxt.append(c)
        cells = nxt
    cells.sort()
    level = np.array([c[0] for c in cells], dtype=np.uint8)
    idx = np.array([c[1:] for c in cells], dtype=np.int32).reshape(len(cells), n)
    return level, idx


def _alg1_brute_force(grid, level, idx, kept, rule):
    """Algorithm 1 (Sec. 3.1.1) evaluated literally in exact rationals.  Each
    kept cell is enlarged by delta = (finest cell width) / 4 per side; a probe
    point of the enlarged box that lies in no closed kept cell (a point outside
    X lies in none) makes the cell a boundary cell.  Probes: the 2^n vertices
    of the enlarged box ("corners", the algorithm as printed), or for "shell"
    also the points of the enlarged box's faces above the centres of the
    finest-level cells along the cell's faces and edges (the edge points of
    Remark 1, taken at every finest position)."""
    n = grid.n
    Lf = int(level.max())
    lo = [Fraction(v) for v in grid.lo]
    w0 = [(Fraction(grid.hi[d]) - Fraction(grid.lo[d])) / grid.n0[d] for d in range(n)]
    wf = [w / 2 ** Lf for w in w0]
    boxes = []
    for c in range(level.shape[0]):
        w = [w0[d] / 2 ** int(level[c]) for d in range(n)]
        a = [lo[d] + int(idx[c, d]) * w[d] for d in range(n)]
        boxes.append((a, [a[d] + w[d] for d in range(n)]))
    kept_boxes = [boxes[c] for c in range(len(boxes)) if kept[c]]
    out = np.zeros(level.shape[0], dtype=np.uint8)
    for c in np.nonzero(kept)[0]:
        a, b = boxes[c]
        axes = []
        for d in range(n):
            delta = wf[d] / 4
            pts = [a[d] - delta, b[d] + delta]
            if rule == "shell":
                m = int((b[d] - a[d]) / wf[d])
                pts += [a[d] + (k + Fraction(1, 2)) * wf[d] for k in range(m)]
            axes.append(pts)
        for p in itertools.product(*axes):
            on_face = [p[d] < a[d] or p[d] > b[d] for d in range(n)]
            if rule == "corners" and not all(on_face):
                continue
            if not any(on_face):
                continue
            if not any(all(ka[d] <= p[d] <= kb[d] for d in range(n)) for ka, kb in kept_boxes):
                out[c] = 1
                break
    return out


@pytest.mark.parametrize("n0,splits,seed", [((5, 4), 2, 3), ((4, 4), 3, 4), ((3, 3, 2), 2, 5)])
@pytest.mark.parametrize("rule", ["shell", "corners"])
def test_boundary_on_mixed_level_coverings_against_algorithm_1(oracle_lib, n0, splits, seed, rule):
    """Boundary selection on coverings whose cells have different levels, with
    holes (dropped cells), against Algorithm 1 evaluated literally in exact
    arithmetic.  The probes of a coarse cell next to finely refined
    neighbours must look at finest-level positions, not at the cell's own
    level: a dropped fine cell beside a coarse one makes it a boundary cell."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(n0)
    grid = W.Grid(n0, tuple([-1.0] * n), tuple([-1.0 + 1.25 * k for k in n0]))
    level, idx = _random_mixed_covering(rng, n0, splits)
    assert len(set(level.tolist())) == splits + 1
    for trial in range(3):
        kept = (rng.random(level.shape[0]) < 0.8).astype(np.uint8)
        got = oracle.boundary(grid, level, idx, kept, rule)
        want = _alg1_brute_force(grid, level, idx, kept, rule)
        np.testing.assert_array_equal(got, want, err_msg=f"trial {trial}")
        # the mixed levels matter: some boundary cell is coarser than the finest level
        if trial == 0:
            assert (want.astype(bool) & (level < level.max())).any()
