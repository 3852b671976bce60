"""GPU parity of the standard algorithm's subdivision (Sec. 2.1: every kept
cell halved across a dimension that cycles from one iteration to the next)
through the C ABI (gis_bisect, and gis_solve / gis_solve_batch with
subdivision "bisect") against the oracle.  Cell lists, kept flags, masks,
round statistics and query answers are compared bit for bit.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from conftest import gpu_available
from paper_2202_06111_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]


@pytest.fixture(scope="module")
def G():
    from paper_2202_06111_amd import gis
    return gis


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


def _np(t):
    return t.detach().cpu().numpy()


def _dev(ctx, a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a, dtype), device=ctx.dev)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", [0, 1])
def test_bisect_step(G, ctx, n, seed):
    """Random level-0 coverings with holes, kept subsets and every dimension;
    the input list also shuffled (its order must not matter)."""
    rng = np.random.default_rng(10 * n + seed)
    n0 = tuple(int(v) for v in rng.integers(3, (300, 40, 14, 7)[n - 1], size=n))
    grid = W.Grid(n0, tuple(rng.uniform(-2, -0.5, n)), tuple(rng.uniform(0.5, 2, n)))
    _, idx = oracle.coarse_cells(grid)
    idx = idx[rng.random(idx.shape[0]) < 0.8]          # holes
    kept = (rng.random(idx.shape[0]) < 0.7).astype(np.uint8)
    for dim in range(n):
        want_grid, want_lv, want_ix = oracle.bisect(grid, idx, kept, dim)
        for order in (np.arange(idx.shape[0]), rng.permutation(idx.shape[0])):
            lv = _dev(ctx, np.zeros(idx.shape[0]), np.uint8)
            g2, got_lv, got_ix = G.bisect(ctx, grid, lv, _dev(ctx, idx[order], np.int32),
                                          _dev(ctx, kept[order], np.uint8), dim)
            assert tuple(g2.n0) == tuple(want_grid.n0)
            np.testing.assert_array_equal(_np(got_lv), want_lv)
            np.testing.assert_array_equal(_np(got_ix), want_ix)


def test_bisect_edge_cases(G, ctx):
    grid = W.Grid((4, 3), (0.0, 0.0), (1.0, 1.0))
    lv0, idx = oracle.coarse_cells(grid)
    # nothing kept, everything kept, one cell
    for kept in (np.zeros(12, np.uint8), np.ones(12, np.uint8), np.eye(1, 12, 7, dtype=np.uint8)[0]):
        _, want_lv, want_ix = oracle.bisect(grid, idx, kept, 1)
        _, got_lv, got_ix = G.bisect(ctx, grid, _dev(ctx, lv0, np.uint8), _dev(ctx, idx, np.int32),
                                     _dev(ctx, kept, np.uint8), 1)
        np.testing.assert_array_equal(_np(got_ix), want_ix)
        assert _np(got_lv).shape[0] == want_lv.shape[0]
    # duplicates in the input are merged
    dup = np.concatenate([idx, idx[:5]])
    kd = np.ones(dup.shape[0], np.uint8)
    _, _, got_ix = G.bisect(ctx, grid, _dev(ctx, np.zeros(dup.shape[0]), np.uint8),
                            _dev(ctx, dup, np.int32), _dev(ctx, kd, np.uint8), 0)
    np.testing.assert_array_equal(_np(got_ix), oracle.bisect(grid, idx, np.ones(12, np.uint8), 0)[2])
    # an empty list
    _, e_lv, e_ix = G.bisect(ctx, grid, _dev(ctx, np.zeros(0), np.uint8),
                             _dev(ctx, np.zeros((0, 2)), np.int32), _dev(ctx, np.zeros(0), np.uint8), 0)
    assert e_lv.shape[0] == 0 and e_ix.shape[0] == 0


def test_bisect_errors(G, ctx):
    grid = W.Grid((4, 3), (0.0, 0.0), (1.0, 1.0))
    lv0, idx = oracle.coarse_cells(grid)
    ones = _dev(ctx, np.ones(12), np.uint8)
    # a kept cell of level 1, a kept cell outside the grid, a bad dimension
    lv1 = lv0.copy()
    lv1[3] = 1
    with pytest.raises(G.GisError, match="GIS_E_INVAL"):
        G.bisect(ctx, grid, _dev(ctx, lv1, np.uint8), _dev(ctx, idx, np.int32), ones, 0)
    bad = idx.copy()
    bad[11] = (4, 0)
    with pytest.raises(G.GisError, match="GIS_E_INVAL"):
        G.bisect(ctx, grid, _dev(ctx, lv0, np.uint8), _dev(ctx, bad, np.int32), ones, 1)
    for dim in (-1, 2):
        with pytest.raises(G.GisError, match="GIS_E_INVAL"):
            G.bisect(ctx, grid, _dev(ctx, lv0, np.uint8), _dev(ctx, idx, np.int32), ones, dim)
    # the same cells that are not kept are ignored
    kept = np.ones(12, np.uint8)
    kept[3] = 0
    _, _, got_ix = G.bisect(ctx, grid, _dev(ctx, lv1, np.uint8), _dev(ctx, idx, np.int32),
                            _dev(ctx, kept, np.uint8), 0)
    np.testing.assert_array_equal(_np(got_ix), oracle.bisect(grid, idx, kept, 0)[2])
    # the context still works after the errors
    _, _, got_ix = G.bisect(ctx, grid, _dev(ctx, lv0, np.uint8), _dev(ctx, idx, np.int32), ones, 1)
    np.testing.assert_array_equal(_np(got_ix), oracle.bisect(grid, idx, np.ones(12, np.uint8), 1)[2])


def _standard(name, analysis, rounds, precision="fp64"):
    base = {
        "vdp": (W.vdp(), W.Grid((12, 10), *W.VDP_BOX), W.evenly_spaced(-1, 1, 5), W.LATTICE3),
        "vdp_fine": (W.vdp(), W.Grid((48, 40), *W.VDP_BOX), W.evenly_spaced(-1, 1, 5), W.LATTICE3),
        "lorenz": (W.lorenz(), W.Grid((6, 7, 5), (-20., -25., 0.), (20., 25., 50.)),
                   W.evenly_spaced(-10, 10, 4), W.CORNERS_CENTER),
        "vdp2": (W.vdp2(), W.Grid((4, 5, 4, 5), (-2.5, -3., -2.5, -3.), (2.5, 3., 2.5, 3.)),
                 W.input_grid(-1, 1, 3, 2), W.CORNERS_CENTER),
        "linear1": (W.linear([[0.7]], [[1.0]], 0.1, 3), W.Grid((9,), (-2.,), (2.,)),
                    W.evenly_spaced(-1, 1, 7), W.LATTICE3),
    }[name]
    system, grid, u, samples = base
    return W.Workload(f"{name}_standard_r{rounds}", system, grid, u, samples, rounds, precision,
                      analysis=analysis, subdivision="bisect")


# (the controlled analysis keeps nothing on coarse Van der Pol and Lorenz
# grids, so its Van der Pol case starts finer)
CASES = [("vdp", "nonleaving", 5), ("vdp", "controlled", 2), ("vdp_fine", "controlled", 3),
         ("lorenz", "nonleaving", 3), ("vdp2", "nonleaving", 2), ("linear1", "controlled", 6),
         ("linear1", "nonleaving", 6)]


def _check(G, ctx, wl, sol):
    want = oracle.solve(wl.system, wl.grid, wl.samples, wl.u, wl.rounds, analysis=wl.analysis,
                        subdivision="bisect")
    info = sol.info()
    lv, ix, kept, mask = (_np(t) for t in sol.export())
    assert info["n0"] == tuple(want["grid"].n0), wl.name
    np.testing.assert_array_equal(lv, want["level"])
    np.testing.assert_array_equal(ix, want["idx"])
    np.testing.assert_array_equal(kept, want["kept"])
    np.testing.assert_array_equal(mask.view(np.uint64), want["mask"])
    assert info["n_rounds"] == len(want["stats"])
    for got_r, want_r in zip(info["rounds"], want["stats"]):
        for k in ("n_cells", "n_rows", "n_edges", "n_out", "n_kept"):
            assert got_r[k] == want_r[k], (wl.name, k, got_r, want_r)
        assert got_r["max_level"] == 0
    for got_r, want_r in zip(info["rounds"][:-1], want["stats"][:-1]):
        assert got_r["n_boundary"] == want_r["n_boundary"], (wl.name, got_r, want_r)
    states = _dev(ctx, W.query_states(wl.grid, 3000, seed=5, margin=0.02), np.float64)
    m_w, a_w = oracle.query(want["grid"], want["level"], want["idx"], want["kept"], want["mask"],
                            _np(states))
    np.testing.assert_array_equal(_np(sol.query_membership(states)), m_w)
    np.testing.assert_array_equal(_np(sol.query_admissible(states)).view(np.uint64), a_w)
    return want


@pytest.mark.parametrize("name,analysis,rounds", CASES, ids=[f"{a}-{b}-r{c}" for a, b, c in CASES])
def test_solve_standard(G, ctx, name, analysis, rounds):
    wl = _standard(name, analysis, rounds)
    _check(G, ctx, wl, G.solve_workload(ctx, wl))


def test_solve_standard_fp32_recheck(G, ctx):
    wl = _standard("vdp", "nonleaving", 5, precision="fp32_recheck")
    _check(G, ctx, wl, G.solve_workload(ctx, wl))


def test_solve_batch_standard(G, ctx):
    """Jobs on different grids and parameters in shared launches: each equals
    its own solve and the oracle (their grids are halved independently)."""
    base = _standard("vdp", "nonleaving", 4)
    wls = [base,
           dataclasses.replace(base, name="vdp_mu15", system=W.vdp(mu=1.5),
                               grid=W.Grid((7, 9), *W.VDP_BOX)),
           dataclasses.replace(base, name="vdp_small_box", grid=W.Grid((10, 10), (-1., -1.), (1., 1.)))]
    sols = G.solve_batch(ctx, wls)
    for wl, sol in zip(wls, sols):
        _check(G, ctx, wl, sol)


def test_solve_standard_workload_full_size(G, ctx):
    """The benchmarked standard-loop workload itself (Van der Pol 32x32, six
    halvings to 256x256, 21 inputs, FP32 + FP64 recheck), whole solve."""
    wl = W.vdp_standard_32()
    _check(G, ctx, wl, G.solve_workload(ctx, wl))


def test_solve_standard_timed_frontier_schedule(G, ctx):
    """Solves timed with HIP events (the build's, and the phases') on a
    schedule that sends the non-leaving analysis of the larger rounds to the
    frontier phase (no witness sweeps, row sweeps only below 2 M edges): the
    host learns that a round has finished from the counters' sequence number,
    not from the runtime, so the library waits for the events before it reads
    their times.  Every call returns, with times, and equals the oracle."""
    wl = W.vdp_standard_32()
    prev = ctx.set_tuning(wit_sweeps=0, sweep_edges=2_000_000)
    try:
        first = None
        for _ in range(4):
            sol = G.solve_workload(ctx, wl, timing=2)
            rounds = sol.info()["rounds"]
            assert all(r["ms_image"] > 0 for r in rounds)
            got = [_np(t) for t in sol.export()]
            if first is None:
                _check(G, ctx, wl, sol)
                first = got
            else:
                for a, b in zip(got, first):
                    np.testing.assert_array_equal(a, b)
            sol.free()
    finally:
        ctx.set_tuning(**prev)


def test_bisect_cell_count_limit(G, ctx):
    """A halving that would put more than 2^30 cells along a dimension is
    refused before any work (GIS_E_UNSUPPORTED), and the context still works."""
    grid = W.Grid(((1 << 29) + 1, 2), (0.0, 0.0), (1.0, 1.0))
    idx = np.array([[5, 1]], np.int32)
    lv = _dev(ctx, np.zeros(1), np.uint8)
    kept = _dev(ctx, np.ones(1), np.uint8)
    with pytest.raises(G.GisError, match="GIS_E_UNSUPPORTED"):
        G.bisect(ctx, grid, lv, _dev(ctx, idx, np.int32), kept, 0)
    small = W.Grid((7, 2), (0.0, 0.0), (1.0, 1.0))
    g2, _, got = G.bisect(ctx, small, lv, _dev(ctx, idx, np.int32), kept, 1)
    assert tuple(g2.n0) == (7, 4)
    np.testing.assert_array_equal(_np(got), [[5, 2], [5, 3]])
