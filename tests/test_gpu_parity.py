"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar: integer, index and flag outputs (edges, OUT flags, kept cells, masks,
cell lists, query answers) bit-exact; FP64 sample images within 1e-10
relative (|a - b| <= 1e-10 max(|a|, |b|, hi_d - lo_d)) -- the canonical
operation order is expected to give 0 ulp, which is asserted separately.
The FP32-with-FP64-recheck path must give the very same graph as FP64.
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


def _cells(ctx, level, idx):
    return (torch.as_tensor(np.ascontiguousarray(level, np.uint8), device=ctx.dev),
            torch.as_tensor(np.ascontiguousarray(idx, np.int32), device=ctx.dev))


def _adaptive_cells(rng, n0, splits, drop_frac=0.1):
    import itertools
    n = len(n0)
    cells = {(0,) + c for c in itertools.product(*[range(k) for k in n0])}
    for _ in range(splits):
        c = sorted(cells)[rng.integers(0, len(cells))]
        cells.remove(c)
        for ch in itertools.product((0, 1), repeat=n):
            cells.add((c[0] + 1,) + tuple(2 * c[1 + d] + ch[d] for d in range(n)))
    cells = sorted(cells)
    keep = rng.random(len(cells)) >= drop_frac
    cells = [c for c, k in zip(cells, keep) if k]
    return (np.array([c[0] for c in cells], np.uint8),
            np.array([c[1:] for c in cells], np.int32).reshape(len(cells), n))


SMALL = {
    "vdp": (W.vdp(), W.Grid((24, 20), *W.VDP_BOX), W.evenly_spaced(-1, 1, 5), W.LATTICE3),
    "lorenz": (W.lorenz(), W.Grid((10, 12, 9), (-20., -25., 0.), (20., 25., 50.)),
               W.evenly_spaced(-10, 10, 4), W.CORNERS_CENTER),
    "vdp2": (W.vdp2(), W.Grid((5, 6, 5, 6), (-2.5, -3., -2.5, -3.), (2.5, 3., 2.5, 3.)),
             W.input_grid(-1, 1, 3, 2), W.CORNERS_CENTER),
    "linear1": (W.linear([[0.7]], [[1.0]], 0.1, 3), W.Grid((37,), (-2.,), (2.,)),
                W.evenly_spaced(-1, 1, 7), W.LATTICE3),
    "linear3": (W.random_linear(5, 3, 2), W.Grid((7, 6, 5), (-1.,) * 3, (1.,) * 3),
                W.input_grid(-1, 1, 2, 2), W.LATTICE3),
    "cstr": (W.cstr(), W.Grid((24, 20), *W.CSTR_BOX), W.evenly_spaced(285, 315, 7), W.LATTICE3),
}


# ------------------------------------------------------------------ images
@pytest.mark.parametrize("name", list(SMALL))
def test_images_fp64_bitexact(G, ctx, name):
    system, grid, u, samples = SMALL[name]
    level, idx = oracle.coarse_cells(grid)
    want = oracle.images(system, grid, samples, level, idx, u)
    dl, di = _cells(ctx, level, idx)
    got = _np(G.images(ctx, system, grid, u, dl, di, samples, "fp64"))
    scale = np.maximum(np.maximum(np.abs(got), np.abs(want)),
                       (np.array(grid.hi) - np.array(grid.lo))[None, None, :])
    assert (np.abs(got - want) <= 1e-10 * scale).all()
    assert np.array_equal(got.view(np.int64), want.view(np.int64)), "expected 0-ulp agreement"


# ------------------------------------------------------------------ build
def _check_graph(G, ctx, system, grid, u, samples, level, idx, precision="fp64", band=None,
                 fast_out=False):
    want = oracle.build_graph(system, grid, samples, level, idx, u, fast_out=fast_out)
    dl, di = _cells(ctx, level, idx)
    opts = G.opts_t(samples=samples, precision=precision, band=band, fast_out=fast_out)
    g = G.build_graph(ctx, system, grid, u, dl, di, opts)
    np.testing.assert_array_equal(_np(g.row_ptr), want["row_ptr"])
    np.testing.assert_array_equal(_np(g.col), want["col"])
    np.testing.assert_array_equal(_np(g.out), want["out"])
    assert g.n_edges == want["col"].shape[0] and g.n_out == int(want["out"].sum())
    return g, want


@pytest.mark.parametrize("name", list(SMALL))
def test_build_uniform_matches_oracle(G, ctx, name):
    system, grid, u, samples = SMALL[name]
    level, idx = oracle.coarse_cells(grid)
    _check_graph(G, ctx, system, grid, u, samples, level, idx)


@pytest.mark.parametrize("name", ["vdp", "lorenz", "vdp2", "linear1", "cstr"])
@pytest.mark.parametrize("seed", [0, 1])
def test_build_adaptive_matches_oracle(G, ctx, name, seed):
    """Mixed-level coverings with holes: edges to coarse and fine cells, holes -> OUT."""
    system, grid, u, samples = SMALL[name]
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    level, idx = _adaptive_cells(rng, grid.n0, splits=12 if grid.n < 4 else 6)
    g, want = _check_graph(G, ctx, system, grid, u, samples, level, idx)
    assert want["out"].sum() > 0


def test_build_fast_out(G, ctx):
    system, grid, u, samples = SMALL["vdp"]
    level, idx = oracle.coarse_cells(grid)
    _check_graph(G, ctx, system, grid, u, samples, level, idx, fast_out=True)


@pytest.mark.parametrize("name", ["vdp", "lorenz", "vdp2", "cstr"])
def test_build_fp32_recheck_equals_fp64(G, ctx, name):
    system, grid, u, samples = SMALL[name]
    rng = np.random.Generator(np.random.PCG64(7))
    level, idx = _adaptive_cells(rng, grid.n0, splits=8 if grid.n < 4 else 4)
    dl, di = _cells(ctx, level, idx)
    band = G.calibrate_band(ctx, system, grid, u, dl, di, samples, safety=8.0, floor_rel=1e-7)
    assert (band > 0).all()
    g, _ = _check_graph(G, ctx, system, grid, u, samples, level, idx, precision="fp32_recheck",
                        band=band)
    assert 0 <= g.n_recheck < g.n_rows


# ------------------------------------------------------------------ prune
@pytest.mark.parametrize("analysis", ["controlled", "nonleaving"])
@pytest.mark.parametrize("name", ["vdp", "lorenz", "vdp2", "linear1", "cstr"])
def test_prune_matches_oracle(G, ctx, name, analysis):
    system, grid, u, samples = SMALL[name]
    rng = np.random.Generator(np.random.PCG64(3))
    level, idx = _adaptive_cells(rng, grid.n0, splits=6, drop_frac=0.05)
    g, want = _check_graph(G, ctx, system, grid, u, samples, level, idx)
    kept_w, mask_w, _ = oracle.prune(want["row_ptr"], want["col"], want["out"], level.shape[0],
                                     u.shape[0], analysis)
    kept, mask, nk = G.prune(ctx, g, level.shape[0], u.shape[0], analysis)
    np.testing.assert_array_equal(_np(kept), kept_w)
    np.testing.assert_array_equal(_np(mask).view(np.uint64), mask_w)
    assert nk == int(kept_w.sum())


def test_prune_deep_peel(G, ctx):
    """Pure drift: every cell is removed, one layer at a time (deep frontier)."""
    grid = W.Grid((3000,), (-1.0,), (1.0,))
    system = W.linear([[0.0]], [[1.0]], dt=0.0005, nsub=1)
    u = np.array([[1.0]])
    level, idx = oracle.coarse_cells(grid)
    g, want = _check_graph(G, ctx, system, grid, u, W.LATTICE3, level, idx)
    kept, mask, nk = G.prune(ctx, g, level.shape[0], 1, "controlled")
    assert nk == 0 and _np(kept).sum() == 0


# Schedule parameters never change results: the frontier phase from the
# start (sweep_edges = 0 and no witness sweeps), the row sweeps instead of
# the witness sweeps for the non-leaving analysis, the frontier phase taking
# over from a few witness sweeps, one sweep or step per convergence check,
# and one-block grids all give the oracle's fixed point.
TUNINGS = {
    "frontier_only": dict(sweep_edges=0, wit_sweeps=0),
    "row_frontier_only": dict(sweep_edges=0, row_frontier=1, wit_sweeps=0),
    "row_sweeps": dict(wit_sweeps=0),
    "witness_then_frontier": dict(wit_sweeps=2, first_sweeps=1, sweep_batch=1),
    "one_sweep_per_check": dict(first_sweeps=1, sweep_batch=1),
    "tiny_grids": dict(sweep_edges=0, front_blocks=1, frontier_batch=1, wit_sweeps=0),
    "tiny_sweep_grid": dict(sweep_blocks=1, first_sweeps=3, sweep_batch=2),
}


@pytest.mark.parametrize("tuning", sorted(TUNINGS))
@pytest.mark.parametrize("analysis", ["controlled", "nonleaving"])
@pytest.mark.parametrize("name", ["vdp", "lorenz", "vdp2"])
def test_prune_tunings_match_oracle(G, ctx, name, analysis, tuning):
    system, grid, u, samples = SMALL[name]
    rng = np.random.Generator(np.random.PCG64(4))
    level, idx = _adaptive_cells(rng, grid.n0, splits=6, drop_frac=0.05)
    g, want = _check_graph(G, ctx, system, grid, u, samples, level, idx)
    kept_w, mask_w, _ = oracle.prune(want["row_ptr"], want["col"], want["out"], level.shape[0],
                                     u.shape[0], analysis)
    prev = ctx.set_tuning(**TUNINGS[tuning])
    try:
        kept, mask, nk = G.prune(ctx, g, level.shape[0], u.shape[0], analysis)
    finally:
        ctx.set_tuning(**prev)
    np.testing.assert_array_equal(_np(kept), kept_w)
    np.testing.assert_array_equal(_np(mask).view(np.uint64), mask_w)
    assert nk == int(kept_w.sum())


@pytest.mark.parametrize("analysis", ["controlled", "nonleaving"])
def test_prune_frontier_dense_rows(G, ctx, analysis):
    """A coarse 4-D covering whose rows have tens of targets: a 256-row block
    of the reverse-CSR scatter holds more edges than its LDS stage, so the
    scatter takes its direct path; the frontier result equals the oracle."""
    system = W.vdp2()
    grid = W.Grid((5, 5, 5, 5), (-2.5, -3, -2.5, -3), (2.5, 3, 2.5, 3))
    u = W.input_grid(-1, 1, 3, 2)
    level, idx = oracle.coarse_cells(grid)
    g, want = _check_graph(G, ctx, system, grid, u, W.CORNERS_CENTER, level, idx)
    rp = want["row_ptr"]
    assert max(rp[min(b + 256, len(rp) - 1)] - rp[b] for b in range(0, len(rp) - 1, 256)) > 6144
    kept_w, mask_w, _ = oracle.prune(want["row_ptr"], want["col"], want["out"], level.shape[0],
                                     u.shape[0], analysis)
    prev = ctx.set_tuning(sweep_edges=0, wit_sweeps=0)
    try:
        kept, mask, nk = G.prune(ctx, g, level.shape[0], u.shape[0], analysis)
    finally:
        ctx.set_tuning(**prev)
    np.testing.assert_array_equal(_np(kept), kept_w)
    np.testing.assert_array_equal(_np(mask).view(np.uint64), mask_w)


@pytest.mark.parametrize("analysis", ["controlled", "nonleaving"])
def test_prune_wide_inputs_random_graph(G, ctx, analysis):
    """K = 300 inputs (beyond a sweep block): the frontier phase with a thread
    per cell, on a seeded random graph (0-3 targets per row, 3% OUT rows)."""
    rng = np.random.Generator(np.random.PCG64(21))
    n_cells, K = 60, 300
    n_rows = n_cells * K
    cnt = rng.integers(0, 4, size=n_rows)
    row_ptr = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    col = np.concatenate([np.sort(rng.choice(n_cells, size=c, replace=False)) for c in cnt]
                         ).astype(np.int32)
    out = (rng.random(n_rows) < 0.03).astype(np.uint8)
    kept_w, mask_w, _ = oracle.prune(row_ptr, col, out, n_cells, K, analysis)
    dev = ctx.dev
    g = G.Graph(torch.as_tensor(row_ptr, device=dev), torch.as_tensor(col, device=dev),
                torch.as_tensor(out, device=dev), n_rows, int(col.shape[0]), int(out.sum()), 0)
    kept, mask, nk = G.prune(ctx, g, n_cells, K, analysis)
    np.testing.assert_array_equal(_np(kept), kept_w)
    np.testing.assert_array_equal(_np(mask).view(np.uint64), mask_w)
    assert nk == int(kept_w.sum())


def _cascade_graph(K, max_targets, seed):
    """A seeded random graph with long removal chains: row (c, u) targets a
    window of cells ahead of c (every id of the window twice, so rows repeat
    targets), the last 200 cells have OUT rows without targets, every 97th
    cell keeps one row pointing at itself, and 5% of the other rows are OUT."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_cells = 3000
    n_rows = n_cells * K
    cell = np.arange(n_rows) // K
    u = np.arange(n_rows) % K
    cnt = rng.integers(1, max_targets + 1, size=n_rows)
    sink = cell >= n_cells - 200
    loop = (cell % 97 == 0) & (u == 0)
    cnt[sink] = 0
    cnt[loop] = 1
    row_ptr = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    start = np.where(loop, cell, cell + 1 + (u % 3))
    k = np.arange(row_ptr[-1]) - np.repeat(row_ptr[:-1], cnt)
    col = np.clip(np.repeat(start, cnt) + k // 2 * 2, 0, n_cells - 1).astype(np.int32)
    out = ((rng.random(n_rows) < 0.05) | sink).astype(np.uint8)
    out[loop] = 0
    return row_ptr, col, out, n_cells


@pytest.mark.parametrize("K,max_targets,shuffled", [(1, 40, False), (2, 60, False),
                                                    (5, 6, False), (33, 4, False),
                                                    (64, 3, False), (5, 6, True)])
@pytest.mark.parametrize("analysis", ["controlled", "nonleaving"])
@pytest.mark.parametrize("row_frontier", [0, 1])
def test_prune_frontier_cascade_graph(G, ctx, analysis, K, max_targets, shuffled, row_frontier):
    """The frontier phase alone (up to a few hundred steps), with one reverse
    entry per (source cell, target) or per (row, target).
    K = 1 and K = 2 give blocks with more distinct (cell, target) pairs than
    the block's LDS table holds (its per-edge fallback); K = 64 fills a whole
    input mask; rows may repeat targets and (shuffled) list them in any
    order."""
    row_ptr, col, out, n_cells = _cascade_graph(K, max_targets, 100 + K)
    if shuffled:
        rng = np.random.Generator(np.random.PCG64(7))
        for r in range(n_cells * K):
            rng.shuffle(col[row_ptr[r]:row_ptr[r + 1]])
    n_rows = n_cells * K
    kept_w, mask_w, iters = oracle.prune(row_ptr, col, out, n_cells, K, analysis)
    assert 0 < kept_w.sum() < n_cells
    dev = ctx.dev
    g = G.Graph(torch.as_tensor(row_ptr, device=dev), torch.as_tensor(col, device=dev),
                torch.as_tensor(out, device=dev), n_rows, int(col.shape[0]), int(out.sum()), 0)
    prev = ctx.set_tuning(sweep_edges=0, row_frontier=row_frontier, wit_sweeps=0)
    try:
        kept, mask, nk = G.prune(ctx, g, n_cells, K, analysis)
    finally:
        ctx.set_tuning(**prev)
    np.testing.assert_array_equal(_np(kept), kept_w)
    np.testing.assert_array_equal(_np(mask).view(np.uint64), mask_w)
    assert nk == int(kept_w.sum())


@pytest.mark.parametrize("K,max_targets,shuffled", [(1, 40, False), (2, 60, False),
                                                    (5, 6, False), (49, 9, False),
                                                    (64, 3, False), (5, 6, True)])
@pytest.mark.parametrize("one_per_check", [False, True])
def test_prune_witness_cascade_graph(G, ctx, K, max_targets, shuffled, one_per_check):
    """The non-leaving analysis by witness sweeps alone, to its fixed point
    over removal chains of a few hundred steps: spans of up to K * 40 edges
    searched 64 at a time, repeated and (shuffled) unordered targets, one
    sweep per convergence check or the default batches."""
    row_ptr, col, out, n_cells = _cascade_graph(K, max_targets, 300 + K)
    if shuffled:
        rng = np.random.Generator(np.random.PCG64(8))
        for r in range(n_cells * K):
            rng.shuffle(col[row_ptr[r]:row_ptr[r + 1]])
    n_rows = n_cells * K
    kept_w, mask_w, iters = oracle.prune(row_ptr, col, out, n_cells, K, "nonleaving")
    assert 0 < kept_w.sum() < n_cells
    dev = ctx.dev
    g = G.Graph(torch.as_tensor(row_ptr, device=dev), torch.as_tensor(col, device=dev),
                torch.as_tensor(out, device=dev), n_rows, int(col.shape[0]), int(out.sum()), 0)
    tun = dict(wit_sweeps=4096)
    if one_per_check:
        tun.update(first_sweeps=1, sweep_batch=1)
    prev = ctx.set_tuning(**tun)
    try:
        kept, mask, nk = G.prune(ctx, g, n_cells, K, "nonleaving")
    finally:
        ctx.set_tuning(**prev)
    np.testing.assert_array_equal(_np(kept), kept_w)
    np.testing.assert_array_equal(_np(mask).view(np.uint64), mask_w)
    assert nk == int(kept_w.sum())


def _zigzag_chains(L):
    """Two chains of L cells each (K = 2): row (c, 0) of every chain cell
    targets the cell before it, row (c, 1) is OUT without targets; chain A
    starts at a dead cell, chain B at a cell whose row 0 targets itself.
    Consecutive chain cells sit at opposite ends of the numbering, so an
    in-place sweep moves a removal by only a link or two and the sweeps give
    up (after 256 of them) long before chain A has died."""
    n_cells, K = 2 * L, 2
    lo, hi, order = 0, n_cells - 1, []
    for k in range(n_cells):
        if k % 2 == 0:
            order.append(lo)
            lo += 1
        else:
            order.append(hi)
            hi -= 1
    order = np.array(order)
    tgt = [[] for _ in range(n_cells * K)]
    out = np.zeros(n_cells * K, np.uint8)
    for chain, pos in (("A", order[0::2]), ("B", order[1::2])):
        for k in range(L):
            c = int(pos[k])
            out[c * K + 1] = 1
            if k > 0:
                tgt[c * K].append(int(pos[k - 1]))
            elif chain == "A":
                out[c * K] = 1
            else:
                tgt[c * K].append(c)
    cnt = np.array([len(t) for t in tgt])
    row_ptr = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    col = np.array([j for t in tgt for j in t], np.int32)
    return row_ptr, col, out, n_cells, K


@pytest.mark.parametrize("analysis,wit_sweeps", [("controlled", 256), ("nonleaving", 256),
                                                 ("nonleaving", 0)])
@pytest.mark.parametrize("row_frontier", [0, 1])
def test_prune_sweeps_then_frontier(G, ctx, analysis, wit_sweeps, row_frontier):
    """The frontier phase taking over from sweeps (row sweeps, or witness
    sweeps for the non-leaving analysis) that have removed cells already: its
    initial state must account for removed targets."""
    row_ptr, col, out, n_cells, K = _zigzag_chains(1500)
    kept_w, mask_w, iters = oracle.prune(row_ptr, col, out, n_cells, K, analysis)
    assert iters == 1500 and kept_w.sum() == 1500
    dev = ctx.dev
    g = G.Graph(torch.as_tensor(row_ptr, device=dev), torch.as_tensor(col, device=dev),
                torch.as_tensor(out, device=dev), n_cells * K, int(col.shape[0]), int(out.sum()),
                0)
    prev = ctx.set_tuning(row_frontier=row_frontier, wit_sweeps=wit_sweeps)
    try:
        kept, mask, nk = G.prune(ctx, g, n_cells, K, analysis)
    finally:
        ctx.set_tuning(**prev)
    np.testing.assert_array_equal(_np(kept), kept_w)
    np.testing.assert_array_equal(_np(mask).view(np.uint64), mask_w)
    assert nk == 1500


@pytest.mark.parametrize("tuning", ["frontier_only", "row_frontier_only", "one_sweep_per_check",
                                    "tiny_grids", "row_sweeps", "witness_then_frontier"])
def test_solve_adaptive_tunings(G, ctx, tuning):
    prev = ctx.set_tuning(**TUNINGS[tuning])
    try:
        _check_solve(G, ctx, W.vdp_adaptive_32("fp64"), "fp64")
    finally:
        ctx.set_tuning(**prev)


def test_graph_replays_match_eager_and_oracle(G):
    """With use_graphs the analysis launch sequence of a round is captured on
    its second sighting and replayed afterwards: solves of two workloads,
    interleaved on a non-default stream with eager work and synchronisations
    between them, all equal the oracle (replays 2, 3 and 4 of each round)."""
    c = G.Context(0)
    st = torch.cuda.Stream()
    try:
        c.set_tuning(use_graphs=1)
        wls = [W.vdp_adaptive_32("fp64"), W.vdp_uniform_64()]
        wants = [_oracle_solve(w) for w in wls]
        for it in range(4):
            for wl, want in zip(wls, wants):
                with torch.cuda.stream(st):
                    sol = G.solve_workload(c, wl, precision="fp64")
                    lv, ix, kept, mask = sol.export()
                    torch.cuda.synchronize()
                    junk = torch.ones(1 << 20, device=c.dev).sum().item()  # eager work between replays
                assert junk == float(1 << 20)
                np.testing.assert_array_equal(_np(lv), want["level"], err_msg=f"iteration {it}")
                np.testing.assert_array_equal(_np(ix), want["idx"])
                np.testing.assert_array_equal(_np(kept), want["kept"])
                np.testing.assert_array_equal(_np(mask).view(np.uint64), want["mask"])
                sol.free()
    finally:
        c.close()


def test_autotune_keeps_results(G):
    """The autotuner only picks schedule parameters: after it, the solve still
    equals the oracle, and the context holds the parameters it returned."""
    c = G.Context(0)
    try:
        wl = W.vdp_adaptive_32("fp64")
        best, ms = G.autotune(c, wl, repeats=1, precision="fp64")
        assert ms > 0
        assert c.get_tuning() == best
        _check_solve(G, c, wl, "fp64")
        with pytest.raises(G.GisError):
            G.autotune(c, wl, repeats=0, precision="fp64")
    finally:
        c.close()


def test_tuning_rejects_out_of_range(G, ctx):
    before = ctx.get_tuning()
    for bad in (dict(first_sweeps=0), dict(sweep_batch=300), dict(sweep_edges=-1),
                dict(front_blocks=0), dict(sweep_blocks=70000), dict(frontier_batch=0),
                dict(edge_hint=-1), dict(edge_hint=5000), dict(row_frontier=2),
                dict(row_frontier=-1), dict(wit_sweeps=-1), dict(wit_sweeps=5000)):
        with pytest.raises(G.GisError):
            ctx.set_tuning(**bad)
        assert ctx.get_tuning() == before


# ------------------------------------------------------------------ subdivide
@pytest.mark.parametrize("rule", ["shell", "corners"])
@pytest.mark.parametrize("name", ["vdp", "lorenz", "linear3"])
def test_subdivide_matches_oracle(G, ctx, name, rule):
    system, grid, u, samples = SMALL[name]
    rng = np.random.Generator(np.random.PCG64(11))
    level, idx = _adaptive_cells(rng, grid.n0, splits=5, drop_frac=0.0)
    kept = (rng.random(level.shape[0]) < 0.8).astype(np.uint8)
    bnd_w = oracle.boundary(grid, level, idx, kept, rule)
    lv_w, ix_w = oracle.subdivide(grid, level, idx, kept, bnd_w)
    dl, di = _cells(ctx, level, idx)
    lv, ix, bnd = G.subdivide(ctx, grid, dl, di, torch.as_tensor(kept, device=ctx.dev), rule)
    np.testing.assert_array_equal(_np(bnd), bnd_w)
    np.testing.assert_array_equal(_np(lv), lv_w)
    np.testing.assert_array_equal(_np(ix), ix_w)


def test_worked_example_5x5_on_gpu(G, ctx):
    grid = W.Grid((5, 5), (0.0, 0.0), (5.0, 5.0))
    level, idx = oracle.coarse_cells(grid)
    for removed, rule, want in [((25,), "corners", [1, 2, 3, 4, 5, 6, 10, 11, 15, 16, 19, 20, 21, 22, 23, 24]),
                                ((4, 25), "corners", [1, 2, 3, 5, 6, 8, 10, 11, 15, 16, 19, 20, 21, 22, 23, 24]),
                                ((4, 25), "shell", [1, 2, 3, 5, 6, 8, 9, 10, 11, 15, 16, 19, 20, 21, 22, 23, 24])]:
        kept = np.ones(25, np.uint8)
        kept[[b - 1 for b in removed]] = 0
        dl, di = _cells(ctx, level, idx)
        _, _, bnd = G.subdivide(ctx, grid, dl, di, torch.as_tensor(kept, device=ctx.dev), rule)
        assert sorted((np.nonzero(_np(bnd))[0] + 1).tolist()) == want


@pytest.mark.parametrize("nn", [1, 3, 7, 20, 64])
@pytest.mark.parametrize("name", ["vdp", "lorenz", "vdp2", "linear1"])
def test_subdivide_neighbours_matches_oracle(G, ctx, name, nn):
    """The neighbourhood selection (Sec. 3.1.2) on random mixed-level
    coverings with removed cells: the cells split (boundary cells and the nn
    kept cells nearest to each) and the new covering equal the oracle's."""
    system, grid, u, samples = SMALL[name]
    rng = np.random.Generator(np.random.PCG64(17 + nn))
    level, idx = _adaptive_cells(rng, grid.n0, splits=5, drop_frac=0.0)
    kept = (rng.random(level.shape[0]) < 0.97).astype(np.uint8)
    bnd_w = oracle.boundary(grid, level, idx, kept, "shell")
    sel_w = oracle.neighbours(grid, level, idx, kept, bnd_w, nn)
    assert sel_w.sum() > bnd_w.sum() or sel_w.sum() == kept.sum()
    lv_w, ix_w = oracle.subdivide(grid, level, idx, kept, sel_w)
    dl, di = _cells(ctx, level, idx)
    lv, ix, bnd = G.subdivide(ctx, grid, dl, di, torch.as_tensor(kept, device=ctx.dev), "shell",
                              neighbours=nn)
    np.testing.assert_array_equal(_np(bnd), bnd_w)
    np.testing.assert_array_equal(_np(lv), lv_w)
    np.testing.assert_array_equal(_np(ix), ix_w)


def test_neighbours_worked_example_on_gpu(G, ctx):
    """Figure 5 of Sec. 3.1.2 on the device: on the 5x5 grid of square cells
    (B25 removed), the nearest 3 (7) kept cells of the corner cell B1 -- which
    the boundary selection marks -- are among the cells split."""
    grid = W.Grid((5, 5), (0.0, 0.0), (5.0, 5.0))
    level, idx = oracle.coarse_cells(grid)
    kept = np.ones(25, np.uint8)
    kept[24] = 0
    dl, di = _cells(ctx, level, idx)
    for nn, near in ((3, [2, 6, 7]), (7, [2, 3, 6, 7, 8, 11, 12])):
        bnd_w = oracle.boundary(grid, level, idx, kept, "shell")
        sel_w = oracle.neighbours(grid, level, idx, kept, bnd_w, nn)
        lv_w, ix_w = oracle.subdivide(grid, level, idx, kept, sel_w)
        lv, ix, bnd = G.subdivide(ctx, grid, dl, di, torch.as_tensor(kept, device=ctx.dev),
                                  "shell", neighbours=nn)
        np.testing.assert_array_equal(_np(lv), lv_w)
        np.testing.assert_array_equal(_np(ix), ix_w)
        split = {int(k) for k in np.nonzero(sel_w)[0] + 1}
        assert set(near) <= split


@pytest.mark.parametrize("nn", [3, 7])
def test_solve_adaptive_with_neighbourhood(G, ctx, nn):
    """The adaptive Van der Pol workload (32x32, 5 rounds) with the
    neighbourhood of Sec. 3.1.2: every round equals the oracle, and the
    selection counts per round are the oracle's."""
    wl = dataclasses.replace(W.vdp_adaptive_32("fp64"), nn=nn)
    sol, want, info = _check_solve(G, ctx, wl, "fp64")
    for got_r, want_r in zip(info["rounds"], want["stats"]):
        if "n_selected" in want_r:
            assert got_r["n_boundary"] == want_r["n_boundary"]
            assert got_r["n_selected"] == want_r["n_selected"]
    sol.free()


def test_neighbours_rejected_with_bisection(G, ctx):
    wl = dataclasses.replace(W.vdp_standard_32("fp64"), nn=3)
    with pytest.raises(G.GisError):
        G.solve_workload(ctx, wl)
    with pytest.raises(G.GisError):
        G.solve_workload(ctx, dataclasses.replace(W.vdp_adaptive_32("fp64"), nn=65))


# ------------------------------------------------------------------ solve + queries
def _oracle_solve(wl, **kw):
    return oracle.solve(wl.system, wl.grid, wl.samples, wl.u, wl.rounds, rule=wl.boundary_rule,
                        analysis=wl.analysis, nn=wl.nn, **kw)


def _check_solve(G, ctx, wl, precision=None):
    want = _oracle_solve(wl)
    over = {} if precision is None else {"precision": precision}
    sol = G.solve_workload(ctx, wl, **over)
    info = sol.info()
    lv, ix, kept, mask = sol.export()
    np.testing.assert_array_equal(_np(lv), want["level"])
    np.testing.assert_array_equal(_np(ix), want["idx"])
    np.testing.assert_array_equal(_np(kept), want["kept"])
    np.testing.assert_array_equal(_np(mask).view(np.uint64), want["mask"])
    assert info["n_rounds"] == len(want["stats"])
    for got_r, want_r in zip(info["rounds"], want["stats"]):
        for k in ("n_cells", "n_rows", "n_edges", "n_out", "n_kept"):
            assert got_r[k] == want_r[k], (k, got_r, want_r)
    return sol, want, info


def test_solve_vdp_uniform_64(G, ctx):
    _check_solve(G, ctx, W.vdp_uniform_64())


@pytest.mark.parametrize("analysis", ["controlled", "nonleaving"])
@pytest.mark.parametrize("name", ["vdp", "lorenz", "vdp2", "linear1", "linear3", "cstr"])
def test_solve_uniform_frontier_from_boxes(G, ctx, name, analysis):
    """One-round solves of full coarse grids straight into the frontier phase
    (the cell-grouped reverse graph built from a solve's job table), 1 to 4
    dimensions, up to 9 inputs."""
    system, grid, u, samples = SMALL[name]
    wl = W.Workload(f"uniform_{name}", system, grid, u, samples, 0, "fp64", analysis=analysis)
    prev = ctx.set_tuning(sweep_edges=0)
    try:
        _check_solve(G, ctx, wl)
    finally:
        ctx.set_tuning(**prev)


@pytest.mark.parametrize("precision", ["fp64", "fp32_recheck"])
def test_solve_vdp_adaptive_32_r5(G, ctx, precision):
    sol, want, info = _check_solve(G, ctx, W.vdp_adaptive_32(precision), precision)
    assert info["n_rounds"] == 6
    if precision == "fp32_recheck":
        assert all(b > 0 for b in info["band"])


def test_solve_controlled_adaptive_small(G, ctx):
    wl = W.Workload("vdp_48_r3_controlled", W.vdp(), W.Grid((48, 48), *W.VDP_BOX),
                    W.evenly_spaced(-1, 1, 9), W.LATTICE3, 3, "fp64", analysis="controlled")
    _check_solve(G, ctx, wl)


def test_solve_corners_rule(G, ctx):
    wl = W.Workload("vdp_32_r3_corners", W.vdp(), W.Grid((32, 32), *W.VDP_BOX),
                    W.evenly_spaced(-1, 1, 7), W.LATTICE3, 3, "fp64", boundary_rule=W.CORNERS,
                    analysis="nonleaving")
    _check_solve(G, ctx, wl)


def test_solve_vdp2_small_rounds(G, ctx):
    wl = W.Workload("vdp2_8_r2", W.vdp2(), W.Grid((8, 8, 8, 8), (-2.5, -3, -2.5, -3), (2.5, 3, 2.5, 3)),
                    W.input_grid(-1, 1, 3, 2), W.CORNERS_CENTER, 2, "fp32_recheck",
                    analysis="nonleaving")
    _check_solve(G, ctx, wl)


@pytest.mark.parametrize("analysis", ["nonleaving", "controlled"])
def test_solve_edge_buffer_regrowth(G, analysis):
    """A fresh context sizes its edge buffer from an estimate (here set to 8
    edges per row) that a coarse 4-D covering exceeds: the round is
    re-emitted, re-analysed and re-subdivided after the buffer grows, and the
    result is unchanged."""
    c = G.Context(0)
    try:
        c.set_tuning(edge_hint=8)
        wl = W.Workload("vdp2_5_r1", W.vdp2(),
                        W.Grid((5, 5, 5, 5), (-2.5, -3, -2.5, -3), (2.5, 3, 2.5, 3)),
                        W.input_grid(-1, 1, 3, 2), W.CORNERS_CENTER, 1, "fp64", analysis=analysis)
        sol, want, info = _check_solve(G, c, wl)
        assert want["stats"][0]["n_edges"] > 10 * want["stats"][0]["n_rows"]
        sol.free()
    finally:
        c.close()


def test_solve_lorenz_small(G, ctx):
    wl = W.Workload("lorenz_24", W.lorenz(), W.Grid((24, 24, 24), (-20., -25., 0.), (20., 25., 50.)),
                    W.evenly_spaced(-10, 10, 5), W.CORNERS_CENTER, 1, "fp32_recheck")
    _check_solve(G, ctx, wl)


@pytest.mark.parametrize("wl", [W.vdp_uniform_64(), W.vdp_adaptive_32("fp64")],
                         ids=["uniform", "adaptive"])
def test_queries_match_oracle(G, ctx, wl):
    want = _oracle_solve(wl)
    sol = G.solve_workload(ctx, wl)
    states = W.query_states(wl.grid, 20000, seed=5, margin=0.05)
    # exact faces and the upper border too
    states[:50] = np.array(wl.grid.hi)[None, :]
    states[50:100, 0] = wl.grid.lo[0]
    m_w, a_w = oracle.query(wl.grid, want["level"], want["idx"], want["kept"], want["mask"], states)
    ds = torch.as_tensor(states, device=ctx.dev)
    np.testing.assert_array_equal(_np(sol.query_membership(ds)), m_w)
    np.testing.assert_array_equal(_np(sol.query_admissible(ds)).view(np.uint64), a_w)


def test_determinism(G, ctx):
    wl = W.vdp_adaptive_32("fp32_recheck")
    a = [_np(t) for t in G.solve_workload(ctx, wl).export()]
    b = [_np(t) for t in G.solve_workload(ctx, wl).export()]
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# ------------------------------------------------------------------ ABI errors
def test_abi_error_paths(G, ctx):
    import ctypes
    L = G.lib()
    system, grid, u, samples = SMALL["vdp"]
    level, idx = oracle.coarse_cells(grid)
    dl, di = _cells(ctx, level, idx)
    du = G.to_device_u(ctx, u)
    st, gt, ct = G.system_t(system), G.grid_t(grid), G.cells_t(dl, di)
    n_rows = level.shape[0] * u.shape[0]
    row_ptr = torch.empty(n_rows + 1, dtype=torch.int64, device=ctx.dev)
    out = torch.empty(n_rows, dtype=torch.uint8, device=ctx.dev)
    col = torch.empty(8, dtype=torch.int32, device=ctx.dev)
    g = G.GraphT()
    g.cap_edges, g.row_ptr, g.col, g.out = 8, G._ptr(row_ptr), G._ptr(col), G._ptr(out)
    opts = G.opts_t(samples=samples)
    s = G._stream_ptr()
    # capacity too small -> GIS_E_CAPACITY with the needed count
    rc = L.gis_build_graph(ctx.handle, ctypes.byref(st), ctypes.byref(gt), G._ptr(du), u.shape[0],
                           ctypes.byref(ct), ctypes.byref(opts), ctypes.byref(g), s)
    assert rc == 4 and g.n_edges > 8
    want = oracle.build_graph(system, grid, samples, level, idx, u)
    assert g.n_edges == want["col"].shape[0]
    np.testing.assert_array_equal(_np(row_ptr), want["row_ptr"])
    # invalid system / grid / opts
    bad = G.system_t(system)
    bad.n = 3
    assert L.gis_build_graph(ctx.handle, ctypes.byref(bad), ctypes.byref(gt), G._ptr(du), u.shape[0],
                             ctypes.byref(ct), ctypes.byref(opts), ctypes.byref(g), s) == 1
    badg = G.grid_t(grid)
    badg.lo[0] = badg.hi[0]
    assert L.gis_build_graph(ctx.handle, ctypes.byref(st), ctypes.byref(badg), G._ptr(du), u.shape[0],
                             ctypes.byref(ct), ctypes.byref(opts), ctypes.byref(g), s) == 1
    fp32 = G.opts_t(samples=samples, precision="fp32_recheck")   # no band -> invalid
    assert L.gis_build_graph(ctx.handle, ctypes.byref(st), ctypes.byref(gt), G._ptr(du), u.shape[0],
                             ctypes.byref(ct), ctypes.byref(fp32), ctypes.byref(g), s) == 1
    assert b"band" in L.gis_last_error()
    # non-canonical / out-of-range / overlapping cell lists
    for lv_bad, ix_bad in [(level, idx[::-1].copy()),
                           (level, np.where(idx == 0, 99, idx).astype(np.int32)),
                           (np.array([0, 1], np.uint8), np.array([[0, 0], [1, 1]], np.int32))]:
        bl, bi = _cells(ctx, lv_bad, ix_bad)
        cb = G.cells_t(bl, bi)
        g.n_rows = 0
        rc = L.gis_build_graph(ctx.handle, ctypes.byref(st), ctypes.byref(gt), G._ptr(du),
                               u.shape[0], ctypes.byref(cb), ctypes.byref(opts), ctypes.byref(g), s)
        assert rc == 1, L.gis_last_error()
    # an inconsistent caller graph is refused by gis_prune
    gg = G.GraphT()
    bad_rp = torch.zeros(n_rows + 1, dtype=torch.int64, device=ctx.dev)
    bad_rp[-1] = 5
    bad_col = torch.full((5,), 10 ** 6, dtype=torch.int32, device=ctx.dev)
    gg.n_rows, gg.n_edges, gg.cap_edges = n_rows, 5, 5
    gg.row_ptr, gg.col, gg.out = G._ptr(bad_rp), G._ptr(bad_col), G._ptr(out)
    kept = torch.empty(level.shape[0], dtype=torch.uint8, device=ctx.dev)
    mask = torch.empty(level.shape[0], dtype=torch.int64, device=ctx.dev)
    assert L.gis_prune(ctx.handle, ctypes.byref(gg), level.shape[0], u.shape[0], 1, G._ptr(kept),
                       G._ptr(mask), None, s) == 1


# ------------------------------------------------------------------ batches
def _batch_workloads(kind):
    rng = np.random.Generator(np.random.PCG64(77))
    out = []
    if kind == "vdp_uniform":          # rounds 0, mixed grid sizes and boxes
        for i, side in enumerate((16, 40, 24, 64, 8)):
            s = rng.uniform(0.6, 1.0)
            out.append(W.Workload(f"b{i}", W.vdp(mu=rng.uniform(0.5, 2.0)),
                                  W.Grid((side, side + 3), *W.scaled_vdp_box(s)),
                                  W.evenly_spaced(-1, 1, 11), W.LATTICE3, 0, "fp64"))
    elif kind == "vdp_controlled_r2":  # the small jobs keep nothing and stop after round 0
        for i, side in enumerate((8, 48, 12, 56)):
            out.append(W.Workload(f"c{i}", W.vdp(mu=rng.uniform(0.8, 1.2)),
                                  W.Grid((side, side), *W.VDP_BOX),
                                  W.evenly_spaced(-1, 1, 9), W.LATTICE3, 2, "fp64"))
    else:                              # adaptive, non-leaving analysis, several levels
        prec = "fp32_recheck" if kind == "vdp_adaptive32" else "fp64"
        for i, side in enumerate((12, 32, 20, 4)):
            out.append(W.Workload(f"a{i}", W.vdp(mu=rng.uniform(0.5, 2.0)),
                                  W.Grid((side, side), *W.VDP_BOX),
                                  W.evenly_spaced(-1, 1, 7), W.LATTICE3, 3, prec,
                                  analysis="nonleaving"))
    return out


@pytest.mark.parametrize("kind", ["vdp_uniform", "vdp_controlled_r2", "vdp_adaptive",
                                  "vdp_adaptive32"])
def test_batch_equals_single_solves_and_oracle(G, ctx, kind):
    wls = _batch_workloads(kind)
    sols = G.solve_batch(ctx, wls)
    for wl, sol in zip(wls, sols):
        got = [_np(t) for t in sol.export()]
        single = [_np(t) for t in G.solve_workload(ctx, wl).export()]
        for a, b in zip(got, single):
            np.testing.assert_array_equal(a, b, err_msg=wl.name)
        want = _oracle_solve(wl)
        np.testing.assert_array_equal(got[0], want["level"])
        np.testing.assert_array_equal(got[1], want["idx"])
        np.testing.assert_array_equal(got[2], want["kept"])
        np.testing.assert_array_equal(got[3].view(np.uint64), want["mask"])
        info = sol.info()
        assert info["n_rounds"] == len(want["stats"]), wl.name
        for got_r, want_r in zip(info["rounds"], want["stats"]):
            for k in ("n_cells", "n_rows", "n_edges", "n_out", "n_kept"):
                assert got_r[k] == want_r[k], (wl.name, k, got_r, want_r)
        states = torch.as_tensor(W.query_states(wl.grid, 3000, seed=3, margin=0.02), device=ctx.dev)
        m_w, a_w = oracle.query(wl.grid, want["level"], want["idx"], want["kept"], want["mask"],
                                states.cpu().numpy())
        np.testing.assert_array_equal(_np(sol.query_membership(states)), m_w)
        np.testing.assert_array_equal(_np(sol.query_admissible(states)).view(np.uint64), a_w)
