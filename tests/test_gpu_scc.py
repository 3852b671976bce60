"""GPU parity of the literal reading of Definition 6 (analysis "largest_scc":
the largest strongly connected component with a cycle plus every cell with a
path into it) through the C ABI, against the oracle: hand-built graphs,
random graphs with planted components of equal and different sizes, whole
solves (uniform, adaptive, standard subdivision) and a batch.  Kept flags,
masks, cell lists and round counts bit for bit.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from conftest import gpu_available
from paper_2202_06111_amd import workloads as W
from test_oracle_scc import CASES, _graph

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


def _prune(G, ctx, n, K, row_ptr, col, **tuning):
    dev = ctx.dev
    out = np.zeros(n * K, np.uint8)
    g = G.Graph(torch.as_tensor(row_ptr, device=dev), torch.as_tensor(col, device=dev),
                torch.as_tensor(out, device=dev), n * K, int(col.shape[0]), 0, 0)
    prev = ctx.set_tuning(**tuning) if tuning else None
    try:
        kept, mask, nk = G.prune(ctx, g, n, K, "largest_scc")
    finally:
        if prev:
            ctx.set_tuning(**prev)
    kept_w, mask_w = oracle.largest_scc(row_ptr, col, n, K)
    np.testing.assert_array_equal(_np(kept), kept_w)
    np.testing.assert_array_equal(_np(mask).view(np.uint64), mask_w)
    assert nk == int(kept_w.sum())


@pytest.mark.parametrize("name", list(CASES))
def test_prune_hand_built(G, ctx, name):
    n, edges, _ = CASES[name]
    row_ptr, col = _graph(n, 2, edges)
    _prune(G, ctx, n, 2, row_ptr, col)


def _planted(seed, n_comp, K):
    """Cycles of random sizes (two of them equally large when seed is even),
    chains between some of them, tails into them and cells with no cycle."""
    rng = np.random.default_rng(seed)
    sizes = [int(v) for v in rng.integers(1, 200, n_comp)]
    if seed % 2 == 0:
        sizes[-1] = sizes[0] = max(sizes)
    perm = rng.permutation(sum(sizes) + 600)
    edges = {}
    comps, at = [], 0
    for sz in sizes:
        cells = [int(v) for v in perm[at:at + sz]]
        at += sz
        comps.append(cells)
        for i, c in enumerate(cells):  # a cycle (a self-loop for one cell)
            edges.setdefault((c, int(rng.integers(0, K))), []).append(cells[(i + 1) % sz])
            if sz > 3 and rng.random() < 0.2:  # chords keep it one component
                edges.setdefault((c, int(rng.integers(0, K))), []).append(
                    cells[int(rng.integers(0, sz))])
    for a in range(len(comps) - 1):  # one-way bridges
        if rng.random() < 0.5:
            edges.setdefault((comps[a][0], 0), []).append(comps[a + 1][-1])
    rest = [int(v) for v in perm[at:]]
    for c in rest:  # tails and dead ends
        if rng.random() < 0.7:
            t = comps[int(rng.integers(0, len(comps)))] if rng.random() < 0.6 else rest
            edges.setdefault((c, int(rng.integers(0, K))), []).append(int(t[int(rng.integers(0, len(t)))]))
    n = len(perm)
    for key in edges:
        edges[key] = sorted(set(edges[key]))
    return n, edges


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("K", [1, 3])
def test_prune_planted_components(G, ctx, seed, K):
    n, edges = _planted(seed, 8 + seed, K)
    row_ptr, col = _graph(n, K, edges)
    _prune(G, ctx, n, K, row_ptr, col)
    _prune(G, ctx, n, K, row_ptr, col, sweep_edges=0, wit_sweeps=0)  # non-leaving phase on the frontier


@pytest.mark.parametrize("K", [1, 2])
def test_prune_wide_hub_and_long_ring(G, ctx, K):
    """A hub cell with the largest id of its component and an edge to each
    of 1,000 cells that all lead back to it (one colour sweep raises more
    cells than a block can queue, so the rest wait for the next sweep), a
    ring of 2,000 cells whose largest id must travel the whole ring (many
    locally followed generations and many sweeps), and tails into both:
    the ring is the largest component."""
    hub = 1000
    edges = {(hub, 0): list(range(hub))}
    for c in range(hub):
        edges[(c, c % K)] = [hub]
    ring = list(range(3000, 1000, -1))  # 3000 -> 2999 -> ... -> 1001 -> 3000
    for i, c in enumerate(ring):
        edges[(c, i % K)] = [ring[(i + 1) % len(ring)]]
    for t in range(3001, 3101):  # tails: into the ring, into the star, and chains of both
        edges[(t, 0)] = [1001 + (t * 7) % 2000] if t % 3 else [t % hub]
        if t % 5 == 0:
            edges[(t, K - 1)] = sorted(set(edges.get((t, K - 1), []) + [t - 1]))
    n = 3101
    row_ptr, col = _graph(n, K, edges)
    _prune(G, ctx, n, K, row_ptr, col)


def _check_solve(G, wl, sols_or_sol, ctx):
    want = oracle.solve(wl.system, wl.grid, wl.samples, wl.u, wl.rounds, rule=wl.boundary_rule,
                        analysis=wl.analysis, subdivision=wl.subdivision)
    sol = sols_or_sol
    lv, ix, kept, mask = (_np(t) for t in sol.export())
    np.testing.assert_array_equal(lv, want["level"])
    np.testing.assert_array_equal(ix, want["idx"])
    np.testing.assert_array_equal(kept, want["kept"])
    np.testing.assert_array_equal(mask.view(np.uint64), want["mask"])
    info = sol.info()
    assert info["n_rounds"] == len(want["stats"])
    for got_r, want_r in zip(info["rounds"], want["stats"]):
        for k in ("n_cells", "n_rows", "n_edges", "n_out", "n_kept"):
            assert got_r[k] == want_r[k], (wl.name, k, got_r, want_r)


def _wl(name):
    vdp = W.vdp()
    return {
        "vdp_uniform": W.Workload("vdp24", vdp, W.Grid((24, 20), *W.VDP_BOX),
                                  W.evenly_spaced(-1, 1, 5), W.LATTICE3, 0, "fp64",
                                  analysis="largest_scc"),
        "vdp_adaptive": W.Workload("vdp16_r3", vdp, W.Grid((16, 16), *W.VDP_BOX),
                                   W.evenly_spaced(-1, 1, 7), W.LATTICE3, 3, "fp32_recheck",
                                   analysis="largest_scc"),
        "vdp_standard": W.Workload("vdp12_std_r4", vdp, W.Grid((12, 10), *W.VDP_BOX),
                                   W.evenly_spaced(-1, 1, 5), W.LATTICE3, 4, "fp64",
                                   analysis="largest_scc", subdivision="bisect"),
        "lorenz": W.Workload("lorenz10", W.lorenz(),
                             W.Grid((10, 12, 9), (-20., -25., 0.), (20., 25., 50.)),
                             W.evenly_spaced(-10, 10, 4), W.CORNERS_CENTER, 1, "fp64",
                             analysis="largest_scc"),
    }[name]


@pytest.mark.parametrize("name", ["vdp_uniform", "vdp_adaptive", "vdp_standard", "lorenz"])
def test_solve_largest_scc(G, ctx, name):
    wl = _wl(name)
    _check_solve(G, wl, G.solve_workload(ctx, wl), ctx)


def test_solve_batch_largest_scc(G, ctx):
    base = _wl("vdp_adaptive")
    wls = [base, dataclasses.replace(base, name="mu2", system=W.vdp(mu=2.0),
                                     grid=W.Grid((12, 14), *W.VDP_BOX))]
    for wl, sol in zip(wls, G.solve_batch(ctx, wls)):
        _check_solve(G, wl, sol, ctx)


def test_solve_largest_scc_default_workload(G, ctx):
    """The default benchmark workload (adaptive Van der Pol 32x32, five
    boundary rounds, 21 inputs) under the literal analysis, whole solve."""
    wl = dataclasses.replace(W.vdp_adaptive_32(), analysis="largest_scc")
    _check_solve(G, wl, G.solve_workload(ctx, wl), ctx)
