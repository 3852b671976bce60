"""gis_prune_static (the analysis in a static device workspace, for callers
that cannot allocate) against gis_prune on the same graphs: kept flags,
masks and kept counts identical, on two calls in a row with the second input
smaller than the first, for both analyses; sizes beyond the workspace and
the unsupported analysis are rejected with an error."""
import numpy as np
import pytest
import torch

from conftest import gpu_available
from paper_2202_06111_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]


@pytest.fixture(scope="module")
def G():
    from paper_2202_06111_amd import gis
    return gis


def _uniform(G, ctx, side, K):
    grid = W.Grid((side, side), *W.VDP_BOX)
    u = W.evenly_spaced(-1.0, 1.0, K)
    level, idx = G.coarse_cells(ctx, grid)
    g = G.build_graph(ctx, W.vdp(), grid, u, level, idx, G.opts_t(samples=W.LATTICE3))
    return g, int(level.shape[0]), K


def _cascade(G, ctx):
    """A seeded graph with removal chains of tens of steps (3000 cells, K = 5)."""
    from test_gpu_parity import _cascade_graph
    row_ptr, col, out, n_cells = _cascade_graph(5, 6, 105)
    dev = ctx.dev
    g = G.Graph(torch.as_tensor(row_ptr, device=dev), torch.as_tensor(col, device=dev),
                torch.as_tensor(out, device=dev), n_cells * 5, int(col.shape[0]), int(out.sum()),
                0)
    return g, n_cells, 5


def _graphs(G, ctx, analysis):
    """A larger graph, then a smaller one."""
    first = _uniform(G, ctx, 96, 11) if analysis == "controlled" else _cascade(G, ctx)
    return [first, _uniform(G, ctx, 24, 7)]


@pytest.mark.parametrize("analysis", ["controlled", "nonleaving"])
def test_static_prune_matches_prune(G, analysis):
    with G.Context(0) as ctx:
        graphs = _graphs(G, ctx, analysis)
        assert graphs[1][1] < graphs[0][1]
        removed_some = False
        for g, n_cells, K in graphs:  # the second call is smaller than the first
            kept_r, mask_r, nk_r = G.prune(ctx, g, n_cells, K, analysis)
            kept_s, mask_s, nk_s = G.prune_static(g, n_cells, K, analysis)
            torch.cuda.synchronize()
            assert nk_s == nk_r and 0 < nk_r, (n_cells, nk_r, nk_s)
            removed_some |= nk_r < n_cells
            assert torch.equal(kept_s, kept_r), n_cells
            assert torch.equal(mask_s, mask_r), n_cells
        assert removed_some


def test_static_prune_caller_buffers_and_repeat(G):
    """Caller-supplied outputs; the same call twice gives the same result (the
    workspace keeps the previous call's contents, which must not leak in)."""
    with G.Context(0) as ctx:
        (g, n, K), (g2, n2, K2) = _graphs(G, ctx, "nonleaving")
        kept = torch.empty(n, dtype=torch.uint8, device=ctx.dev)
        mask = torch.empty((n, 1), dtype=torch.int64, device=ctx.dev)
        a = G.prune_static(g, n, K, "nonleaving", kept=kept, mask=mask)
        first = (a[0].clone(), a[1].clone(), a[2])
        G.prune_static(g2, n2, K2, "controlled")
        b = G.prune_static(g, n, K, "nonleaving", kept=kept, mask=mask)
        assert torch.equal(first[0], b[0]) and torch.equal(first[1], b[1]) and first[2] == b[2]


def test_static_prune_rejects(G):
    with G.Context(0) as ctx:
        (g, n, K), _ = _graphs(G, ctx, "controlled")
        with pytest.raises(G.GisError) as e:
            G.prune_static(g, n, K, "largest_scc")
        assert e.value.status == 1  # GIS_E_INVAL
        big = (1 << 21) + 1
        fake = G.Graph(torch.zeros(big + 1, dtype=torch.int64, device=ctx.dev),
                       torch.zeros(1, dtype=torch.int32, device=ctx.dev),
                       torch.zeros(big, dtype=torch.uint8, device=ctx.dev), big, 0, 0, 0)
        with pytest.raises(G.GisError) as e:
            G.prune_static(fake, big, 1, "controlled",
                           kept=torch.empty(1, dtype=torch.uint8, device=ctx.dev),
                           mask=torch.empty((1, 1), dtype=torch.int64, device=ctx.dev))
        assert e.value.status == 4  # GIS_E_CAPACITY
