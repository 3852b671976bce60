"""Full-size GPU parity on the large workloads against digests of the CPU
oracle's results (tests/golden/digests_fullsize.json, written by
tests/golden/make_digests.py, which calls only oracle/ and the seeded
generators):

* Lorenz-type 128^3 (44 M rows): the graph (row offsets, targets, OUT flags)
  of both image precisions, and kept flags and masks of both analyses;
* coupled Van der Pol 32^4 with two boundary rounds: every round's covering,
  graph and non-leaving analysis through the step entry points (gis_build_graph,
  gis_prune, gis_subdivide), FP64 and FP32 with the FP64 recheck (equal
  element by element on the device), and the whole gis_solve in both
  precisions against the last round's digests; with every row of every round
  checked against the recheck band;
* the reactor of Sec. 4.1 as bench.py times it: the adaptive solve (8x8,
  10 rounds, N = 3) and the standard one (20 halvings, 2.0e9 rows): every
  round's counts, the final covering, kept set and masks, query answers.

Digests are SHA-256 of the arrays' little-endian bytes, the layout of the C
ABI (row_ptr i64, col i32, out u8, level u8, idx i32 cell-major, kept u8,
mask u64 words).  Every round of the coupled solve has its digests (the
oracle's round-2 graph, 1.56e9 rows and 1.2e10 edges, takes an hour on 8
cores); where a round's graph digest is absent, sampled rows are checked
against rows the oracle computes one by one.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
from conftest import gpu_available
from paper_2202_06111_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

DIGESTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "digests_fullsize.json")


@pytest.fixture(scope="module")
def G():
    from paper_2202_06111_amd import gis
    return gis


@pytest.fixture(scope="module")
def D():
    with open(DIGESTS) as f:
        return json.load(f)


def _sha(t: torch.Tensor, chunk: int = 1 << 28) -> str:
    """SHA-256 of a device tensor's bytes, copied to the host in chunks."""
    h = hashlib.sha256()
    flat = t.contiguous().reshape(-1).view(torch.uint8)
    for i in range(0, flat.numel(), chunk):
        h.update(flat[i:i + chunk].cpu().numpy().tobytes())
    return h.hexdigest()


def _check_covering(level, idx, want, what):
    assert int(level.shape[0]) == want["n_cells"], what
    assert _sha(level) == want["level"], what
    assert _sha(idx) == want["idx"], what


def _check_graph(g, want, what):
    assert (g.n_rows, g.n_edges, g.n_out) == (want["n_rows"], want["n_edges"], want["n_out"]), what
    assert _sha(g.row_ptr) == want["row_ptr"], what
    assert _sha(g.col) == want["col"], what
    assert _sha(g.out) == want["out"], what


def _check_analysis(kept, mask, want, what):
    assert int(kept.sum().item()) == want["n_kept"], what
    assert _sha(kept) == want["kept"], what
    assert _sha(mask) == want["mask"], what


def _sample_rows_against_oracle(wl, level, idx, g, n_sample, seed):
    """Edges and OUT flags of sampled rows against the oracle's rows of the
    same covering, computed one by one."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = np.unique(np.concatenate([rng.integers(0, g.n_rows, size=n_sample),
                                     [0, g.n_rows - 1]])).astype(np.int64)
    lv, ix = level.cpu().numpy(), idx.cpu().numpy()
    want = oracle.build_graph(wl.system, wl.grid, wl.samples, lv, ix, wl.u, rows=rows)
    rt = torch.as_tensor(rows, device=g.row_ptr.device)
    a = g.row_ptr[rt].cpu().numpy()
    b = g.row_ptr[rt + 1].cpu().numpy()
    out = g.out[rt].cpu().numpy()
    pos = 0
    for i, r in enumerate(rows):
        got = g.col[int(a[i]):int(b[i])].cpu().numpy()
        c = int(want["cnt"][i])
        np.testing.assert_array_equal(got, want["col"][pos:pos + c], err_msg=f"row {r}")
        pos += c
        assert out[i] == want["out"][i], f"row {r}"


def test_lorenz_128_full_graph(G, D):
    want = D["lorenz_uniform_128^3"]["rounds"][0]
    wl = W.lorenz_uniform_128()
    with G.Context(0) as ctx:
        level, idx = G.coarse_cells(ctx, wl.grid)
        _check_covering(level, idx, want["covering"], "lorenz covering")
        band = G.calibrate_band(ctx, wl.system, wl.grid, wl.u, level, idx, wl.samples,
                                safety=8.0, floor_rel=1e-5)
        g64 = G.build_graph(ctx, wl.system, wl.grid, wl.u, level, idx,
                            G.opts_t(samples=wl.samples, precision="fp64"))
        _check_graph(g64, want["graph"], "lorenz fp64 graph")
        g32 = G.build_graph(ctx, wl.system, wl.grid, wl.u, level, idx,
                            G.opts_t(samples=wl.samples, precision="fp32_recheck", band=band))
        print(f"lorenz 128^3: rows {g64.n_rows} edges {g64.n_edges} out {g64.n_out} "
              f"recheck {g32.n_recheck} band {band}", flush=True)
        assert torch.equal(g32.row_ptr, g64.row_ptr) and torch.equal(g32.col, g64.col)
        assert torch.equal(g32.out, g64.out)
        del g32
        for analysis in ("controlled", "nonleaving"):
            kept, mask, nk = G.prune(ctx, g64, int(level.shape[0]), wl.K, analysis)
            _check_analysis(kept, mask, want[analysis], f"lorenz {analysis}")
            print(f"  {analysis}: kept {nk}", flush=True)
        del g64
    torch.cuda.empty_cache()


def test_vdp2_32_two_rounds_by_steps(G, D):
    """Round by round through the step entry points, both image precisions;
    the FP32 band is calibrated on each round's covering (every row)."""
    want = D["vdp2_adaptive_32^4_r2"]
    rounds = want["rounds"]
    wl = W.vdp2_adaptive_32()
    with G.Context(0) as ctx:
        level, idx = G.coarse_cells(ctx, wl.grid)
        for r in range(wl.rounds + 1):
            wr = rounds[r]
            _check_covering(level, idx, wr["covering"], f"round {r} covering")
            n_cells = int(level.shape[0])
            cap = wr["graph"]["n_edges"] if "graph" in wr else None
            g64 = G.build_graph(ctx, wl.system, wl.grid, wl.u, level, idx,
                                G.opts_t(samples=wl.samples, precision="fp64"), cap_edges=cap)
            if "graph" in wr:
                _check_graph(g64, wr["graph"], f"round {r} graph")
            else:
                _sample_rows_against_oracle(wl, level, idx, g64, 400, seed=40 + r)
            band = G.calibrate_band(ctx, wl.system, wl.grid, wl.u, level, idx, wl.samples,
                                    safety=8.0, floor_rel=1e-5)
            g32 = G.build_graph(ctx, wl.system, wl.grid, wl.u, level, idx,
                                G.opts_t(samples=wl.samples, precision="fp32_recheck", band=band),
                                cap_edges=g64.n_edges)
            print(f"vdp2 round {r}: cells {n_cells} rows {g64.n_rows} edges {g64.n_edges} "
                  f"recheck {g32.n_recheck} band {band}", flush=True)
            assert g32.n_edges == g64.n_edges and g32.n_out == g64.n_out
            assert torch.equal(g32.row_ptr, g64.row_ptr) and torch.equal(g32.out, g64.out)
            assert torch.equal(g32.col, g64.col)
            del g32
            torch.cuda.empty_cache()
            kept, mask, nk = G.prune(ctx, g64, n_cells, wl.K, wl.analysis)
            del g64
            torch.cuda.empty_cache()
            if wl.analysis in wr:
                _check_analysis(kept, mask, wr[wl.analysis], f"round {r} analysis")
            if r < wl.rounds:
                level, idx, bnd = G.subdivide(ctx, wl.grid, level, idx, kept, wl.boundary_rule)
                assert int(bnd.sum().item()) == wr["n_boundary"], f"round {r} boundary"
            del kept, mask
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", ["fp64", "fp32_recheck"])
def test_vdp2_32_two_rounds_full_solve(G, D, precision):
    """The whole gis_solve (the benchmarked path) against the last round's
    digests; FP32: every row of every round is checked against its round's
    recheck band (check_band), and the largest FP32 error stays within it."""
    want = D["vdp2_adaptive_32^4_r2"]["rounds"]
    wl = W.vdp2_adaptive_32()
    torch.cuda.empty_cache()
    with G.Context(0) as ctx:
        over = dict(precision=precision)
        if precision != "fp64":
            over["check_band"] = True
        sol = G.solve(ctx, wl.system, wl.grid, wl.u, wl.rounds, G.workload_opts(wl, **over))
        inf = sol.info()
        for i, rs in enumerate(inf["rounds"]):
            print(f"vdp2 solve {precision} round {i}: cells {rs['n_cells']} rows {rs['n_rows']} "
                  f"edges {rs['n_edges']} kept {rs['n_kept']} recheck {rs['n_recheck']} "
                  f"band {rs['band']} max_err_all {rs['max_err_all']}", flush=True)
            assert rs["n_cells"] == want[i]["covering"]["n_cells"]
            if "graph" in want[i]:
                assert rs["n_edges"] == want[i]["graph"]["n_edges"]
                assert rs["n_out"] == want[i]["graph"]["n_out"]
            if wl.analysis in want[i]:
                assert rs["n_kept"] == want[i][wl.analysis]["n_kept"]
            if precision != "fp64":
                assert all(0 < e <= b for e, b in zip(rs["max_err_all"], rs["band"])), i
        lv, ix, kept, mask = sol.export()
        _check_covering(lv, ix, want[2]["covering"], "final covering")
        if wl.analysis in want[2]:
            _check_analysis(kept, mask, want[2][wl.analysis], "final analysis")
        sol.free()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["cstr_adaptive_8x8_r10_n3", "cstr_standard_8x8_r20"])
def test_cstr_full_solve(G, D, name):
    """The reactor experiment's two solves (Sec. 4.1-4.2) as bench.py times
    them -- 10 adaptive rounds with the N = 3 neighbourhood, and the standard
    algorithm's 20 halvings (2.0e9 rows in all, 5.0e9 edges in its last
    round) -- against the oracle's digests: every round's counts, the final
    covering, kept set and masks, and the answers to 10^5 seeded queries."""
    if "cstr" not in D or name not in D["cstr"]:
        pytest.skip("the oracle's digests of this solve are not recorded")
    want = D["cstr"][name]
    wl = W.ALL[name]()
    torch.cuda.empty_cache()
    with G.Context(0) as ctx:
        sol = G.solve_workload(ctx, wl)
        inf = sol.info()
        assert inf["n_rounds"] == len(want["rounds"])
        assert list(inf["n0"]) == want["n0"]
        for i, (got_r, want_r) in enumerate(zip(inf["rounds"], want["rounds"])):
            for k in ("n_cells", "n_rows", "n_edges", "n_out", "n_kept"):
                assert got_r[k] == want_r[k], (name, i, k, got_r[k], want_r[k])
            for k in ("n_boundary", "n_selected"):
                if k in want_r:
                    assert got_r[k] == want_r[k], (name, i, k, got_r[k], want_r[k])
        print(f"{name}: rounds {inf['n_rounds']} final cells {inf['rounds'][-1]['n_cells']} "
              f"edges {inf['rounds'][-1]['n_edges']}", flush=True)
        lv, ix, kept, mask = sol.export()
        _check_covering(lv, ix, want["covering"], f"{name} covering")
        _check_analysis(kept, mask, want[wl.analysis], f"{name} analysis")
        qa = want["queries"]
        states = torch.as_tensor(W.query_states(wl.grid, qa["n"], seed=qa["seed"],
                                                margin=qa["margin"]), device=ctx.dev)
        assert _sha(sol.query_membership(states)) == want["member"]
        assert _sha(sol.query_admissible(states)) == want["admissible"]
        sol.free()
    torch.cuda.empty_cache()
