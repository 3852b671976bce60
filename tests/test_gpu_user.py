"""GPU parity of user-supplied fields (gis_set_user_field: the f of Eq. 1
given as code, compiled at run time with the library's build kernels)
against the CPU oracle's twin of the same code, through the C ABI.

Bar: sample images 0 ulp; graphs, kept sets, masks, coverings bit-exact.
Cases: built-in fields written as user code equal the built-ins on the
device too (images and whole solves); the damped Duffing oscillator, a field
outside the built-ins, equals the oracle (images, build on refined coverings,
both analyses, adaptive solves in FP64 and FP32 + recheck, a batch); the
error paths (no field, mismatched dimensions, a body that does not compile).
"""
import numpy as np
import pytest
import torch

import oracle
from conftest import gpu_available
from paper_2202_06111_amd import workloads as W
from test_oracle_user import CSTR, DUFFING, DUFFING_P, VDP, VDP2, as_user

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


DUFF = W.user(DUFFING, 2, 1, 0.1, 2, DUFFING_P)
DUFF_GRID = W.Grid((20, 18), (-2.0, -2.0), (2.0, 2.0))
DUFF_U = W.evenly_spaced(-0.5, 0.5, 5)

CASES = {
    "vdp": (W.vdp(mu=1.3), VDP, W.Grid((24, 20), *W.VDP_BOX), W.LATTICE3, W.evenly_spaced(-1, 1, 5)),
    "vdp2": (W.vdp2(), VDP2, W.Grid((5, 6, 5, 6), (-2.5, -3., -2.5, -3.), (2.5, 3., 2.5, 3.)),
             W.CORNERS_CENTER, W.input_grid(-1, 1, 3, 2)),
    "cstr": (W.cstr(), CSTR, W.Grid((24, 20), *W.CSTR_BOX), W.LATTICE3,
             W.evenly_spaced(285, 315, 7)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_builtin_as_user_images_bitexact(G, ctx, name):
    system, body, grid, samples, u = CASES[name]
    level, idx = oracle.coarse_cells(grid)
    dl, di = _dev(ctx, level, np.uint8), _dev(ctx, idx, np.int32)
    builtin = _np(G.images(ctx, system, grid, u, dl, di, samples, "fp64"))
    user = _np(G.images(ctx, as_user(system, body), grid, u, dl, di, samples, "fp64"))
    assert np.array_equal(user.view(np.int64), builtin.view(np.int64))


def test_duffing_images_match_oracle(G, ctx):
    level, idx = oracle.coarse_cells(DUFF_GRID)
    want = oracle.images(DUFF, DUFF_GRID, W.LATTICE3, level, idx, DUFF_U)
    got = _np(G.images(ctx, DUFF, DUFF_GRID, DUFF_U, _dev(ctx, level, np.uint8),
                       _dev(ctx, idx, np.int32), W.LATTICE3, "fp64"))
    assert np.array_equal(got.view(np.int64), want.view(np.int64))


def _refined(rng, n0, splits):
    import itertools
    cells = {(0,) + c for c in itertools.product(*[range(k) for k in n0])}
    for _ in range(splits):
        c = sorted(cells)[rng.integers(0, len(cells))]
        cells.remove(c)
        for ch in itertools.product((0, 1), repeat=len(n0)):
            cells.add((c[0] + 1,) + tuple(2 * c[1 + d] + ch[d] for d in range(len(n0))))
    cells = sorted(cells)
    keep = rng.random(len(cells)) >= 0.1
    cells = [c for c, k in zip(cells, keep) if k]
    return (np.array([c[0] for c in cells], np.uint8),
            np.array([c[1:] for c in cells], np.int32).reshape(len(cells), len(n0)))


@pytest.mark.parametrize("analysis", ["controlled", "nonleaving"])
def test_duffing_build_and_prune_match_oracle(G, ctx, analysis):
    level, idx = _refined(np.random.Generator(np.random.PCG64(5)), DUFF_GRID.n0, 20)
    want = oracle.build_graph(DUFF, DUFF_GRID, W.LATTICE3, level, idx, DUFF_U)
    g = G.build_graph(ctx, DUFF, DUFF_GRID, DUFF_U, _dev(ctx, level, np.uint8),
                      _dev(ctx, idx, np.int32), G.opts_t(samples=W.LATTICE3, precision="fp64"))
    np.testing.assert_array_equal(_np(g.row_ptr), want["row_ptr"])
    np.testing.assert_array_equal(_np(g.col), want["col"])
    np.testing.assert_array_equal(_np(g.out), want["out"])
    kept_w, mask_w, _ = oracle.prune(want["row_ptr"], want["col"], want["out"], level.shape[0],
                                     DUFF_U.shape[0], analysis)
    kept, mask, nk = G.prune(ctx, g, level.shape[0], DUFF_U.shape[0], analysis)
    np.testing.assert_array_equal(_np(kept), kept_w)
    np.testing.assert_array_equal(_np(mask).view(np.uint64), mask_w)


def _check_solve(G, ctx, wl, sol):
    want = oracle.solve(wl.system, wl.grid, wl.samples, wl.u, wl.rounds, analysis=wl.analysis,
                        nn=wl.nn)
    lv, ix, kept, mask = (_np(t) for t in sol.export())
    np.testing.assert_array_equal(lv, want["level"])
    np.testing.assert_array_equal(ix, want["idx"])
    np.testing.assert_array_equal(kept, want["kept"])
    np.testing.assert_array_equal(mask.view(np.uint64), want["mask"])
    info = sol.info()
    assert info["n_rounds"] == len(want["stats"])
    for got_r, want_r in zip(info["rounds"], want["stats"]):
        for k in ("n_cells", "n_edges", "n_out", "n_kept"):
            assert got_r[k] == want_r[k], (k, got_r, want_r)
    return info


@pytest.mark.parametrize("precision", ["fp64", "fp32_recheck"])
def test_duffing_adaptive_solve(G, ctx, precision):
    wl = W.Workload("duffing_20x18_r3", DUFF, DUFF_GRID, DUFF_U, W.LATTICE3, 3, precision,
                    analysis="nonleaving", nn=3)
    sol = G.solve_workload(ctx, wl, check_band=precision != "fp64")
    info = _check_solve(G, ctx, wl, sol)
    assert info["rounds"][-1]["n_kept"] > 0
    sol.free()


def test_vdp_as_user_solve_equals_builtin(G, ctx):
    """The adaptive Van der Pol workload (32x32, 5 rounds, FP32 + recheck)
    with the field as user code: the same result as the built-in field."""
    wl = W.vdp_adaptive_32()
    a = G.solve_workload(ctx, wl)
    b = G.solve_workload(ctx, W.Workload(wl.name, as_user(wl.system, VDP), wl.grid, wl.u,
                                         wl.samples, wl.rounds, wl.precision,
                                         analysis=wl.analysis))
    for ta, tb in zip(a.export(), b.export()):
        assert torch.equal(ta, tb)
    assert [r["n_edges"] for r in a.info()["rounds"]] == [r["n_edges"] for r in b.info()["rounds"]]
    a.free()
    b.free()


def test_batch_of_user_fields(G, ctx):
    base = W.Workload("duffing_b", DUFF, DUFF_GRID, DUFF_U, W.LATTICE3, 2, "fp64",
                      analysis="nonleaving")
    other = W.Workload("duffing_b2", W.user(DUFFING, 2, 1, 0.1, 2, (0.5, -1.0, 0.8)),
                       W.Grid((16, 16), (-2.0, -2.0), (2.0, 2.0)), DUFF_U, W.LATTICE3, 2, "fp64",
                       analysis="nonleaving")
    sols = G.solve_batch(ctx, [base, other])
    for wl, sol in zip([base, other], sols):
        _check_solve(G, ctx, wl, sol)
        sol.free()


def test_user_field_errors(G):
    c = G.Context(0)
    try:
        level, idx = oracle.coarse_cells(DUFF_GRID)
        dl, di = _dev(c, level, np.uint8), _dev(c, idx, np.int32)
        # no field installed (a system without code uses the context's field):
        # the launch refuses the user kind
        with pytest.raises(G.GisError, match="no user field"):
            G.images(c, W.System(W.USER, 2, 1, 0.1, 2, DUFFING_P), DUFF_GRID, DUFF_U, dl, di,
                     W.LATTICE3, "fp64")
        # a body that does not compile leaves no field
        with pytest.raises(G.GisError, match="does not compile"):
            c.set_user_field("dx[0] = nope;", 2, 1)
        # a field of another dimension
        c.set_user_field(DUFFING, 2, 1)
        with pytest.raises(G.GisError, match="compiled for n = 2"):
            G.images(c, W.System(W.USER, 2, 2, 0.1, 2, DUFFING_P), DUFF_GRID, np.zeros((3, 2)),
                     dl, di, W.LATTICE3, "fp64")
        # still usable afterwards
        got = _np(G.images(c, DUFF, DUFF_GRID, DUFF_U, dl, di, W.LATTICE3, "fp64"))
        want = oracle.images(DUFF, DUFF_GRID, W.LATTICE3, level, idx, DUFF_U)
        assert np.array_equal(got.view(np.int64), want.view(np.int64))
    finally:
        c.close()
