"""User-supplied fields (the f of Eq. 1 given as code): pins of the oracle's
CPU twin, and the library's compile-only check (no device needed).

* Each built-in field written as user code gives the built-in field's sample
  images bit for bit (the built-ins are pinned in test_oracle_rk4.py and
  test_oracle_cstr.py), so the twin's compilation adds nothing and drops
  nothing.
* A field outside the built-ins, the damped Duffing oscillator
  x'' = -delta x' - alpha x - beta x^3 + u, against scipy's DOP853 on the
  textbook equation and the fourth-order error ratio of RK4.
* The library compiles the same bodies for gfx950 with hipRTC, with its own
  build kernels (gis_set_user_field with no context), and reports a body
  that does not compile with the compiler's message.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_2202_06111_amd import workloads as W

VDP = "dx[0] = x[1];\ndx[1] = fmaT(p[0] * fmaT(-x[0], x[0], (R)1), x[1], u[0] - x[0]);"
LORENZ = """dx[0] = p[0] * (x[1] - x[0]);
dx[1] = fmaT(x[0], p[1] - x[2], u[0] - x[1]);
dx[2] = fmaT(x[0], x[1], -(p[2] * x[2]));"""
VDP2 = """dx[0] = x[1];
dx[1] = fmaT(fmaT(-x[0], x[0], (R)1), x[1], fmaT(p[0], x[2] - x[0], u[0] - x[0]));
dx[2] = x[3];
dx[3] = fmaT(fmaT(-x[2], x[2], (R)1), x[3], fmaT(p[0], x[0] - x[2], u[1] - x[2]));"""
CSTR = """const R e = expT(-(p[3] / x[1]));
const R rate = (p[4] * e) * x[0];
dx[0] = fmaT(p[0], p[1] - x[0], -rate);
dx[1] = fmaT(p[0], p[2] - x[1], fmaT(p[5], rate, p[6] * (u[0] - x[1])));"""
# damped Duffing oscillator, p = (delta, alpha, beta)
DUFFING = """dx[0] = x[1];
dx[1] = fmaT(-p[2] * x[0], x[0] * x[0], fmaT(-p[1], x[0], fmaT(-p[0], x[1], u[0])));"""
DUFFING_P = (0.3, -1.0, 1.0)


def as_user(system, body):
    return W.user(body, system.n, system.m, system.dt, system.nsub, system.params)


BUILTIN = {
    "vdp": (W.vdp(mu=1.3), VDP, W.Grid((6, 5), *W.VDP_BOX), W.LATTICE3, W.evenly_spaced(-1, 1, 3)),
    "lorenz": (W.lorenz(), LORENZ, W.Grid((3, 4, 3), (-20., -25., 0.), (20., 25., 50.)),
               W.CORNERS_CENTER, W.evenly_spaced(-10, 10, 3)),
    "vdp2": (W.vdp2(), VDP2, W.Grid((2, 3, 2, 3), (-2.5, -3., -2.5, -3.), (2.5, 3., 2.5, 3.)),
             W.CORNERS_CENTER, W.input_grid(-1, 1, 2, 2)),
    "cstr": (W.cstr(), CSTR, W.Grid((7, 6), *W.CSTR_BOX), W.LATTICE3,
             W.evenly_spaced(285, 315, 4)),
}


@pytest.mark.parametrize("name", sorted(BUILTIN))
def test_builtin_fields_as_user_code_are_bit_identical(oracle_lib, name):
    system, body, grid, samples, u = BUILTIN[name]
    level, idx = oracle.coarse_cells(grid)
    want = oracle.images(system, grid, samples, level, idx, u)
    got = oracle.images(as_user(system, body), grid, samples, level, idx, u)
    assert np.array_equal(got.view(np.int64), want.view(np.int64))


def _duffing_rhs(t, s, u):
    d, a, b = DUFFING_P
    return [s[1], -d * s[1] - a * s[0] - b * s[0] ** 3 + u[0]]


def test_duffing_against_independent_integrator(oracle_lib):
    system = W.user(DUFFING, 2, 1, 0.1, 2, DUFFING_P)
    rng = np.random.Generator(np.random.PCG64(41))
    for _ in range(8):
        x = rng.uniform(-2, 2, size=2)
        u = rng.uniform(-0.5, 0.5, size=1)
        got = oracle.step(system, x, u)
        ref = solve_ivp(_duffing_rhs, (0, system.dt), x, args=(u,), method="DOP853",
                        rtol=1e-13, atol=1e-13).y[:, -1]
        # RK4's truncation scale (a wrong sign or term gives 1e-2 and more)
        assert np.abs(got - ref).max() <= 3e-5 * max(1.0, np.abs(ref).max()), (got, ref)


def test_duffing_fourth_order_error_ratio(oracle_lib):
    x, u = np.array([1.2, -0.4]), np.array([0.2])
    dt = 0.8
    ref = solve_ivp(_duffing_rhs, (0, dt), x, args=(u,), method="DOP853",
                    rtol=3e-14, atol=1e-14).y[:, -1]
    errs = [np.abs(oracle.step(W.user(DUFFING, 2, 1, dt, k, DUFFING_P), x, u) - ref).max()
            for k in (4, 8)]
    assert 11.0 < errs[0] / errs[1] < 22.0, errs


def test_user_and_builtin_solve_agree(oracle_lib):
    """A whole oracle solve of the Van der Pol field as user code equals the
    built-in one (covering, kept cells, masks)."""
    grid = W.Grid((16, 16), *W.VDP_BOX)
    u = W.evenly_spaced(-1, 1, 5)
    a = oracle.solve(W.vdp(), grid, W.LATTICE3, u, 2, analysis="nonleaving")
    b = oracle.solve(as_user(W.vdp(), VDP), grid, W.LATTICE3, u, 2, analysis="nonleaving")
    for k in ("level", "idx", "kept", "mask"):
        np.testing.assert_array_equal(a[k], b[k])


# ---------------------------------------------------------------- library, compile only
@pytest.fixture(scope="module")
def G():
    from paper_2202_06111_amd import gis
    return gis


@pytest.mark.parametrize("body,n,m", [(VDP, 2, 1), (LORENZ, 3, 1), (VDP2, 4, 2), (CSTR, 2, 1),
                                      (DUFFING, 2, 1)])
def test_library_compiles_user_fields(G, body, n, m):
    G.check_user_field(body, n, m)


def test_library_reports_compile_errors(G):
    with pytest.raises(G.GisError, match="user field:2:"):
        G.check_user_field("dx[0] = x[1];\ndx[1] = undefined_name;", 2, 1)
    with pytest.raises(G.GisError, match="GIS_E_INVAL"):
        G.check_user_field(VDP, 5, 1)
