"""Pins of the oracle's one-step map x+ = f(x, u) (Eq. 1) and its sample points.

The oracle discretises the ODE with nsub classical RK4 substeps.  These tests
pin it to things outside the oracle:
  * the closed form of RK4 on a linear field x' = A x + B u: one substep is
    x+ = P(hA) x + h Q(hA) B u with P(Z) = I + Z + Z^2/2 + Z^3/6 + Z^4/24 and
    Q(Z) = I + Z/2 + Z^2/6 + Z^3/24 (non-symmetric A catches a transposed
    operand);
  * an independent high-order integrator (scipy DOP853) applied to each ODE
    written from its textbook statement, and the fourth-order error ratio;
  * exact dyadic sample coordinates of the two sample schemes.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_2202_06111_amd import workloads as W


def _rk4_linear_closed_form(A, B, u, x, dt, nsub):
    n = A.shape[0]
    h = dt / nsub
    Z = h * A
    I = np.eye(n)
    Z2 = Z @ Z
    Z3 = Z2 @ Z
    Z4 = Z3 @ Z
    P = I + Z + Z2 / 2 + Z3 / 6 + Z4 / 24
    Q = I + Z / 2 + Z2 / 6 + Z3 / 24
    for _ in range(nsub):
        x = P @ x + h * (Q @ (B @ u))
    return x


@pytest.mark.parametrize("n,m,nsub", [(1, 1, 1), (2, 1, 3), (3, 2, 2), (4, 2, 4)])
def test_linear_closed_form(oracle_lib, n, m, nsub):
    rng = np.random.Generator(np.random.PCG64(100 + n))
    for trial in range(5):
        A = rng.uniform(-2, 2, size=(n, n))
        B = rng.uniform(-1, 1, size=(n, m))
        system = W.linear(A, B, dt=0.3, nsub=nsub)
        x = rng.uniform(-3, 3, size=n)
        u = rng.uniform(-1, 1, size=m)
        got = oracle.step(system, x, u)
        want = _rk4_linear_closed_form(A, B, u, x, 0.3, nsub)
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def _vdp_rhs(mu):
    def f(t, s, u):
        x1, x2 = s
        return [x2, mu * (1 - x1 ** 2) * x2 - x1 + u[0]]
    return f


def _lorenz_rhs(t, s, u):
    x1, x2, x3 = s
    return [10 * (x2 - x1), x1 * (28 - x3) - x2 + u[0], x1 * x2 - (8 / 3) * x3]


def _vdp2_rhs(t, s, u):
    x1, v1, x2, v2 = s
    return [v1, (1 - x1 ** 2) * v1 - x1 + 0.2 * (x2 - x1) + u[0],
            v2, (1 - x2 ** 2) * v2 - x2 + 0.2 * (x1 - x2) + u[1]]


CASES = [
    (W.vdp(mu=1.7), _vdp_rhs(1.7), ((-2.5, -3.0), (2.5, 3.0)), 1, 3e-5),
    (W.lorenz(), _lorenz_rhs, ((-20, -25, 0), (20, 25, 50)), 1, 3e-5),
    (W.vdp2(), _vdp2_rhs, ((-2.5, -3, -2.5, -3), (2.5, 3, 2.5, 3)), 2, 3e-5),
]


@pytest.mark.parametrize("system,rhs,box,m,tol", CASES, ids=["vdp", "lorenz", "vdp2"])
def test_step_matches_independent_integrator(oracle_lib, system, rhs, box, m, tol):
    rng = np.random.Generator(np.random.PCG64(7))
    lo, hi = np.array(box[0], float), np.array(box[1], float)
    for trial in range(6):
        x = rng.uniform(lo, hi)
        u = rng.uniform(-1, 1, size=m)
        got = oracle.step(system, x, u)
        ref = solve_ivp(rhs, (0, system.dt), x, args=(u,), method="DOP853",
                        rtol=1e-13, atol=1e-13).y[:, -1]
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() <= tol * scale, (trial, got, ref)


@pytest.mark.parametrize("system,rhs,box,m,tol", CASES, ids=["vdp", "lorenz", "vdp2"])
def test_fourth_order_error_ratio(oracle_lib, system, rhs, box, m, tol):
    """Halving the substep divides the one-interval error by about 2^4."""
    rng = np.random.Generator(np.random.PCG64(8))
    lo, hi = np.array(box[0], float), np.array(box[1], float)
    x = 0.5 * rng.uniform(lo, hi)
    u = rng.uniform(-1, 1, size=m)
    dt = system.dt * 4  # a longer interval keeps the errors far above rounding
    ref = solve_ivp(rhs, (0, dt), x, args=(u,), method="DOP853", rtol=3e-14, atol=1e-14).y[:, -1]
    errs = []
    for nsub in (4, 8):
        s = W.System(system.kind, system.n, system.m, dt, nsub, system.params)
        errs.append(np.abs(oracle.step(s, x, u) - ref).max())
    ratio = errs[0] / errs[1]
    assert 11.0 < ratio < 22.0, (errs, ratio)


def _exact_samples(grid, samples, level, idx):
    n = grid.n
    pts = set()
    for d_offsets in itertools.product(range(3), repeat=n):
        if samples == W.CORNERS_CENTER:
            if not (all(k in (0, 2) for k in d_offsets) or all(k == 1 for k in d_offsets)):
                continue
        p = []
        for d in range(n):
            h = (Fraction(grid.hi[d]) - Fraction(grid.lo[d])) / grid.n0[d] / 2 ** level
            p.append(Fraction(grid.lo[d]) + (idx[d] + Fraction(d_offsets[d], 2)) * h)
        pts.add(tuple(p))
    return pts


@pytest.mark.parametrize("samples", [W.LATTICE3, W.CORNERS_CENTER])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_sample_points_on_dyadic_grid(oracle_lib, samples, n):
    """With a zero field the images are the sample points themselves; on a
    dyadic grid they must be exactly the cell's 3^n lattice (faces, centre)
    or its 2^n corners plus the centre."""
    grid = W.Grid(tuple([8] * n), tuple([-2.5] * n), tuple([2.5] * n))
    system = W.linear(np.zeros((n, n)), np.zeros((n, 1)), dt=0.1, nsub=2)
    level = np.array([0, 1, 2], dtype=np.uint8)
    idx = np.array([[3] * n, [0] * n, [31] * n], dtype=np.int32)
    u = np.zeros((1, 1))
    imgs = oracle.images(system, grid, samples, level, idx, u)
    for c in range(3):
        got = {tuple(Fraction(v) for v in p) for p in imgs[c]}
        assert got == _exact_samples(grid, samples, int(level[c]), idx[c])
        assert imgs[c].shape[0] == (3 ** n if samples == W.LATTICE3 else 2 ** n + 1)
