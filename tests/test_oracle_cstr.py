"""Pins of the oracle's CSTR model (Sec. 4.1, Eq. 4, Table 2) and of its own
exponential, against facts outside the oracle:

  * exp: the C library's exp within 1 ulp on the CSTR's argument range and on
    the whole finite range, exact results at 0 and at the limits, NaN and
    infinities, and the subnormal range;
  * the field, through one RK4 step (the oracle's x+ = f(x, u)), on special
    cases whose RK4 result has a closed form:
      - no reaction (k0 = 0): a linear field, one RK4 step is
        P(hA) x + h Q(hA) b (the classical closed form);
      - an isothermal batch reactor (no flow, no heat of reaction, no
        cooling): T is unchanged and cA is multiplied by the RK4 stability
        polynomial R(-k h) with k = k0 exp(-(E/R)/T) (C library exp);
      - no cooling (UA = 0): the energy-balance combination
        z = (-dH/(rho cp)) cA + T loses the reaction term and obeys
        z' = q/V (z_f - z), so z+ = z_f + (z0 - z_f) R(-h q/V);
  * the textbook steady state of this reactor, (cA, T) = (0.5, 350) at
    Tc = 300 K, where the field nearly vanishes;
  * an independent high-order integrator (scipy DOP853) applied to Eq. (4)
    written with the C library's exp, and the fourth-order error ratio;
  * the packed parameters against Table 2.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_2202_06111_amd import workloads as W


def _ulps(got, want):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    return np.abs(got - want) / np.spacing(np.abs(want))


# ------------------------------------------------------------------ exp
def test_exp_within_one_ulp_cstr_range(oracle_lib):
    """-(E/R)/T for T in about [300, 400] K: the Arrhenius arguments."""
    x = np.random.Generator(np.random.PCG64(11)).uniform(-30.0, -20.0, 200_000)
    got = oracle.exp(x)
    want = np.array([math.exp(v) for v in x])
    u = _ulps(got, want)
    assert u.max() <= 1.0
    assert (u == 0).mean() > 0.9


def test_exp_within_one_ulp_everywhere(oracle_lib):
    rng = np.random.Generator(np.random.PCG64(12))
    x = np.concatenate([rng.uniform(-708.0, 709.7, 200_000), rng.uniform(-1.0, 1.0, 50_000),
                        rng.uniform(-1e-8, 1e-8, 10_000)])
    got = oracle.exp(x)
    want = np.array([math.exp(v) for v in x])
    assert _ulps(got, want).max() <= 1.0


def test_exp_subnormal_results(oracle_lib):
    """exp(x) for x in (-745, -708): subnormal results, within one unit of the
    smallest subnormal of math.exp."""
    x = np.random.Generator(np.random.PCG64(13)).uniform(-745.0, -708.5, 20_000)
    got = oracle.exp(x)
    want = np.array([math.exp(v) for v in x])
    assert (np.abs(got - want) <= 5e-324).all()
    assert (got > 0).all()


def test_exp_special_values(oracle_lib):
    got = oracle.exp(np.array([0.0, -0.0, np.inf, -np.inf, 709.78, 709.79, 710.0, 1e300,
                               -745.2, -746.0, -1e300]))
    assert got[0] == 1.0 and got[1] == 1.0
    assert got[2] == np.inf and got[3] == 0.0
    assert np.isfinite(got[4]) and got[4] > 1.7e308      # just below the largest double
    assert got[5] == np.inf and got[6] == np.inf and got[7] == np.inf
    assert got[8] == 0.0 and got[9] == 0.0 and got[10] == 0.0
    assert np.isnan(oracle.exp(np.array([np.nan]))[0])


def test_exp_functional_equation(oracle_lib):
    """exp(a) exp(b) = exp(a + b) within a few ulp when a + b is exact."""
    rng = np.random.Generator(np.random.PCG64(14))
    a = np.round(rng.uniform(-20, 20, 5000) * 1024) / 1024   # dyadic: a + b is exact
    b = np.round(rng.uniform(-20, 20, 5000) * 1024) / 1024
    s = a + b
    ea, eb, es = oracle.exp(a), oracle.exp(b), oracle.exp(s)
    assert _ulps(ea * eb, es).max() <= 4.0


# ------------------------------------------------------------------ field / step
TABLE2 = dict(q=100.0, V=100.0, cAf=1.0, Tf=350.0, E_over_R=8750.0, k0=7.2e10,
              minus_dH=5.0e4, UA=5.0e4, cp=0.239, rho=1000.0)


def _R(z):
    """Stability polynomial of classical RK4."""
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def test_parameters_packed_from_table2():
    s = W.cstr()
    assert s.kind == W.CSTR and (s.n, s.m) == (2, 1) and s.dt == 0.1 and s.nsub == 1
    p = s.params
    assert p[0] == 1.0 and p[1] == 1.0 and p[2] == 350.0 and p[3] == 8750.0 and p[4] == 7.2e10
    assert p[5] == pytest.approx(5.0e4 / 239.0, rel=1e-15)      # -dH / (rho cp), K L / mol
    assert p[6] == pytest.approx(5.0e4 / 23900.0, rel=1e-15)    # UA / (V rho cp), 1 / min


@pytest.mark.parametrize("nsub", [1, 3])
def test_no_reaction_is_the_linear_closed_form(oracle_lib, nsub):
    s = W.cstr(k0=0.0, nsub=nsub, dt=0.25)
    qv, cAf, Tf, ua = s.params[0], s.params[1], s.params[2], s.params[6]
    A = np.array([[-qv, 0.0], [0.0, -qv - ua]])
    rng = np.random.Generator(np.random.PCG64(21))
    h = s.dt / nsub
    Z = h * A
    I = np.eye(2)
    P = I + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24
    Q = I + Z / 2 + Z @ Z / 6 + Z @ Z @ Z / 24
    for _ in range(8):
        x = np.array([rng.uniform(0, 1), rng.uniform(345, 355)])
        Tc = rng.uniform(285, 315)
        b = np.array([qv * cAf, qv * Tf + ua * Tc])
        want = x.copy()
        for _ in range(nsub):
            want = P @ want + h * (Q @ b)
        got = oracle.step(s, x, np.array([Tc]))
        np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("nsub", [1, 2])
def test_isothermal_batch_reactor(oracle_lib, nsub):
    """q = 0, -dH = 0, UA = 0: T stays put exactly and cA decays by R(-k h)."""
    s = W.cstr(q=0.0, minus_dH=0.0, UA=0.0, nsub=nsub, dt=0.1)
    rng = np.random.Generator(np.random.PCG64(22))
    for _ in range(10):
        cA, T = rng.uniform(0.05, 1.0), rng.uniform(330, 370)
        got = oracle.step(s, np.array([cA, T]), np.array([300.0]))
        k = 7.2e10 * math.exp(-8750.0 / T)
        want = cA * _R(-k * s.dt / nsub) ** nsub
        assert got[1] == T
        assert abs(got[0] - want) <= 4e-16 * max(cA, 1.0) * 8


@pytest.mark.parametrize("nsub", [1, 4])
def test_energy_balance_invariant_without_cooling(oracle_lib, nsub):
    """UA = 0: z = (-dH/(rho cp)) cA + T follows the linear feed relaxation
    whatever the reaction does, so one RK4 step maps z exactly as R(-h q/V)."""
    s = W.cstr(UA=0.0, nsub=nsub, dt=0.1)
    qv, cAf, Tf, beta = s.params[0], s.params[1], s.params[2], s.params[5]
    zf = beta * cAf + Tf
    rng = np.random.Generator(np.random.PCG64(23))
    for _ in range(10):
        x = np.array([rng.uniform(0, 1), rng.uniform(345, 355)])
        got = oracle.step(s, x, np.array([rng.uniform(285, 315)]))
        z0 = beta * x[0] + x[1]
        z1 = beta * got[0] + got[1]
        want = zf + (z0 - zf) * _R(-qv * s.dt / nsub) ** nsub
        assert abs(z1 - want) <= 1e-11 * abs(want)
        # the reaction term does act: cA itself is not the feed relaxation
        assert abs(got[0] - (cAf + (x[0] - cAf) * _R(-qv * s.dt / nsub) ** nsub)) > 1e-6


def test_textbook_steady_state(oracle_lib):
    """(cA, T) = (0.5, 350) with Tc = 300 balances Eq. (4) with Table 2
    (k(350) = 7.2e10 exp(-25) = 0.99996... per minute): one step moves the
    state by the small residual only, and each balance term is needed for it."""
    s = W.cstr()
    x = np.array([0.5, 350.0])
    got = oracle.step(s, x, np.array([300.0]))
    assert abs(got[0] - 0.5) < 5e-6
    assert abs(got[1] - 350.0) < 1e-3
    # a 10 K warmer coolant: over a very short interval T rises at the
    # cooling term's rate UA/(V rho cp) * 10 K = 20.92 K/min (the other terms
    # still balance), and cA does not move at first order
    tiny = W.cstr(dt=1e-4)
    warm = oracle.step(tiny, x, np.array([310.0]))
    assert (warm[1] - 350.0) / 1e-4 == pytest.approx(5.0e4 / 23900.0 * 10, rel=1e-3)
    assert abs(warm[0] - 0.5) / 1e-4 < 1e-3


def _cstr_rhs(t, s, u):
    cA, T = s
    r = 7.2e10 * math.exp(-8750.0 / T) * cA
    return [(100.0 / 100.0) * (1.0 - cA) - r,
            (100.0 / 100.0) * (350.0 - T) + 5.0e4 / (1000.0 * 0.239) * r
            + 5.0e4 / (100.0 * 1000.0 * 0.239) * (u[0] - T)]


def test_step_matches_independent_integrator(oracle_lib):
    s = W.cstr(nsub=4)
    rng = np.random.Generator(np.random.PCG64(24))
    for _ in range(8):
        x = np.array([rng.uniform(0, 1), rng.uniform(345, 355)])
        u = np.array([rng.uniform(285, 315)])
        got = oracle.step(s, x, u)
        ref = solve_ivp(_cstr_rhs, (0, s.dt), x, args=(u,), method="DOP853",
                        rtol=1e-13, atol=1e-13).y[:, -1]
        # the RK4 error relative to the state's change over the interval
        # (up to 16 K in 0.1 min near the runaway corner)
        rel = np.abs(got - ref) / np.maximum(np.abs(ref - x), 1e-3)
        assert (rel < 2e-4).all(), (got, ref, x)


def test_fourth_order_error_ratio(oracle_lib):
    # a state that relaxes (from (0.6, 352) with Tc = 295 the reactor runs
    # away within 0.4 min and the coarse steps are far from the asymptote)
    x = np.array([0.5, 348.0])
    u = np.array([300.0])
    dt = 0.4
    ref = solve_ivp(_cstr_rhs, (0, dt), x, args=(u,), method="DOP853",
                    rtol=3e-14, atol=1e-14).y[:, -1]
    errs = [np.abs(oracle.step(W.cstr(dt=dt, nsub=k), x, u) - ref).max() for k in (4, 8)]
    assert 11.0 < errs[0] / errs[1] < 22.0, errs
