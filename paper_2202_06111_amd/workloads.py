"""Seeded synthetic workloads: systems, state boxes, input sets, query states.

This module holds no arithmetic of the GIS method itself.  It only describes
problems in the terms of the paper's problem statement (Eq. 1: a map
x+ = f(x, u) with compact state set X and input set U) and draws the
synthetic inputs that both the HIP library and the CPU oracle consume, so the
two sides always see bit-identical arrays.

The named workloads are the controlled Van der Pol, Lorenz-type and coupled
Van der Pol problems used to exercise the graph-construction path, and the
paper's own example, the continuously stirred tank reactor of Sec. 4.1
(Eq. 4, Table 2).
"""
from __future__ import annotations

import dataclasses
from typing import Sequence, Tuple

import numpy as np

# system kinds (names; each side maps them to its own numbering)
LINEAR = "linear"
VDP = "vdp"
LORENZ = "lorenz"
VDP2 = "vdp2"
CSTR = "cstr"
USER = "user"       # the caller's own field, given as code (see user())

LATTICE3 = "lattice3"            # 3^n points: offsets {0, 1/2, 1} of the cell width
CORNERS_CENTER = "corners_center"  # 2^n corners + the centre

SHELL = "shell"        # every finest cell adjacent to the cell (Remark 1 edge points included)
CORNERS = "corners"    # the 2^n diagonal corners only (Algorithm 1 as printed)


@dataclasses.dataclass(frozen=True)
class System:
    """x+ = RK4^nsub(x, u) over one sampling interval dt of an ODE x' = g(x, u)."""
    kind: str
    n: int
    m: int
    dt: float
    nsub: int
    params: Tuple[float, ...]
    # kind "user": the body of g, setting dx[0..n-1] from x, u and p (type R,
    # fmaT and expT available); the library compiles it for the device and
    # the oracle compiles it for the host
    source: str = ""

    def param_array(self) -> np.ndarray:
        p = np.zeros(32, dtype=np.float64)
        p[: len(self.params)] = self.params
        return p


@dataclasses.dataclass(frozen=True)
class Grid:
    """Closed state box X = prod [lo_d, hi_d] with n0_d coarse cells per dimension."""
    n0: Tuple[int, ...]
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]

    @property
    def n(self) -> int:
        return len(self.n0)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    system: System
    grid: Grid
    u: np.ndarray            # K x m, float64
    samples: str
    rounds: int
    precision: str           # "fp64" or "fp32_recheck"
    boundary_rule: str = SHELL
    # graph analysis: "controlled" (every image of some input stays in the kept
    # set) or "nonleaving" (cells with an infinite admissible path, the
    # paper's analysis).  Boundary-only refinement needs the latter: under the
    # controlled analysis a 32x32 Van der Pol covering keeps no cell at all.
    analysis: str = "controlled"
    # subdivision between rounds: "boundary" (2^n children of the boundary
    # cells, Sec. 3.1) or "bisect" (every kept cell halved across a cycled
    # dimension, the standard algorithm of Sec. 2.1)
    subdivision: str = "boundary"
    # neighbourhood size N of Sec. 3.1.2: the N kept cells nearest to each
    # boundary cell are subdivided with it (0: boundary cells only)
    nn: int = 0

    @property
    def K(self) -> int:
        return int(self.u.shape[0])


# ---------------------------------------------------------------- systems
def vdp(mu: float = 1.0, dt: float = 0.1, nsub: int = 4) -> System:
    """x1' = x2, x2' = mu (1 - x1^2) x2 - x1 + u."""
    return System(VDP, 2, 1, dt, nsub, (float(mu),))


def lorenz(sigma: float = 10.0, rho: float = 28.0, beta: float = 8.0 / 3.0,
           dt: float = 0.01, nsub: int = 2) -> System:
    """x1' = sigma (x2 - x1), x2' = x1 (rho - x3) - x2 + u, x3' = x1 x2 - beta x3."""
    return System(LORENZ, 3, 1, dt, nsub, (float(sigma), float(rho), float(beta)))


def vdp2(coupling: float = 0.2, dt: float = 0.1, nsub: int = 4) -> System:
    """Two oscillators, state (x1, v1, x2, v2):
    xi'' = (1 - xi^2) xi' - xi + c (xj - xi) + ui."""
    return System(VDP2, 4, 2, dt, nsub, (float(coupling),))


def cstr(dt: float = 0.1, nsub: int = 1, q: float = 100.0, V: float = 100.0,
         cAf: float = 1.0, Tf: float = 350.0, E_over_R: float = 8750.0, k0: float = 7.2e10,
         minus_dH: float = 5.0e4, UA: float = 5.0e4, cp: float = 0.239,
         rho: float = 1000.0) -> System:
    """The CSTR of Sec. 4.1 (Eq. 4), state (cA [mol/L], T [K]), input the
    coolant temperature Tc [K]; defaults are Table 2 and the sampling interval
    h = 0.1 min, one RK4 step per interval:
        cA' = q/V (cAf - cA) - k0 exp(-(E/R) / T) cA
        T'  = q/V (Tf - T) + (-dH)/(rho cp) k0 exp(-(E/R) / T) cA + UA/(V rho cp) (Tc - T)
    Parameters packed as (q/V, cAf, Tf, E/R, k0, -dH/(rho cp), UA/(V rho cp))."""
    return System(CSTR, 2, 1, float(dt), int(nsub),
                  (q / V, float(cAf), float(Tf), float(E_over_R), float(k0),
                   minus_dH / (rho * cp), UA / (V * rho * cp)))


def user(body: str, n: int, m: int, dt: float, nsub: int,
         params: Sequence[float] = ()) -> System:
    """x+ = RK4^nsub(x, u) of the field whose code is `body` (Eq. 1 with the
    caller's f): C statements setting dx[0..n-1] from x[0..n-1], u[0..m-1]
    and p[0..23], all of type R; fmaT(a, b, c) and expT(v) may be called.
    Written in the common subset of C and C++ (casts as (R)v), it compiles
    both for the device and for the CPU oracle."""
    assert 1 <= n <= 4 and 1 <= m <= 2 and len(params) <= 24
    return System(USER, n, m, float(dt), int(nsub), tuple(float(v) for v in params), body)


def linear(A: Sequence[Sequence[float]], B: Sequence[Sequence[float]], dt: float,
           nsub: int) -> System:
    """x' = A x + B u (n <= 4, m <= 2); parameters packed as A (stride 4) then B (stride 2)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    n, m = A.shape[0], B.shape[1]
    assert A.shape == (n, n) and B.shape[0] == n and n <= 4 and m <= 2
    p = np.zeros(24)
    for d in range(n):
        p[4 * d: 4 * d + n] = A[d]
        p[16 + 2 * d: 16 + 2 * d + m] = B[d]
    return System(LINEAR, n, m, float(dt), int(nsub), tuple(float(v) for v in p))


# ---------------------------------------------------------------- inputs
def evenly_spaced(a: float, b: float, K: int) -> np.ndarray:
    """K values a + (b - a) k / (K - 1), endpoints included (K x 1)."""
    if K == 1:
        return np.array([[float(a)]])
    k = np.arange(K, dtype=np.float64)
    return (((b - a) * k) / (K - 1) + a).reshape(K, 1)


def input_grid(a: float, b: float, per_dim: int, m: int) -> np.ndarray:
    """Cartesian product of evenly spaced values, row-major, first input slowest."""
    axis = evenly_spaced(a, b, per_dim)[:, 0]
    mesh = np.meshgrid(*([axis] * m), indexing="ij")
    return np.stack([g.reshape(-1) for g in mesh], axis=1)


# ---------------------------------------------------------------- named workloads
VDP_BOX = ((-2.5, -3.0), (2.5, 3.0))


def vdp_uniform_64() -> Workload:
    """Controlled Van der Pol on a uniform 64x64 grid, 11 inputs on [-1, 1], FP64."""
    return Workload("vdp_uniform_64x64", vdp(), Grid((64, 64), *VDP_BOX),
                    evenly_spaced(-1.0, 1.0, 11), LATTICE3, 0, "fp64")


def vdp_adaptive_32(precision: str = "fp32_recheck") -> Workload:
    """Van der Pol, 32x32 coarse grid, 5 boundary-only refinement rounds, 21 inputs."""
    return Workload("vdp_adaptive_32x32_r5", vdp(), Grid((32, 32), *VDP_BOX),
                    evenly_spaced(-1.0, 1.0, 21), LATTICE3, 5, precision,
                    analysis="nonleaving")


def vdp_standard_32(precision: str = "fp32_recheck") -> Workload:
    """Van der Pol, 32x32 coarse grid, 6 rounds of the standard algorithm
    (every kept cell halved, dimensions cycled: 256x256 cells at the end),
    21 inputs: the baseline that the adaptive workload is compared with."""
    return Workload("vdp_standard_32x32_r6", vdp(), Grid((32, 32), *VDP_BOX),
                    evenly_spaced(-1.0, 1.0, 21), LATTICE3, 6, precision,
                    analysis="nonleaving", subdivision="bisect")


def lorenz_uniform_128() -> Workload:
    """Lorenz-type system on a uniform 128^3 grid, 21 inputs on [-10, 10]."""
    return Workload("lorenz_uniform_128^3", lorenz(),
                    Grid((128, 128, 128), (-20.0, -25.0, 0.0), (20.0, 25.0, 50.0)),
                    evenly_spaced(-10.0, 10.0, 21), CORNERS_CENTER, 0, "fp32_recheck")


def vdp2_adaptive_32() -> Workload:
    """Two coupled Van der Pol oscillators, 32^4 coarse grid + 2 boundary rounds, 7x7 inputs."""
    return Workload("vdp2_adaptive_32^4_r2", vdp2(),
                    Grid((32, 32, 32, 32), (-2.5, -3.0, -2.5, -3.0), (2.5, 3.0, 2.5, 3.0)),
                    input_grid(-1.0, 1.0, 7, 2), CORNERS_CENTER, 2, "fp32_recheck",
                    analysis="nonleaving")


def vdp2_adaptive_32_r1() -> Workload:
    """The coupled Van der Pol workload with one boundary round instead of two."""
    wl = vdp2_adaptive_32()
    return dataclasses.replace(wl, name="vdp2_adaptive_32^4_r1", rounds=1)


CSTR_BOX = ((0.0, 345.0), (1.0, 355.0))   # 0 <= cA <= 1 mol/L, 345 <= T <= 355 K (Sec. 4.1)
CSTR_U = (285.0, 315.0)                   # 285 <= Tc <= 315 K


def cstr_adaptive(nn: int = 3, rounds: int = 10, n0: int = 8, K: int = 31,
                  precision: str = "fp64") -> Workload:
    """The CSTR of Sec. 4.1 with adaptive subdivision: an n0 x n0 coarse grid
    of X, K coolant temperatures evenly spaced on U, the boundary cells and
    their nn nearest kept cells split into 4 children per round (Sec. 3.1).
    A round halves the finest width in both dimensions, as two iterations of
    the standard algorithm do, so 10 rounds match the paper's 20 iterations."""
    return Workload(f"cstr_adaptive_{n0}x{n0}_r{rounds}_n{nn}", cstr(),
                    Grid((n0, n0), *CSTR_BOX), evenly_spaced(*CSTR_U, K), LATTICE3, rounds,
                    precision, analysis="nonleaving", nn=nn)


def cstr_standard(rounds: int = 20, n0: int = 8, K: int = 31,
                  precision: str = "fp64") -> Workload:
    """The CSTR with the standard algorithm (every kept cell halved, the cut
    dimension cycled: Sec. 2.1; the paper's N = 1000 case of Sec. 4.2, where
    all cells are subdivided), on the grid and inputs of cstr_adaptive."""
    return Workload(f"cstr_standard_{n0}x{n0}_r{rounds}", cstr(), Grid((n0, n0), *CSTR_BOX),
                    evenly_spaced(*CSTR_U, K), LATTICE3, rounds, precision,
                    analysis="nonleaving", subdivision="bisect")


def scaled_vdp_box(scale: float) -> Tuple[Tuple[float, ...], Tuple[float, ...]]:
    return ((-2.5 * scale, -3.0 * scale), (2.5 * scale, 3.0 * scale))


@dataclasses.dataclass(frozen=True)
class ServeRequest:
    rid: int
    arrival_s: float
    workload: Workload
    n_queries: int
    query_seed: int

    @property
    def queries(self) -> np.ndarray:
        """n_queries x n float64 states, uniform in the request's box (seeded)."""
        return query_states(self.workload.grid, self.n_queries, seed=self.query_seed)

    @property
    def kinds(self) -> np.ndarray:
        """Query kinds alternating 0 (membership) and 1 (admissible-input mask)."""
        return (np.arange(self.n_queries) % 2).astype(np.uint8)


def serving_stream(n_requests: int, rate_per_s: float, seed: int = 0,
                   n_queries: int = 100_000,
                   sides: Sequence[int] = (32, 64, 128, 256)) -> list:
    """Poisson arrivals of Van der Pol solves with mu ~ U[0.5, 2], box scale
    ~ U[0.6, 1], grid side uniform over `sides`, 11 inputs on [-1, 1], and
    n_queries uniform query states in the request's box alternating between
    the two query kinds (generated on demand from the recorded seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        mu = rng.uniform(0.5, 2.0)
        s = rng.uniform(0.6, 1.0)
        side = int(sides[rng.integers(0, len(sides))])
        lo, hi = scaled_vdp_box(s)
        wl = Workload(f"serve_{rid}", vdp(mu=mu), Grid((side, side), lo, hi),
                      evenly_spaced(-1.0, 1.0, 11), LATTICE3, 0, "fp64")
        reqs.append(ServeRequest(rid, t, wl, n_queries, seed * 1_000_003 + rid + 1))
    return reqs


def query_states(grid: Grid, count: int, seed: int, margin: float = 0.0) -> np.ndarray:
    """count states uniform in the box enlarged by `margin` (relative) per side."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = np.asarray(grid.lo, dtype=np.float64)
    hi = np.asarray(grid.hi, dtype=np.float64)
    w = hi - lo
    return rng.uniform(lo - margin * w, hi + margin * w, size=(count, grid.n))


def random_linear(seed: int, n: int, m: int) -> System:
    """A seeded random linear system x' = A x + B u for property tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.uniform(-1.0, 1.0, size=(n, n)) - 0.5 * np.eye(n)
    B = rng.uniform(-1.0, 1.0, size=(n, m))
    return linear(A, B, dt=0.1, nsub=2)


ALL = {
    "vdp_uniform_64x64": vdp_uniform_64,
    "vdp_adaptive_32x32_r5": vdp_adaptive_32,
    "vdp_standard_32x32_r6": vdp_standard_32,
    "lorenz_uniform_128^3": lorenz_uniform_128,
    "vdp2_adaptive_32^4_r2": vdp2_adaptive_32,
    "vdp2_adaptive_32^4_r1": vdp2_adaptive_32_r1,
    "cstr_adaptive_8x8_r10_n3": cstr_adaptive,
    "cstr_standard_8x8_r20": cstr_standard,
}


def sample_count(samples: str, n: int) -> int:
    return 3 ** n if samples == LATTICE3 else 2 ** n + 1


def mask_words(K: int) -> int:
    return (K + 63) // 64


def canonical_flops_per_row(system: System, samples: str) -> int:
    """Algorithmic flop count of one (cell, input) image: S samples x nsub
    substeps x (4 F + 12 n), F = flops of one field evaluation in its
    canonical operation order (an FMA counts two)."""
    # CSTR: the division (E/R)/T (1), exp (1 multiply, 2 + 13 FMAs: 31), the
    # rate (2), cA' (3), T' (7); negations are free, as in the other fields
    F = {VDP: 6, LORENZ: 9, VDP2: 16, CSTR: 44}.get(system.kind)
    if F is None:  # linear: n (m + n) FMAs
        F = 2 * system.n * (system.m + system.n)
    return sample_count(samples, system.n) * system.nsub * (4 * F + 12 * system.n)
