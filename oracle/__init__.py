"""CPU oracle of the GIS graph-construction path -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
import this package.  It wraps gis_oracle.c (plain single-threaded FP64 C,
compiled with gcc -ffp-contract=off) through ctypes and composes its steps
into the paper's iteration loop (Sec. 2 and Sec. 3.1 of Decardi-Nelson and
Liu, arXiv 2202.06111).  It shares no code with the HIP library.

Parity status per function (what pins each one is in tests/test_oracle_*.py):
  step / images   pinned: RK4 closed form on linear fields, scipy integration
                  of the stated ODEs, 4th-order error ratio; the CSTR field
                  (Sec. 4.1, Eq. 4) also by the RK4 stability polynomial on
                  its linear and isothermal special cases, its energy-balance
                  invariant and its textbook steady state
  exp             pinned: the C library's exp within 1 ulp, exact powers of
                  two, overflow, underflow and NaN
  user fields     the caller's field code compiled for the host (gcc, FP64,
                  no contraction); pinned: the built-in fields written as
                  user code give the same bits, and a field outside the
                  built-ins (Duffing) against scipy DOP853 and the 4th-order
                  error ratio
  cover           pinned: exact rational brute force on dyadic grids
  build           pinned: identity-map stencil, brute-force box/cell overlap
  prune           pinned: brute-force subset enumeration, drift/contraction
                  special cases, 1-D linear closed-form invariant interval,
                  textbook non-leaving set via strongly connected components
  neighbours      pinned: the 5x5 worked example of Sec. 3.1.2 (Figure 5);
                  brute force with exact rational centre distances on
                  dyadic mixed-level coverings; closed-form nearest cells on
                  a grid of non-square cells
  boundary        pinned: the 5x5 worked example of Sec. 3.1.1 and Remark 1;
                  Algorithm 1 evaluated literally in exact rationals (enlarged
                  cells, vertex and edge-point probes) on random mixed-level
                  coverings with holes
  subdivide/solve pinned: union preservation and monotone shrinking
  largest_scc     pinned: hand-built graphs, brute-force transitive closure
                  on random small graphs, inclusion in the non-leaving set
  bisect          pinned: hand-derived 2x2 example, exact halving of every
                  kept cell, loop with nothing removed = the uniform grid
  query           pinned: brute-force point location over the cell list
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gis_oracle.c")
_LIB = os.path.join(_HERE, "libgis_oracle.so")

_KINDS = {"linear": 0, "vdp": 1, "lorenz": 2, "vdp2": 3, "cstr": 4, "user": 5}
_SCHEMES = {"lattice3": 1, "corners_center": 2}
_RULES = {"shell": 1, "corners": 2}


def build() -> str:
    """Compile the oracle with gcc (FP64, no contraction, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Sys(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("nsub", ctypes.c_int32), ("dt", ctypes.c_double), ("p", ctypes.c_double * 32)]


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n0", ctypes.c_int32 * 4),
                ("lo", ctypes.c_double * 4), ("hi", ctypes.c_double * 4)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        # global symbols: a user field's library calls or_exp
        lib = ctypes.CDLL(_LIB, mode=ctypes.RTLD_GLOBAL)
        P = ctypes.c_void_p
        I32, I64 = ctypes.c_int32, ctypes.c_int64
        lib.or_step.argtypes = [P, P, P, P]
        lib.or_exp_vec.argtypes = [P, I64, P]
        lib.or_set_user_field.argtypes = [P]
        lib.or_num_samples.argtypes = [I32, I32]
        lib.or_num_samples.restype = I32
        lib.or_images.argtypes = [P, P, I32, P, P, I64, P, I32, P]
        lib.or_cover.argtypes = [P, I32, P, P, P, P]
        lib.or_cover.restype = I32
        lib.or_max_level.argtypes = [P, I64]
        lib.or_max_level.restype = I32
        lib.or_build.argtypes = [P, P, I32, P, P, I64, P, I32, I32, P, I64, P, P, P]
        lib.or_build.restype = I64
        lib.or_free.argtypes = [P]
        lib.or_bboxes.argtypes = [P, P, I32, P, P, P, I32, P, I64, P, P, P]
        lib.or_prune.argtypes = [P, P, P, I64, I32, I32, P, P, I32]
        lib.or_prune.restype = I32
        lib.or_boundary.argtypes = [P, P, P, I64, P, I32, P]
        lib.or_boundary.restype = I32
        lib.or_neighbours.argtypes = [P, P, P, I64, P, P, I32, P]
        lib.or_neighbours.restype = I32
        lib.or_subdivide.argtypes = [P, P, P, I64, P, P, P, P, I64]
        lib.or_subdivide.restype = I64
        lib.or_query.argtypes = [P, P, P, I64, P, P, I32, P, I64, P, P]
        lib.or_query.restype = I32
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


_TWIN = r'''/* CPU twin of a user field, written by oracle/__init__.py: the field's
 * code compiled as C99 in FP64, operation by operation. */
#include <math.h>
typedef double R;
double or_exp(double x);
static double fmaT(double a, double b, double c) { return fma(a, b, c); }
static double expT(double v) { return or_exp(v); }
void user_field_twin(const double* p, const double* x, const double* u, double* dx) {
  (void)p; (void)x; (void)u;
#line 1 "user field"
%s
}
'''
_twins = {}   # body -> (library, function pointer)
_twin_dir = None


def _install_user_field(body: str) -> None:
    """Compiles the body of a user field for the host (gcc, FP64, no
    contraction, like the oracle) and installs it as the oracle's field of
    kind "user"."""
    global _twin_dir
    lib = _load()
    if body not in _twins:
        import hashlib
        import tempfile
        if _twin_dir is None:
            _twin_dir = tempfile.mkdtemp(prefix="gis_oracle_fields_")
        key = hashlib.sha256(body.encode()).hexdigest()[:16]
        src = os.path.join(_twin_dir, f"field_{key}.c")
        so = os.path.join(_twin_dir, f"field_{key}.so")
        with open(src, "w") as f:
            f.write(_TWIN % body)
        subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-o", so, src, "-lm"], check=True)
        twin = ctypes.CDLL(so)
        _twins[body] = (twin, ctypes.cast(twin.user_field_twin, ctypes.c_void_p).value)
    lib.or_set_user_field(_twins[body][1])


def _sys(system) -> _Sys:
    if system.kind == "user":
        if not system.source:
            raise ValueError("the oracle needs the code of a user field")
        _install_user_field(system.source)
    s = _Sys()
    s.kind = _KINDS[system.kind]
    s.n, s.m, s.nsub, s.dt = system.n, system.m, system.nsub, system.dt
    p = np.zeros(32)
    p[: len(system.params)] = system.params
    for i in range(32):
        s.p[i] = p[i]
    return s


def _grid(grid) -> _Grid:
    g = _Grid()
    g.n = grid.n
    for d in range(grid.n):
        g.n0[d] = grid.n0[d]
        g.lo[d] = grid.lo[d]
        g.hi[d] = grid.hi[d]
    return g


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def mask_words(K: int) -> int:
    return (K + 63) // 64


# ------------------------------------------------------------------ steps
def step(system, x: np.ndarray, u: np.ndarray) -> np.ndarray:
    """x+ = f(x, u) of Eq. (1) for one state (nsub RK4 substeps)."""
    lib = _load()
    s = _sys(system)
    x = _c(x, np.float64)
    u = _c(u, np.float64)
    y = np.zeros(system.n)
    lib.or_step(ctypes.byref(s), _ptr(x), _ptr(u), _ptr(y))
    return y


def exp(x: np.ndarray) -> np.ndarray:
    """The oracle's own exponential (Cody-Waite reduction + degree-13 Taylor
    polynomial), used by the CSTR field of Sec. 4.1."""
    x = _c(np.atleast_1d(x), np.float64)
    y = np.zeros_like(x)
    _load().or_exp_vec(_ptr(x), x.size, _ptr(y))
    return y


def num_samples(samples: str, n: int) -> int:
    return int(_load().or_num_samples(_SCHEMES[samples], n))


def coarse_cells(grid):
    """The full coarse covering C_{d_0}: every level-0 cell, row-major."""
    axes = [np.arange(k, dtype=np.int32) for k in grid.n0]
    mesh = np.meshgrid(*axes, indexing="ij")
    idx = np.stack([g.reshape(-1) for g in mesh], axis=1).astype(np.int32)
    level = np.zeros(idx.shape[0], dtype=np.uint8)
    return level, np.ascontiguousarray(idx)


def images(system, grid, samples: str, level, idx, u) -> np.ndarray:
    """Sample images of every row: array [n_cells*K, S, n]."""
    lib = _load()
    level, idx, u = _c(level, np.uint8), _c(idx, np.int32), _c(u, np.float64)
    K = u.shape[0]
    S = num_samples(samples, grid.n)
    out = np.zeros((level.shape[0] * K, S, grid.n))
    s, g = _sys(system), _grid(grid)
    lib.or_images(ctypes.byref(s), ctypes.byref(g), _SCHEMES[samples], _ptr(level), _ptr(idx),
                  level.shape[0], _ptr(u), K, _ptr(out))
    return out


def bboxes(system, grid, samples: str, level, idx, u, rows):
    lib = _load()
    level, idx, u = _c(level, np.uint8), _c(idx, np.int32), _c(u, np.float64)
    rows = _c(rows, np.int64)
    a = np.zeros((rows.shape[0], grid.n))
    b = np.zeros((rows.shape[0], grid.n))
    fin = np.zeros(rows.shape[0], dtype=np.uint8)
    s, g = _sys(system), _grid(grid)
    lib.or_bboxes(ctypes.byref(s), ctypes.byref(g), _SCHEMES[samples], _ptr(level), _ptr(idx),
                  _ptr(u), u.shape[0], _ptr(rows), rows.shape[0], _ptr(a), _ptr(b), _ptr(fin))
    return a, b, fin.astype(bool)


def cover(grid, Lstar: int, a, b):
    """Closed range R, interior range Ri (each [n,2] int64) and OUT_X of a box."""
    lib = _load()
    a, b = _c(a, np.float64), _c(b, np.float64)
    R = np.zeros((grid.n, 2), dtype=np.int64)
    Ri = np.zeros((grid.n, 2), dtype=np.int64)
    g = _grid(grid)
    outx = lib.or_cover(ctypes.byref(g), Lstar, _ptr(a), _ptr(b), _ptr(R), _ptr(Ri))
    return R, Ri, bool(outx)


def build_graph(system, grid, samples: str, level, idx, u, fast_out: bool = False, rows=None):
    """Symbolic image of the covering (Definition 1) with OUT flags.

    rows=None: every row; returns dict(row_ptr, col, out).
    rows=array: only those rows; returns dict(cnt, col, out) with col the
    concatenation of the rows' edge lists in the given order."""
    lib = _load()
    level, idx, u = _c(level, np.uint8), _c(idx, np.int32), _c(u, np.float64)
    K = u.shape[0]
    n_cells = level.shape[0]
    if rows is not None:
        rows = _c(rows, np.int64)
        n_rows = rows.shape[0]
    else:
        n_rows = n_cells * K
    cnt = np.zeros(n_rows, dtype=np.int64)
    out = np.zeros(n_rows, dtype=np.uint8)
    colp = ctypes.c_void_p()
    s, g = _sys(system), _grid(grid)
    total = lib.or_build(ctypes.byref(s), ctypes.byref(g), _SCHEMES[samples], _ptr(level),
                         _ptr(idx), n_cells, _ptr(u), K, int(fast_out), _ptr(rows), n_rows,
                         _ptr(cnt), _ptr(out), ctypes.byref(colp))
    if total < 0:
        raise ValueError(f"oracle build failed ({total}): invalid covering or out of memory")
    col = np.zeros(total, dtype=np.int32)
    if total > 0:
        ctypes.memmove(col.ctypes.data, colp.value, total * 4)
    lib.or_free(colp)
    if rows is not None:
        return {"cnt": cnt, "col": col, "out": out}
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(cnt, out=row_ptr[1:])
    return {"row_ptr": row_ptr, "col": col, "out": out}


_ANALYSES = {"controlled": 1, "nonleaving": 2}


def prune(row_ptr, col, out, n_cells: int, K: int, analysis: str = "controlled"):
    """Graph analysis of Sec. 2.3: kept cells K* and per-cell input masks.

    analysis="controlled": largest set in which every cell has an input whose
    image is not OUT and whose edges all end in the set.
    analysis="nonleaving": vertices with an infinite admissible path in the
    input-union symbolic image (Definitions 5-6).
    analysis="largest_scc": Definition 6 read literally (largest_scc)."""
    if analysis == "largest_scc":
        kept, mask = largest_scc(row_ptr, col, n_cells, K)
        return kept, mask, 0
    lib = _load()
    row_ptr, col, out = _c(row_ptr, np.int64), _c(col, np.int32), _c(out, np.uint8)
    W = mask_words(K)
    kept = np.zeros(n_cells, dtype=np.uint8)
    mask = np.zeros((n_cells, W), dtype=np.uint64)
    sweeps = lib.or_prune(_ptr(row_ptr), _ptr(col), _ptr(out), n_cells, K,
                          _ANALYSES[analysis], _ptr(kept), _ptr(mask), W)
    return kept, mask, int(sweeps)


def largest_scc(row_ptr, col, n_cells: int, K: int):
    """Definition 6 read literally (Sec. 2.3): the vertices of the largest
    strongly connected component of the input-union symbolic image, plus
    every vertex with a path into it.  Only components with an infinite path
    through them count (two or more vertices, or one with an edge to itself);
    none: the set is empty.  Equally large components: the one holding the
    smallest cell id.  Mask bit u of a kept cell: row (cell, u) has an edge
    into the set.  The components come from scipy's strongly connected
    components; the rest is written out below."""
    from collections import deque
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    row_ptr, col = _c(row_ptr, np.int64), _c(col, np.int64)
    rows = np.arange(n_cells * K, dtype=np.int64)
    src = np.repeat(rows // K, np.diff(row_ptr))
    A = csr_matrix((np.ones(col.shape[0], dtype=np.int8), (src, col)), shape=(n_cells, n_cells))
    _, label = connected_components(A, directed=True, connection="strong")
    members = {}
    for c in range(n_cells):
        members.setdefault(int(label[c]), []).append(c)
    self_loop = set(int(v) for v in src[src == col])
    best = None
    for comp in members.values():  # comp is ascending: comp[0] is its smallest id
        if len(comp) < 2 and comp[0] not in self_loop:
            continue
        if best is None or len(comp) > len(best) or (len(comp) == len(best) and comp[0] < best[0]):
            best = comp
    kept = np.zeros(n_cells, dtype=np.uint8)
    if best is not None:
        preds = [[] for _ in range(n_cells)]
        for a, b in zip(src.tolist(), col.tolist()):
            preds[b].append(a)
        todo = deque(best)
        for c in best:
            kept[c] = 1
        while todo:
            v = todo.popleft()
            for a in preds[v]:
                if not kept[a]:
                    kept[a] = 1
                    todo.append(a)
    W = mask_words(K)
    mask = np.zeros((n_cells, W), dtype=np.uint64)
    for r in range(n_cells * K):
        c, u = divmod(r, K)
        if kept[c] and kept[col[row_ptr[r]:row_ptr[r + 1]]].any():
            mask[c, u // 64] |= np.uint64(1) << np.uint64(u % 64)
    return kept, mask


def boundary(grid, level, idx, kept, rule: str = "shell") -> np.ndarray:
    lib = _load()
    level, idx, kept = _c(level, np.uint8), _c(idx, np.int32), _c(kept, np.uint8)
    bnd = np.zeros(level.shape[0], dtype=np.uint8)
    g = _grid(grid)
    rc = lib.or_boundary(ctypes.byref(g), _ptr(level), _ptr(idx), level.shape[0], _ptr(kept),
                         _RULES[rule], _ptr(bnd))
    if rc != 0:
        raise ValueError(f"oracle boundary failed ({rc})")
    return bnd


def neighbours(grid, level, idx, kept, bnd, N: int) -> np.ndarray:
    """Cells selected for subdivision with a neighbourhood (Sec. 3.1.2): the
    boundary cells and, for each, the N kept cells with the nearest centres
    (the cell itself excluded; equal distances ordered by cell id)."""
    lib = _load()
    level, idx = _c(level, np.uint8), _c(idx, np.int32)
    kept, bnd = _c(kept, np.uint8), _c(bnd, np.uint8)
    sel = np.zeros(level.shape[0], dtype=np.uint8)
    g = _grid(grid)
    rc = lib.or_neighbours(ctypes.byref(g), _ptr(level), _ptr(idx), level.shape[0], _ptr(kept),
                           _ptr(bnd), int(N), _ptr(sel))
    if rc != 0:
        raise ValueError(f"oracle neighbourhood failed ({rc})")
    return sel


def subdivide(grid, level, idx, kept, bnd):
    lib = _load()
    level, idx = _c(level, np.uint8), _c(idx, np.int32)
    kept, bnd = _c(kept, np.uint8), _c(bnd, np.uint8)
    g = _grid(grid)
    need = lib.or_subdivide(ctypes.byref(g), _ptr(level), _ptr(idx), level.shape[0], _ptr(kept),
                            _ptr(bnd), None, None, 0)
    lv = np.zeros(max(need, 1), dtype=np.uint8)
    ix = np.zeros((max(need, 1), grid.n), dtype=np.int32)
    got = lib.or_subdivide(ctypes.byref(g), _ptr(level), _ptr(idx), level.shape[0], _ptr(kept),
                           _ptr(bnd), _ptr(lv), _ptr(ix), need)
    assert got == need
    return lv[:need].copy(), ix[:need].copy()


def bisect(grid, idx, kept, dim: int):
    """Subdivision step of the standard algorithm (Sec. 2.1): every kept cell
    of a level-0 covering is cut in half across dimension `dim`.  The halves
    are the level-0 cells of the grid with twice as many cells along `dim`
    (same box X), returned with that grid, in canonical (row-major) order."""
    idx, kept = _c(idx, np.int32), _c(kept, np.uint8)
    n = grid.n
    n0 = list(grid.n0)
    n0[dim] *= 2
    new_grid = type(grid)(tuple(n0), tuple(grid.lo), tuple(grid.hi))
    halves = []
    for c in np.nonzero(kept)[0]:
        for h in (0, 1):
            k = [int(v) for v in idx[c]]
            k[dim] = 2 * k[dim] + h
            halves.append(tuple(k))
    halves.sort()  # lexicographic on (i_0, ..., i_{n-1}): dimension 0 slowest
    out = np.array(halves, dtype=np.int32).reshape(len(halves), n)
    return new_grid, np.zeros(len(halves), dtype=np.uint8), out


def query(grid, level, idx, kept, mask, states):
    lib = _load()
    level, idx, kept = _c(level, np.uint8), _c(idx, np.int32), _c(kept, np.uint8)
    mask = _c(mask, np.uint64)
    states = _c(states, np.float64)
    W = mask.shape[1]
    member = np.zeros(states.shape[0], dtype=np.uint8)
    adm = np.zeros((states.shape[0], W), dtype=np.uint64)
    g = _grid(grid)
    rc = lib.or_query(ctypes.byref(g), _ptr(level), _ptr(idx), level.shape[0], _ptr(kept),
                      _ptr(mask), W, _ptr(states), states.shape[0], _ptr(member), _ptr(adm))
    if rc != 0:
        raise ValueError(f"oracle query failed ({rc})")
    return member, adm


def solve(system, grid, samples: str, u, rounds: int, rule: str = "shell",
          fast_out: bool = False, keep_graphs: bool = False, analysis: str = "controlled",
          subdivision: str = "boundary", nn: int = 0):
    """The iteration loop: build and prune on the coarse covering, then
    `rounds` times subdivide, rebuild and prune.  subdivision "boundary":
    the 2^n children of the boundary cells (Sec. 3.1); "bisect": the
    standard algorithm's halving of every kept cell (Sec. 2.1), across
    dimension 0 in the first subdivision, 1 in the second, ... cyclically.
    nn > 0 ("boundary" only): the nn kept cells nearest to each boundary cell
    are subdivided as well (Sec. 3.1.2).  Stops early when nothing is kept.  The result holds the grid of the
    final covering (the coarse grid unless cells were bisected)."""
    u = _c(u, np.float64)
    K = u.shape[0]
    level, idx = coarse_cells(grid)
    stats = []
    graphs = []
    kept = mask = None
    for r in range(rounds + 1):
        if r > 0:
            if subdivision == "bisect":
                grid, level, idx = bisect(grid, idx, kept, (r - 1) % grid.n)
                stats[-1]["n_boundary"] = int(kept.sum())
            else:
                bnd = boundary(grid, level, idx, kept, rule)
                sel = neighbours(grid, level, idx, kept, bnd, nn) if nn > 0 else bnd
                level, idx = subdivide(grid, level, idx, kept, sel)
                stats[-1]["n_boundary"] = int(bnd.sum())
                stats[-1]["n_selected"] = int(sel.sum())
        if level.shape[0] == 0:
            break
        g = build_graph(system, grid, samples, level, idx, u, fast_out=fast_out)
        kept, mask, sweeps = prune(g["row_ptr"], g["col"], g["out"], level.shape[0], K, analysis)
        stats.append({"round": r, "n_cells": int(level.shape[0]), "n_rows": int(level.shape[0] * K),
                      "n_edges": int(g["col"].shape[0]), "n_out": int(g["out"].sum()),
                      "n_kept": int(kept.sum()), "sweeps": sweeps, "n0": tuple(grid.n0)})
        if keep_graphs:
            graphs.append(g)
        if kept.sum() == 0:
            break
    res = {"level": level, "idx": idx, "kept": kept, "mask": mask, "stats": stats, "grid": grid}
    if keep_graphs:
        res["graphs"] = graphs
    return res
