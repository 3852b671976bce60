"""Python binding of libgis (the C ABI of include/gis.h).

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch provides device memory (tensors passed by data_ptr()) and streams
(torch.cuda.current_stream().cuda_stream).  Importing this module loads the
library and fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import workloads as W

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgis.so")

KIND = {W.LINEAR: 0, W.VDP: 1, W.LORENZ: 2, W.VDP2: 3, W.CSTR: 4, W.USER: 5}
SAMPLES = {W.LATTICE3: 1, W.CORNERS_CENTER: 2}
PRECISION = {"fp64": 1, "fp32_recheck": 2}
RULE = {W.SHELL: 1, W.CORNERS: 2}
ANALYSIS = {"controlled": 1, "nonleaving": 2, "largest_scc": 3}
SUBDIVISION = {"boundary": 0, "bisect": 1}
STATUS = {0: "GIS_OK", 1: "GIS_E_INVAL", 2: "GIS_E_NOMEM", 3: "GIS_E_HIP", 4: "GIS_E_CAPACITY",
          5: "GIS_E_UNSUPPORTED", 6: "GIS_E_INTERNAL"}
MAX_ROUNDS = 32

P = ctypes.c_void_p
I32, I64, F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class SystemT(ctypes.Structure):
    _fields_ = [("kind", I32), ("n", I32), ("m", I32), ("nsub", I32), ("dt", F64),
                ("params", F64 * 32)]


class GridT(ctypes.Structure):
    _fields_ = [("n", I32), ("n0", I32 * 4), ("lo", F64 * 4), ("hi", F64 * 4)]


class OptsT(ctypes.Structure):
    _fields_ = [("samples", I32), ("precision", I32), ("boundary_rule", I32), ("analysis", I32),
                ("fast_out", I32), ("timing", I32), ("subdivision", I32), ("check_band", I32),
                ("neighbours", I32), ("reserved", I32), ("band", F64 * 4)]


class CellsT(ctypes.Structure):
    _fields_ = [("n_cells", I64), ("cap", I64), ("level", P), ("idx", P)]


class GraphT(ctypes.Structure):
    _fields_ = [("n_rows", I64), ("n_edges", I64), ("n_out", I64), ("n_recheck", I64),
                ("cap_edges", I64), ("row_ptr", P), ("col", P), ("out", P)]


class TuningT(ctypes.Structure):
    _fields_ = [("first_sweeps", I32), ("sweep_batch", I32), ("sweep_edges", I64),
                ("frontier_batch", I32), ("sweep_blocks", I32), ("front_blocks", I32),
                ("use_graphs", I32), ("edge_hint", I32), ("row_frontier", I32),
                ("wit_sweeps", I32)]


TUNING_FIELDS = ("first_sweeps", "sweep_batch", "sweep_edges", "frontier_batch", "sweep_blocks",
                 "front_blocks", "use_graphs", "edge_hint", "row_frontier", "wit_sweeps")


class JobT(ctypes.Structure):
    _fields_ = [("sys", SystemT), ("grid", GridT), ("d_u", P)]


class RoundStatsT(ctypes.Structure):
    _fields_ = [("n_cells", I64), ("n_rows", I64), ("n_edges", I64), ("n_out", I64),
                ("n_kept", I64), ("n_boundary", I64), ("n_recheck", I64), ("max_level", I32),
                ("reserved", I32), ("ms_build", F64), ("ms_prune", F64), ("ms_subdivide", F64),
                ("ms_image", F64), ("ms_recheck", F64), ("ms_host", F64), ("ms_host_wait", F64),
                ("band", F64 * 4), ("max_err", F64 * 4), ("max_err_all", F64 * 4),
                ("n_selected", I64)]


class SolveInfoT(ctypes.Structure):
    _fields_ = [("n_rounds", I32), ("n", I32), ("K", I32), ("mask_words", I32), ("n0", I32 * 4),
                ("n_cells", I64), ("n_kept", I64), ("band", F64 * 4),
                ("rounds", RoundStatsT * MAX_ROUNDS)]


class GisError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """The loaded libgis.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "gis_ctx_create": ([I32, ctypes.POINTER(P)], I32),
            "gis_ctx_destroy": ([P], None),
            "gis_get_tuning": ([P, P], I32),
            "gis_set_tuning": ([P, P], I32),
            "gis_autotune": ([P, P, P, P, I32, I32, P, I32, P, P, P], I32),
            "gis_build_graph": ([P, P, P, P, I32, P, P, P, P], I32),
            "gis_prune": ([P, P, I64, I32, I32, P, P, P, P], I32),
            "gis_prune_static": ([P, I64, I32, I32, P, P, P, P], I32),
            "gis_exp": ([P, I64, P, P], I32),
            "gis_set_user_field": ([P, ctypes.c_char_p, I32, I32], I32),
            "gis_subdivide": ([P, P, P, P, I32, I32, P, P, P], I32),
            "gis_bisect": ([P, P, P, P, I32, P, P, P], I32),
            "gis_solve": ([P, P, P, P, I32, I32, P, ctypes.POINTER(P), P], I32),
            "gis_solve_batch": ([P, I32, P, I32, I32, P, P, P], I32),
            "gis_solution_info": ([P, P], I32),
            "gis_solution_export": ([P, P, P, P, P], I32),
            "gis_solution_free": ([P], None),
            "gis_query_membership": ([P, P, I64, P, P], I32),
            "gis_query_admissible": ([P, P, I64, P, P], I32),
            "gis_images": ([P, P, P, P, I32, P, I32, I32, P, P], I32),
            "gis_calibrate_band": ([P, P, P, P, I32, P, I32, F64, F64, P, P], I32),
            "gis_last_error": ([], ctypes.c_char_p),
            "gis_version": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


EXPORTED = ("gis_ctx_create", "gis_ctx_destroy", "gis_get_tuning", "gis_set_tuning", "gis_autotune", "gis_build_graph", "gis_prune", "gis_prune_static", "gis_subdivide", "gis_bisect",
            "gis_solve", "gis_solve_batch", "gis_solution_info", "gis_solution_export", "gis_solution_free",
            "gis_query_membership", "gis_query_admissible", "gis_images", "gis_exp", "gis_set_user_field",
            "gis_calibrate_band",
            "gis_last_error", "gis_version")


def _check(rc: int) -> None:
    if rc != 0:
        raise GisError(rc, lib().gis_last_error().decode())


def _stream_ptr(stream=None) -> P:
    s = torch.cuda.current_stream() if stream is None else stream
    return P(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> P:
    return P(0 if t is None else t.data_ptr())


# ------------------------------------------------------------------ structs
def system_t(system: W.System, ctx: Optional["Context"] = None) -> SystemT:
    """The gis_system of a system; a system with its own field code (kind
    "user", non-empty source) first installs that field in ctx
    (gis_set_user_field); with an empty source the context's field is used."""
    if system.kind == W.USER and system.source:
        if ctx is None:
            raise ValueError("a system with a user field needs the context it runs in")
        ctx.use_field(system.source, system.n, system.m)
    s = SystemT()
    s.kind = KIND[system.kind]
    s.n, s.m, s.nsub, s.dt = system.n, system.m, system.nsub, system.dt
    for i, v in enumerate(system.param_array()):
        s.params[i] = float(v)
    return s


def grid_t(grid: W.Grid) -> GridT:
    g = GridT()
    g.n = grid.n
    for d in range(grid.n):
        g.n0[d], g.lo[d], g.hi[d] = grid.n0[d], grid.lo[d], grid.hi[d]
    return g


def opts_t(samples: str = W.LATTICE3, precision: str = "fp64", boundary_rule: str = W.SHELL,
           analysis: str = "controlled", fast_out: bool = False,
           band: Optional[Sequence[float]] = None, timing: int = 0,
           subdivision: str = "boundary", check_band: bool = False,
           neighbours: int = 0) -> OptsT:
    o = OptsT()
    o.samples = SAMPLES[samples]
    o.precision = PRECISION[precision]
    o.boundary_rule = RULE[boundary_rule]
    o.analysis = ANALYSIS[analysis]
    o.fast_out = int(bool(fast_out))
    o.timing = int(timing)
    o.subdivision = SUBDIVISION[subdivision]
    o.check_band = int(bool(check_band))
    o.neighbours = int(neighbours)
    for d, v in enumerate([] if band is None else list(band)):
        o.band[d] = float(v)
    return o


def workload_opts(wl: W.Workload, **over) -> OptsT:
    kw = dict(samples=wl.samples, precision=wl.precision, boundary_rule=wl.boundary_rule,
              analysis=wl.analysis, subdivision=wl.subdivision, neighbours=wl.nn)
    kw.update(over)
    return opts_t(**kw)


# ------------------------------------------------------------------ context
class Context:
    """A libgis context (device workspace) on one device."""

    def __init__(self, device: int = 0):
        self.device = device
        h = P()
        _check(lib().gis_ctx_create(device, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self) -> P:
        if self._h is None:
            raise RuntimeError("context is closed")
        return self._h

    def close(self) -> None:
        if self._h is not None:
            lib().gis_ctx_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dev(self) -> torch.device:
        return torch.device("cuda", self.device)

    def set_user_field(self, body: str, n: int, m: int) -> None:
        """gis_set_user_field: compiles the field body for this context's
        device (kind GIS_SYS_USER)."""
        _check(lib().gis_set_user_field(self.handle, body.encode(), n, m))
        self._field = (body, n, m)

    def use_field(self, body: str, n: int, m: int) -> None:
        """Installs the field unless it is the one installed already."""
        if getattr(self, "_field", None) != (body, n, m):
            self.set_user_field(body, n, m)

    def get_tuning(self) -> dict:
        t = TuningT()
        _check(lib().gis_get_tuning(self.handle, ctypes.byref(t)))
        return {f: int(getattr(t, f)) for f in TUNING_FIELDS}

    def set_tuning(self, **fields) -> dict:
        """Replaces the named schedule parameters; returns the previous set."""
        prev = self.get_tuning()
        t = TuningT()
        for f in TUNING_FIELDS:
            setattr(t, f, int(fields.pop(f, prev[f])))
        if fields:
            raise TypeError(f"unknown tuning fields {sorted(fields)}")
        _check(lib().gis_set_tuning(self.handle, ctypes.byref(t)))
        return prev


def to_device_u(ctx: Context, u) -> torch.Tensor:
    if isinstance(u, torch.Tensor):
        return u.to(device=ctx.dev, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(u, dtype=np.float64), device=ctx.dev)


def cells_t(level: torch.Tensor, idx: torch.Tensor, cap: Optional[int] = None) -> CellsT:
    c = CellsT()
    c.n_cells = int(level.shape[0])
    c.cap = int(level.shape[0] if cap is None else cap)
    c.level = _ptr(level)
    c.idx = _ptr(idx)
    return c


@dataclasses.dataclass
class Graph:
    row_ptr: torch.Tensor
    col: torch.Tensor
    out: torch.Tensor
    n_rows: int
    n_edges: int
    n_out: int
    n_recheck: int

    def graph_t(self) -> GraphT:
        g = GraphT()
        g.n_rows, g.n_edges, g.n_out, g.n_recheck = self.n_rows, self.n_edges, self.n_out, self.n_recheck
        g.cap_edges = int(self.col.shape[0])
        g.row_ptr, g.col, g.out = _ptr(self.row_ptr), _ptr(self.col), _ptr(self.out)
        return g


def coarse_cells(ctx: Context, grid: W.Grid):
    """The full level-0 covering as device tensors (canonical order)."""
    axes = [torch.arange(k, dtype=torch.int32) for k in grid.n0]
    mesh = torch.meshgrid(*axes, indexing="ij")
    idx = torch.stack([m.reshape(-1) for m in mesh], dim=1).contiguous().to(ctx.dev)
    level = torch.zeros(idx.shape[0], dtype=torch.uint8, device=ctx.dev)
    return level, idx


def build_graph(ctx: Context, system: W.System, grid: W.Grid, u, level: torch.Tensor,
                idx: torch.Tensor, opts: OptsT, cap_edges: Optional[int] = None, stream=None) -> Graph:
    """Symbolic image of a covering; grows col and retries once on a capacity miss."""
    du = to_device_u(ctx, u)
    K = int(du.shape[0])
    n_rows = int(level.shape[0]) * K
    row_ptr = torch.empty(n_rows + 1, dtype=torch.int64, device=ctx.dev)
    out = torch.empty(max(n_rows, 1), dtype=torch.uint8, device=ctx.dev)
    cap = int(cap_edges if cap_edges is not None else max(16, 12 * n_rows))
    st, gt, ct = system_t(system, ctx), grid_t(grid), cells_t(level, idx)
    for attempt in range(2):
        col = torch.empty(max(cap, 1), dtype=torch.int32, device=ctx.dev)
        g = GraphT()
        g.cap_edges = cap
        g.row_ptr, g.col, g.out = _ptr(row_ptr), _ptr(col), _ptr(out)
        rc = lib().gis_build_graph(ctx.handle, ctypes.byref(st), ctypes.byref(gt), _ptr(du), K,
                                   ctypes.byref(ct), ctypes.byref(opts), ctypes.byref(g),
                                   _stream_ptr(stream))
        if rc == 4 and attempt == 0:
            cap = int(g.n_edges)
            continue
        _check(rc)
        return Graph(row_ptr, col[: g.n_edges], out[:n_rows], n_rows, int(g.n_edges), int(g.n_out),
                     int(g.n_recheck))
    raise GisError(4, "capacity retry failed")


def prune(ctx: Context, graph: Graph, n_cells: int, K: int, analysis: str = "controlled",
          stream=None):
    """Graph analysis; returns (kept uint8 [n_cells], mask int64 [n_cells, W], n_kept)."""
    Wd = (K + 63) // 64
    kept = torch.empty(max(n_cells, 1), dtype=torch.uint8, device=ctx.dev)
    mask = torch.empty((max(n_cells, 1), Wd), dtype=torch.int64, device=ctx.dev)
    nk = I64(0)
    g = graph.graph_t()
    _check(lib().gis_prune(ctx.handle, ctypes.byref(g), n_cells, K, ANALYSIS[analysis], _ptr(kept),
                           _ptr(mask), ctypes.byref(nk), _stream_ptr(stream)))
    return kept[:n_cells], mask[:n_cells], int(nk.value)


def prune_static(graph: Graph, n_cells: int, K: int, analysis: str = "controlled", stream=None,
                 kept: Optional[torch.Tensor] = None, mask: Optional[torch.Tensor] = None):
    """gis_prune_static: the analysis without device allocation in the
    library (its workspace is a static device array).  kept [n_cells] uint8
    and mask [n_cells, ceil(K/64)] int64 may be passed in, so that the call
    allocates nothing at all; returns (kept, mask, n_kept)."""
    Wd = (K + 63) // 64
    dev = graph.row_ptr.device
    if kept is None:
        kept = torch.empty(max(n_cells, 1), dtype=torch.uint8, device=dev)
    if mask is None:
        mask = torch.empty((max(n_cells, 1), Wd), dtype=torch.int64, device=dev)
    nk = I64(0)
    g = graph.graph_t()
    _check(lib().gis_prune_static(ctypes.byref(g), n_cells, K, ANALYSIS[analysis], _ptr(kept),
                                  _ptr(mask), ctypes.byref(nk), _stream_ptr(stream)))
    return kept[:n_cells], mask[:n_cells], int(nk.value)


def subdivide(ctx: Context, grid: W.Grid, level: torch.Tensor, idx: torch.Tensor,
              kept: torch.Tensor, rule: str = W.SHELL, stream=None, neighbours: int = 0):
    """Boundary selection (with the `neighbours` nearest kept cells of each
    boundary cell) and subdivision; returns (level, idx, boundary flags)."""
    n_cells = int(level.shape[0])
    cap = max(1, int(kept.sum().item()) << grid.n) if n_cells else 1
    lv = torch.empty(cap, dtype=torch.uint8, device=ctx.dev)
    ix = torch.empty((cap, grid.n), dtype=torch.int32, device=ctx.dev)
    bnd = torch.empty(max(n_cells, 1), dtype=torch.uint8, device=ctx.dev)
    cin = cells_t(level, idx)
    cout = cells_t(lv, ix, cap)
    gt = grid_t(grid)
    _check(lib().gis_subdivide(ctx.handle, ctypes.byref(gt), ctypes.byref(cin), _ptr(kept),
                               RULE[rule], int(neighbours), _ptr(bnd), ctypes.byref(cout),
                               _stream_ptr(stream)))
    n = int(cout.n_cells)
    return lv[:n], ix[:n], bnd[:n_cells]


def bisect(ctx: Context, grid: W.Grid, level: torch.Tensor, idx: torch.Tensor,
           kept: torch.Tensor, dim: int, stream=None):
    """Standard subdivision: every kept level-0 cell halved across `dim`;
    returns (grid of the halves, level, idx)."""
    n_cells = int(idx.shape[0])
    cap = max(1, 2 * int(kept.sum().item())) if n_cells else 1
    lv = torch.empty(cap, dtype=torch.uint8, device=ctx.dev)
    ix = torch.empty((cap, grid.n), dtype=torch.int32, device=ctx.dev)
    cin = cells_t(level, idx)
    cout = cells_t(lv, ix, cap)
    gt, go = grid_t(grid), GridT()
    _check(lib().gis_bisect(ctx.handle, ctypes.byref(gt), ctypes.byref(cin), _ptr(kept), int(dim),
                            ctypes.byref(go), ctypes.byref(cout), _stream_ptr(stream)))
    n = int(cout.n_cells)
    return W.Grid(tuple(go.n0[: grid.n]), grid.lo, grid.hi), lv[:n], ix[:n]


def check_user_field(body: str, n: int, m: int) -> None:
    """Compiles a field body for gfx950 without a device (gis_set_user_field
    with no context); raises GisError with the compiler's messages."""
    _check(lib().gis_set_user_field(None, body.encode(), n, m))


def exp(x: torch.Tensor, stream=None) -> torch.Tensor:
    """gis_exp: the library's FP64 exponential (the CSTR field's) on a
    device float64 tensor, elementwise."""
    x = x.contiguous()
    assert x.dtype == torch.float64 and x.is_cuda
    y = torch.empty_like(x)
    _check(lib().gis_exp(_ptr(x), x.numel(), _ptr(y), _stream_ptr(stream)))
    return y


def images(ctx: Context, system: W.System, grid: W.Grid, u, level, idx, samples: str,
           precision: str = "fp64", stream=None) -> torch.Tensor:
    du = to_device_u(ctx, u)
    K = int(du.shape[0])
    S = W.sample_count(samples, grid.n)
    out = torch.empty((int(level.shape[0]) * K, S, grid.n), dtype=torch.float64, device=ctx.dev)
    st, gt, ct = system_t(system, ctx), grid_t(grid), cells_t(level, idx)
    _check(lib().gis_images(ctx.handle, ctypes.byref(st), ctypes.byref(gt), _ptr(du), K,
                            ctypes.byref(ct), SAMPLES[samples], PRECISION[precision], _ptr(out),
                            _stream_ptr(stream)))
    return out


def calibrate_band(ctx: Context, system: W.System, grid: W.Grid, u, level, idx, samples: str,
                   safety: float = 8.0, floor_rel: float = 1e-5, stream=None) -> np.ndarray:
    du = to_device_u(ctx, u)
    band = (F64 * 4)()
    st, gt, ct = system_t(system, ctx), grid_t(grid), cells_t(level, idx)
    _check(lib().gis_calibrate_band(ctx.handle, ctypes.byref(st), ctypes.byref(gt), _ptr(du),
                                    int(du.shape[0]), ctypes.byref(ct), SAMPLES[samples], safety,
                                    floor_rel, band, _stream_ptr(stream)))
    return np.array(band[: grid.n])


def info_dict(inf: SolveInfoT) -> dict:
    """gis_solve_info as a dict with one dict per round."""
    rounds = []
    for r in range(inf.n_rounds):
        s = inf.rounds[r]
        d = {}
        for k, t in RoundStatsT._fields_:
            if k == "reserved":
                continue
            v = getattr(s, k)
            d[k] = list(v[: inf.n]) if isinstance(t, type) and issubclass(t, ctypes.Array) else v
        rounds.append(d)
    return {"n_rounds": inf.n_rounds, "n": inf.n, "K": inf.K, "mask_words": inf.mask_words,
            "n0": tuple(inf.n0[: inf.n]), "n_cells": inf.n_cells, "n_kept": inf.n_kept, "band": list(inf.band[: inf.n]),
            "rounds": rounds}


class Solution:
    """A solve result resident on the device (library-owned handle)."""

    def __init__(self, handle: P, device: int):
        self._h = handle
        self.device = device

    @property
    def handle(self) -> P:
        if self._h is None:
            raise RuntimeError("solution is freed")
        return self._h

    def info_raw(self) -> SolveInfoT:
        """The solve statistics as the C struct (no conversion)."""
        inf = SolveInfoT()
        _check(lib().gis_solution_info(self.handle, ctypes.byref(inf)))
        return inf

    def info(self) -> dict:
        return info_dict(self.info_raw())

    def export(self, stream=None):
        inf = self.info()
        n, nc, Wd = inf["n"], inf["n_cells"], inf["mask_words"]
        dev = torch.device("cuda", self.device)
        lv = torch.empty(max(nc, 1), dtype=torch.uint8, device=dev)
        ix = torch.empty((max(nc, 1), n), dtype=torch.int32, device=dev)
        kept = torch.empty(max(nc, 1), dtype=torch.uint8, device=dev)
        mask = torch.empty((max(nc, 1), Wd), dtype=torch.int64, device=dev)
        c = cells_t(lv, ix, max(nc, 1))
        _check(lib().gis_solution_export(self.handle, ctypes.byref(c), _ptr(kept), _ptr(mask),
                                         _stream_ptr(stream)))
        return lv[:nc], ix[:nc], kept[:nc], mask[:nc]

    def query_membership(self, states: torch.Tensor, stream=None) -> torch.Tensor:
        states = states.to(dtype=torch.float64).contiguous()
        out = torch.empty(max(states.shape[0], 1), dtype=torch.uint8, device=states.device)
        _check(lib().gis_query_membership(self.handle, _ptr(states), int(states.shape[0]),
                                          _ptr(out), _stream_ptr(stream)))
        return out[: states.shape[0]]

    def query_admissible(self, states: torch.Tensor, stream=None) -> torch.Tensor:
        states = states.to(dtype=torch.float64).contiguous()
        Wd = self.info()["mask_words"]
        out = torch.empty((max(states.shape[0], 1), Wd), dtype=torch.int64, device=states.device)
        _check(lib().gis_query_admissible(self.handle, _ptr(states), int(states.shape[0]),
                                          _ptr(out), _stream_ptr(stream)))
        return out[: states.shape[0]]

    def free(self) -> None:
        if self._h is not None:
            lib().gis_solution_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def solve(ctx: Context, system: W.System, grid: W.Grid, u, rounds: int, opts: OptsT,
          stream=None) -> Solution:
    du = to_device_u(ctx, u)
    h = P()
    st, gt = system_t(system, ctx), grid_t(grid)
    _check(lib().gis_solve(ctx.handle, ctypes.byref(st), ctypes.byref(gt), _ptr(du),
                           int(du.shape[0]), rounds, ctypes.byref(opts), ctypes.byref(h),
                           _stream_ptr(stream)))
    return Solution(h, ctx.device)


def autotune(ctx: Context, wl: W.Workload, repeats: int = 3, stream=None, **opt_over):
    """Chooses ctx's schedule parameters for the workload by timing whole solves
    (gis_autotune); returns (parameters, median ms per solve)."""
    du = to_device_u(ctx, wl.u)
    st, gt = system_t(wl.system, ctx), grid_t(wl.grid)
    opts = workload_opts(wl, **opt_over)
    best = TuningT()
    ms = F64(0.0)
    _check(lib().gis_autotune(ctx.handle, ctypes.byref(st), ctypes.byref(gt), _ptr(du),
                              int(du.shape[0]), wl.rounds, ctypes.byref(opts), int(repeats),
                              ctypes.byref(best), ctypes.byref(ms), _stream_ptr(stream)))
    return {f: int(getattr(best, f)) for f in TUNING_FIELDS}, float(ms.value)


class Solver:
    """One workload's solve with its arguments marshalled once: each call is a
    single gis_solve on the given stream (for loops of identical solves)."""

    def __init__(self, ctx: Context, wl: W.Workload, stream=None, **opt_over):
        self.ctx = ctx
        self.du = to_device_u(ctx, wl.u)
        self.st, self.gt = system_t(wl.system, ctx), grid_t(wl.grid)
        self.opts = workload_opts(wl, **opt_over)
        self.rounds = wl.rounds
        self.sp = _stream_ptr(stream)
        self._args = (ctx.handle, ctypes.byref(self.st), ctypes.byref(self.gt), _ptr(self.du),
                      int(self.du.shape[0]), self.rounds, ctypes.byref(self.opts))

    def __call__(self) -> Solution:
        h = P()
        _check(lib().gis_solve(*self._args, ctypes.byref(h), self.sp))
        return Solution(h, self.ctx.device)


def solve_workload(ctx: Context, wl: W.Workload, stream=None, **opt_over) -> Solution:
    return solve(ctx, wl.system, wl.grid, wl.u, wl.rounds, workload_opts(wl, **opt_over), stream)


def solve_batch(ctx: Context, workloads, stream=None, **opt_over) -> list:
    """Solves several workloads (same system kind, dimensions, K, rounds and
    options) through shared launches; returns one Solution per workload."""
    wls = list(workloads)
    w0 = wls[0]
    for w in wls:
        assert (w.system.kind, w.system.n, w.system.m, w.K, w.rounds) == \
            (w0.system.kind, w0.system.n, w0.system.m, w0.K, w0.rounds), "incompatible batch"
    dus = [to_device_u(ctx, w.u) for w in wls]
    jobs = (JobT * len(wls))()
    for i, w in enumerate(wls):
        jobs[i].sys = system_t(w.system, ctx)
        jobs[i].grid = grid_t(w.grid)
        jobs[i].d_u = _ptr(dus[i])
    outs = (P * len(wls))()
    opts = workload_opts(w0, **opt_over)
    _check(lib().gis_solve_batch(ctx.handle, len(wls), jobs, w0.K, w0.rounds, ctypes.byref(opts),
                                 outs, _stream_ptr(stream)))
    return [Solution(P(outs[i]), ctx.device) for i in range(len(wls))]
