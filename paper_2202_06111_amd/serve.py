"""Continuous-batching serving loop for GIS solves.

Requests (a system, a state box, a grid, an input set, and a batch of query
states) arrive on a Poisson clock.  Whenever one of the server's slots is
free, the dispatcher takes the requests waiting at that moment, in arrival
order, as long as their estimated device memory fits in what is left of the
budget, and runs them as one batch: one gis_solve_batch call pushes all of
them through shared kernel launches.  Each slot owns a libgis context and its
own HIP stream, so batches of different slots overlap on the device (the
library releases the GIL inside every call), and requests arriving while
batches run join the next batch as soon as a slot and memory free up.  A
solve's result stays on the device until its membership and admissible-input
queries are answered.  Latency is measured from the request's arrival to the
answer of its last query.
"""
from __future__ import annotations

import collections
import dataclasses
import statistics
import threading
import time
from typing import List, Optional

import numpy as np
import torch

from . import gis
from . import workloads as W


def estimate_bytes(wl: W.Workload, edges_per_row: float = 8.0) -> int:
    """Device memory one solve of `wl` needs at its largest round (upper
    estimate): per row the ranges, counts, OUT flag, CSR offsets, edges and
    reverse edges; per cell the list, index and prune state."""
    cells = int(np.prod(wl.grid.n0)) << (wl.grid.n * max(wl.rounds, 0))
    rows = cells * wl.K
    per_row = 2 * 4 * wl.grid.n + 4 + 1 + 8 + 8 + 8 * edges_per_row
    per_cell = 1 + 4 * wl.grid.n + 5 + 32 + 8 * ((wl.K + 63) // 64)
    return int(rows * per_row + cells * per_cell + (1 << 20))


@dataclasses.dataclass
class Result:
    rid: int
    arrival_s: float
    start_s: float
    done_s: float
    slot: int
    n_cells: int
    n_kept: int
    member: np.ndarray
    admissible: np.ndarray
    # with Server(export_results=True): the final covering, kept flags and
    # admissible-input masks (level, idx, kept, mask), copied to the host
    export: Optional[tuple] = None

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class Admission:
    """Slots plus a device-memory budget.  admit() blocks until a slot is free
    and the request's estimate fits in what is left of the budget (a request
    larger than the whole budget is admitted alone)."""

    def __init__(self, n_slots: int, budget_bytes: int):
        self.budget = int(budget_bytes)
        self._cv = threading.Condition()
        self._in_use = 0
        self._free = list(range(n_slots))
        self.max_in_use = 0
        self.deferred = 0

    def admit(self, need: int) -> int:
        need = min(int(need), self.budget)
        with self._cv:
            waited = False
            while not self._free or self._in_use + need > self.budget:
                waited = True
                self._cv.wait()
            self.deferred += int(waited)
            self._in_use += need
            self.max_in_use = max(self.max_in_use, self._in_use)
            return self._free.pop()

    def acquire_slot(self) -> int:
        """Blocks until a slot is free and takes it."""
        with self._cv:
            while not self._free:
                self._cv.wait()
            return self._free.pop()

    def reserve(self, need: int, block: bool) -> bool:
        """Takes `need` bytes of the budget; without `block`, only if they fit now."""
        need = min(int(need), self.budget)
        with self._cv:
            if self._in_use + need > self.budget:
                self.deferred += 1
                if not block:
                    return False
                while self._in_use + need > self.budget:
                    self._cv.wait()
            self._in_use += need
            self.max_in_use = max(self.max_in_use, self._in_use)
            return True

    def release(self, slot: int, need: int) -> None:
        need = min(int(need), self.budget)
        with self._cv:
            self._in_use -= need
            self._free.append(slot)
            self._cv.notify_all()

    @property
    def in_use(self) -> int:
        with self._cv:
            return self._in_use


@dataclasses.dataclass
class Queries:
    """A request's query states as they arrive with it: the membership and the
    admissible-input queries, each an (N x n) float64 array in pinned host
    memory."""
    member_states: torch.Tensor
    admissible_states: torch.Tensor

    @staticmethod
    def of(req: W.ServeRequest) -> "Queries":
        states, kinds = req.queries, req.kinds
        return Queries(torch.from_numpy(np.ascontiguousarray(states[kinds == 0])).pin_memory(),
                       torch.from_numpy(np.ascontiguousarray(states[kinds == 1])).pin_memory())


# Schedule parameters of the serving contexts: the serving mix (controlled
# analysis, grids up to 256^2) needs long removal chains, which the frontier
# phase handles better than sweeps (measured on the mix: 2.9k against 1.6k
# solves/s at saturation with the default switch at 8 M edges).
SERVING_TUNING = {"sweep_edges": 0}


class Server:
    def __init__(self, n_slots: int = 4, mem_budget_bytes: int = 8 << 30, device: int = 0,
                 tuning: Optional[dict] = None, export_results: bool = False):
        self.n_slots = n_slots
        self.device = device
        self.export_results = export_results
        self.adm = Admission(n_slots, mem_budget_bytes)
        self.ctxs = [gis.Context(device) for _ in range(n_slots)]
        for c in self.ctxs:
            c.set_tuning(**(SERVING_TUNING if tuning is None else tuning))
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_slots)]

    def close(self) -> None:
        for c in self.ctxs:
            c.close()

    # -------------------------------------------------------------- queries
    @staticmethod
    def _enqueue_queries(ctx: gis.Context, sol: gis.Solution, q: Queries, stream):
        """Copies the query states in, answers both kinds and copies the answers
        out to pinned host memory, all enqueued on `stream` (no synchronisation)."""
        ms = q.member_states.to(ctx.dev, non_blocking=True)
        as_ = q.admissible_states.to(ctx.dev, non_blocking=True)
        member = sol.query_membership(ms, stream)
        adm = sol.query_admissible(as_, stream)
        member_h = torch.empty(member.shape, dtype=member.dtype, pin_memory=True)
        adm_h = torch.empty(adm.shape, dtype=adm.dtype, pin_memory=True)
        member_h.copy_(member, non_blocking=True)
        adm_h.copy_(adm, non_blocking=True)
        return member_h, adm_h

    # -------------------------------------------------------------- one request
    def _serve_one(self, slot: int, req: W.ServeRequest, q: Queries, t0: float) -> Result:
        ctx, stream = self.ctxs[slot], self.streams[slot]
        start = time.perf_counter() - t0
        wl = req.workload
        with torch.cuda.stream(stream):
            du = gis.to_device_u(ctx, wl.u)
            sol = gis.solve(ctx, wl.system, wl.grid, du, wl.rounds, gis.workload_opts(wl), stream)
            try:
                member_h, adm_h = self._enqueue_queries(ctx, sol, q, stream)
                info = sol.info()
                ex = sol.export(stream) if self.export_results else None
                stream.synchronize()
            finally:
                sol.free()
        done = time.perf_counter() - t0
        return Result(req.rid, req.arrival_s, start, done, slot, info["n_cells"], info["n_kept"],
                      member_h.numpy(), adm_h.numpy().view(np.uint64),
                      None if ex is None else tuple(t.cpu().numpy() for t in ex))

    @staticmethod
    def _compatible(a: W.Workload, b: W.Workload) -> bool:
        key = lambda w: (w.system.kind, w.system.n, w.system.m, w.K, w.rounds, w.samples,
                         w.precision, w.boundary_rule, w.analysis)
        return key(a) == key(b)

    def _serve_batch(self, slot: int, reqs: List[W.ServeRequest], qs: List[Queries],
                     t0: float) -> List[Result]:
        """One gis_solve_batch for the requests, then every query of the batch
        enqueued on the slot's stream and one synchronisation."""
        ctx, stream = self.ctxs[slot], self.streams[slot]
        start = time.perf_counter() - t0
        with torch.cuda.stream(stream):
            sols = gis.solve_batch(ctx, [r.workload for r in reqs], stream)
            try:
                answers = [self._enqueue_queries(ctx, sol, q, stream) for sol, q in zip(sols, qs)]
                infos = [sol.info() for sol in sols]
                exports = [sol.export(stream) if self.export_results else None for sol in sols]
                stream.synchronize()
            finally:
                for sol in sols:
                    sol.free()
        done = time.perf_counter() - t0
        return [Result(req.rid, req.arrival_s, start, done, slot, info["n_cells"], info["n_kept"],
                       m.numpy(), a.numpy().view(np.uint64),
                       None if ex is None else tuple(t.cpu().numpy() for t in ex))
                for req, info, (m, a), ex in zip(reqs, infos, answers, exports)]

    def run(self, requests: List[W.ServeRequest], realtime: bool = True,
            max_batch: int = 16) -> dict:
        """Serves the stream; returns per-request results and summary stats.
        Each request's query states are materialised (pinned host memory)
        before the clock starts: they arrive with the request."""
        queries = [Queries.of(r) for r in requests]
        results: List[Optional[Result]] = [None] * len(requests)
        errors: List[BaseException] = []
        pending = collections.deque(sorted(range(len(requests)),
                                           key=lambda i: requests[i].arrival_s))
        waiting: collections.deque = collections.deque()
        batch_sizes: List[int] = []
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()

        def arrivals() -> None:
            now = time.perf_counter() - t0
            while pending and (not realtime or requests[pending[0]].arrival_s <= now):
                waiting.append(pending.popleft())

        def worker(slot: int, idx: List[int], need: int) -> None:
            try:
                for i, r in zip(idx, self._serve_batch(slot, [requests[i] for i in idx],
                                                       [queries[i] for i in idx], t0)):
                    results[i] = r
            except BaseException as e:  # reported after the run
                errors.append(e)
            finally:
                self.adm.release(slot, need)

        threads = []
        while pending or waiting:
            arrivals()
            if not waiting:
                time.sleep(max(0.0, requests[pending[0]].arrival_s - (time.perf_counter() - t0)))
                continue
            slot = self.adm.acquire_slot()
            arrivals()  # requests that came while every slot was busy join this batch
            first = waiting.popleft()
            need = min(estimate_bytes(requests[first].workload), self.adm.budget)
            self.adm.reserve(need, block=True)
            idx = [first]
            while waiting and len(idx) < max_batch:
                nxt = waiting[0]
                if not self._compatible(requests[nxt].workload, requests[first].workload):
                    break
                nd = min(estimate_bytes(requests[nxt].workload), self.adm.budget)
                if not self.adm.reserve(nd, block=False):
                    break
                need += nd
                idx.append(waiting.popleft())
            batch_sizes.append(len(idx))
            th = threading.Thread(target=worker, args=(slot, idx, need), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        wall = time.perf_counter() - t0
        if errors:
            raise errors[0]
        lat = sorted(r.latency_s for r in results)
        q = sum(len(r.member) + len(r.admissible) for r in results)
        return {
            "results": results,
            "wall_s": wall,
            "solves_per_s": len(results) / wall,
            "queries_per_s": q / wall,
            "latency_ms": {"p50": 1e3 * statistics.median(lat),
                           "p99": 1e3 * lat[min(len(lat) - 1, int(0.99 * len(lat)))],
                           "max": 1e3 * lat[-1]},
            "batches": len(batch_sizes),
            "mean_batch": sum(batch_sizes) / max(len(batch_sizes), 1),
            "max_bytes_in_use": self.adm.max_in_use,
            "budget_bytes": self.adm.budget,
            "deferred": self.adm.deferred,
        }


def serve_alone(requests: List[W.ServeRequest], device: int = 0,
                export_results: bool = False) -> List[Result]:
    """Each request solved and queried by itself, one after the other."""
    srv = Server(n_slots=1, device=device, export_results=export_results)
    try:
        queries = [Queries.of(r) for r in requests]
        t0 = time.perf_counter()
        return [srv._serve_one(0, r, q, t0) for r, q in zip(requests, queries)]
    finally:
        srv.close()
