"""Writes tests/golden/digests_fullsize.json: SHA-256 digests of what the CPU
oracle computes on the full-size workloads, for the GPU parity tests.

Only oracle/ and the seeded generators of paper_2202_06111_amd/workloads.py
are called here.  The oracle is single-threaded; this script runs several
oracle processes over disjoint row ranges of one covering (the rows of the
symbolic image are independent, Sec. 2.2, Definition 1) and concatenates their
results in row order, which is exactly what one call over every row returns.

Contents (per workload, per round):
  covering   level (u8) and multi-index (i32, cell-major) of the cell list
  graph      row_ptr (i64), col (i32), out (u8) of the symbolic image
             (Definition 1; OUT rows of Sec. 2.3)
  <analysis> kept (u8) and admissible-input masks (u64, ceil(K/64) words per
             cell) of the graph analysis (Sec. 2.3)
Digests are over the arrays' little-endian bytes.  Workloads:
  lorenz_uniform_128^3   the uniform 128^3 grid, 21 inputs: graph, both analyses
  vdp2_adaptive_32^4_r2  the coupled Van der Pol solve: rounds 0 and 1 in full
                         (covering, graph, non-leaving analysis), and the round-2
                         covering, i.e. the oracle's boundary selection and
                         subdivision (Sec. 3.1.1) of round 1's result; with
                         --only vdp2r2 also round 2's graph and analysis (the
                         graph, 62 GB, is written to files under --workdir and
                         the oracle's analysis runs on them memory-mapped)
  cstr                   the reactor of Sec. 4.1: the adaptive solve (8x8, 10
                         rounds, N = 3) and the standard one (20 halvings):
                         per-round counts, final covering, kept set, masks and
                         the answers to 10^5 seeded queries
  serving stream         every request of the seeded serving test stream
                         (Van der Pol, grids 32^2 .. 256^2): final covering,
                         kept set, masks, and the answers to its queries

Usage: python tests/golden/make_digests.py [--procs 8] [--only NAME] [--workdir DIR]
Takes about 10 minutes with 8 processes and about 30 GB of memory (the
round-1 graph of the coupled Van der Pol solve has 2.75e9 edges); vdp2r2
about an hour more and 62 GB of disk.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2202_06111_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "digests_fullsize.json")

# the serving test stream (tests/test_serving.py uses the same arguments)
SERVE_STREAM = dict(n_requests=24, rate_per_s=1e6, seed=11, n_queries=4000)


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


_job = {}


def _init(wl, level, idx):
    _job["wl"], _job["level"], _job["idx"] = wl, level, idx


def _chunk(bounds):
    a, b = bounds
    wl = _job["wl"]
    g = oracle.build_graph(wl.system, wl.grid, wl.samples, _job["level"], _job["idx"], wl.u,
                           rows=np.arange(a, b, dtype=np.int64))
    return g["cnt"], g["col"], g["out"]


def build_graph(wl, level, idx, procs):
    """oracle.build_graph over every row, split over processes by row range."""
    n_rows = level.shape[0] * wl.K
    n_chunks = max(1, min(256, n_rows // 200_000))
    cuts = np.linspace(0, n_rows, n_chunks + 1).astype(np.int64)
    cnts, cols, outs = [], [], []
    ctx = mp.get_context("fork")
    with ctx.Pool(procs, initializer=_init, initargs=(wl, level, idx)) as pool:
        for cnt, col, out in pool.imap(_chunk, list(zip(cuts[:-1], cuts[1:]))):
            cnts.append(cnt)
            cols.append(col)
            outs.append(out)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(np.concatenate(cnts), out=row_ptr[1:])
    del cnts
    col = np.concatenate(cols)
    del cols
    return {"row_ptr": row_ptr, "col": col, "out": np.concatenate(outs)}


def covering_entry(level, idx):
    return {"n_cells": int(level.shape[0]), "level": sha(level), "idx": sha(idx)}


def graph_entry(g):
    return {"n_rows": int(g["out"].shape[0]), "n_edges": int(g["col"].shape[0]),
            "n_out": int(g["out"].sum()), "row_ptr": sha(g["row_ptr"]), "col": sha(g["col"]),
            "out": sha(g["out"])}


def analysis_entry(kept, mask, sweeps):
    return {"n_kept": int(kept.sum()), "kept": sha(kept), "mask": sha(mask), "sweeps": sweeps}


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def lorenz(procs):
    wl = W.lorenz_uniform_128()
    level, idx = oracle.coarse_cells(wl.grid)
    log(f"{wl.name}: build {level.shape[0] * wl.K} rows")
    g = build_graph(wl, level, idx, procs)
    rnd = {"covering": covering_entry(level, idx), "graph": graph_entry(g)}
    for analysis in ("controlled", "nonleaving"):
        log(f"{wl.name}: {analysis} analysis")
        kept, mask, sweeps = oracle.prune(g["row_ptr"], g["col"], g["out"], level.shape[0], wl.K,
                                          analysis)
        rnd[analysis] = analysis_entry(kept, mask, sweeps)
    return {"cite": "Sec. 2.2 Definition 1 (graph), Sec. 2.3 (both analyses)",
            "rounds": [rnd]}


def vdp2(procs):
    wl = W.vdp2_adaptive_32()
    level, idx = oracle.coarse_cells(wl.grid)
    rounds = []
    for r in range(wl.rounds + 1):
        entry = {"covering": covering_entry(level, idx)}
        if r == wl.rounds:  # the last covering only: its graph is too large for this host
            rounds.append(entry)
            break
        log(f"{wl.name}: round {r}: build {level.shape[0] * wl.K} rows")
        g = build_graph(wl, level, idx, procs)
        entry["graph"] = graph_entry(g)
        log(f"{wl.name}: round {r}: {wl.analysis} analysis ({g['col'].shape[0]} edges)")
        kept, mask, sweeps = oracle.prune(g["row_ptr"], g["col"], g["out"], level.shape[0], wl.K,
                                          wl.analysis)
        del g
        entry[wl.analysis] = analysis_entry(kept, mask, sweeps)
        bnd = oracle.boundary(wl.grid, level, idx, kept, wl.boundary_rule)
        entry["n_boundary"] = int(bnd.sum())
        rounds.append(entry)
        level, idx = oracle.subdivide(wl.grid, level, idx, kept, bnd)
    return {"cite": "Sec. 2.2 Definition 1, Sec. 2.3 (non-leaving cells, Definitions 5-6), "
                    "Sec. 3.1.1 (Algorithm 1, Remark 1)",
            "analysis": wl.analysis, "rounds": rounds}


class _Sha:
    """Running SHA-256 over the little-endian bytes of arrays fed in order."""

    def __init__(self):
        self.h = hashlib.sha256()

    def feed(self, a):
        self.h.update(np.ascontiguousarray(a).tobytes())

    def hex(self):
        return self.h.hexdigest()


def build_graph_to_disk(wl, level, idx, procs, workdir, what):
    """oracle.build_graph over every row by row ranges, streamed to files
    under workdir (row offsets i64, targets i32, OUT flags u8) while running
    digests are taken; returns the memory-mapped arrays and the graph entry."""
    n_rows = level.shape[0] * wl.K
    os.makedirs(workdir, exist_ok=True)
    f_rp, f_col, f_out = (os.path.join(workdir, f) for f in ("row_ptr.i64", "col.i32", "out.u8"))
    h_rp, h_col, h_out = _Sha(), _Sha(), _Sha()
    n_chunks = 1024
    cuts = np.linspace(0, n_rows, n_chunks + 1).astype(np.int64)
    total = 0
    log(f"{what}: build {n_rows} rows into {workdir}")
    ctx = mp.get_context("fork")
    with open(f_rp, "wb") as frp, open(f_col, "wb") as fcol, open(f_out, "wb") as fout, \
            ctx.Pool(procs, initializer=_init, initargs=(wl, level, idx)) as pool:
        zero = np.zeros(1, dtype=np.int64)
        frp.write(zero.tobytes())
        h_rp.feed(zero)
        for i, (cnt, col, out) in enumerate(pool.imap(_chunk, list(zip(cuts[:-1], cuts[1:])))):
            rp = np.cumsum(cnt) + total
            total = int(rp[-1]) if rp.shape[0] else total
            for f, h, a in ((frp, h_rp, rp), (fcol, h_col, col), (fout, h_out, out)):
                f.write(np.ascontiguousarray(a).tobytes())
                h.feed(a)
            if i % 64 == 0:
                log(f"  chunk {i}/{n_chunks}: {total} edges so far")
    entry = {"n_rows": int(n_rows), "n_edges": int(total), "row_ptr": h_rp.hex(),
             "col": h_col.hex(), "out": h_out.hex()}
    rp = np.memmap(f_rp, dtype=np.int64, mode="r")
    col = np.memmap(f_col, dtype=np.int32, mode="r") if total > 0 else np.zeros(0, np.int32)
    out = np.memmap(f_out, dtype=np.uint8, mode="r")
    entry["n_out"] = int(np.sum(out, dtype=np.int64))
    return {"row_ptr": rp, "col": col, "out": out}, entry


def vdp2_round2(procs, workdir):
    """Round 2 of the coupled Van der Pol solve: the round-2 covering is
    recomputed (rounds 0 and 1, checked against the stored digest), its
    graph built by row ranges and streamed to files (row offsets, targets,
    OUT flags) while the digests run, then the oracle's analysis reads the
    files memory-mapped."""
    wl = W.vdp2_adaptive_32()
    level, idx = oracle.coarse_cells(wl.grid)
    for r in range(2):
        log(f"{wl.name}: round {r}: build {level.shape[0] * wl.K} rows (to reach round 2)")
        g = build_graph(wl, level, idx, procs)
        kept, mask, _ = oracle.prune(g["row_ptr"], g["col"], g["out"], level.shape[0], wl.K,
                                     wl.analysis)
        del g
        bnd = oracle.boundary(wl.grid, level, idx, kept, wl.boundary_rule)
        level, idx = oracle.subdivide(wl.grid, level, idx, kept, bnd)
    n_cells = level.shape[0]
    cov = covering_entry(level, idx)
    g, graph = build_graph_to_disk(wl, level, idx, procs, workdir, f"{wl.name}: round 2")
    log(f"{wl.name}: round 2: {wl.analysis} analysis ({graph['n_edges']} edges, memory-mapped)")
    kept, mask, sweeps = oracle.prune(g["row_ptr"], g["col"], g["out"], n_cells, wl.K, wl.analysis)
    return {"covering": cov, "graph": graph, wl.analysis: analysis_entry(kept, mask, sweeps)}


def solve_rounds(wl, procs, workdir):
    """The loop of oracle.solve (Sec. 2.1 and Sec. 3.1) with each round's
    graph built by row ranges in parallel processes (rounds of more than
    2e8 rows streamed to files under workdir and analysed memory-mapped);
    returns the final grid, covering, kept flags, masks and the per-round
    counts."""
    grid = wl.grid
    level, idx = oracle.coarse_cells(grid)
    stats, kept = [], None
    for r in range(wl.rounds + 1):
        if r > 0:
            if wl.subdivision == "bisect":
                grid, level, idx = oracle.bisect(grid, idx, kept, (r - 1) % grid.n)
                stats[-1]["n_boundary"] = int(kept.sum())
            else:
                bnd = oracle.boundary(grid, level, idx, kept, wl.boundary_rule)
                sel = oracle.neighbours(grid, level, idx, kept, bnd, wl.nn) if wl.nn > 0 else bnd
                level, idx = oracle.subdivide(grid, level, idx, kept, sel)
                stats[-1]["n_boundary"] = int(bnd.sum())
                stats[-1]["n_selected"] = int(sel.sum())
        if level.shape[0] == 0:
            break
        wl_r = dataclasses.replace(wl, grid=grid)
        if level.shape[0] * wl.K > 200_000_000:
            g, _ = build_graph_to_disk(wl_r, level, idx, procs, workdir, f"{wl.name}: round {r}")
        else:
            log(f"{wl.name}: round {r}: build {level.shape[0] * wl.K} rows")
            g = build_graph(wl_r, level, idx, procs)
        kept, mask, sweeps = oracle.prune(g["row_ptr"], g["col"], g["out"], level.shape[0], wl.K,
                                          wl.analysis)
        stats.append({"n_cells": int(level.shape[0]), "n_rows": int(level.shape[0] * wl.K),
                      "n_edges": int(g["col"].shape[0]),
                      "n_out": int(np.sum(g["out"], dtype=np.int64)),
                      "n_kept": int(kept.sum()), "sweeps": sweeps})
        del g
        if kept.sum() == 0:
            break
    return grid, level, idx, kept, mask, stats


# seeded query states of the CSTR solves (tests/test_gpu_fullsize.py draws the same)
CSTR_QUERIES = dict(n=100_000, seed=9, margin=0.02)


def cstr(procs, workdir):
    out = {}
    for wl in (W.cstr_adaptive(), W.cstr_standard()):
        t = time.time()
        grid, level, idx, kept, mask, stats = solve_rounds(wl, procs, workdir)
        q = W.query_states(wl.grid, CSTR_QUERIES["n"], seed=CSTR_QUERIES["seed"],
                           margin=CSTR_QUERIES["margin"])
        member, adm = oracle.query(grid, level, idx, kept, mask, q)
        out[wl.name] = {"cite": "Sec. 4.1 (Eq. 4, Table 2); Sec. 2.2-2.3; Sec. 3.1 (Algorithm 1, "
                                "Remark 1, N-NN of Sec. 3.1.2) or Sec. 2.1 (halving)",
                        "analysis": wl.analysis, "n0": list(grid.n0), "rounds": stats,
                        "covering": covering_entry(level, idx),
                        wl.analysis: analysis_entry(kept, mask, stats[-1]["sweeps"]),
                        "queries": dict(CSTR_QUERIES), "member": sha(member),
                        "admissible": sha(adm), "oracle_seconds": round(time.time() - t, 1)}
        log(f"{wl.name}: {len(stats)} rounds, final cells {stats[-1]['n_cells']}, "
            f"kept {stats[-1]['n_kept']}")
    return out


def serving():
    reqs = W.serving_stream(SERVE_STREAM["n_requests"], SERVE_STREAM["rate_per_s"],
                            seed=SERVE_STREAM["seed"], n_queries=SERVE_STREAM["n_queries"])
    out = []
    for r in reqs:
        wl = r.workload
        res = oracle.solve(wl.system, wl.grid, wl.samples, wl.u, wl.rounds,
                           rule=wl.boundary_rule, analysis=wl.analysis)
        q, kinds = r.queries, r.kinds
        member, adm = oracle.query(wl.grid, res["level"], res["idx"], res["kept"], res["mask"], q)
        out.append({"rid": r.rid, "side": int(wl.grid.n0[0]),
                    "covering": covering_entry(res["level"], res["idx"]),
                    wl.analysis: analysis_entry(res["kept"], res["mask"], res["stats"][-1]["sweeps"]),
                    "member": sha(member[kinds == 0]), "admissible": sha(adm[kinds == 1])})
        log(f"serving request {r.rid}: side {wl.grid.n0[0]}, kept {int(res['kept'].sum())}")
    return {"cite": "Sec. 2.2-2.3 on each request; queries: membership and admissible inputs",
            "stream": SERVE_STREAM, "requests": out}


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--procs", type=int, default=8)
    p.add_argument("--only", default=None, help="lorenz, vdp2, serving, cstr or vdp2r2")
    p.add_argument("--workdir", default=os.path.join(ROOT, "_work", "big"),
                   help="where vdp2r2 and cstr write their largest graphs (62 GB, 29 GB)")
    a = p.parse_args()
    oracle._load()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    jobs = {"serving": lambda: serving(), "lorenz": lambda: lorenz(a.procs),
            "vdp2": lambda: vdp2(a.procs), "cstr": lambda: cstr(a.procs, a.workdir)}
    keys = {"serving": "serving_stream", "lorenz": "lorenz_uniform_128^3",
            "vdp2": "vdp2_adaptive_32^4_r2", "cstr": "cstr"}
    if a.only == "vdp2r2":
        t = time.time()
        r2 = vdp2_round2(a.procs, a.workdir)
        entry = data["vdp2_adaptive_32^4_r2"]
        if r2["covering"] != entry["rounds"][2]["covering"]:
            raise SystemExit("round-2 covering differs from the stored one")
        entry["rounds"][2] = r2
        entry["round2_oracle_seconds"] = round(time.time() - t, 1)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        log(f"vdp2r2 done in {time.time() - t:.0f} s")
        return
    for name, fn in jobs.items():
        if a.only and a.only != name:
            continue
        t = time.time()
        data[keys[name]] = fn()
        data[keys[name]]["oracle_seconds"] = round(time.time() - t, 1)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        log(f"{name} done in {time.time() - t:.0f} s")


if __name__ == "__main__":
    main()
