"""Benchmark of the GIS graph-construction path on one MI355X.

A step is one whole solve of the workload: coarse covering, then per round
build the symbolic image (RK4 images -> bounding boxes -> covering ranges ->
CSR edges), analyse it (prune to the fixed point) and refine the boundary
cells.  The reported value is (cell x input) rows imaged per second of
wall-clock over the timed steps; inputs are resident on the device before the
timed region starts.  The default workload is the largest one that fits one
GPU: two coupled Van der Pol oscillators, 32^4 coarse cells, two boundary
rounds, 7x7 inputs (1.84e9 rows per solve), FP32 images with the FP64
recheck; the same solve with plain FP64 images is timed beside it
("other_precision").

A measurement "cstr" reruns the paper's own experiment (the reactor of
Sec. 4.1): adaptive solves with neighbourhoods N = 0, 1, 3, 5 against the
standard algorithm at the same finest cell width, time per solve and cells.

A second measurement, "serving", runs the mixed stream of smaller solves
(with their membership and admissible-input queries) through the
continuous-batching server and reports solves/s and p50/p99 latency.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--precision fp64|fp32_recheck] [--other-steps N]
                       [--analysis controlled|nonleaving|largest_scc] [--no-cpu-baseline]
                       [--autotune] [--tuning field=value,...] [--serve-requests N]
                       [--cstr-steps N]

With --autotune the library's autotuner first picks the schedule parameters
(sweep and frontier batching, grid shapes) for the workload by timing whole
solves; the parameters used are reported under "schedule".
Prints one JSON line on stdout.
"""
import argparse
import dataclasses
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X vector peaks (256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz):
# FP64 FMA runs at full rate, 78.6 TFLOP/s.  FP32 reaches 157.3 TFLOP/s only through
# packed (two-per-lane) FP32 instructions, which the kernels do not use; its
# unpacked FP32 FMA rate is the same 78.6 TFLOP/s.
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Published MI355X HBM3E bandwidth.
PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="vdp2_adaptive_32^4_r2")
    p.add_argument("--precision", default=None, help="fp64 or fp32_recheck (default: workload's)")
    p.add_argument("--other-steps", type=int, default=5,
                   help="timed solves with the other image precision (0: skip that leg)")
    p.add_argument("--analysis", default=None,
                   help="controlled, nonleaving or largest_scc (default: workload's)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--autotune", action="store_true",
                   help="run the autotuner (gis_autotune, untimed, before the warm-up) instead "
                        "of keeping the default schedule parameters")
    p.add_argument("--tuning", default="",
                   help="schedule parameters to start from, as field=value[,field=value...] "
                        "(fields of gis_tuning)")
    p.add_argument("--cpu-budget-s", type=float, default=15.0)
    p.add_argument("--cstr-steps", type=int, default=3,
                   help="solves per configuration of the reactor experiment (0: skip it)")
    p.add_argument("--serve-requests", type=int, default=1000,
                   help="requests of the Poisson pass of the serving measurement (0: skip it); "
                        "the saturation pass takes a quarter of them")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="first run one plain device-to-device copy of this many MiB, as the "
                        "reference kernel for scaling HBM byte counters")
    return p.parse_args()


TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "traffic_k_build.md")
KERNEL_SOURCES = ("k_build_dev.h", "k_build.hip", "dynamics.h", "gis_internal.h")
ANALYSIS_TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "traffic_analysis.md")
ANALYSIS_SOURCES = ("k_prune.hip", "k_frontier.hip", "gis_internal.h")


def kernel_sources_digest(sources=KERNEL_SOURCES):
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2202_06111_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, precision, table=TRAFFIC_TABLE, sources=KERNEL_SOURCES):
    """HBM bytes per build-kernel launch (or per solve, for the analysis
    table) from the committed counter summary (FETCH_SIZE + WRITE_SIZE,
    scaled by a plain copy of known size), provided it was taken for this
    workload and precision with the current kernel sources; None otherwise."""
    if not os.path.exists(table):
        return None
    digest = kernel_sources_digest(sources)
    with open(table) as fh:
        for line in fh:
            cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            if len(cells) >= 8 and cells[0] == workload and cells[1] == precision and cells[2] == digest:
                try:
                    return float(cells[7])
                except ValueError:
                    return None
    return None


def host_cpu():
    """Model name of the host CPU and the number of cores this process may use."""
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count()
    return model, n


def cpu_baseline(wl, budget_s, gpu_rows_per_solve):
    """The CPU oracle (single-threaded FP64) timed on a bounded sample of the
    same workload.  Workloads whose whole solve the oracle finishes within the
    budget are timed on whole solves; otherwise on seeded random rows of the
    round-0 covering (the symbolic image of those rows: images, boxes, cover
    ranges, edges), in chunks until the budget is spent."""
    import numpy as np
    import oracle
    oracle._load()
    model, ncpu = host_cpu()
    base = {"unit": "images/s", "cores": 1, "kind": "oracle", "cpu_model": model,
            "host_cores": ncpu}
    # whole solves when one of them takes a few seconds at most (about 4e5
    # images/s per core for the planar field)
    if gpu_rows_per_solve <= 2_000_000:
        reps, rows, t0 = 0, 0, time.perf_counter()
        while True:
            res = oracle.solve(wl.system, wl.grid, wl.samples, wl.u, wl.rounds,
                               rule=wl.boundary_rule, analysis=wl.analysis,
                               subdivision=wl.subdivision)
            rows += sum(s["n_rows"] for s in res["stats"])
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget_s or reps >= 50:
                break
        return {"value": rows / el, **base,
                "sample": f"{reps} whole solve(s) of {wl.name} in {el:.1f} s, single thread"}
    level, idx = oracle.coarse_cells(wl.grid)
    n_rows = level.shape[0] * wl.K
    rng = np.random.Generator(np.random.PCG64(12345))
    done, t0 = 0, time.perf_counter()
    while True:
        rows = np.sort(rng.choice(n_rows, size=2000, replace=False)).astype(np.int64)
        oracle.build_graph(wl.system, wl.grid, wl.samples, level, idx, wl.u, rows=rows)
        done += rows.shape[0]
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": done / el, **base,
            "sample": f"graph build of {done} seeded random rows (PCG64 seed 12345, chunks of "
                      f"2000) of the round-0 covering of {wl.name} in {el:.1f} s, single thread"}


def serving(n_req):
    """The serving mix (Van der Pol solves with mu ~ U[0.5, 2], box scale ~ U[0.6, 1],
    grids 32^2..256^2, 11 inputs, 10^5 queries each) through the continuous-batching
    server: first n_req / 4 requests at once (saturation throughput), then a
    Poisson stream of n_req requests at 0.7x that rate (latency)."""
    from paper_2202_06111_amd import serve
    from paper_2202_06111_amd import workloads as W
    srv = serve.Server(n_slots=4, mem_budget_bytes=32 << 30)
    n_sat = max(n_req // 4, 8)
    try:
        srv.run(W.serving_stream(8, 1e6, seed=99), realtime=False)  # warm-up
        sat = srv.run(W.serving_stream(n_sat, 1e6, seed=0), realtime=False)
        rate = 0.7 * sat["solves_per_s"]
        lat = srv.run(W.serving_stream(n_req, rate, seed=1), realtime=True)
    finally:
        srv.close()
    return {"queries_per_request": 100_000, "slots": 4,
            "saturation": {"requests": n_sat, "solves_per_s": sat["solves_per_s"],
                           "queries_per_s": sat["queries_per_s"],
                           "mean_batch": sat["mean_batch"], "latency_ms": sat["latency_ms"]},
            "poisson": {"requests": n_req, "seed": 1, "rate_per_s": rate,
                        "solves_per_s": lat["solves_per_s"], "mean_batch": lat["mean_batch"],
                        "latency_ms": lat["latency_ms"],
                        "latency_samples": len(lat["results"])}}


def timed_solves(gis, ctx, wl, stream, precision, steps, warmup):
    """warmup + steps whole solves; returns (per-solve stats of the timed ones,
    seconds over the timed region, per-solve wall seconds).  timing 1: HIP
    events around the build kernel only, on the solve's stream."""
    import torch
    solver = gis.Solver(ctx, wl, stream=stream, precision=precision, timing=1)

    def step():
        sol = solver()  # gis_solve synchronises its stream before returning
        raw = sol.info_raw()
        sol.free()
        return raw

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    raws, lat = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        raws.append(step())
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return [gis.info_dict(r) for r in raws], el, lat


def phase_times(gis, ctx, wl, stream, precision, n=2):
    """Per-phase device times from a few more solves with HIP events between
    the phases (outside the timed region: each event record costs host time)."""
    phased = gis.Solver(ctx, wl, stream=stream, precision=precision, timing=2)
    out = []
    for _ in range(n):
        sol = phased()
        out.append(sol.info())
        sol.free()
    return out


def build_roofline(W, wl, infos, precision):
    """k_build: canonical image flops of its launches over their summed
    duration (HIP events on the launch stream) against the VALU peak."""
    rows = sum(r["n_rows"] for inf in infos for r in inf["rounds"])
    flops_row = W.canonical_flops_per_row(wl.system, wl.samples)
    img_ms = sum(r["ms_image"] for inf in infos for r in inf["rounds"])
    launches = sum(len(inf["rounds"]) for inf in infos)
    achieved = rows * flops_row / (img_ms * 1e-3) / 1e12 if img_ms > 0 else 0.0
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
            "traffic": recorded_traffic(wl.name, precision),
            "kernel": "k_build<%s> (images + boxes + cover + CSR emit, one pass)" %
                      ("fp64" if precision == "fp64" else "fp32+fp64 recheck"),
            "launches_per_solve": launches / max(len(infos), 1),
            "avg_launch_ms": img_ms / max(launches, 1),
            "flops_per_row": flops_row}


def analysis_roofline(wl, phase_infos, precision):
    """The analysis (every launch from the end of the build to the start of
    the subdivision): its algorithmic bytes -- one read of the targets (4 B
    per edge) and row offsets (8 B per row), one write of the kept flags and
    masks (1 + 8 ceil(K/64) B per cell) -- over its HIP-event duration,
    against the HBM peak."""
    words = (wl.K + 63) // 64
    byts = sum(4 * r["n_edges"] + 8 * r["n_rows"] + (1 + 8 * words) * r["n_cells"]
               for inf in phase_infos for r in inf["rounds"])
    ms = sum(r["ms_prune"] for inf in phase_infos for r in inf["rounds"])
    achieved = byts / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": recorded_traffic(wl.name, precision, ANALYSIS_TRAFFIC_TABLE,
                                        ANALYSIS_SOURCES),
            "traffic_per": "solve",
            "kernel": f"graph analysis ({wl.analysis}), all of its launches",
            "bytes_per_solve": byts / max(len(phase_infos), 1),
            "ms_per_solve": ms / max(len(phase_infos), 1)}


def cstr_experiment(gis, W, ctx, stream, steps, cpu_budget_s):
    """The paper's reactor experiment (Sec. 4.1-4.2) on this GPU: adaptive
    subdivision with neighbourhoods N = 0, 1, 3, 5 over 10 rounds against the
    standard algorithm (every kept cell halved, the paper's N = 1000) over 20
    halvings -- the same finest cell width -- from the same 8x8 grid with 31
    coolant temperatures, FP64 images.  The paper reports N = 3 about 8x
    faster than N = 1000 after 20 iterations on its CPU."""
    def one(wl):
        infos, el, _ = timed_solves(gis, ctx, wl, stream, "fp64", steps, 1)
        last = infos[-1]
        rows = sum(r["n_rows"] for r in last["rounds"])
        return {"workload": wl.name, "ms_per_solve": 1e3 * el / steps, "rows_per_solve": rows,
                "images_per_s": rows * steps / el, "final_cells": last["n_cells"],
                "final_kept": last["n_kept"],
                "cells_per_round": [r["n_cells"] for r in last["rounds"]],
                "k_build": build_roofline(W, wl, infos, "fp64")}

    res = {"grid0": [8, 8], "inputs": 31, "precision": "fp64", "steps": steps,
           "adaptive": [{"N": nn, **one(W.cstr_adaptive(nn=nn))} for nn in (0, 1, 3, 5)],
           "standard": one(W.cstr_standard())}
    n3 = next(r for r in res["adaptive"] if r["N"] == 3)
    res["standard_over_adaptive_N3"] = res["standard"]["ms_per_solve"] / n3["ms_per_solve"]
    if cpu_budget_s > 0:
        # the oracle on this host: whole 6-round adaptive solves (N = 3)
        import oracle
        oracle._load()
        wl = W.cstr_adaptive(nn=3, rounds=6)
        reps, rows, t0 = 0, 0, time.perf_counter()
        while True:
            r = oracle.solve(wl.system, wl.grid, wl.samples, wl.u, wl.rounds,
                             analysis=wl.analysis, nn=wl.nn)
            rows += sum(x["n_rows"] for x in r["stats"])
            reps += 1
            el = time.perf_counter() - t0
            if el >= cpu_budget_s:
                break
        res["cpu_oracle"] = {"value": rows / el, "unit": "images/s", "cores": 1, "kind": "oracle",
                             "sample": f"{reps} whole solve(s) of {wl.name} in {el:.1f} s, "
                                       "single thread"}
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {a.gpus} is not supported "
              "(the path has no multi-GPU sharding).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2202_06111_amd import gis
    from paper_2202_06111_amd import workloads as W

    if a.workload not in W.ALL:
        sys.exit(f"unknown workload {a.workload}; choose from {sorted(W.ALL)}")
    wl = W.ALL[a.workload]()
    if a.analysis:
        wl = dataclasses.replace(wl, analysis=a.analysis)
    precision = a.precision or wl.precision
    other = "fp64" if precision != "fp64" else "fp32_recheck"
    if a.copy_calibration_mib > 0:
        n = a.copy_calibration_mib << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = gis.Context(0)
    # a stream of its own (default priority): the null stream cannot be captured as a graph
    stream = torch.cuda.Stream()
    if a.tuning:
        ctx.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in a.tuning.split(","))})
    schedule = {"autotuned": False, **ctx.get_tuning()}
    if a.autotune:
        best, tuned_ms = gis.autotune(ctx, wl, repeats=3, stream=stream, precision=precision)
        schedule = {"autotuned": True, "tuned_ms_per_solve": tuned_ms, **best}

    infos, el, lat = timed_solves(gis, ctx, wl, stream, precision, a.steps, a.warmup)
    phase_infos = phase_times(gis, ctx, wl, stream, precision)
    rows = sum(r["n_rows"] for inf in infos for r in inf["rounds"])
    last = infos[-1]
    broof = build_roofline(W, wl, infos, precision)
    aroof = analysis_roofline(wl, phase_infos, precision)
    res = {
        "metric": "cell x input images/s in graph build (whole solve)",
        "value": rows / el,
        "unit": "images/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * el / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64recheck",
        "data": "synthetic",
        "config": {"workload": wl.name, "system": wl.system.kind, "grid0": list(wl.grid.n0),
                   "rounds": wl.rounds, "inputs": wl.K, "samples": wl.samples,
                   "analysis": wl.analysis, "subdivision": wl.subdivision, "precision": precision,
                   "rows_per_solve": rows // a.steps, "final_cells": last["n_cells"],
                   "final_kept": last["n_kept"],
                   "rounds_detail": [{k: r[k] for k in ("n_cells", "n_rows", "n_edges", "n_kept",
                                                        "n_recheck")}
                                     for r in last["rounds"]]},
        "roofline": broof,
        "rooflines": {"k_build": broof, "analysis": aroof},
        "schedule": schedule,
        "phases_ms_per_solve": {
            k: sum(r[k] for inf in phase_infos for r in inf["rounds"]) / len(phase_infos)
            for k in ("ms_build", "ms_image", "ms_prune", "ms_subdivide")},
        "host_ms_per_solve": {
            "busy": sum(r["ms_host"] for inf in infos for r in inf["rounds"]) / a.steps,
            "blocked_in_sync": sum(r["ms_host_wait"] for inf in infos for r in inf["rounds"]) / a.steps},
        "recheck_rows_per_solve": sum(r["n_recheck"] for inf in infos for r in inf["rounds"]) / a.steps,
        "solves_per_s": a.steps / el,
        "latency_ms": {"p50": 1e3 * statistics.median(lat),
                       "p99": 1e3 * sorted(lat)[min(len(lat) - 1, int(0.99 * len(lat)))]},
    }
    if precision != "fp64":
        res["recheck_band"] = [{"band": r["band"], "max_err_sample": r["max_err"]}
                               for r in last["rounds"]]
    if a.other_steps > 0:
        # the same solve with the other image precision, on the same GPU
        o_infos, o_el, _ = timed_solves(gis, ctx, wl, stream, other, a.other_steps, 1)
        o_rows = sum(r["n_rows"] for inf in o_infos for r in inf["rounds"])
        same = all(r1["n_edges"] == r2["n_edges"] and r1["n_kept"] == r2["n_kept"]
                   for r1, r2 in zip(o_infos[-1]["rounds"], last["rounds"]))
        res["other_precision"] = {
            "precision": other, "dtype": "f64" if other == "fp64" else "f32+f64recheck",
            "steps": a.other_steps, "value": o_rows / o_el, "unit": "images/s",
            "ms_per_step": 1e3 * o_el / a.other_steps,
            "k_build": build_roofline(W, wl, o_infos, other),
            "same_edge_and_kept_counts": same}
    if a.cstr_steps > 0:
        res["cstr"] = cstr_experiment(gis, W, ctx, stream, a.cstr_steps,
                                      0.0 if a.no_cpu_baseline else 5.0)
    ctx.close()
    if a.serve_requests > 0:
        res["serving"] = serving(a.serve_requests)
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, a.cpu_budget_s, rows // a.steps)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
