"""Benchmark of the GIS graph-construction path on one MI355X.

A step is one whole solve of the workload: coarse covering, then per round
build the symbolic image (RK4 images -> bounding boxes -> covering ranges ->
CSR edges), analyse it (prune to the fixed point) and refine the boundary
cells.  The reported value is (cell x input) rows imaged per second of
wall-clock over the timed steps; inputs are resident on the device before the
timed region starts.

A second measurement, "serving", runs the mixed stream of smaller solves
(with their membership and admissible-input queries) through the
continuous-batching server and reports solves/s and p50/p99 latency.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--precision fp64|fp32_recheck]
                       [--analysis controlled|nonleaving|largest_scc] [--no-cpu-baseline]
                       [--no-autotune] [--tuning field=value,...] [--serve-requests N]

Before the warm-up, the library's autotuner picks the schedule parameters
(sweep and frontier batching, grid shapes) for the workload by timing whole
solves; the chosen parameters are reported under "schedule".
Prints one JSON line on stdout.
"""
import argparse
import dataclasses
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X vector peaks (256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz):
# FP64 FMA runs at full rate, 78.6 TFLOP/s.  FP32 reaches 157.3 TFLOP/s only through
# packed (two-per-lane) FP32 instructions, which this build does not emit; its
# unpacked FP32 FMA rate is the same 78.6 TFLOP/s.
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="vdp_adaptive_32x32_r5")
    p.add_argument("--precision", default=None, help="fp64 or fp32_recheck (default: workload's)")
    p.add_argument("--analysis", default=None,
                   help="controlled, nonleaving or largest_scc (default: workload's)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the default schedule parameters instead of running the autotuner "
                        "(gis_autotune, untimed, before the warm-up)")
    p.add_argument("--tuning", default="",
                   help="schedule parameters to start from, as field=value[,field=value...] "
                        "(fields of gis_tuning)")
    p.add_argument("--cpu-budget-s", type=float, default=12.0)
    p.add_argument("--serve-requests", type=int, default=64,
                   help="requests per pass of the serving measurement (0: skip it)")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="first run one plain device-to-device copy of this many MiB, as the "
                        "reference kernel for scaling HBM byte counters")
    return p.parse_args()


TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "traffic_k_build.md")
KERNEL_SOURCES = ("k_build.hip", "dynamics.h", "gis_internal.h")


def kernel_sources_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2202_06111_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, precision):
    """HBM bytes per build-kernel launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), provided
    it was taken for this workload and precision with the current kernel
    sources; None otherwise."""
    if not os.path.exists(TRAFFIC_TABLE):
        return None
    digest = kernel_sources_digest()
    with open(TRAFFIC_TABLE) as fh:
        for line in fh:
            cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            if len(cells) >= 8 and cells[0] == workload and cells[1] == precision and cells[2] == digest:
                try:
                    return float(cells[7])
                except ValueError:
                    return None
    return None


def cpu_baseline(wl, budget_s):
    """The CPU oracle (single-threaded FP64) timed on whole solves of the same workload."""
    import oracle
    oracle._load()
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
    return {"value": rows / el, "unit": "images/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} whole solve(s) of {wl.name} in {el:.1f} s, single thread"}


def serving(n_req):
    """The serving mix (Van der Pol solves with mu ~ U[0.5, 2], box scale ~ U[0.6, 1],
    grids 32^2..256^2, 11 inputs, 10^5 queries each) through the continuous-batching
    server: first all requests at once (saturation throughput), then a Poisson
    stream at 0.7x that rate (latency)."""
    from paper_2202_06111_amd import serve
    from paper_2202_06111_amd import workloads as W
    srv = serve.Server(n_slots=4, mem_budget_bytes=32 << 30)
    try:
        srv.run(W.serving_stream(8, 1e6, seed=99), realtime=False)  # warm-up
        sat = srv.run(W.serving_stream(n_req, 1e6, seed=0), realtime=False)
        rate = 0.7 * sat["solves_per_s"]
        lat = srv.run(W.serving_stream(n_req, rate, seed=1), realtime=True)
    finally:
        srv.close()
    return {"requests_per_pass": n_req, "queries_per_request": 100_000, "slots": 4,
            "saturation": {"solves_per_s": sat["solves_per_s"],
                           "queries_per_s": sat["queries_per_s"],
                           "mean_batch": sat["mean_batch"], "latency_ms": sat["latency_ms"]},
            "poisson": {"rate_per_s": rate, "solves_per_s": lat["solves_per_s"],
                        "mean_batch": lat["mean_batch"], "latency_ms": lat["latency_ms"]}}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {a.gpus} is not supported by this build "
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
    if not a.no_autotune:
        best, tuned_ms = gis.autotune(ctx, wl, repeats=3, stream=stream, precision=precision)
        schedule = {"autotuned": True, "tuned_ms_per_solve": tuned_ms, **best}
    # timing 1: HIP events around the build kernel only (the roofline needs them)
    solver = gis.Solver(ctx, wl, stream=stream, precision=precision, timing=1)

    def step():
        sol = solver()  # gis_solve synchronises its stream before returning
        raw = sol.info_raw()
        sol.free()
        return raw

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    raws, lat = [], []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ts = time.perf_counter()
        raws.append(step())
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    infos = [gis.info_dict(r) for r in raws]
    # per-phase device times from a few more solves with events between phases
    # (outside the timed region: each event record costs host time)
    phased = gis.Solver(ctx, wl, stream=stream, precision=precision, timing=2)
    phase_infos = []
    for _ in range(3):
        sol = phased()
        phase_infos.append(sol.info())
        sol.free()

    rows = sum(r["n_rows"] for inf in infos for r in inf["rounds"])
    flops_row = W.canonical_flops_per_row(wl.system, wl.samples)
    img_ms = sum(r["ms_image"] for inf in infos for r in inf["rounds"])
    launches = sum(len(inf["rounds"]) for inf in infos)
    achieved = rows * flops_row / (img_ms * 1e-3) / 1e12 if img_ms > 0 else 0.0
    last = infos[-1]
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
                   "final_kept": last["n_kept"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
                     "traffic": recorded_traffic(wl.name, precision),
                     "kernel": "k_build<%s> (images + boxes + cover + CSR emit, one pass)" %
                               ("fp64" if precision == "fp64" else "fp32+fp64 recheck"),
                     "avg_launch_ms": img_ms / max(launches, 1),
                     "flops_per_row": flops_row},
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
    ctx.close()
    if a.serve_requests > 0:
        res["serving"] = serving(a.serve_requests)
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, a.cpu_budget_s)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
