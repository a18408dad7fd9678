"""Benchmark of the split step on one MI355X.

Workload: circular cylinder (radius 0.1, 1024-gon) crossing a stationary Mach-2 shock on
[0,2]x[0,1] with 1024 x 512 cells, moving at +1.0 along x, CFL 0.8.  One step = the CFL
time step (device reduction, read back) + the full split step (stage and end geometry,
two sweeps with every cut-cell operation).  Timed after W warm-up steps, K steps
bracketed by device synchronisation; value = cells x steps / time.

Reported: cell-updates/s of the FP32-state / FP64-geometry mode (headline) and of the FP64
mode, p50/p99 step latency, the roofline of the dominant kernel (the dense sweep) from HIP
events on the library's stream, and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def run_mode(precision, steps, warmup, w):
    import numpy as np
    import torch
    from paper_1711_11361_amd import cc

    s = cc.Solver(w["grid"], w["body"], precision=precision)
    s.set_prim(w["prim"])
    tiles = s.autotune()
    cfl = w["cfl"]
    for _ in range(warmup):
        s.step(s.cfl_dt(cfl))
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    # timed region: each step is the CFL reduction plus one replay of the captured step graph
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(s.stream)
        s.step(s.cfl_dt(cfl))
        ev[k][1].record(s.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    info = s.info()
    if info["status"] != 0:
        raise RuntimeError(f"device status {info['status']}")
    # kernel timing pass (same kernels and grids, launched one by one): every dense-sweep
    # launch records its own start and stop events
    nt = min(steps, 100)
    cc.cc_timing(s.ctx, 1)
    cc.cc_timing_read(s.ctx)
    for _ in range(nt):
        s.step(s.cfl_dt(cfl))
    tim = cc.cc_timing_read(s.ctx)
    # phase breakdown: events bracket the box and geometry phases
    cc.cc_timing(s.ctx, 2)
    for _ in range(nt):
        s.step(s.cfl_dt(cfl))
    phases = cc.cc_timing_read(s.ctx)
    cc.cc_timing(s.ctx, 0)
    tim["box"], tim["geometry"] = phases["box"], phases["geometry"]
    tim["phase_steps"] = nt
    U = s.get_u()
    assert np.isfinite(U).all()
    cells = w["grid"]["nx"] * w["grid"]["ny"]
    T = t1 - t0
    return {"value": cells * steps / T, "ms_per_step": 1e3 * T / steps, "lat": lat, "timing": tim,
            "t_end": info["t"], "collapses": info["collapses"], "box_cells": info["box_cells"],
            "tiles": {"x_rows_per_block": info["tile_x_rows"], "y_rows_per_tile": info["tile_y_rows"]}}


def cpu_baseline(w, budget_s=15.0):
    from oracle import ref
    o = ref.Oracle(w["grid"], w["body"])
    o.set_prim(w["prim"])
    cells = w["grid"]["nx"] * w["grid"]["ny"]
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(o.cfl_dt(w["cfl"]))
        n += 1
    T = time.perf_counter() - t0
    return {"value": cells * n / T, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} steps of the same 1024x512 workload from t=0 (FP64 C oracle, one thread, "
                      f"{T:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W

    w = W.cylinder()
    nx, ny = w["grid"]["nx"], w["grid"]["ny"]
    r32 = run_mode(cc.CC_FP32_GEOM64, args.steps, args.warmup, w)
    r64 = run_mode(cc.CC_FP64, args.steps, args.warmup, w)

    def roofline(r, bytes_per_value):
        tim = r["timing"]
        kern = max(("dense_x", "dense_y"), key=lambda k: tim[k][0])
        ms, cnt = tim[kern]
        avg_s = ms / cnt / 1e3
        alg = nx * ny * 4 * 2 * bytes_per_value  # read + write of the state, one sweep
        ach = alg / avg_s / 1e9
        return {"bound": "hbm", "kernel": f"k_{kern}", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": round(avg_s * 1e6, 2),
                "other_dense_us": round(1e3 * tim["dense_y" if kern == "dense_x" else "dense_x"][0] /
                                        max(tim["dense_y" if kern == "dense_x" else "dense_x"][1], 1), 2),
                "box_kernels_us_per_step": round(1e3 * tim["box"][0] / tim["phase_steps"], 2),
                "geometry_us_per_step": round(1e3 * tim["geometry"][0] / tim["phase_steps"], 2),
                "tiles": r["tiles"]}

    out = {
        "metric": "cell-updates/s per split step (FP32+FP64-geom vs FP64) + p50/p99 step latency",
        "value": r32["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state and fluxes, f64 geometry and cut-cell arithmetic",
        "data": "synthetic",
        "config": {"workload": "cylinder r=0.1 crossing a stationary Mach-2 shock, 1024x512 on [0,2]x[0,1], "
                               "body speed 1.0, CFL 0.8", "grid": [nx, ny], "cells": nx * ny},
        "latency_ms": {"p50": float(np.percentile(r32["lat"], 50)), "p99": float(np.percentile(r32["lat"], 99))},
        "fp64": {"value": r64["value"], "ms_per_step": r64["ms_per_step"], "dtype": "f64",
                 "latency_ms": {"p50": float(np.percentile(r64["lat"], 50)),
                                "p99": float(np.percentile(r64["lat"], 99))},
                 "roofline": roofline(r64, 8)},
        "roofline": roofline(r32, 4),
        "sim_time_reached": r32["t_end"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
