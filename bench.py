"""Benchmark of the split step on one MI355X.

Headline workload: circular cylinder (radius 0.1, 1024-gon) crossing a stationary Mach-2
shock on [0,2]x[0,1] with 1024 x 512 cells, moving at +1.0 along x, CFL 0.8.  One step =
the CFL time step of its start state + the full split step (stage and end geometry, two
sweeps with every cut-cell operation).  The timed steps are planned on the device
(cc_advance: dt, poses and boxes computed at the head of each captured step, no host round
trip between steps).  Timed after W warm-up steps, K steps bracketed by device
synchronisation; value = cells x steps / time, FP32 state with FP64 geometry (the FP64 mode
beside it).

Also reported, each measured in this run:
* the roofline of the dominant kernel: the merged first-box-phase + dense-sweep launch the
  captured step runs, its duration from HIP events around that very launch (the step's
  launches issued one by one, same kernels, grids and arguments), and the whole step's
  fraction of the HBM roofline;
* accuracy of the FP32 state on the same workload: relative L1 of density against the FP64
  path with identical time steps, and the mass drift of both (from the conservation budget);
* the other configurations: the inclined piston (200 x 20, FP64), 16 triangle seeds at
  2048 x 1024 stepped as one batch (FP32), the pitching NACA 0012 at 4096 x 4096 (FP32 and
  FP64, tuned tiles), each with its rate and roofline;
* copies of the headline workload stepped as one batch against per-instance FP64 launches;
* the FP64 CPU oracle on a bounded sample of the headline workload, one thread and all
  host cores.
"""
import argparse
import hashlib
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def rate(cells, steps, seconds):
    return cells * steps / seconds


def timed_kernels(step_fn, nsteps, enable, read):
    """Average duration (us) of the dense launches of each direction over nsteps steps
    issued one by one with events around every dense launch."""
    enable(1)
    read()
    for _ in range(nsteps):
        step_fn()
    t = read()
    enable(0)
    return {k: (1e3 * t[k][0] / t[k][1] if t[k][1] > 0 else None) for k in ("dense_x", "dense_y")}


def roofline(kern_us, cells, bytes_per_value, table, names, grid=None):
    """Roofline of the slower dense launch: algorithmic bytes (read and write of the
    4-component state of every cell, per sweep) over its average duration; traffic: the
    counter bytes of the same launch on the same grid (`grid` "NXxNY"), when measured."""
    kern = max((k for k in kern_us if kern_us[k]), key=lambda k: kern_us[k])
    us = kern_us[kern]
    alg = cells * 4 * 2 * bytes_per_value
    ach = alg / (us * 1e-6) / 1e9
    name = names[kern]
    t = table.get(f"{name}@{grid}") if grid else None
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": None if t is None else t["fetch_bytes"] + t["write_bytes"],
            "kernel": name, "algorithmic_bytes": alg, "avg_launch_us": round(us, 2),
            "other_dense_us": {k: round(v, 2) for k, v in kern_us.items() if k != kern and v}}


def kernel_names(s, prec32):
    info = s.info()
    r = "float" if prec32 else "double"
    y = f"kb_wall_dense_yc<{r}, {info['tile_y_rows']}>" if info["tile_y_walk"] else \
        f"kb_wall_dense_y<{r}, {info['tile_y_rows']}>"
    x = "kb_wall_dense_x" if info["x_with_box"] else "kb_dense_x"
    return {"dense_x": f"{x}<{r}, {info['tile_x_rows']}>", "dense_y": y}


def run_mode(precision, steps, warmup, w, table, tune_cache=None):
    import numpy as np
    import torch
    from paper_1711_11361_amd import cc

    s = cc.Solver(w["grid"], w["body"], precision=precision)
    s.set_prim(w["prim"])
    prec32 = precision == cc.CC_FP32_GEOM64
    if tune_cache is not None:
        s.autotune(reps=5, cache_path=tune_cache)
    cfl = w["cfl"]
    cells = w["grid"]["nx"] * w["grid"]["ny"]
    # host-planned steps (cc_cfl_dt read back, then the captured step), for comparison
    for _ in range(5):
        s.step(s.cfl_dt(cfl))
    torch.cuda.synchronize()
    nh = min(steps, 50)
    h0 = time.perf_counter()
    for _ in range(nh):
        s.step(s.cfl_dt(cfl))
    torch.cuda.synchronize()
    host_ms = 1e3 * (time.perf_counter() - h0) / nh
    s.advance(warmup, cfl)
    torch.cuda.synchronize()
    # timed region: K device-planned steps (each: the CFL reduction of its start state, the
    # time step, the poses and boxes, and the split step), queued without host round trips;
    # cc_advance returns after the last one has finished
    t0 = time.perf_counter()
    s.advance(steps, cfl)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    info = s.info()
    if info["status"] & ~1:  # bit 0 (a cell with no donor) is only reported
        raise RuntimeError(f"device status {info['status']}")
    # latency pass after the timed region: an event pair around every step
    _, ms = s.advance(min(steps, 100), cfl, want_ms=True)
    lat = np.asarray(ms, dtype=np.float64)
    # kernel pass: the captured step's launches issued one by one, events around each dense
    # (merged first box phase + tiles) launch
    kern_us = timed_kernels(lambda: s.step(s.cfl_dt(cfl)), min(steps, 50), lambda m: cc.cc_timing(s.ctx, m),
                            lambda: cc.cc_timing_read(s.ctx))
    # phase breakdown of single sweeps (events between the box and geometry launches)
    cc.cc_timing(s.ctx, 2)
    cc.cc_timing_read(s.ctx)
    nph = min(steps, 20)
    for _ in range(nph):
        s.step(s.cfl_dt(cfl))
    ph = cc.cc_timing_read(s.ctx)
    cc.cc_timing(s.ctx, 0)
    info = s.info()
    if info["status"] & ~1:  # bit 0 (a cell with no donor) is only reported
        raise RuntimeError(f"device status {info['status']}")
    out = {"value": rate(cells, steps, T), "ms_per_step": 1e3 * T / steps, "host_planned_ms_per_step": host_ms,
           "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
           "t_end": info["t"], "collapses": info["collapses"],
           "tiles": {"x_rows_per_block": info["tile_x_rows"], "y_rows_per_tile": info["tile_y_rows"],
                     "y_column_walk": info["tile_y_walk"]},
           "box_phases_us_per_step": round(1e3 * ph["box"][0] / nph, 2),
           "geometry_us_per_step": round(1e3 * ph["geometry"][0] / nph, 2)}
    bpv = 4 if prec32 else 8
    out["roofline"] = roofline(kern_us, cells, bpv, table, kernel_names(s, prec32),
                               f"{w['grid']['nx']}x{w['grid']['ny']}")
    step_bytes = cells * 2 * 4 * 2 * bpv
    ach = step_bytes / (out["ms_per_step"] * 1e-3) / 1e9
    out["step_roofline"] = {"algorithmic_bytes": step_bytes, "achieved": round(ach, 1), "unit": "GB/s",
                            "frac": round(ach / HBM_PEAK_GBS, 4)}
    out["solver"] = s
    return out


def accuracy(w, nsteps):
    """FP32 state against the FP64 path on the same workload with identical time steps:
    relative L1 of density (volume-weighted), and the mass drift of each (change of the
    mass total minus the conservation budget, per initial mass)."""
    import numpy as np
    from paper_1711_11361_amd import cc

    res = {}
    s32 = cc.Solver(w["grid"], w["body"], precision=cc.CC_FP32_GEOM64)
    s32.set_prim(w["prim"])
    s32.set_budget(True)
    T0 = {"f32": s32.totals()}
    dts, _ = s32.advance(nsteps, w["cfl"])
    s64 = cc.Solver(w["grid"], w["body"], precision=cc.CC_FP64)
    s64.set_prim(w["prim"])
    s64.set_budget(True)
    T0["f64"] = s64.totals()
    for dt in dts:
        s64.step(dt)
    for name, s in (("f32", s32), ("f64", s64)):
        T1, (bnd, wall, lost) = cc.cc_totals(s.ctx, True)
        res[name] = abs((T1[0] - T0[name][0]) - bnd[0] - wall[0] + lost[0]) / T0[name][0]
    al = s64.geometry_dump(0)["alpha"]
    U32, U64 = s32.get_u(), s64.get_u()
    m = (al > 0) & (U64[0] > 0) & (U32[0] > 0)
    l1 = float((np.abs(U32[0][m] - U64[0][m])).sum() / U64[0][m].sum())
    s32.close()
    s64.close()
    return {"steps": nsteps, "fp32_l1_density_vs_fp64": l1, "mass_drift": {"f32": res["f32"], "f64": res["f64"]},
            "note": "same workload from t=0 with the conservation budget tracked, the FP64 path given the FP32 "
                    "run's time steps"}


def piston_leg(steps, warmup):
    """Config 1: the inclined piston, 200 x 20, FP64 (launch-bound at 4000 cells)."""
    import torch
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W

    w = W.piston()
    s = cc.Solver(w["grid"], w["body"], precision=cc.CC_FP64)
    s.set_prim(w["prim"])
    s.advance(warmup, w["cfl"])
    torch.cuda.synchronize()
    n = min(steps, 150)  # the run to t = 0.5 takes about 190 steps
    t0 = time.perf_counter()
    s.advance(n, w["cfl"])
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    cells = w["grid"]["nx"] * w["grid"]["ny"]
    s.close()
    return {"workload": "inclined piston (30 degrees) into gas at rest, 200x20 on [0,1]x[0,0.1], FP64",
            "value": rate(cells, n, T), "unit": "cell-updates/s", "ms_per_step": 1e3 * T / n, "steps": n}


def triangle_batch_leg(steps, warmup, table, seeds=16):
    """Config 3: 16 triangle seeds at 2048 x 1024 stepped as one batch, FP32 state, dense
    tile shapes picked by the batch tuner."""
    import numpy as np
    import torch
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W

    ws = [W.triangle_case(k) for k in range(seeds)]
    sol = []
    b = cc.Batch(seeds, cc.CC_FP32_GEOM64)
    for w in ws:
        s = cc.Solver(w["grid"], w["body"], precision=cc.CC_FP32_GEOM64)
        s.set_prim(w["prim"])
        b.add(s)
        sol.append(s)
    tx, ty = b.autotune(reps=10)
    b.advance(warmup, 0.8)
    torch.cuda.synchronize()
    n = min(steps, 100)
    t0 = time.perf_counter()
    b.advance(n, 0.8)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    _, lat = b.advance(min(n, 50), 0.8, want_ms=True)

    def step():
        dts = b.cfl_dt(0.8)
        b.step(dts)

    kern_us = timed_kernels(step, 10, lambda m: cc.cc_batch_timing(b.b, m), lambda: cc.cc_batch_timing_read(b.b))
    cells = sum(w["grid"]["nx"] * w["grid"]["ny"] for w in ws)
    # the library gives an x sweep over more than 2^21 cells per launch its dense kernel alone
    x = "kb_dense_x" if cells > (1 << 21) else "kb_wall_dense_x"
    rows_x = (1, 2, 4, 8)[tx]
    y = f"kb_wall_dense_yc<float, {(4, 8)[ty - 4]}>" if ty >= 4 else f"kb_wall_dense_y<float, {(8, 12, 16, 24)[ty]}>"
    names = {"dense_x": f"{x}<float, {rows_x}>", "dense_y": y}
    rf = roofline(kern_us, cells, 4, table, names)
    for s in sol:
        b.remove(s)
        s.close()
    b.close()
    lat = np.asarray(lat, dtype=np.float64)
    step_bytes = cells * 64
    ach = step_bytes / (T / n) / 1e9
    return {"workload": f"{seeds} triangle seeds crossing the Mach-2 shock, 2048x1024 each, one batch, "
                        "FP32 state / FP64 geometry, tiles tuned",
            "tiles": {"x_rows_per_block": rows_x, "y_rows_per_tile": (8, 12, 16, 24, 4, 8)[ty],
                      "y_column_walk": ty >= 4},
            "value": rate(cells, n, T), "unit": "cell-updates/s", "ms_per_iteration": 1e3 * T / n, "steps": n,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "roofline": rf,
            "step_roofline": {"algorithmic_bytes": step_bytes, "achieved": round(ach, 1), "unit": "GB/s",
                              "frac": round(ach / HBM_PEAK_GBS, 4)}}


def naca_leg(steps, warmup, table):
    """Config 4: the pitching NACA 0012 at 4096 x 4096, tiles tuned, captured steps."""
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W

    w = W.naca()
    out = {"workload": "NACA 0012 pitching 2 deg at reduced frequency 0.1 in a Mach-0.7 stream, 4096x4096 on "
                       "[-2,4]x[-3,3], tiles tuned"}
    cache = os.path.join("/tmp", f"cc_tiles_{os.getpid()}.txt")
    n = 500 if steps >= 50 else steps  # a 500-step window (about 0.25 s FP32, 0.45 s FP64)
    for prec, key in ((cc.CC_FP32_GEOM64, "f32"), (cc.CC_FP64, "f64")):
        r = run_mode(prec, n, warmup, w, table, tune_cache=cache)
        r.pop("solver").close()
        r["steps"] = n
        out[key] = r
    out["value"] = out["f32"]["value"]
    out["unit"] = "cell-updates/s"
    return out


def naca_lift_series(n=1024, cycles=3, per_cycle=48):
    """Config 4's pitching aerofoil on an n x n grid over `cycles` pitch periods (device-
    planned steps, FP32 state): lift, drag and moment coefficients C = F / (rho U^2 c / 2)
    (moment about the quarter chord, counter-clockwise positive) from the surface loads
    against the angle of attack, sampled per_cycle times a period (the last period
    reported), and the range of the wall cells' pressure coefficients at the end."""
    import numpy as np
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W

    w = W.naca(nx=n, ny=n)
    b = w["body"]
    s = cc.Solver(w["grid"], b, precision=cc.CC_FP32_GEOM64)
    s.set_prim(w["prim"])
    U, rho, chord = 0.7, 1.0, 1.0  # the free stream of the workload
    q = 0.5 * rho * U * U * chord
    period = 2.0 * math.pi / b["pitch_omega"]
    dt0 = s.cfl_dt(w["cfl"])
    chunk = max(1, int(period / dt0 / per_cycle))
    samples = []
    t0 = time.perf_counter()
    while s.info()["t"] < cycles * period:
        s.advance(chunk, w["cfl"])
        t = s.info()["t"]
        fx, fy, mz, _ = s.surface_loads()
        # the pose angle turns the body counter-clockwise, which lowers the leading edge (on
        # the upstream side): the angle of attack is its negative
        aoa = -math.degrees(b["theta0"] + b["pitch_amp"] * math.sin(b["pitch_omega"] * t))
        samples.append((t, aoa, fy / q, fx / q, mz / (q * chord)))
    wall = time.perf_counter() - t0
    r = s.surface_pressure()
    cp = (r[:, 3] - 1.0 / 1.4) / q  # free-stream pressure 1/gamma
    steps = s.info()["steps"]
    s.close()
    last = [x for x in samples if x[0] >= (cycles - 1) * period]
    return {"workload": f"NACA 0012 pitching 2 deg at reduced frequency 0.1, Mach 0.7, {n}x{n}, FP32 state",
            "cycles": cycles, "steps": steps, "wall_s": round(wall, 2),
            "last_cycle": {"angle_of_attack_deg": [round(x[1], 4) for x in last],
                           "c_l": [round(x[2], 5) for x in last],
                           "c_d": [round(x[3], 5) for x in last], "c_m": [round(x[4], 5) for x in last]},
            "c_l_range": [round(min(x[2] for x in last), 5), round(max(x[2] for x in last), 5)],
            "wall_cells": int(len(cp)), "cp_range": [round(float(cp.min()), 4), round(float(cp.max()), 4)]}


def run_to(s, cfl, t_end):
    """Host-planned CFL steps of a context with several bodies up to time t_end; returns
    (steps, seconds)."""
    import torch
    n = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = 0.0
    while t < t_end - 1e-12:
        dt = min(s.cfl_dt(cfl), t_end - t)
        s.step(dt)
        t += dt
        n += 1
    torch.cuda.synchronize()
    return n, time.perf_counter() - t0


def channel_leg():
    """Sloped moving channel (Sec. 3.1): a density pulse advected along two parallel walls at
    30 degrees that move together along +x, FP64, to t = 0.5; error norms of the density
    against the exact (advected) solution over full cells and their orders, at a fixed CFL
    number and with the CFL number halved per refinement (Eq. CFLvarying)."""
    import numpy as np
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W

    def one(ny, cfl):
        w = W.channel(ny, cfl=cfl)
        s = cc.Solver(w["grid"], bodies=w["bodies"], precision=cc.CC_FP64)
        s.set_prim(w["prim"])
        n, T = run_to(s, cfl, w["t_end"])
        st = s.info()["status"]
        P = s.get_prim()
        full = s.geometry_dump(0)["alpha"] == 1.0
        s.close()
        ex = W.channel_exact(w, w["t_end"])
        e = np.abs(P[0][full] - ex[0][full])
        h2 = (3.0 / w["grid"]["nx"]) * (1.0 / ny)
        cells = w["grid"]["nx"] * ny
        print(f"channel {w['grid']['nx']}x{ny} cfl {cfl}: {n} steps in {T:.2f} s", file=sys.stderr, flush=True)
        return {"grid": [w["grid"]["nx"], ny], "cfl": cfl, "steps": n, "status": int(st),
                "L1": float(e.sum() * h2), "L2": float(np.sqrt((e * e).sum() * h2)), "Linf": float(e.max()),
                "cell_updates_per_s": rate(cells, n, T), "ms_per_step": 1e3 * T / n}

    def orders(rows):
        for a, b in zip(rows, rows[1:]):
            b["orders"] = {k: float(np.log2(a[k] / b[k])) for k in ("L1", "L2", "Linf")}
        return rows

    fixed = orders([one(ny, 0.5) for ny in (32, 64, 128, 256, 512)])
    halved = orders([one(ny, 0.5 / 2 ** k) for k, ny in enumerate((128, 256, 512))])
    return {"workload": "sloped channel (30 degrees, width 0.25) moving at 0.5 along +x, density pulse advected "
                        "along it at 1.0, domain [-1.5,1.5]x[-0.5,0.5], FP64, t = 0.5",
            "fixed_cfl": fixed, "cfl_halved": halved}


def tube_leg(ny=512):
    """Two bodies in relative motion (the planar open-ended shock tube after Sec. 3.5): a
    piston driven at the Mach-1.76 piston speed along a static tube wall, 2.5 ny x ny cells,
    to t = 3 (the shock has left the tube), FP32 and FP64."""
    import numpy as np
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W

    out = {}
    for name, prec in (("fp32", cc.CC_FP32_GEOM64), ("fp64", cc.CC_FP64)):
        w = W.piston_tube(ny)
        s = cc.Solver(w["grid"], bodies=w["bodies"], precision=prec)
        s.set_prim(w["prim"])
        n1, _ = run_to(s, w["cfl"], 0.2)  # warm-up
        n, T = run_to(s, w["cfl"], 1.2)
        P = s.get_prim()
        full = s.geometry_dump(0)["alpha"] == 1.0
        up, S = w["piston_speed"], w["shock_speed"]
        X, Y = W.cell_centres(w["grid"])
        m = (X > 0.5 + up * 1.2 + 0.2) & (X < 0.5 + S * 1.2 - 0.3) & (Y < 0.3) & full
        n2, _ = run_to(s, w["cfl"], 1.8)
        st = s.info()["status"]
        s.close()
        cells = w["grid"]["nx"] * ny
        out[name] = {"cell_updates_per_s": rate(cells, n, T), "ms_per_step": 1e3 * T / n, "steps": n,
                     "status": int(st), "plateau_at_t1.2": {"rho": float(P[0][m].mean()), "u": float(P[1][m].mean()),
                                                            "p": float(P[3][m].mean())}}
    w = W.piston_tube(ny)
    up, S = w["piston_speed"], w["shock_speed"]
    out["closed_form_sealed_tube"] = {"rho": S / (S - up), "u": up, "p": 1.0 + S * up}
    out["workload"] = (f"piston (speed {up:.4f}, Mach-1.76 shock) inside a static tube wall, clearance 1/16, "
                       f"{int(2.5 * ny)}x{ny} on [0,10]x[0,4], reflective centre line")
    return out


def tube_overpressure_leg(ny=512, t_end=4.5, every=8):
    """The open-ended shock tube in axisymmetric form (Sec. 3.5; planar alongside): overpressure
    history on the axis 1.5 diameters downstream of the tube's exit (the probe of Fig.
    Piston_PressureTimeHistory), FP64, host-planned steps."""
    import numpy as np
    import torch
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W

    out = {}
    for name, axi in (("axisymmetric", True), ("planar", False)):
        w = W.piston_tube(ny, axisymmetric=axi)
        g = w["grid"]
        s = cc.Solver(g, bodies=w["bodies"], precision=cc.CC_FP64)
        s.set_prim(w["prim"])
        hx = (g["x_hi"] - g["x_lo"]) / g["nx"]
        ip = int((7.5 - g["x_lo"]) / hx)  # probe cell: x = 7.5 (1.5 D past the exit), first row
        ts, ps = [], []
        n, t = 0, 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while t < t_end - 1e-12:
            dt = min(s.cfl_dt(w["cfl"]), t_end - t)
            s.step(dt)
            t += dt
            n += 1
            if n % every == 0:
                u = s.get_u_tensor()[:, 0, ip].cpu().numpy()
                ts.append(t)
                ps.append(0.4 * (u[3] - 0.5 * (u[1] ** 2 + u[2] ** 2) / u[0]))
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        st = s.info()["status"]
        s.close()
        ps = np.array(ps) - 1.0
        k = int(np.argmax(ps))
        arrive = next((ts[q] for q in range(len(ps)) if ps[q] > 0.05), None)
        out[name] = {"steps": n, "wall_s": T, "status": int(st), "peak_overpressure": float(ps[k]),
                     "peak_time": float(ts[k]), "arrival_time": arrive,
                     "history": [[round(a, 4), round(float(b), 4)] for a, b in zip(ts[::4], ps[::4])]}
        print(f"tube {name}: {n} steps in {T:.2f} s, peak {ps[k]:.3f} at t = {ts[k]:.3f}", file=sys.stderr,
              flush=True)
    out["workload"] = (f"piston in the open-ended tube, {int(2.5 * ny)}x{ny} on [0,10]x[0,4] (lengths in tube "
                       f"diameters), probe on the axis at x = 7.5, overpressure p - p_inf (p_inf = 1), to t = {t_end}")
    return out


def batched(w, instances, steps, warmup):
    """Copies of the headline workload stepped as one batch (device-planned, dense tiles picked
    by the batch tuner), and the same copies as plain FP64 contexts advanced one after
    another with launches of their own."""
    import numpy as np
    import torch
    from paper_1711_11361_amd import cc

    sol = []
    for _ in range(instances):
        s = cc.Solver(w["grid"], w["body"], precision=cc.CC_FP32_GEOM64)
        s.set_prim(w["prim"])
        sol.append(s)
    b = cc.Batch(instances, cc.CC_FP32_GEOM64)
    for s in sol:
        b.add(s)
    tx, ty = b.autotune(reps=10)
    b.advance(warmup, w["cfl"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.advance(steps, w["cfl"])
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    _, lat = b.advance(min(steps, 100), w["cfl"], want_ms=True)
    cells = w["grid"]["nx"] * w["grid"]["ny"] * instances
    for s in sol:
        b.remove(s)
        s.close()
    b.close()
    s64 = []
    for _ in range(instances):
        s = cc.Solver(w["grid"], w["body"], precision=cc.CC_FP64)
        s.set_prim(w["prim"])
        s.advance(warmup, w["cfl"])
        s64.append(s)
    n64 = min(steps, 100)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for s in s64:
        s.advance(n64, w["cfl"])
    torch.cuda.synchronize()
    T64 = time.perf_counter() - p0
    for s in s64:
        s.close()
    lat = np.asarray(lat, dtype=np.float64)
    return {"instances": instances, "precision": "f32 state, f64 geometry", "planning": "device",
            "tiles": {"x_rows_per_block": (1, 2, 4, 8)[tx], "y_rows_per_tile": (8, 12, 16, 24, 4, 8)[ty],
                      "y_column_walk": ty >= 4},
            "cell_updates_per_s": cells * steps / T, "ms_per_iteration": 1e3 * T / steps,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "per_instance_fp64": {"cell_updates_per_s": cells * n64 / T64, "steps_each": n64}}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s=10.0):
    """The FP64 oracle as it stands, on a bounded sample of the headline workload from t=0:
    the plain build on one thread, and the OpenMP build of the same source on all host
    threads (identical results)."""
    from oracle import ref
    cells = w["grid"]["nx"] * w["grid"]["ny"]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    res = {}
    for parallel in (False, True):
        o = ref.Oracle(w["grid"], w["body"], parallel=parallel)
        o.set_prim(w["prim"])
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            o.step(o.cfl_dt(w["cfl"]))
            n += 1
        T = time.perf_counter() - t0
        o.close()
        res[parallel] = (rate(cells, n, T), n, T)
    v, n, T = res[True]
    v1, n1, T1 = res[False]
    return {"value": v, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} steps of the same 1024x512 workload from t=0 ({T:.1f} s, FP64 C oracle, OpenMP over "
                      f"rows and lines, {threads} threads)",
            "single_thread": {"value": v1, "sample": f"{n1} steps ({T1:.1f} s, one thread)"},
            "host": {"cpu_model": cpu_model(), "logical_cpus": os.cpu_count()}}


def serving(n, budget_gib, slots):
    """The serving mix: n requests (Poisson arrivals at 50/s, 500 steps each) served once
    batched in FP32 state / FP64 geometry and once as plain per-request FP64 launches."""
    import numpy as np
    from paper_1711_11361_amd import serving as S

    # first use of both modes (module load, graph capture paths) outside the measured runs
    for mode in ("batched", "plain"):
        srv = S.Server(mode, slots=4)
        srv.run(S.make_requests(4, rate=1e9, steps=3, seed=99, first=10000))
        srv.close()
    check = set(range(0, n, 16))  # requests whose end states are compared between the modes
    out = {}
    res = {}
    for mode in ("batched", "plain"):
        reqs = S.make_requests(n, rate=50.0, steps=500, seed=0)
        srv = S.Server(mode, budget_bytes=budget_gib * (1 << 30), slots=slots, keep_results=check)
        try:
            out[mode] = srv.run(reqs)
        except Exception as e:  # reported in the line; the run releases its contexts first
            out[mode] = {"error": f"{type(e).__name__}: {e}"}
            return out
        finally:
            srv.close()
        res[mode] = {r.rid: r.result[0] for r in reqs if r.result is not None}
    l1 = {}
    for rid in sorted(res["plain"]):
        a, b = res["batched"][rid].astype(np.float64), res["plain"][rid]
        den = np.abs(b).sum()
        l1[rid] = float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())
    worst = max(l1, key=l1.get)
    out["fp32_vs_fp64_l1_density"] = {"max": l1[worst], "worst_request": worst,
                                      "median": float(np.median(list(l1.values()))),
                                      "requests_compared": len(l1), "per_request": l1}
    out["speedup_cell_updates"] = out["batched"]["cell_updates_per_s"] / out["plain"]["cell_updates_per_s"]
    out["config"] = {"requests": n, "arrivals_per_s": 50.0, "steps_each": 500, "budget_gib": budget_gib,
                     "slots": slots}
    return out


def serving_child(n, budget_gib, slots, timeout_s=900):
    """The serving mix in a child process of its own (its own device context and memory
    pool), so that whatever happens there cannot take the rest of the line with it."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--serving-only", "--serving", str(n), "--budget-gib",
           str(budget_gib), "--slots", str(slots)]
    try:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout_s)
    except subprocess.TimeoutExpired:
        return {"error": f"serving run exceeded {timeout_s} s"}
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": f"serving run ended with status {r.returncode}", "stderr_tail": r.stderr[-2000:]}
    return json.loads(lines[-1])


def probe():
    """Dispatches for counter runs (one process, the step's launches one by one): the dense
    launches of the headline workload in both precisions and of the 4096 x 4096 aerofoil in
    FP32 and FP64 (every x-block height), then a plain 512 MiB fill and five 512 MiB device copies (larger than the
    last-level cache) whose counter readings scale FETCH_SIZE and WRITE_SIZE to bytes."""
    import torch
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W

    # (workload, precisions, tile pairs): the default tiles, and on the aerofoil also every
    # x-block height with the y column walks its tuner picks
    for w, precs, tiles in ((W.cylinder(), (cc.CC_FP32_GEOM64, cc.CC_FP64), ((0, 0),)),
                            (W.naca(), (cc.CC_FP32_GEOM64, cc.CC_FP64), ((0, 0), (1, 5), (2, 5), (3, 5)))):
        for prec in precs:
            s = cc.Solver(w["grid"], w["body"], precision=prec)
            s.set_prim(w["prim"])
            for _ in range(4):
                s.step(s.cfl_dt(w["cfl"]))
            for tx, ty in tiles:
                if prec == cc.CC_FP64 and ty == 5:
                    ty = 4  # an FP64 column walk takes 4 rows
                s.set_tiles(tx, ty)
                cc.cc_timing(s.ctx, 1)  # the step's launches one by one
                for _ in range(2):
                    s.step(s.cfl_dt(w["cfl"]))
                cc.cc_timing_read(s.ctx)
                cc.cc_timing(s.ctx, 0)
            print("probe", w["name"], "fp32" if prec == cc.CC_FP32_GEOM64 else "fp64", s.info(), flush=True)
            s.close()
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print("probe done", flush=True)


COPY_BYTES = 512 << 20
TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "dense_sweep_hbm_traffic.md")
DENSE_SOURCES = ("cc_device.h", "sweep.h", "engine.h")


def dense_fingerprint():
    """Hash of the sources the dense-sweep kernels are compiled from."""
    h = hashlib.sha256()
    for f in DENSE_SOURCES:
        with open(os.path.join(ROOT, "paper_1711_11361_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_table():
    """Per-dispatch HBM bytes of the dense launches from the committed counter summary (its
    JSON block), or {} when it is absent or was taken from other kernel sources."""
    try:
        txt = open(TRAFFIC_TABLE).read()
        d = json.loads(txt.split("```json")[1].split("```")[0])
        return d["kernels"] if d.get("source") == dense_fingerprint() else {}
    except (OSError, IndexError, KeyError, ValueError):
        return {}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the legs of the other configurations")
    ap.add_argument("--legs", default="piston,triangle,naca,lift,batched,channel,tube,axisym",
                    help="legs of the other configurations to run (comma list of piston, triangle, naca, lift, "
                         "batched, channel, tube, axisym)")
    ap.add_argument("--serving", type=int, default=256,
                    help="requests of the serving mix, run in a child process (0: skip)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving mix and print its JSON (the child of the default run)")
    ap.add_argument("--probe", action="store_true", help="dispatches for rocprofv3 counter runs only")
    ap.add_argument("--budget-gib", type=float, default=16.0)
    ap.add_argument("--slots", type=int, default=64)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(how the path would shard is described in the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.probe:
        probe()
        return
    if args.serving_only:
        print(json.dumps(serving(args.serving, args.budget_gib, args.slots)), flush=True)
        return
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W

    w = W.cylinder()
    table = traffic_table()
    nx, ny = w["grid"]["nx"], w["grid"]["ny"]
    r32 = run_mode(cc.CC_FP32_GEOM64, args.steps, args.warmup, w, table)
    s32 = r32.pop("solver")
    fluid = int((s32.geometry_dump(0)["alpha"] > 0.0).sum())  # cells with fluid at the end
    loads = s32.surface_loads()
    s32.close()
    r64 = run_mode(cc.CC_FP64, args.steps, args.warmup, w, table)
    r64.pop("solver").close()
    print(f"headline done: {r32['ms_per_step']:.4f} ms/step FP32, {r64['ms_per_step']:.4f} FP64", file=sys.stderr,
          flush=True)
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
        "latency_ms": r32["latency_ms"],
        "host_planned_ms_per_step": r32["host_planned_ms_per_step"],
        "fluid_cell_updates_per_s": fluid * args.steps / (r32["ms_per_step"] * 1e-3 * args.steps),
        "fluid_cells": fluid,
        "surface_loads": {"force": [float(loads[0]), float(loads[1])], "moment": float(loads[2])},
        "roofline": r32["roofline"],
        "step_roofline": r32["step_roofline"],
        "phases_us_per_step": {"box": r32["box_phases_us_per_step"], "geometry": r32["geometry_us_per_step"]},
        "fp64": {k: r64[k] for k in ("value", "ms_per_step", "host_planned_ms_per_step", "latency_ms", "roofline",
                                     "step_roofline")},
        "tiles": r32["tiles"],
        "sim_time_reached": r32["t_end"],
    }
    out["fp64"]["dtype"] = "f64"
    out["accuracy"] = accuracy(w, 200)
    print("accuracy done", file=sys.stderr, flush=True)
    legs = set(args.legs.split(",")) if not args.no_configs else set()
    out["configs"] = {}
    if "piston" in legs:
        out["configs"]["piston_200x20"] = piston_leg(args.steps, min(args.warmup, 10))
    if "triangle" in legs:
        out["configs"]["triangle_16x2048x1024_batched"] = triangle_batch_leg(args.steps, min(args.warmup, 10), table)
        print("triangle batch done", file=sys.stderr, flush=True)
    if "naca" in legs:
        out["configs"]["naca_4096x4096"] = naca_leg(args.steps, min(args.warmup, 10), table)
        print("naca done", file=sys.stderr, flush=True)
    if "lift" in legs:
        out["naca_lift"] = naca_lift_series()
        print("lift series done", file=sys.stderr, flush=True)
    if "batched" in legs:
        out["batched_copies"] = [batched(w, k, min(args.steps, 200), min(args.warmup, 20)) for k in (4, 16)]
    if "channel" in legs:
        out["sloped_channel"] = channel_leg()
        print("channel done", file=sys.stderr, flush=True)
    if "tube" in legs:
        out["piston_tube"] = tube_leg()
        print("tube done", file=sys.stderr, flush=True)
    if "axisym" in legs:
        out["tube_overpressure"] = tube_overpressure_leg()
        print("axisymmetric tube done", file=sys.stderr, flush=True)
    if args.serving > 0:
        out["serving"] = serving_child(args.serving, args.budget_gib, args.slots)
        print("serving done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
