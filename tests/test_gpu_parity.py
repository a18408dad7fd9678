"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle.

* geometry: vertex classes bit-exact, apertures and volume fractions to round-off;
* per sweep from identical inputs: relative L-infinity of U <= 1e-12 (FP64), per
  component, momentum relative to the characteristic momentum rho (|u| + a);
* end time (config 1, the inclined piston, 200 x 20 to t = 0.5): relative L1 <= 1e-9,
  with the oracle's time steps;
* the CFL time step to 1e-12; conservation totals to round-off;
* FP32 state with FP64 geometry against the FP64 oracle: relative L1 of density <= 1e-4;
* full-size workloads (1024 x 512 cylinder, 2048 x 1024 triangle, 4096 x 4096 aerofoil):
  one step each, in the launch configuration the benchmark uses.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from oracle import ref  # noqa: E402
from paper_1711_11361_amd import cc  # noqa: E402
from paper_1711_11361_amd import workloads as W  # noqa: E402

FP64_TOL = 1e-12


def pair(w, precision=cc.CC_FP64, prim=None):
    o = ref.Oracle(w["grid"], w["body"])
    s = cc.Solver(w["grid"], w["body"], precision=precision)
    p = w["prim"] if prim is None else prim
    o.set_prim(p)
    s.set_prim(p)
    return o, s


def scales(U, gamma=1.4):
    """Per-component scales of a conserved state: max|rho|, max|E|, and for both momentum
    components the characteristic momentum max rho (|u| + a).  A momentum component of a
    quiescent or one-directional flow is nearly zero everywhere, so its own maximum would
    measure round-off of near-cancelling terms rather than disagreement."""
    r = np.where(U[0] > 0, U[0], 1.0)
    p = (gamma - 1.0) * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / r)
    a = np.sqrt(np.maximum(gamma * p / r, 0.0))
    mom = np.where(U[0] > 0, np.hypot(U[1], U[2]) + U[0] * a, 0.0).max()
    sc = np.array([np.abs(U[0]).max(), mom, mom, np.abs(U[3]).max()])
    return np.where(sc > 0, sc, 1.0)


def worst_cell(a, b):
    sc = scales(b)[:, None, None]
    k, j, i = np.unravel_index(np.argmax(np.abs(a - b) / sc), a.shape)
    return int(k), int(j), int(i)


def rel_linf(a, b):
    """max over components of max|a-b| / scale (scales() of the oracle state)."""
    sc = scales(b)
    return max(np.abs(a[k] - b[k]).max() / sc[k] for k in range(4))


def geometry_cases():
    yield "piston30", W.piston()
    yield "piston_ragged", W.piston(nx=37, ny=23, angle_deg=47.0, face=(0.3, 0.04))
    yield "cylinder", W.cylinder(nx=128, ny=64)
    for seed in (0, 5):
        yield f"triangle{seed}", W.triangle_case(seed, nx=96, ny=48)
    w = W.naca(nx=96, ny=96)
    yield "naca", w
    # many edges per item: vertex tiles and chain searches one item per thread
    w = W.naca(nx=512, ny=512)
    w["body"]["pitch_amp"] = math.radians(8.0)
    w["body"]["pitch_omega"] = 2.0
    yield "naca_fine_pitch", w
    # a 2048-gon a few cells across: more uncertain edges per vertex tile than the tile lists
    yield "circle2048_coarse", W.cylinder(nx=32, ny=16, radius=0.3, n_poly=2048)
    for k in (0, 1, 2, 3, 7, 11):
        r = W.serving_request(k)
        yield f"req{k}", r


@pytest.mark.parametrize("name,w", list(geometry_cases()), ids=[c[0] for c in geometry_cases()])
def test_geometry_matches_oracle(name, w):
    o = ref.Oracle(w["grid"], w["body"])
    s = cc.Solver(w["grid"], w["body"])
    for t in (0.0, 0.0123, 0.37):
        o.geometry(t, 0)
        s.geometry(t, 0)
        a, b = s.geometry_dump(0), o.geometry_dump(0)
        assert np.array_equal(a["vcls"], b["vcls"]), name
        # the compacted cut-cell list: bit-exact, sorted by linear index
        assert np.array_equal(a["cut"], o.cut_list(0)), name
        for key in ("alpha", "bx", "by"):
            # two different exact clipping algorithms: round-off of the polygon coordinates
            # relative to the cell (the piston quads reach ~4 units away) is the bound
            assert np.abs(a[key] - b[key]).max() <= 1e-12, (name, key, np.abs(a[key] - b[key]).max())
            # open / closed classification of faces and cells is exact
            assert np.array_equal(a[key] == 1.0, b[key] == 1.0) and np.array_equal(a[key] == 0.0, b[key] == 0.0)


def sweep_cases():
    """(name, workload, oracle-only steps before the comparison, compared steps)."""
    yield "piston30", W.piston(), 0, 6
    yield "piston_reflective", W.piston(nx=64, ny=16, bc=(1, 1, 1, 1)), 0, 6
    yield "cylinder", W.cylinder(nx=128, ny=64), 0, 6
    yield "cylinder_no_threshold", W.cylinder(nx=128, ny=64, alpha_min=0.0), 0, 4
    # cut cells collapse before (from step 64) and after covering (step 99)
    yield "cylinder_collapses", W.cylinder(nx=128, ny=64), 60, 45
    yield "triangle", W.triangle_case(2, nx=96, ny=48), 0, 6
    w = W.naca(nx=96, ny=96)
    w["body"]["pitch_amp"] = math.radians(8.0)
    w["body"]["pitch_omega"] = 2.0
    yield "naca_pitch", w, 0, 6
    yield "nobody_ragged", {**W.cylinder(nx=61, ny=29), "body": None}, 0, 4
    for k in (0, 3, 7):
        yield f"req{k}", W.serving_request(k), 0, 4
    # impulsive starts: collapses before and after covering in the first step
    for k in (4, 10):
        yield f"req{k}_impulsive", W.serving_request(k), 0, 2


@pytest.mark.parametrize("name,w,skip,nsteps", list(sweep_cases()), ids=[c[0] for c in sweep_cases()])
def test_sweeps_match_oracle_from_identical_inputs(name, w, skip, nsteps):
    o, s = pair(w)
    for _ in range(skip):
        o.step(o.cfl_dt(w["cfl"]))
    if skip:
        s.set_clock(o.t, o.steps)
    c0 = o.collapses
    worst = 0.0
    for k in range(nsteps):
        dt = o.cfl_dt(w["cfl"])
        s.set_u(o.get_u())  # identical inputs for the time step as well
        dg = s.cfl_dt(w["cfl"])
        assert abs(dg - dt) <= 1e-12 * dt, (name, dg, dt)
        o.begin_step(dt)
        s.begin_step(dt)
        for sw in range(2):
            d = o.parity if sw == 0 else 1 - o.parity
            s.set_u(o.get_u())  # identical inputs
            o.sweep(d, dt)
            s.sweep(d, dt)
            Ug, Uo = s.get_u(), o.get_u()
            e = rel_linf(Ug, Uo)
            worst = max(worst, e)
            if e > FP64_TOL:
                c, j, i = worst_cell(Ug, Uo)
                gs = o.geometry_dump(0 if sw == 0 else 1)["alpha"][j, i]
                ge = o.geometry_dump(1 if sw == 0 else 2)["alpha"][j, i]
                raise AssertionError(f"{name} step {k} sweep {sw}: rel {e:.3e} at comp {c} cell ({i},{j}) "
                                     f"alpha_s {gs:.3e} alpha_e {ge:.3e} gpu {Ug[:, j, i]} oracle {Uo[:, j, i]}")
        o.end_step()
        s.end_step()
    assert s.info()["status"] == 0 and o.status == 0
    assert s.info()["collapses"] == o.collapses - c0


def test_end_time_parity_config1():
    w = W.piston()
    o, s = pair(w)
    dts = o.run(w["cfl"], t_end=w["t_end"])
    s.run(w["cfl"], dts=dts)
    Ug, Uo = s.get_u(), o.get_u()
    for k in range(4):
        den = np.abs(Uo[k]).sum()
        if den > 0:
            assert np.abs(Ug[k] - Uo[k]).sum() / den <= 1e-9, k
    # totals are sums of U times the cell area, so |Tg - To| <= area sum|Ug - Uo| per
    # component: the end-time L1 bar above bounds them by 1e-9 area sum|Uo|
    To, Tg = o.totals(), s.totals()
    area = (w["grid"]["x_hi"] - w["grid"]["x_lo"]) / o.nx * (w["grid"]["y_hi"] - w["grid"]["y_lo"]) / o.ny
    for k in range(4):
        assert abs(Tg[k] - To[k]) <= 1e-9 * area * np.abs(Uo[k]).sum(), k


def test_fp32_state_against_fp64_oracle():
    w = W.cylinder(nx=256, ny=128)
    o, s = pair(w, precision=cc.CC_FP32_GEOM64)
    dts = o.run(w["cfl"], nsteps=60)
    s.run(w["cfl"], dts=dts)
    Po, Pg = o.get_prim(), s.get_prim()
    al = o.geometry_dump(0)["alpha"]
    l1 = (al * np.abs(Pg[0] - Po[0])).sum() / (al * np.abs(Po[0])).sum()
    assert l1 <= 1e-4, l1


def vw_l1_density(Ug, Uo, alpha):
    """Volume-weighted relative L1 of the density, (sum alpha |rho_g - rho_o|) / sum alpha
    rho_o over cells with gas in both (densities per unit fluid volume)."""
    m = (alpha > 0) & (Uo[0] > 0) & (Ug[0] > 0)
    rg, ro = Ug[0][m] / alpha[m], Uo[0][m] / alpha[m]
    return float((alpha[m] * np.abs(rg - ro)).sum() / (alpha[m] * ro).sum())


@pytest.mark.parametrize("which", ["cylinder_1024x512", "triangle_2048x1024", "naca_4096x4096"])
def test_full_size_one_step(which):
    """One step at full size in both precisions against one FP64 oracle step: FP64 to the
    per-step bar; FP32 state within its own rounding (about 1e-7 relative per operation, a
    few hundred operations per cell: 1e-4 of the scale at any cell, 1e-5 in L1 density)."""
    if which.startswith("cylinder"):
        w = W.cylinder()
    elif which.startswith("triangle"):
        w = W.triangle_case(0)
    else:
        w = W.naca()
    o = ref.Oracle(w["grid"], w["body"], parallel=True)
    o.set_prim(w["prim"])
    dt = o.cfl_dt(w["cfl"])
    o.step(dt)
    Uo = o.get_u()
    al = o.geometry_dump(0)["alpha"]
    for prec in (cc.CC_FP64, cc.CC_FP32_GEOM64):
        s = cc.Solver(w["grid"], w["body"], precision=prec)
        s.set_prim(w["prim"])
        dg = s.cfl_dt(w["cfl"])
        s.step(dt)
        Ug = s.get_u()
        e = rel_linf(Ug, Uo)
        if prec == cc.CC_FP64:
            assert abs(dg - dt) <= 1e-12 * dt
            assert e <= FP64_TOL, e
        else:
            assert abs(dg - dt) <= 1e-5 * dt
            l1 = vw_l1_density(Ug, Uo, al)
            print(f"{which} FP32 state, one step: rel Linf {e:.2e}, L1 density {l1:.2e}")
            assert e <= 1e-4 and l1 <= 1e-5, (e, l1)
        s.close()


def test_fp32_state_at_the_benchmark_size_over_200_steps():
    """The headline configuration (1024 x 512 cylinder crossing the Mach-2 shock, FP32 state
    with FP64 geometry) against the FP64 oracle over 200 steps with the oracle's time steps:
    relative L1 of density <= 1e-4 (the stated accuracy); the GPU's mass drift over the run
    (mass change minus its budget, per initial mass) is stated."""
    w = W.cylinder()
    o = ref.Oracle(w["grid"], w["body"], parallel=True)
    o.set_prim(w["prim"])
    dts = o.run(w["cfl"], nsteps=200)
    s = cc.Solver(w["grid"], w["body"], precision=cc.CC_FP32_GEOM64)
    s.set_prim(w["prim"])
    s.set_budget(True)
    T0 = s.totals()
    s.run(w["cfl"], dts=dts)
    T1, (bnd, wall, lost) = cc.cc_totals(s.ctx, True)
    l1 = vw_l1_density(s.get_u(), o.get_u(), o.geometry_dump(0)["alpha"])
    drift = abs((T1[0] - T0[0]) - bnd[0] - wall[0] + lost[0]) / T0[0]
    print(f"1024x512 cylinder, 200 steps, FP32 state: L1 density {l1:.2e}, mass drift {drift:.2e}")
    assert l1 <= 1e-4, l1
    assert drift <= 1e-5, drift
    assert s.info()["status"] == 0 and o.status == 0


def test_sixteen_triangle_seeds_batched_against_the_oracle():
    """The 16-seed triangle workload at 2048 x 1024 (FP32 state, FP64 geometry) stepped as one
    batch, each member compared with its own FP64 oracle run over two steps (the oracle's
    time steps): relative L1 of density <= 1e-5 for every member."""
    seeds = range(16)
    b = cc.Batch(16, cc.CC_FP32_GEOM64)
    sol, dts = [], []
    for seed in seeds:
        w = W.triangle_case(seed)
        s = cc.Solver(w["grid"], w["body"], precision=cc.CC_FP32_GEOM64)
        s.set_prim(w["prim"])
        b.add(s)
        sol.append(s)
    ref_states = []
    for seed in seeds:
        w = W.triangle_case(seed)
        o = ref.Oracle(w["grid"], w["body"], parallel=True)
        o.set_prim(w["prim"])
        d = o.run(w["cfl"], nsteps=2)
        dts.append(d)
        ref_states.append((o.get_u(), o.geometry_dump(0)["alpha"]))
        o.close()
    for k in range(2):
        b.step([d[k] for d in dts])
    for seed, s, (Uo, al) in zip(seeds, sol, ref_states):
        l1 = vw_l1_density(s.get_u(), Uo, al)
        assert l1 <= 1e-5, (seed, l1)
    for s in sol:
        b.remove(s)
        s.close()
    b.close()


def test_restart_from_saved_state_is_bit_exact():
    """cc_set_clock + cc_set_u resume a saved (t, step count, U) bit for bit."""
    w = W.cylinder(nx=128, ny=64)
    s = cc.Solver(w["grid"], w["body"])
    s.set_prim(w["prim"])
    dts, saved = [], None
    for k in range(9):
        if k == 4:
            saved = (s.get_u(), s.info()["t"])
        dt = s.cfl_dt(w["cfl"])
        dts.append(dt)
        s.step(dt)
    r = cc.Solver(w["grid"], w["body"])
    r.set_prim(w["prim"])
    r.run(w["cfl"], dts=[0.6 * dt for dt in dts[:6]])
    r.set_clock(saved[1], 4)
    r.set_u(saved[0])
    for dt in dts[4:]:
        r.step(dt)
    assert r.info()["steps"] == 9
    assert np.array_equal(r.get_u(), s.get_u())


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
def test_every_tile_shape_gives_identical_results(precision):
    """The dense-sweep tile shapes only change the schedule: two steps from the same state
    agree bit for bit across all shapes, on a ragged grid with reflective walls and a body;
    the tuner's choice is one of them."""
    w = W.cylinder(nx=203, ny=77)
    w["grid"]["bc"] = (1, 0, 1, 1)
    # 64-column tiles staged in LDS (8, 12 rows; 16, 24 with FP32 state) and column walks
    # (4, 8 rows of 256 columns)
    ys = [0, 1, 2, 3, 4, 5] if precision == cc.CC_FP32_GEOM64 else [0, 1, 4]
    ref_u = None
    for tx in range(4):
        for ty in ys:
            s = cc.Solver(w["grid"], w["body"], precision=precision)
            s.set_prim(w["prim"])
            s.set_tiles(tx, ty)
            for dt in (1.5e-3, 1.8e-3):
                s.step(dt)
            U = s.get_u()
            if ref_u is None:
                ref_u = U
            assert np.array_equal(U, ref_u), (tx, ty)
    s = cc.Solver(w["grid"], w["body"], precision=precision)
    s.set_prim(w["prim"])
    tx, ty = s.autotune(reps=3)
    assert 0 <= tx < 4 and ty in ys
    with pytest.raises(cc.CCError):
        s.set_tiles(0, 9)


def loads_cases():
    """(name, workload, oracle steps before the comparison)."""
    yield "piston30", W.piston(), 40
    yield "piston_aligned", W.piston(angle_deg=0.0), 40
    yield "cylinder", W.cylinder(nx=128, ny=64), 30
    w = W.naca(nx=96, ny=96)
    w["body"]["pitch_amp"] = math.radians(8.0)
    w["body"]["pitch_omega"] = 2.0
    yield "naca_pitch", w, 10
    yield "req3", W.serving_request(3), 10


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
@pytest.mark.parametrize("name,w,nsteps", list(loads_cases()), ids=[c[0] for c in loads_cases()])
def test_surface_loads_match_oracle(name, w, nsteps, precision):
    """Force and moment on the body from identical states: round-off in FP64 (the sums run
    in another order), the state's FP32 rounding otherwise; relative to sum p*|N|."""
    o, s = pair(w, precision)
    for _ in range(nsteps):
        o.step(o.cfl_dt(w["cfl"]))
    s.set_clock(o.t, o.steps)
    s.set_u(o.get_u())
    lo, lg = o.surface_loads(), s.surface_loads()
    g = w["grid"]
    size = max(g["x_hi"] - g["x_lo"], g["y_hi"] - g["y_lo"])
    tol = 1e-12 if precision == cc.CC_FP64 else 1e-5
    assert lo[3] > 0.0
    assert abs(lg[0] - lo[0]) <= tol * lo[3] and abs(lg[1] - lo[1]) <= tol * lo[3], (name, lg, lo)
    assert abs(lg[2] - lo[2]) <= tol * lo[3] * size and abs(lg[3] - lo[3]) <= tol * lo[3], (name, lg, lo)


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
@pytest.mark.parametrize("name,w,nsteps", list(loads_cases()), ids=[c[0] for c in loads_cases()])
def test_surface_pressure_matches_oracle(name, w, nsteps, precision):
    """The wall pressure distribution from identical states: the same wall cells in the
    same order (bit-exact indices), wall points and normals to round-off, p* to round-off in
    FP64 (relative to the largest p*, and to the cell's own p* over its volume fraction) and
    to the state's FP32 rounding otherwise."""
    o, s = pair(w, precision)
    for _ in range(nsteps):
        o.step(o.cfl_dt(w["cfl"]))
    s.set_clock(o.t, o.steps)
    s.set_u(o.get_u())
    ro, rg = o.surface_pressure(), s.surface_pressure()
    assert len(ro) > 0 and np.array_equal(rg[:, 0], ro[:, 0]), name
    g = w["grid"]
    size = max(g["x_hi"] - g["x_lo"], g["y_hi"] - g["y_lo"])
    h = size / max(g["nx"], g["ny"])
    assert np.abs(rg[:, 1:3] - ro[:, 1:3]).max() <= 1e-12 * size, name
    assert np.abs(rg[:, 4:6] - ro[:, 4:6]).max() <= 1e-12 * h, name
    if precision == cc.CC_FP64:
        # p* follows the cell's state U / alpha, so the rounding in which the two exact
        # clipping algorithms differ (~1e-14 of a cell in alpha for coordinates of a few
        # units) appears divided by alpha in cells a body barely enters
        al = o.geometry_dump(0)["alpha"].reshape(-1)[ro[:, 0].astype(np.int64)]
        bound = 1e-12 * np.abs(ro[:, 3]).max() + 1e-13 * np.abs(ro[:, 3]) / al
        assert (np.abs(rg[:, 3] - ro[:, 3]) <= bound).all(), name
    else:
        assert np.abs(rg[:, 3] - ro[:, 3]).max() <= 1e-5 * np.abs(ro[:, 3]).max(), name
