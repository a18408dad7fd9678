"""The conservation budget on the GPU (Sec. 3.3: mass-conservation error), through the C ABI.

* per sweep, from identical inputs: the change of the GPU's budget (domain-boundary fluxes,
  wall terms, residuals without recipients) equals the oracle's, to round-off of sums taken
  in another order;
* the GPU's own totals change by boundary + wall - lost, to round-off (FP64 state), and up to
  the state's rounding with FP32 state (the mass drift, stated);
* captured steps, device-planned steps and batches track the same budget as single sweeps.
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

EPS = 2.0 ** -52


def area_of(g):
    return (g["x_hi"] - g["x_lo"]) / g["nx"] * (g["y_hi"] - g["y_lo"]) / g["ny"]


def cases():
    yield "piston30", W.piston(), 6          # body box on the domain boundary: faces in the box
    yield "piston_reflective", W.piston(nx=64, ny=16, bc=(1, 1, 1, 1)), 4
    yield "cylinder", W.cylinder(nx=128, ny=64), 5
    yield "req10_impulsive", W.serving_request(10), 2   # collapses before and after covering
    w = W.naca(nx=96, ny=96)
    w["body"]["pitch_amp"] = math.radians(8.0)
    w["body"]["pitch_omega"] = 2.0
    yield "naca_pitch", w, 4
    yield "nobody_ragged", {**W.cylinder(nx=61, ny=29), "body": None}, 3


@pytest.mark.parametrize("name,w,nsteps", list(cases()), ids=[c[0] for c in cases()])
def test_budget_per_sweep_matches_oracle(name, w, nsteps):
    o = ref.Oracle(w["grid"], w["body"])
    s = cc.Solver(w["grid"], w["body"])
    o.set_prim(w["prim"])
    s.set_prim(w["prim"])
    s.set_budget(True)
    area = area_of(w["grid"])
    for k in range(nsteps):
        dt = o.cfl_dt(w["cfl"])
        o.begin_step(dt)
        s.begin_step(dt)
        for sw in range(2):
            d = o.parity if sw == 0 else 1 - o.parity
            s.set_u(o.get_u())  # identical inputs
            ob0, gb0 = o.budget(), s.budget()
            T0 = s.totals()
            # round-off scale: the total magnitude of the state (a component that cancels,
            # such as the y-momentum wall force on a symmetric body, has no scale of its own)
            mag = np.abs(o.get_u()).sum() * area
            o.sweep(d, dt)
            s.sweep(d, dt)
            ob1, gb1 = o.budget(), s.budget()
            T1 = s.totals()
            for part in range(3):
                do, dg = ob1[part] - ob0[part], gb1[part] - gb0[part]
                tol = 1e-11 * np.abs(do) + 1e-14 * mag
                assert (np.abs(dg - do) <= tol).all(), (name, k, sw, part, dg, do)
            # the GPU's totals move by its own budget
            resid = (T1 - T0) - (gb1[0] - gb0[0]) - (gb1[1] - gb0[1]) + (gb1[2] - gb0[2])
            bound = 64 * EPS * mag * max(1.0, math.sqrt(o.nx * o.ny) / 64)
            assert (np.abs(resid) <= bound).all(), (name, k, sw, resid)
        o.end_step()
        s.end_step()
    if name == "req10_impulsive":
        assert o.collapses > 0


def run_budget(w, precision, mode, nsteps):
    """(totals at start, totals at end, budget) of nsteps CFL steps taken as `mode`."""
    s = cc.Solver(w["grid"], w["body"], precision=precision)
    s.set_prim(w["prim"])
    s.set_budget(True)
    T0 = s.totals()
    if mode == "captured":
        for _ in range(nsteps):
            s.step(s.cfl_dt(w["cfl"]))
    elif mode == "planned":
        s.advance(nsteps, w["cfl"])
    else:
        b = cc.Batch(2, precision)
        other = cc.Solver(w["grid"], w["body"], precision=precision)
        other.set_prim(w["prim"])
        b.add(other)
        b.add(s)
        b.advance(nsteps, w["cfl"])
        b.remove(other)
        b.remove(s)
        b.close()
    return T0, s.totals(), s.budget(), s


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
def test_budget_is_the_same_in_every_launch_path(precision):
    """Single sweeps, captured steps, device-planned steps and a batch member track one
    budget (bit for bit: the same kernels with the same partial sums)."""
    w = W.cylinder(nx=160, ny=80)
    ref_run = None
    for mode in ("captured", "planned", "batch"):
        T0, T1, bud, _ = run_budget(w, precision, mode, 12)
        if ref_run is None:
            ref_run = (T1, bud)
        else:
            assert np.array_equal(T1, ref_run[0]), mode
            for part in range(3):
                assert np.array_equal(bud[part], ref_run[1][part]), (mode, part)


def test_fp32_mass_drift_is_small_and_fp64_is_round_off():
    """Mass drift = (change of the mass total - boundary - wall + lost mass) / initial mass:
    round-off with FP64 state, the FP32 state's rounding otherwise (stated, and bounded)."""
    w = W.cylinder(nx=256, ny=128)
    drift = {}
    for prec in (cc.CC_FP64, cc.CC_FP32_GEOM64):
        T0, T1, bud, s = run_budget(w, prec, "planned", 100)
        drift[prec] = abs((T1[0] - T0[0]) - bud[0][0] - bud[1][0] + bud[2][0]) / T0[0]
    assert drift[cc.CC_FP64] < 1e-13, drift
    assert drift[cc.CC_FP32_GEOM64] < 1e-5, drift
    print(f"mass drift over 100 steps: FP64 {drift[cc.CC_FP64]:.2e}, FP32 state {drift[cc.CC_FP32_GEOM64]:.2e}")


def test_budget_refused_in_the_persistent_mode():
    w = W.cylinder(nx=64, ny=32)
    s = cc.Solver(w["grid"], w["body"])
    s.set_prim(w["prim"])
    s.set_budget(True)
    with pytest.raises(cc.CCError) as e:
        s.set_launch_mode(cc.CC_LAUNCH_PERSISTENT)
    assert e.value.status == cc.CC_ERR_UNSUPPORTED
    s.set_budget(False)
    s.set_launch_mode(cc.CC_LAUNCH_PERSISTENT)
    with pytest.raises(cc.CCError) as e:
        s.set_budget(True)
    assert e.value.status == cc.CC_ERR_UNSUPPORTED
