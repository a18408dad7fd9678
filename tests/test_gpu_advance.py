"""Steps planned on the device (cc_advance: the CFL time step, poses, regions and sweep
boxes computed by a block at the head of each step) against the host-planned path
(cc_cfl_dt + cc_step): the same time steps and states, bit for bit, for bodies that do not
turn; for a pitching body, whose angle comes from the device's sin and cos, agreement to
round-off; the same refusal at the same step; the host's bookkeeping (clock, step count,
direction order, level regions) taken over exactly, so host and device steps interleave."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1711_11361_amd import cc  # noqa: E402
from paper_1711_11361_amd import workloads as W  # noqa: E402


def solver(w, precision):
    s = cc.Solver(w["grid"], w["body"], precision=precision)
    s.set_prim(w["prim"])
    return s


def fixed_bodies():
    yield "cylinder", W.cylinder(nx=128, ny=64)
    yield "piston", W.piston()
    yield "triangle", W.triangle_case(3, nx=96, ny=48)
    yield "nobody", {**W.cylinder(nx=61, ny=29), "body": None}
    for k in range(40):
        r = W.serving_request(k)
        if r["body"]["pitch_amp"] == 0.0 and r["grid"]["nx"] * r["grid"]["ny"] <= 256 * 128:
            yield f"req{k}", r
            break


def host_steps(s, cfl, n):
    dts = []
    for _ in range(n):
        dt = s.cfl_dt(cfl)
        s.step(dt)
        dts.append(dt)
    return np.array(dts)


@pytest.mark.parametrize("timed", [True, False], ids=["per_step_graphs", "runs_of_steps"])
@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
@pytest.mark.parametrize("name,w", list(fixed_bodies()), ids=[c[0] for c in fixed_bodies()])
def test_device_planned_steps_equal_host_planned(name, w, precision, timed):
    """Timed runs launch one graph per step (events between steps); untimed runs launch
    graphs of several steps and single steps for the remainder (9 = 4 + 4 + 1)."""
    n = 9
    a, b = solver(w, precision), solver(w, precision)
    da = host_steps(a, w["cfl"], n)
    db, ms = b.advance(n, w["cfl"], want_ms=timed)
    assert np.array_equal(da, db), (name, da, db)
    assert np.array_equal(a.get_u(), b.get_u()), name
    ia, ib = a.info(), b.info()
    for key in ("t", "steps", "parity", "status", "collapses", "box_cells"):
        assert ia[key] == ib[key], (name, key, ia[key], ib[key])
    if timed:
        assert ms.shape == (n,) and np.all(ms > 0.0)
    else:
        assert ms is None
    # the host's bookkeeping continues from the device's: further steps either way agree
    da2 = host_steps(a, w["cfl"], 3)
    db2 = host_steps(b, w["cfl"], 3)
    assert np.array_equal(da2, db2)
    assert np.array_equal(a.get_u(), b.get_u()), name
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
def test_interleaved_host_and_device_steps(precision):
    w = W.cylinder(nx=128, ny=64)
    a, b = solver(w, precision), solver(w, precision)
    da = host_steps(a, w["cfl"], 10)
    d1 = host_steps(b, w["cfl"], 3)
    d2, _ = b.advance(4, w["cfl"])
    d3 = host_steps(b, w["cfl"], 3)
    assert np.array_equal(da, np.concatenate([d1, d2, d3]))
    assert np.array_equal(a.get_u(), b.get_u())


def test_pitching_body_agrees_to_round_off():
    w = W.naca(nx=96, ny=96)
    w["body"]["pitch_amp"] = np.radians(8.0)
    w["body"]["pitch_omega"] = 2.0
    a, b = solver(w, cc.CC_FP64), solver(w, cc.CC_FP64)
    n = 8
    da = host_steps(a, w["cfl"], n)
    db, _ = b.advance(n, w["cfl"])
    assert np.abs(da - db).max() <= 1e-13 * da.max()
    Ua, Ub = a.get_u(), b.get_u()
    err = max(np.abs(Ua[k] - Ub[k]).max() / np.abs(Ua[k]).max() for k in range(4))
    assert err <= 1e-10, err
    assert a.info()["steps"] == b.info()["steps"] == n


def test_refusal_at_the_same_step():
    # a body faster than every signal of the gas at CFL 1.5 moves more than a cell per sweep
    w = W.cylinder(nx=64, ny=32, speed=6.0)
    a, b = solver(w, cc.CC_FP64), solver(w, cc.CC_FP64)
    dt = a.cfl_dt(1.5)
    with pytest.raises(cc.CCError) as ea:
        a.step(dt)
    with pytest.raises(cc.CCError) as eb:
        b.advance(3, 1.5)
    assert ea.value.status == eb.value.status == cc.CC_ERR_MOTION
    assert eb.value.done == 0
    assert np.array_equal(a.get_u(), b.get_u())
    assert b.info()["steps"] == 0
    # a smaller CFL number still steps afterwards, the same way on both paths
    da = host_steps(a, 0.3, 2)
    db, _ = b.advance(2, 0.3)
    assert np.array_equal(da, db)
    assert np.array_equal(a.get_u(), b.get_u())


@pytest.mark.parametrize("name", ["cylinder_1024x512", "naca_4096x4096"])
def test_full_size_device_planned_steps(name):
    """The benchmark's grid (bit for bit) and the pitching aerofoil's (round-off)."""
    w = W.cylinder() if name.startswith("cylinder") else W.naca()
    a, b = solver(w, cc.CC_FP32_GEOM64), solver(w, cc.CC_FP32_GEOM64)
    n = 4
    da = host_steps(a, w["cfl"], n)
    db, _ = b.advance(n, w["cfl"])
    Ua, Ub = a.get_u(), b.get_u()
    if name.startswith("cylinder"):
        assert np.array_equal(da, db) and np.array_equal(Ua, Ub)
    else:
        assert np.abs(da - db).max() <= 1e-12 * da.max()
        err = max(np.abs(Ua[k] - Ub[k]).max() / np.abs(Ua[k]).max() for k in range(4))
        assert err <= 1e-5, err  # FP32 state: one rounding of the state apart at most
    assert a.info()["status"] == b.info()["status"] == 0
    a.close()
    b.close()


def small_mix():
    out = []
    for k in range(40):
        r = W.serving_request(k)
        if r["grid"]["nx"] * r["grid"]["ny"] <= 256 * 128:
            out.append(r)
        if len(out) == 6:
            break
    return out


@pytest.mark.parametrize("timed", [True, False], ids=["per_step_graphs", "runs_of_steps"])
@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
def test_batch_advance_equals_members_advanced_alone(precision, timed):
    """A batch of mixed requests (turning and translating bodies, both direction orders
    after an odd step) planned on the device equals each member advanced alone, bit for
    bit; and, for the members that do not turn, the host-planned batch step."""
    reqs = small_mix()
    cfl = reqs[0]["cfl"]
    alone = [solver(w, precision) for w in reqs]
    mem = [solver(w, precision) for w in reqs]
    host = [solver(w, precision) for w in reqs]
    # one host step first, so that the members' direction orders differ from the batch's start
    for s in alone + mem + host:
        s.step(s.cfl_dt(cfl))
    n = 7
    da = [s.advance(n, cfl)[0] for s in alone]
    b = cc.Batch(len(mem), precision)
    for s in mem:
        b.add(s)
    db, ms = b.advance(n, cfl, want_ms=timed)
    assert ms is None if not timed else (ms.shape == (n,) and np.all(ms > 0))
    hb = cc.Batch(len(host), precision)
    for s in host:
        hb.add(s)
    dh = []
    d = hb.cfl_dt(cfl)
    for _ in range(n):
        dh.append(d)
        hb.step(d)
        d, st = hb.last_dt(cfl)
    for k, (w, a, m, h) in enumerate(zip(reqs, alone, mem, host)):
        assert np.array_equal(da[k], db[k]), k
        assert np.array_equal(a.get_u(), m.get_u()), k
        assert a.info()["steps"] == m.info()["steps"]
        if w["body"]["pitch_amp"] == 0.0:
            assert np.array_equal(np.array([x[k] for x in dh]), db[k]), k
            assert np.array_equal(h.get_u(), m.get_u()), k
    for s in mem:
        b.remove(s)
    for s in host:
        hb.remove(s)
    b.close()
    hb.close()


def test_reset_of_an_advanced_context():
    """cc_set_clock / cc_set_state on a context whose body has travelled far (its level
    slots hold cut-cell boxes of a later time) start the run again exactly as a fresh
    context: the same time steps and states, bit for bit, device- and host-planned."""
    w = W.cylinder(nx=256, ny=128)
    fresh = solver(w, cc.CC_FP64)
    d_ref, _ = fresh.advance(40, w["cfl"])
    u_ref = fresh.get_u()
    fresh.close()
    s = solver(w, cc.CC_FP64)
    for reset in ("state", "clock", "host"):
        s.advance(500, w["cfl"])
        assert s.info()["t"] > 0.5  # the cylinder has moved more than 64 cells
        if reset == "clock":
            s.set_clock(0.0, 0)
        s.set_prim(w["prim"])
        if reset == "host":
            for dt in d_ref:
                s.step(dt)
        else:
            d, _ = s.advance(40, w["cfl"])
            assert np.array_equal(np.asarray(d), np.asarray(d_ref)), reset
        assert np.array_equal(s.get_u(), u_ref), reset
    s.close()
