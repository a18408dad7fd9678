"""Batched stepping (one launch per phase over many contexts, one captured graph per
membership) against contexts stepped alone, and the captured single-context step against
its individual launches: bit-identical states, with members joining and leaving between
steps (continuous batching)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1711_11361_amd import cc  # noqa: E402
from paper_1711_11361_amd import workloads as W  # noqa: E402


def small_requests():
    out = []
    for k in range(40):
        r = W.serving_request(k)
        if r["grid"]["nx"] * r["grid"]["ny"] <= 256 * 128:
            out.append(r)
        if len(out) == 6:
            break
    return out


def solver(w, precision):
    s = cc.Solver(w["grid"], w["body"], precision=precision)
    s.set_prim(w["prim"])
    return s


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
@pytest.mark.parametrize("mode", [cc.CC_LAUNCH_PER_PHASE, cc.CC_LAUNCH_PERSISTENT])
def test_graph_step_equals_individual_launches(precision, mode):
    w = W.cylinder(nx=128, ny=64)
    a, b = solver(w, precision), solver(w, precision)
    a.set_launch_mode(mode)
    for _ in range(7):
        dt = a.cfl_dt(w["cfl"])  # from the speeds the captured step folded in
        assert dt == b.cfl_dt(w["cfl"])  # from a separate reduction of the state
        a.step(dt)  # captured graph
        b.begin_step(dt)
        for d in (b.parity, 1 - b.parity):
            b.sweep(d, dt)
        b.end_step()
    assert np.array_equal(a.get_u(), b.get_u())
    assert a.info()["status"] == 0


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
def test_folded_speeds_after_collapse_rounds(precision):
    """A cylinder started impulsively into gas at rest, moving down and to the right, has
    its fastest gas in the lower front of its box and collapses cut cells in its first
    steps.  When a step's last sweep ran collapse rounds, its combine block recomputes the
    speeds of the box cells (about nine per thread here), and the time step from the
    folded speeds must equal a separate reduction of the state."""
    g = W.grid(128, 128, 0.0, 2.0, 0.0, 1.0, alpha_min=W.SMALL_CELL)
    bd = W.body(W.circle(0.2, 40), ref=(0.5, 0.5), vel=(2.0, -1.2))
    w = {"grid": g, "body": bd, "prim": W.uniform_prim(g, 1.0, 0.0, 0.0, 1.0)}
    a, b = solver(w, precision), solver(w, precision)
    for _ in range(5):
        dt = a.cfl_dt(0.5)  # folded into the previous captured step
        assert dt == b.cfl_dt(0.5)  # separate reduction
        a.step(dt)
        b.begin_step(dt)
        for d in (b.parity, 1 - b.parity):
            b.sweep(d, dt)
        b.end_step()
    assert a.info()["collapses"] == b.info()["collapses"] > 0
    assert np.array_equal(a.get_u(), b.get_u())
    assert a.cfl_dt(0.5) == b.cfl_dt(0.5)


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
@pytest.mark.parametrize("mode", [cc.CC_LAUNCH_PER_PHASE, cc.CC_LAUNCH_PERSISTENT])
def test_batch_equals_members_alone(precision, mode):
    reqs = small_requests()
    alone = [solver(w, precision) for w in reqs]
    mem = [solver(w, precision) for w in reqs]
    dts = []
    for s, w in zip(alone, reqs):
        d = []
        for _ in range(6):
            dt = s.cfl_dt(w["cfl"])
            s.step(dt)
            d.append(dt)
        dts.append(d)
    B = cc.Batch(8, precision)
    B.set_launch_mode(mode)
    for s in mem:
        B.add(s)
    for k in range(6):
        st = B.step([d[k] for d in dts])
        assert st == [0] * len(mem)
    for a, m in zip(alone, mem):
        assert np.array_equal(a.get_u(), m.get_u())
        assert a.info()["steps"] == m.info()["steps"] == 6
    # the speeds the batch reduced give the same next time steps as each member's own
    nxt, status = B.last_dt(reqs[0]["cfl"])
    own = [m.cfl_dt(w["cfl"]) for m, w in zip(mem, reqs)]
    assert status == [0] * len(mem)
    np.testing.assert_allclose(nxt, own, rtol=0, atol=0)


def test_members_join_and_leave():
    reqs = small_requests()
    p = cc.CC_FP32_GEOM64
    alone = [solver(w, p) for w in reqs]
    mem = [solver(w, p) for w in reqs]
    # member k joins at step k and leaves after 4 steps; the batch steps 9 times
    B = cc.Batch(4, p)
    active = []
    for step in range(9):
        for k in range(len(reqs)):
            if k == step and len(active) < 4:
                B.add(mem[k])
                active.append(k)
        dts = [alone[k].cfl_dt(reqs[k]["cfl"]) for k in active]
        for k, dt in zip(active, dts):
            alone[k].step(dt)
        B.step(dts)
        for k in list(active):
            if mem[k].info()["steps"] == 4:
                B.remove(mem[k])
                active.remove(k)
    for a, m in zip(alone, mem):
        assert np.array_equal(a.get_u(), m.get_u())
    # a removed member steps on its own again
    mem[0].step(mem[0].cfl_dt(reqs[0]["cfl"]))


def test_batch_refuses_misuse():
    reqs = small_requests()
    s64 = solver(reqs[0], cc.CC_FP64)
    s32 = solver(reqs[1], cc.CC_FP32_GEOM64)
    B = cc.Batch(1, cc.CC_FP64)
    with pytest.raises(cc.CCError):
        B.add(s32)  # other precision
    B.add(s64)
    with pytest.raises(cc.CCError):
        B.add(solver(reqs[2], cc.CC_FP64))  # full
    with pytest.raises(cc.CCError):
        s64.step(1e-4)  # stepped by its batch


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
def test_large_batch_with_its_own_box_launch_equals_members_alone(precision):
    """Five 1024 x 512 cylinders (2.6 M cells) in one batch: its x sweeps run the box cells'
    first phase in a launch of its own, the members alone in the x launch; the results are
    the same bit for bit."""
    ws = []
    for q in range(5):
        w = W.cylinder()
        w["body"]["vel"] = (0.6 + 0.2 * q, 0.05 * (q - 2))
        ws.append(w)
    alone = []
    for w in ws:
        s = solver(w, precision)
        assert s.info()["x_with_box"]
        dts = []
        for _ in range(4):
            dt = s.cfl_dt(w["cfl"])
            dts.append(dt)
            s.step(dt)
        alone.append((dts, s.get_u()))
        s.close()
    b = cc.Batch(len(ws), precision)
    members = []
    for w in ws:
        s = solver(w, precision)
        b.add(s)
        members.append(s)
    for k in range(4):
        b.step([a[0][k] for a in alone])
    for q, s in enumerate(members):
        assert np.array_equal(s.get_u(), alone[q][1]), q
        b.remove(s)
        s.close()
    b.close()
