"""C-ABI calls of the step's boundary beyond the step itself: the time step written to
device memory (cc_cfl_dt's d_dt), and the tile tuner of a batch with its cache file."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1711_11361_amd import cc  # noqa: E402
from paper_1711_11361_amd import workloads as W  # noqa: E402


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
def test_device_time_step_equals_host_time_step(precision):
    """d_dt is the host path's dt bit for bit, also for a pitching body (the wall speeds of
    its vertices enter) and after captured steps."""
    w = W.naca(nx=128, ny=128)
    w["body"]["pitch_amp"] = 0.2
    w["body"]["pitch_omega"] = 3.0
    s = cc.Solver(w["grid"], w["body"], precision=precision)
    s.set_prim(w["prim"])
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(5):
        with torch.cuda.stream(s.stream):
            s.cfl_dt_device(w["cfl"], out)
        s.stream.synchronize()
        dd = float(out.cpu().item())
        dh = s.cfl_dt(w["cfl"])
        assert dd == dh and dh > 0.0
        s.step(dh)


def test_batch_tuner_with_cache(tmp_path):
    """The batch tuner picks valid shapes, a second call takes them from the cache file
    without timing, and the results of a step do not depend on the shapes."""
    reqs = [W.serving_request(k) for k in (0, 3, 7)]
    b = cc.Batch(4, cc.CC_FP32_GEOM64)
    sol = []
    for r in reqs:
        s = cc.Solver(r["grid"], r["body"], precision=cc.CC_FP32_GEOM64)
        s.set_prim(r["prim"])
        b.add(s)
        sol.append(s)
    cache = str(tmp_path / "tiles.txt")
    tx, ty = b.autotune(reps=3, cache_path=cache)
    assert 0 <= tx < 4 and 0 <= ty < 6
    lines = open(cache).read().split("\n")
    assert len([ln for ln in lines if ln]) == 1 and lines[0].endswith(f" {tx} {ty}")
    key = lines[0].split()[0]
    assert all(f"{r['grid']['nx']}x{r['grid']['ny']}" in key for r in reqs)
    # a planted entry for the same key is taken as it is (no timing)
    with open(cache, "a") as f:
        f.write(f"{key} 3 4\n")
    assert b.autotune(reps=3, cache_path=cache) == (3, 4)
    dts = b.cfl_dt(0.8)
    b.step(dts)
    U_a = [s.get_u() for s in sol]
    # the same requests stepped alone with the default shapes
    for r, Ua in zip(reqs, U_a):
        s = cc.Solver(r["grid"], r["body"], precision=cc.CC_FP32_GEOM64)
        s.set_prim(r["prim"])
        s.step(s.cfl_dt(0.8))
        assert np.array_equal(s.get_u(), Ua)
    # a context's tuner uses the same cache format
    s = cc.Solver(reqs[0]["grid"], reqs[0]["body"], precision=cc.CC_FP32_GEOM64)
    s.set_prim(reqs[0]["prim"])
    c1 = s.autotune(reps=2, cache_path=cache)
    assert s.autotune(reps=2, cache_path=cache) == c1
    assert os.path.getsize(cache) > 0


@pytest.mark.parametrize("precision", [cc.CC_FP64, cc.CC_FP32_GEOM64])
def test_timed_steps_equal_captured_steps(precision):
    """The timing mode issues the captured step's launches one by one with events around the
    dense launches: the same results bit for bit, for a context and a batch, and one timed
    dense launch per sweep (per direction present in a batch)."""
    w = W.cylinder(nx=200, ny=96)
    runs = []
    for timed in (False, True):
        s = cc.Solver(w["grid"], w["body"], precision=precision)
        s.set_prim(w["prim"])
        cc.cc_timing(s.ctx, 1 if timed else 0)
        for _ in range(6):
            s.step(s.cfl_dt(w["cfl"]))
        t = cc.cc_timing_read(s.ctx)
        runs.append(s.get_u())
        if timed:
            assert t["dense_x"][1] == 6 and t["dense_y"][1] == 6 and t["dense_x"][0] > 0 and t["dense_y"][0] > 0
    assert np.array_equal(runs[0], runs[1])
    # a batch whose members sweep in different orders (one started a step later)
    res = []
    for timed in (False, True):
        b = cc.Batch(2, precision)
        sol = []
        for lag in (0, 1):
            s = cc.Solver(w["grid"], w["body"], precision=precision)
            s.set_prim(w["prim"])
            for _ in range(lag):
                s.step(s.cfl_dt(w["cfl"]))
            b.add(s)
            sol.append(s)
        cc.cc_batch_timing(b.b, 1 if timed else 0)
        dts = b.cfl_dt(w["cfl"])
        for _ in range(4):
            b.step(dts)
            dts, _ = b.last_dt(w["cfl"])
        t = cc.cc_batch_timing_read(b.b)
        if timed:
            assert t["dense_x"][1] == 8 and t["dense_y"][1] == 8
        res.append([s.get_u() for s in sol])
        for s in sol:
            b.remove(s)
        b.close()
    for a, c in zip(res[0], res[1]):
        assert np.array_equal(a, c)
