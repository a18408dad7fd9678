"""Serving with continuous batching: requests that arrive while others run are admitted
when a slot and memory free up, and each request's result is the same as when it runs
alone (bit for bit: the batched step computes exactly what the single-context step does,
and each request keeps its own CFL time step)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1711_11361_amd import cc, serving  # noqa: E402


def small_requests(n, steps):
    out, k = [], 0
    while len(out) < n:
        r = serving.Request(k, serving.W.serving_request(k), 0.0, steps)
        g = r.work["grid"]
        if g["nx"] * g["ny"] <= 256 * 128:
            out.append(r)
        k += 1
    # all arrive at once; with fewer slots than requests and uneven step counts, waiting
    # requests join while others are still running
    for j, r in enumerate(out):
        r.arrival = 0.0
        r.steps = steps + 2 * j
    return out


def alone(r, precision):
    s = cc.Solver(r.work["grid"], r.work["body"], precision=precision)
    s.set_prim(r.work["prim"])
    for _ in range(r.steps):
        s.step(s.cfl_dt(r.work["cfl"]))
    return s.get_u()


def test_each_result_is_the_same_alone_and_in_the_mix():
    reqs = small_requests(6, 10)
    budget = 3 * max(serving.workspace_bytes(r.work, cc.CC_FP32_GEOM64) for r in reqs)
    srv = serving.Server("batched", budget_bytes=budget, slots=3, keep_results=True)
    rep = srv.run(reqs)
    assert rep["requests"] == 6 and rep["max_concurrent"] == 3
    # requests admitted after the first ones left ran beside requests admitted before them
    late = [r for r in reqs if r.admit_iter > 0]
    assert late
    for r in late:
        assert any(q.admit_iter < r.admit_iter < q.admit_iter + q.steps for q in reqs), r.rid
    for r in reqs:
        assert r.done == r.steps
        assert np.array_equal(r.result, alone(r, cc.CC_FP32_GEOM64)), r.rid


def test_plain_mode_matches_fp64_alone():
    reqs = small_requests(3, 6)
    srv = serving.Server("plain", slots=2, keep_results=True)
    rep = srv.run(reqs)
    assert rep["requests"] == 3
    for r in reqs:
        assert np.array_equal(r.result, alone(r, cc.CC_FP64)), r.rid


def test_large_requests_the_same_alone_and_in_the_mix():
    """The mix's larger grids (512 x 512 and 1024 x 512) under continuous batching."""
    out, k = [], 0
    while len(out) < 4:
        r = serving.Request(k, serving.W.serving_request(k), 0.0, 8)
        g = r.work["grid"]
        if g["nx"] * g["ny"] >= 512 * 512:
            out.append(r)
        k += 1
    for j, r in enumerate(out):
        r.steps = 8 + 3 * j
    assert {(r.work["grid"]["nx"], r.work["grid"]["ny"]) for r in out} == {(512, 512), (1024, 512)}
    budget = 2 * max(serving.workspace_bytes(r.work, cc.CC_FP32_GEOM64) for r in out)
    srv = serving.Server("batched", budget_bytes=budget, slots=2, keep_results=True)
    rep = srv.run(out)
    srv.close()
    assert rep["requests"] == 4 and rep["max_concurrent"] == 2
    for r in out:
        assert r.done == r.steps
        assert np.array_equal(r.result, alone(r, cc.CC_FP32_GEOM64)), r.rid
