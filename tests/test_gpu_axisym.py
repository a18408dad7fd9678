"""The axisymmetric form (reading R33) through the C ABI against the FP64 oracle: the
uniform expansion away from the axis and the piston inside a cylindrical tube (two bodies).

* per sweep from identical inputs (the source acts at the start of the step): relative
  L-infinity of U <= 1e-12 (FP64);
* with the oracle's time steps through captured steps: relative L1 <= 1e-10 (expansion) and
  <= 1e-9 (tube) at the end; FP32 state: relative L1 of density <= 1e-5;
* the calls an axisymmetric context does not support refuse.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from oracle import ref  # noqa: E402
from paper_1711_11361_amd import cc  # noqa: E402
from paper_1711_11361_amd import workloads as W  # noqa: E402


def scales(U, gamma=1.4):
    r = np.where(U[0] > 0, U[0], 1.0)
    p = (gamma - 1.0) * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / r)
    a = np.sqrt(np.maximum(gamma * p / r, 0.0))
    mom = np.where(U[0] > 0, np.hypot(U[1], U[2]) + U[0] * a, 0.0).max()
    sc = np.array([np.abs(U[0]).max(), mom, mom, np.abs(U[3]).max()])
    return np.where(sc > 0, sc, 1.0)


def rel_linf(a, b):
    sc = scales(b)
    return max(np.abs(a[k] - b[k]).max() / sc[k] for k in range(4))


def pair(w, precision=cc.CC_FP64):
    if "bodies" in w:
        o = ref.Oracle(w["grid"], bodies=w["bodies"])
        s = cc.Solver(w["grid"], bodies=w["bodies"], precision=precision)
    else:
        o = ref.Oracle(w["grid"], w["body"])
        s = cc.Solver(w["grid"], w["body"], precision=precision)
    o.set_prim(w["prim"])
    s.set_prim(w["prim"])
    return o, s


def cases():
    yield "expansion", W.uniform_expansion(32)
    yield "expansion_ragged", {**W.uniform_expansion(29, nx=13)}
    yield "tube", W.piston_tube(64, axisymmetric=True)


@pytest.mark.parametrize("name,w", list(cases()), ids=[c[0] for c in cases()])
def test_sweeps_match_oracle_from_identical_inputs(name, w):
    o, s = pair(w)
    for k in range(6):
        dt = o.cfl_dt(w["cfl"])
        s.set_u(o.get_u())
        assert abs(s.cfl_dt(w["cfl"]) - dt) <= 1e-12 * dt
        o.begin_step(dt)
        s.begin_step(dt)
        for sw in range(2):
            d = o.parity if sw == 0 else 1 - o.parity
            s.set_u(o.get_u())  # identical inputs (after the source, which begin_step applies)
            o.sweep(d, dt)
            s.sweep(d, dt)
            e = rel_linf(s.get_u(), o.get_u())
            assert e <= 1e-12, (name, k, sw, e)
        o.end_step()
        s.end_step()
    assert s.info()["status"] == o.status == 0


@pytest.mark.parametrize("name,w,nsteps,tol", [("expansion", W.uniform_expansion(32), 40, 1e-10),
                                               ("tube", W.piston_tube(64, axisymmetric=True), 120, 1e-9)],
                         ids=["expansion", "tube"])
def test_end_time_parity(name, w, nsteps, tol):
    o, s = pair(w)
    dts = o.run(w["cfl"], nsteps=nsteps)
    s.run(w["cfl"], dts=dts)
    Ug, Uo = s.get_u(), o.get_u()
    for k in range(4):
        den = np.abs(Uo[k]).sum()
        if den > 0:
            assert np.abs(Ug[k] - Uo[k]).sum() / den <= tol, (name, k)
    assert s.info()["collapses"] == o.collapses


def test_fp32_expansion_against_fp64_oracle():
    w = W.uniform_expansion(64)
    o, s = pair(w, precision=cc.CC_FP32_GEOM64)
    dts = o.run(w["cfl"], nsteps=60)
    s.run(w["cfl"], dts=dts)
    Po, Pg = o.get_prim(), s.get_prim()
    assert np.abs(Pg[0] - Po[0]).sum() / np.abs(Po[0]).sum() <= 1e-5


def test_unsupported_calls_refuse():
    w = W.uniform_expansion(16)
    s = cc.Solver(w["grid"], None)
    s.set_prim(w["prim"])
    for call in (lambda: s.advance(2, 0.5), lambda: s.set_launch_mode(1)):
        with pytest.raises(cc.CCError) as e:
            call()
        assert e.value.status == cc.CC_ERR_UNSUPPORTED
    b = cc.Batch(2, cc.CC_FP64)
    with pytest.raises(cc.CCError) as e:
        b.add(s)
    assert e.value.status == cc.CC_ERR_UNSUPPORTED
    b.close()
