"""Surface loads of the oracle (force and moment of the gas on the body at level n) against
what the geometry and the gas dynamics fix:

* a closed body in gas at rest feels no net force (the effective wall normals of a closed
  polygon telescope to zero, and the wall pressure of gas at rest against a wall at rest
  is the gas pressure);
* a half-plane piston at rest whose face crosses the whole domain feels p L (-n): the
  normals telescope to the face's length inside the domain, L = H / cos(angle), and the
  moment about the face's mid point vanishes (the cells are point-symmetric about it);
* a piston driven into gas at rest feels the exact post-shock pressure on its face
  (Sec. 3.2's piston problem);
* the wall pressure distribution lists the terms the loads sum: at rest every wall cell's
  p* is the gas pressure, and the records' sums reproduce the force and moment.
"""
import math

import numpy as np

from oracle import exact, ref
from paper_1711_11361_amd import workloads as W


def make(w, prim=None):
    o = ref.Oracle(w["grid"], w["body"])
    o.set_prim(w["prim"] if prim is None else prim)
    return o


def test_closed_body_at_rest_feels_no_net_force():
    w = W.cylinder(nx=128, ny=64, speed=0.0, alpha_min=0.0)
    o = make(w, W.uniform_prim(w["grid"], 1.0, 0.0, 0.0, 1.0))
    fx, fy, mz, scale = o.surface_loads()
    assert scale > 0.6  # ~ the circumference 2 pi r at unit pressure
    assert abs(fx) <= 1e-13 * scale and abs(fy) <= 1e-13 * scale


def test_piston_at_rest_feels_pressure_times_face_length():
    w = W.piston(speed=0.0)
    p = 1.7
    o = make(w, W.uniform_prim(w["grid"], 1.0, 0.0, 0.0, p))
    fx, fy, mz, scale = o.surface_loads()
    n = w["normal"]
    L = 0.1 / n[0]  # the face crosses the whole height 0.1 of the domain
    assert abs(fx - (-p * L * n[0])) <= 1e-12 * scale
    assert abs(fy - (-p * L * n[1])) <= 1e-12 * scale
    assert abs(scale - p * L) <= 1e-12 * scale  # every wall cell's normal points along -n
    assert abs(mz) <= 1e-12 * scale * 0.1


def test_driven_piston_feels_the_post_shock_pressure():
    # the face normal to x: the flow is one-dimensional, the exact solution of Sec. 3.2's
    # piston problem holds across the whole channel (an inclined face in this channel
    # is not: the zero-gradient top and bottom boundaries bend its flow)
    w = W.piston(angle_deg=0.0)
    o = make(w)
    o.run(0.8, t_end=w["t_end"])
    fx, fy, mz, scale = o.surface_loads()
    S, r1, p1 = exact.piston_shock(1.4, 1.0, 1.0, w["speed"])
    pw = -fx / 0.1  # mean pressure on the face (height 0.1)
    assert abs(pw / p1 - 1) < 1e-4, (pw, p1)
    assert fy == 0.0 and abs(mz) <= 1e-15 * scale


def test_no_body_no_loads():
    w = {**W.cylinder(nx=32, ny=16), "body": None}
    o = make(w)
    assert np.array_equal(o.surface_loads(), np.zeros(4))


def test_pressure_distribution_lists_the_terms_of_the_loads():
    # at rest: p* = p in every wall cell, the normals sum to zero around the closed body
    w = W.cylinder(nx=128, ny=64, speed=0.0, alpha_min=0.0)
    o = make(w, W.uniform_prim(w["grid"], 1.0, 0.0, 0.0, 1.3))
    r = o.surface_pressure()
    assert len(r) > 30 and np.all(np.diff(r[:, 0]) > 0)  # increasing cell index
    assert np.abs(r[:, 3] - 1.3).max() <= 1e-13
    # a moving, pitching body in a stream: the records' sums are the loads
    w = W.naca(nx=192, ny=192)
    w["body"]["pitch_amp"] = math.radians(6.0)
    w["body"]["pitch_omega"] = 1.5
    o = make(w)
    for _ in range(6):
        o.step(o.cfl_dt(w["cfl"]))
    r = o.surface_pressure()
    fx, fy, mz, scale = o.surface_loads()
    cx, cy = w["body"]["ref"]
    assert abs((r[:, 3] * r[:, 4]).sum() - fx) <= 1e-13 * scale
    assert abs((r[:, 3] * r[:, 5]).sum() - fy) <= 1e-13 * scale
    m = ((r[:, 1] - cx) * (r[:, 3] * r[:, 5]) - (r[:, 2] - cy) * (r[:, 3] * r[:, 4])).sum()
    assert abs(m - mz) <= 1e-13 * scale
    # wall points lie in their cells
    g = w["grid"]
    hx, hy = (g["x_hi"] - g["x_lo"]) / g["nx"], (g["y_hi"] - g["y_lo"]) / g["ny"]
    i, j = r[:, 0].astype(int) % g["nx"], r[:, 0].astype(int) // g["nx"]
    assert np.all(r[:, 1] >= g["x_lo"] + i * hx - 1e-12) and np.all(r[:, 1] <= g["x_lo"] + (i + 1) * hx + 1e-12)
    assert np.all(r[:, 2] >= g["y_lo"] + j * hy - 1e-12) and np.all(r[:, 2] <= g["y_lo"] + (j + 1) * hy + 1e-12)
