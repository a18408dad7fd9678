"""Pins of the axisymmetric form (reading R33: the Euler equations in (x, r), r = y, with the
geometric source -(1/r) (rho v, rho u v, rho v^2, v (E + p)) applied before each step's
first sweep; the open-ended shock tube of Sec. 3.5 is computed in this form).

* a flow without radial velocity is the planar flow, bit for bit (the source vanishes);
* the uniform expansion rho = 1/(1+t)^2, u = 0, v = r/(1+t), p = (1+t)^(-2 gamma) (an exact
  solution of the axisymmetric equations: the gas spreads away from the axis, and in planar
  form the density would fall only as 1/(1+t)) is approached at first order (the source is
  split off in time) as the grid is refined, with the reflective axis as the lower boundary.
"""
import math

import numpy as np

from oracle import ref
from paper_1711_11361_amd import workloads as W

G = 1.4


def test_flow_without_radial_velocity_is_planar():
    out = []
    for axi in (False, True):
        g = W.grid(64, 8, 0.0, 1.0, 0.0, 0.125, bc=(0, 0, 1, 0))
        g["axisymmetric"] = axi
        prim = W.split_prim(g, 0.5, (1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1))
        o = ref.Oracle(g)
        o.set_prim(prim)
        o.run(0.8, nsteps=30)
        out.append(o.get_u())
    assert np.array_equal(out[0], out[1])


def expansion(ny, axi=True, t_end=0.1, cfl=0.5):
    g = W.grid(8, ny, 0.0, 8.0 / ny, 0.0, 1.0, bc=(0, 0, 1, 0))
    g["axisymmetric"] = axi
    X, Y = W.cell_centres(g)
    prim = np.empty((4, ny, 8))
    prim[0], prim[1], prim[2], prim[3] = 1.0, 0.0, Y, 1.0
    o = ref.Oracle(g)
    o.set_prim(prim)
    while o.t < t_end - 1e-12:
        o.step(min(o.cfl_dt(cfl), t_end - o.t))
    P = o.get_prim()
    m = Y < 0.6  # away from the outer boundary, whose zero-gradient ghost cells are not exact
    return (np.abs(P[0][m] - (1.0 + t_end) ** -2).mean(), np.abs(P[3][m] - (1.0 + t_end) ** (-2 * G)).mean(),
            np.abs(P[2][m] - Y[m] / (1.0 + t_end)).mean())


def test_uniform_expansion_converges_to_the_exact_solution():
    e = [expansion(ny) for ny in (16, 32, 64)]
    for q in range(3):
        orders = [math.log2(e[k][q] / e[k + 1][q]) for k in range(2)]
        assert min(orders) > 0.9, (q, e, orders)
    assert e[0][0] < 2e-3 and e[0][1] < 3e-3
    planar = expansion(16, axi=False)
    assert planar[0] > 0.05  # without the source the density falls too slowly
