"""Pins of the oracle parts that the consistency and conservation tests cannot see.

* the CFL time step (Sec. 4, reading R17), computed by hand from the primitive field and
  the body's posed vertices, on a grid with hx != hy, once with the gas and once with the
  wall setting the step;
* the rigid-body velocity against a centred difference of the pose, and the step's
  displacement against the difference of the poses at the step's ends (Sec. 2.3.4);
* MUSCL-Hancock (end of Sec. 2.3.5): the half-step evolution of a linear profile with
  uniform velocity and pressure is that profile advected by half a step;
* the stabilised flux of a static cut cell whose low face is shielded (Eqs.
  Klein2shieldedFluxMethod2, Klein2DtotalfluxaMethod2, Klein2DcompleteMovingMethod2a/b in
  the static limit): the update is dt/h [beta_hi (F_lo - F_hi) + ahat (F_lo - F^B)], a
  convex combination without division by the volume fraction, with the apertures and the
  shielded volume from the closed form of the cell's wall;
* why a cell that becomes fluid takes a state but no content (reading R13): with the
  content moving as printed, a body moving with a uniform flow no longer leaves it uniform.
"""
import math

import numpy as np
import pytest

from oracle import ref
from paper_1711_11361_amd import workloads as W

GAMMA = 1.4
EPS = 2.0 ** -52


def cons(rho, u, v, p, g=GAMMA):
    return np.array([rho, rho * u, rho * v, p / (g - 1.0) + 0.5 * rho * (u * u + v * v)])


# ------------------------------------------------------------------ CFL time step
def posed_vertices_and_velocities(body, t):
    """The body's vertices at time t and their rigid velocities, written out from the
    prescribed motion: theta(t) = theta0 + A sin(w t), centre ref + v t."""
    A, w = body["pitch_amp"], body["pitch_omega"]
    th = body["theta0"] + A * math.sin(w * t)
    thd = A * w * math.cos(w * t)
    cx = body["ref"][0] + body["vel"][0] * t
    cy = body["ref"][1] + body["vel"][1] * t
    V = np.asarray(body["verts"])
    X = math.cos(th) * V[:, 0] - math.sin(th) * V[:, 1] + cx
    Y = math.sin(th) * V[:, 0] + math.cos(th) * V[:, 1] + cy
    UX = body["vel"][0] - thd * (Y - cy)
    UY = body["vel"][1] + thd * (X - cx)
    return X, Y, UX, UY


def cfl_case(wall_dominated):
    g = W.grid(40, 20, 0.0, 2.0, 0.0, 0.5)  # hx = 0.05, hy = 0.025
    rng = np.random.default_rng(11)
    prim = np.empty((4, 20, 40))
    if wall_dominated:  # slow, cold gas; a fast, fast-turning body
        prim[0] = rng.uniform(0.8, 1.2, (20, 40))
        prim[1] = rng.uniform(-0.05, 0.05, (20, 40))
        prim[2] = rng.uniform(-0.05, 0.05, (20, 40))
        prim[3] = rng.uniform(0.005, 0.01, (20, 40))
        b = W.body(W.triangle(0.3), ref=(1.0, 0.25), theta0=0.3, vel=(2.5, -1.7), pitch_amp=0.5,
                   pitch_omega=4.0)
    else:
        prim[0] = rng.uniform(0.5, 2.0, (20, 40))
        prim[1] = rng.uniform(-1.0, 1.0, (20, 40))
        prim[2] = rng.uniform(-0.5, 0.5, (20, 40))
        prim[3] = rng.uniform(0.3, 3.0, (20, 40))
        prim[1, 7, 31] = -3.1  # the fastest cell, moving to -x
        b = W.body(W.triangle(0.3), ref=(1.0, 0.25), theta0=0.3, vel=(0.4, -0.3), pitch_amp=0.2,
                   pitch_omega=3.0)
    return g, b, prim


@pytest.mark.parametrize("wall_dominated", [False, True])
def test_cfl_time_step_by_hand(wall_dominated):
    g, b, prim = cfl_case(wall_dominated)
    t0 = 0.7
    o = ref.Oracle(g, b)
    o.set_prim(prim, t0)
    live = o.geometry_dump(0)["alpha"] > 0.0
    rho, u, v, p = prim
    a = np.sqrt(GAMMA * p / rho)
    sx_gas = (np.abs(u) + a)[live].max()
    sy_gas = (np.abs(v) + a)[live].max()
    _, _, UX, UY = posed_vertices_and_velocities(b, t0)
    sx = max(sx_gas, np.abs(UX).max())
    sy = max(sy_gas, np.abs(UY).max())
    hx, hy = 0.05, 0.025
    dt = 0.8 * min(hx / sx, hy / sy)
    assert abs(o.cfl_dt(0.8) - dt) <= 1e-14 * dt
    # the case really decides what it claims to (so that a dropped term would show)
    if wall_dominated:
        assert np.abs(UX).max() > sx_gas and np.abs(UY).max() > sy_gas
    else:
        assert np.abs(UX).max() < sx_gas and np.abs(UY).max() < sy_gas
    assert abs(0.8 * min(hy / sx, hx / sy) - dt) > 1e-3 * dt  # swapped cell sizes differ
    assert np.allclose(o.wave_speeds(), [sx, sy], rtol=1e-14, atol=0.0)


def test_body_velocity_is_the_derivative_of_the_pose():
    b = W.body(W.naca00(0.12, 1.0, 32, 0.25), ref=(0.3, -0.2), theta0=0.4, vel=(0.7, -0.35),
               pitch_amp=0.3, pitch_omega=2.5)
    o = ref.Oracle(W.grid(16, 16, -2.0, 2.0, -2.0, 2.0), b)
    eps = 1e-5
    for t in (0.0, 0.37, 1.9):
        P = o.pose(t)
        dP = (o.pose(t + eps) - o.pose(t - eps)) / (2.0 * eps)
        for k in range(len(P)):
            uw = o.body_velocity(t, P[k, 0], P[k, 1])
            assert np.abs(uw - dP[k]).max() < 1e-8, (t, k, uw, dP[k])
        # and against the motion written out here
        X, Y, UX, UY = posed_vertices_and_velocities(b, t)
        assert np.abs(P[:, 0] - X).max() < 1e-15 and np.abs(P[:, 1] - Y).max() < 1e-15
        for k in range(len(P)):
            assert np.abs(o.body_velocity(t, X[k], Y[k]) - (UX[k], UY[k])).max() < 1e-15


def test_step_displacement_is_the_difference_of_the_poses():
    b = W.body(W.triangle(0.4), ref=(0.1, 0.2), theta0=0.2, vel=(0.9, 0.4), pitch_amp=0.6, pitch_omega=3.0)
    o = ref.Oracle(W.grid(32, 32, -1.0, 1.0, -1.0, 1.0), b)
    o.set_prim(W.uniform_prim(o.grid, 1.0, 0.0, 0.0, 1.0), 0.25)
    dt = 0.013
    P0, P1 = o.pose(0.25), o.pose(0.25 + dt)
    o.begin_step(dt)
    for k in range(len(P0)):
        for d in (0, 1):
            D = o.step_disp(d, P0[k, 0], P0[k, 1])
            assert abs(D - (P1[k, d] - P0[k, d])) < 1e-15, (k, d)


# ------------------------------------------------------------------ MUSCL-Hancock
@pytest.mark.parametrize("d", [0, 1])
@pytest.mark.parametrize("slopes", [(0.1, 0.1), (0.06, 0.14), (-0.2, -0.05)])
def test_muscl_half_step_advects_a_linear_profile(d, slopes):
    """With uniform velocity and pressure every conserved component is linear in the
    density, so the van Leer slope is 2ab/(a+b) of the density differences a, b (times the
    component's factor), and the half-step evolution moves the face states exactly as
    advection by u_d dt/2 would: rho_face = rho +- s/2 - (lam/2) u_d s."""
    rho0, u, v, p = 1.1, 0.7, -0.45, 0.9
    a, b = slopes
    lam = 0.37
    qm, q, qp = cons(rho0 - a, u, v, p), cons(rho0, u, v, p), cons(rho0 + b, u, v, p)
    el, er = ref.muscl(qm, q, qp, True, lam, d)
    s = 2.0 * a * b / (a + b)
    ud = u if d == 0 else v
    rl = rho0 - 0.5 * s - 0.5 * lam * ud * s
    rr = rho0 + 0.5 * s - 0.5 * lam * ud * s
    assert np.allclose(el, cons(rl, u, v, p), rtol=1e-14, atol=1e-15)
    assert np.allclose(er, cons(rr, u, v, p), rtol=1e-14, atol=1e-15)
    # slopes of opposite sign: first order
    el0, er0 = ref.muscl(qm, q, cons(rho0 - 0.5 * b, u, v, p), True, lam, d)
    assert np.array_equal(el0, q) and np.array_equal(er0, q)


# ------------------------------------------------------------------ stabilised flux
def shielded_cell_case(d):
    """A static convex body whose top boundary rises across cell c = (4, 5) of a 10 x 10
    grid on the unit square (h = 0.1) and runs flat east of a vertex inside it: in cell
    units the wall meets the cell's low x-face at height 0.3, the vertex sits at (0.6,
    0.7), then the wall runs flat at 0.7.  Closed forms: beta_lo = 0.7, beta_hi = 0.3,
    alpha = 1 - (0.6 (0.3 + 0.7) / 2 + 0.4 * 0.7) = 0.42, shielded part of the low face
    s = 0.4, shielded volume ahat = 0.6 * 0.4 / 2 = 0.12.  The face between c and its east
    neighbour is shielded by neither (the wall is flat there), so
        U_e - U = lam [beta_hi (F_lo - F_hi) + ahat (F_lo - F^B)].
    d = 1: the same configuration mirrored about the diagonal (cell (5, 4), y-sweep)."""
    poly = np.array([[-0.245, 0.1], [0.95, 0.1], [0.95, 0.57], [0.46, 0.57]])
    cell = (4, 5)
    if d == 1:
        poly = poly[::-1, ::-1].copy()  # swap x and y, keep counter-clockwise order
        cell = (5, 4)
    g = W.grid(10, 10, 0.0, 1.0, 0.0, 1.0)
    X, Y = W.cell_centres(g)
    prim = np.empty((4, 10, 10))
    prim[0] = 1.0 + 0.3 * np.sin(7.0 * X + 3.0 * Y)
    prim[1] = 0.4 + 0.3 * np.cos(5.0 * Y - 2.0 * X)
    prim[2] = -0.3 + 0.2 * np.sin(4.0 * X * Y + 1.0)
    prim[3] = 1.0 + 0.4 * np.cos(6.0 * X - 5.0 * Y)
    return g, W.body(poly), prim, cell


@pytest.mark.parametrize("d", [0, 1])
def test_static_shielded_cut_cell_update_is_a_convex_combination(d):
    g, b, prim, (ci, cj) = shielded_cell_case(d)
    o = ref.Oracle(g, b)
    o.set_prim(prim)
    o.trace(ci, cj)
    dt = 0.2 * o.cfl_dt(0.8)
    o.begin_step(dt)
    if d == 1:  # step 0 sweeps x first; the y-sweep of this cell comes second
        o.sweep(0, dt)
    U0 = o.get_u()[:, cj, ci].copy()
    o.sweep(d, dt)
    U1 = o.get_u()[:, cj, ci]
    r = o.trace_get()
    assert r["wall"] and r["has"]
    for key, val in (("alpha_s", 0.42), ("alpha_e", 0.42), ("bt_lo", 0.7), ("bt_hi", 0.3), ("ahat", 0.12)):
        assert abs(r[key] - val) < 1e-14, (key, r[key])
    lam = dt / 0.1
    F_lo, F_hi, FB = r["F_lo"], r["F_hi"], r["FB"]
    expect = lam * (0.3 * (F_lo - F_hi) + 0.12 * (F_lo - FB))
    scale = np.abs(U0) + lam * (0.3 * (np.abs(F_lo) + np.abs(F_hi)) + 0.12 * (np.abs(F_lo) + np.abs(FB)))
    assert (np.abs((U1 - U0) - expect) <= 16 * EPS * scale).all(), ((U1 - U0), expect)
    # the stabilised fluxes themselves: the low face carries beta F - (s - ahat)(F - F^B),
    # the high face its plain aperture-weighted flux
    assert np.allclose(r["phi_lo"], 0.7 * F_lo - (0.4 - 0.12) * (F_lo - FB), rtol=0, atol=8 * EPS * np.abs(F_lo).max())
    assert np.array_equal(r["phi_hi"], r["bt_hi"] * F_hi)
    # the fluxes differ, so the identity is not vacuous
    assert np.abs(F_lo - F_hi).max() > 1e-3 and np.abs(F_lo - FB).max() > 1e-3


# ------------------------------------------------------------------ reading R13
def test_moving_content_into_uncovered_cells_breaks_the_consistency_condition():
    """Reading R13: with exact time-averaged apertures, fluid swept into a cell that
    becomes fluid already enters through its faces.  Moving the donors' content into it as
    well (Eq. cutCellInitialisationDonorCellUpdate as printed) counts that fluid twice: a
    body moving with a uniform flow then leaves density spikes in the cells it uncovers,
    while the state-only reading keeps the flow uniform to round-off."""
    out = {}
    for literal in (False, True):
        w = W.cylinder(nx=96, ny=48, speed=0.5, alpha_min=0.0)
        o = ref.Oracle(w["grid"], w["body"])
        o.set_uncover_moves_content(literal)
        o.set_prim(W.uniform_prim(w["grid"], 1.3, 0.5, 0.0, 0.9))
        o.run(0.8, nsteps=25)
        P = o.get_prim()
        m = P[0] > 0
        out[literal] = np.abs(P[0][m] / 1.3 - 1.0).max()
    assert out[False] < 1e-8
    assert out[True] > 0.5, out
