"""Seeded synthetic workloads shaped like the paper's tests (input construction only).

Nothing here computes any part of the cut-cell method: it only builds grids, body polygons
(in the body frame), prescribed motions and primitive initial fields.  Both the GPU tests
and the CPU oracle read workloads from this module, so that the two sides always see
identical inputs.

Workloads (non-dimensional stand-ins for the paper's SI set-ups):

* ``piston``   -- a half-plane piston inclined at 30 degrees driven into gas at rest
                  (the set-up of the paper's shock-tube piston, Sec. 3.5, made planar);
* ``cylinder`` -- a circular cylinder crossing a stationary Mach-2 shock (Sec. 3.2);
* ``triangle`` -- an equilateral-triangle cylinder crossing the same shock (Sec. 3.3),
                  orientation and speed drawn per seed;
* ``naca``     -- a NACA 0012 aerofoil pitching about its quarter chord in a Mach-0.7
                  free stream (Sec. 3.4);
* ``serving_request`` -- the mixed request population of the serving benchmark;
* ``channel``  -- two parallel walls at 30 degrees moving together along +x, a density
                  pulse advected along the channel (Sec. 3.1), with its exact solution;
* ``piston_tube`` -- a rectangular piston driven along the inside of a static open-ended
                  tube wall (two bodies in relative motion; the planar form of Sec. 3.5).
"""
import math

import numpy as np

GAMMA = 1.4


# --------------------------------------------------------------------------- grids / fields
# Small-cell threshold of the shock-crossing and serving workloads: cut cells below 1 % of a
# cell count as solid.  Their bodies move at speeds unrelated to the gas around them, so
# front cells shrink to ~1e-7 of a cell while holding content they cannot contain; without
# the threshold the 1024 x 512 cylinder run fails within 300 steps.
SMALL_CELL = 1e-2


def grid(nx, ny, x_lo, x_hi, y_lo, y_hi, bc=(0, 0, 0, 0), gamma=GAMMA, alpha_min=0.0):
    return {"nx": int(nx), "ny": int(ny), "x_lo": float(x_lo), "x_hi": float(x_hi),
            "y_lo": float(y_lo), "y_hi": float(y_hi), "bc": tuple(int(b) for b in bc),
            "gamma": float(gamma), "alpha_min": float(alpha_min)}


def cell_centres(g):
    hx = (g["x_hi"] - g["x_lo"]) / g["nx"]
    hy = (g["y_hi"] - g["y_lo"]) / g["ny"]
    xc = g["x_lo"] + (np.arange(g["nx"]) + 0.5) * hx
    yc = g["y_lo"] + (np.arange(g["ny"]) + 0.5) * hy
    return np.meshgrid(xc, yc)


def uniform_prim(g, rho, u, v, p):
    prim = np.empty((4, g["ny"], g["nx"]))
    prim[0], prim[1], prim[2], prim[3] = rho, u, v, p
    return prim


def split_prim(g, x_split, left, right):
    """Two primitive states (rho, u, v, p) separated by the vertical line x = x_split,
    assigned by cell centre."""
    X, _ = cell_centres(g)
    prim = np.empty((4, g["ny"], g["nx"]))
    lm = X < x_split
    for k in range(4):
        prim[k] = np.where(lm, left[k], right[k])
    return prim


def mach2_stationary_shock(gamma=GAMMA):
    """Upstream (rho=1, p=1, Mach 2) and the Rankine-Hugoniot downstream state of a
    stationary normal shock, as (rho, u, v, p) tuples."""
    rho1, p1 = 1.0, 1.0
    u1 = 2.0 * math.sqrt(gamma * p1 / rho1)
    M2 = 4.0
    r = (gamma + 1.0) * M2 / ((gamma - 1.0) * M2 + 2.0)
    pr = 1.0 + 2.0 * gamma * (M2 - 1.0) / (gamma + 1.0)
    return (rho1, u1, 0.0, p1), (rho1 * r, u1 / r, 0.0, p1 * pr)


# --------------------------------------------------------------------------- body polygons
def circle(r, n=1024):
    """Regular n-gon inscribed in a circle of radius r, counter-clockwise."""
    k = np.arange(n)
    a = 2.0 * np.pi * k / n
    return np.stack([r * np.cos(a), r * np.sin(a)], axis=1)


def triangle(side):
    """Equilateral triangle with its centroid at the origin, counter-clockwise."""
    R = side / math.sqrt(3.0)
    a = np.deg2rad(np.array([90.0, 210.0, 330.0]))
    return np.stack([R * np.cos(a), R * np.sin(a)], axis=1)


def naca00(thickness, chord=1.0, n_side=512, pivot=0.25):
    """Symmetric NACA 4-digit section with a closed trailing edge (reading: last
    coefficient -0.1036), leading edge at x = -pivot*chord, body-frame origin at the pivot.
    Cosine-spaced, n_side points per surface (shared leading and trailing edges),
    counter-clockwise (upper surface from trailing to leading edge, then lower)."""
    k = np.arange(n_side)
    x = 0.5 * (1.0 + np.cos(np.pi * k / (n_side - 1)))  # 1 -> 0
    t = thickness
    yt = 5.0 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2 + 0.2843 * x ** 3
                    - 0.1036 * x ** 4)
    yt[0] = 0.0
    yt[-1] = 0.0
    upper = np.stack([x, yt], axis=1)
    lower = np.stack([x[::-1][1:-1], -yt[::-1][1:-1]], axis=1)
    pts = np.concatenate([upper, lower], axis=0)
    pts[:, 0] = (pts[:, 0] - pivot) * chord
    pts[:, 1] = pts[:, 1] * chord
    return pts


def half_plane_quad(L=2.0):
    """A large quad standing in for the half-plane {x_b <= 0} of the body frame."""
    return np.array([[-L, -L], [0.0, -L], [0.0, L], [-L, L]])


def clipped_half_plane(normal, offset, box):
    """The convex polygon {x in box : normal . x <= offset}, counter-clockwise, for a box
    (x0, x1, y0, y1) (a wall's solid side, cut off well outside the domain)."""
    x0, x1, y0, y1 = box
    pts = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
    nx_, ny_ = normal
    out = []
    for k in range(4):
        a, b = pts[k - 1], pts[k]
        da = nx_ * a[0] + ny_ * a[1] - offset
        db = nx_ * b[0] + ny_ * b[1] - offset
        if (da <= 0.0) != (db <= 0.0):
            t = da / (da - db)
            out.append((a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])))
        if db <= 0.0:
            out.append(b)
    return np.array(out, dtype=np.float64)


def rectangle(x0, x1, y0, y1):
    return np.array([[x0, y0], [x1, y0], [x1, y1], [x0, y1]], dtype=np.float64)


def body(verts, ref=(0.0, 0.0), theta0=0.0, vel=(0.0, 0.0), pitch_amp=0.0, pitch_omega=0.0):
    return {"verts": np.ascontiguousarray(verts, dtype=np.float64), "ref": tuple(map(float, ref)),
            "theta0": float(theta0), "vel": tuple(map(float, vel)),
            "pitch_amp": float(pitch_amp), "pitch_omega": float(pitch_omega)}


# --------------------------------------------------------------------------- workloads
def piston(nx=200, ny=20, angle_deg=30.0, speed=0.3, face=(0.1, 0.05), bc=(0, 0, 0, 0)):
    """Inclined piston into quiescent gas: domain [0,1]x[0,0.1], rho=1, u=v=0, p=1; the
    piston face passes through `face` with normal at `angle_deg` and moves along it."""
    g = grid(nx, ny, 0.0, 1.0, 0.0, 0.1, bc=bc)
    th = math.radians(angle_deg)
    n = (math.cos(th), math.sin(th))
    b = body(half_plane_quad(0.6), ref=face, theta0=th, vel=(speed * n[0], speed * n[1]))
    return {"name": "piston", "grid": g, "body": b, "prim": uniform_prim(g, 1.0, 0.0, 0.0, 1.0),
            "cfl": 0.8, "t_end": 0.5, "normal": n, "speed": speed, "face": face}


def cylinder(nx=1024, ny=512, radius=0.1, centre=(0.5, 0.5), speed=1.0, n_poly=1024, alpha_min=SMALL_CELL):
    """Circular cylinder crossing a stationary Mach-2 shock at x = 1 on [0,2]x[0,1]."""
    g = grid(nx, ny, 0.0, 2.0, 0.0, 1.0, alpha_min=alpha_min)
    up, down = mach2_stationary_shock()
    b = body(circle(radius, n_poly), ref=centre, vel=(speed, 0.0))
    return {"name": "cylinder", "grid": g, "body": b, "prim": split_prim(g, 1.0, up, down),
            "cfl": 0.8, "steps": 2000}


def triangle_case(seed, nx=2048, ny=1024, side=0.2, centre=(0.5, 0.5), alpha_min=SMALL_CELL):
    """Equilateral triangle crossing the Mach-2 stationary shock; orientation uniform in
    [0, 60) degrees and speed uniform in [0.5, 1.5] drawn from the seed."""
    rng = np.random.default_rng(seed)
    ang = math.radians(rng.uniform(0.0, 60.0))
    spd = rng.uniform(0.5, 1.5)
    g = grid(nx, ny, 0.0, 2.0, 0.0, 1.0, alpha_min=alpha_min)
    up, down = mach2_stationary_shock()
    b = body(triangle(side), ref=centre, theta0=ang, vel=(spd, 0.0))
    return {"name": "triangle", "grid": g, "body": b, "prim": split_prim(g, 1.0, up, down),
            "cfl": 0.8, "steps": 2000, "seed": seed}


def naca(nx=4096, ny=4096, amp_deg=2.0, reduced_freq=0.1, mach=0.7, n_side=512):
    """NACA 0012, chord 1, leading edge at the origin, pitching about the quarter chord
    theta(t) = amp sin(omega t), omega = 2 k U / c, in a free stream rho=1, p=1/gamma."""
    g = grid(nx, ny, -2.0, 4.0, -3.0, 3.0)
    U = mach
    omega = 2.0 * reduced_freq * U / 1.0
    b = body(naca00(0.12, 1.0, n_side, 0.25), ref=(0.25, 0.0), pitch_amp=math.radians(amp_deg),
             pitch_omega=omega)
    period = 2.0 * math.pi / omega
    return {"name": "naca", "grid": g, "body": b,
            "prim": uniform_prim(g, 1.0, U, 0.0, 1.0 / GAMMA), "cfl": 0.8,
            "t_end": 3.0 * period}


SERVING_GRIDS = ((64, 64), (256, 128), (512, 512), (1024, 512))


def serving_request(k):
    """Request k of the serving mix, drawn from numpy's default_rng(1000 + k).

    Grid from SERVING_GRIDS (square cells: domain [0, nx/ny] x [0, 1]); body one of circle,
    triangle, NACA 00t (chord 0.3) or inclined piston, centred at (0.25 x_extent, 0.5);
    motion a translation along +x (speed in [0.2, 1.5]) or a pitch oscillation (amplitude
    1-4 degrees, reduced frequency 0.05-0.2); initial state quiescent or the Mach-2
    stationary shock at x_extent/2.  500 steps each."""
    rng = np.random.default_rng(1000 + k)
    nx, ny = SERVING_GRIDS[rng.integers(len(SERVING_GRIDS))]
    xe = nx / ny
    g = grid(nx, ny, 0.0, xe, 0.0, 1.0, alpha_min=SMALL_CELL)
    kind = ["circle", "triangle", "naca", "piston"][rng.integers(4)]
    motion = ["translate", "pitch"][rng.integers(2)]
    centre = (0.25 * xe, 0.5)
    speed = rng.uniform(0.2, 1.5)
    amp = math.radians(rng.uniform(1.0, 4.0))
    kred = rng.uniform(0.05, 0.2)
    if kind == "circle":
        verts = circle(rng.uniform(0.05, 0.15), 256)
        chord = 0.3
    elif kind == "triangle":
        verts = triangle(rng.uniform(0.1, 0.25))
        chord = 0.25
    elif kind == "naca":
        chord = 0.3
        verts = naca00(rng.uniform(0.09, 0.15), chord, 128, 0.25)
    else:
        chord = 0.3
        verts = half_plane_quad(4.0)
        centre = (0.1 * xe, 0.5)
    theta0 = 0.0
    if kind == "piston":
        theta0 = math.radians(rng.uniform(0.0, 60.0))
    shock = bool(rng.integers(2))
    if motion == "translate":
        vel = (speed, 0.0) if kind != "piston" else (speed * math.cos(theta0), speed * math.sin(theta0))
        b = body(verts, ref=centre, theta0=theta0, vel=vel)
    else:
        U = 1.0
        b = body(verts, ref=centre, theta0=theta0, pitch_amp=amp,
                 pitch_omega=2.0 * kred * U / chord)
    if shock:
        up, down = mach2_stationary_shock()
        prim = split_prim(g, 0.5 * xe, up, down)
    else:
        prim = uniform_prim(g, 1.0, 0.0, 0.0, 1.0)
    return {"name": f"req{k}", "grid": g, "body": b, "prim": prim, "cfl": 0.8, "steps": 500,
            "kind": kind, "motion": motion}


# --------------------------------------------------------------------------- several bodies
def wedges():
    """Two static convex bodies facing each other across the open grid line x = 0.4 of the
    unit square (10 x 10 cells, h = 0.1).  The left one's corner cuts cell (3, 5) in the
    triangle (0.3, 0.5), (0.38, 0.5), (0.3, 0.57), and below it a vertical wall at x = 0.38
    cuts column 3 from y = 0.25 to 0.5; the right one's corner cuts cell (4, 5) in the
    triangle (0.43, 0.5), (0.5, 0.5), (0.5, 0.56), and its vertical wall at x = 0.43 cuts
    column 4.  A smooth non-uniform state, so that the fluxes of neighbouring faces and the
    walls differ."""
    g = grid(10, 10, 0.0, 1.0, 0.0, 1.0)
    a = np.array([[0.05, 0.25], [0.38, 0.25], [0.38, 0.5], [0.3, 0.57], [0.05, 0.57]])
    b = np.array([[0.43, 0.25], [0.95, 0.25], [0.95, 0.56], [0.5, 0.56], [0.43, 0.5]])
    X, Y = cell_centres(g)
    prim = np.empty((4, 10, 10))
    prim[0] = 1.0 + 0.3 * np.sin(7.0 * X + 3.0 * Y)
    prim[1] = 0.4 + 0.3 * np.cos(5.0 * Y - 2.0 * X)
    prim[2] = -0.3 + 0.2 * np.sin(4.0 * X * Y + 1.0)
    prim[3] = 1.0 + 0.4 * np.cos(6.0 * X - 5.0 * Y)
    return {"name": "wedges", "grid": g, "bodies": [body(a), body(b)], "prim": prim, "cfl": 0.8}


def channel(ny=32, angle_deg=30.0, width=0.25, speed=0.5, flow=1.0, amp=0.5, sigma=0.1, cfl=0.5):
    """Sloped channel (Sec. 3.1): domain [-1.5, 1.5] x [-0.5, 0.5] (3 ny x ny square cells),
    two parallel walls at `angle_deg` to the x axis, `width` apart about the origin, both
    moving with velocity (speed, 0); their solid sides are half-planes cut off far outside
    the domain.  Gas: p = 1, velocity (speed, 0) + flow t (t the channel direction), and a
    density pulse rho = 1 + amp exp(-(s / sigma)^2) of the distance s along t from the
    origin (uniform across the channel).  The exact solution advects the initial field with
    the gas velocity (channel_exact).  The pulse shape is not given in the paper (reading)."""
    g = grid(3 * ny, ny, -1.5, 1.5, -0.5, 0.5)
    a = math.radians(angle_deg)
    t = (math.cos(a), math.sin(a))
    n = (-math.sin(a), math.cos(a))
    box = (-2.5, 3.0, -1.0, 1.0)  # outside the domain while the walls move by less than 1
    lower = clipped_half_plane(n, -0.5 * width, box)
    upper = clipped_half_plane((-n[0], -n[1]), -0.5 * width, box)
    bodies = [body(lower, vel=(speed, 0.0)), body(upper, vel=(speed, 0.0))]
    vel = (speed + flow * t[0], flow * t[1])
    w = {"name": "channel", "grid": g, "bodies": bodies, "cfl": cfl, "t_end": 0.5,
         "dir": t, "normal": n, "width": width, "speed": speed, "vel": vel, "amp": amp, "sigma": sigma}
    w["prim"] = channel_exact(w, 0.0)
    return w


def channel_exact(w, t):
    """Primitive fields of the channel's exact solution at time t, at the cell centres."""
    g = w["grid"]
    X, Y = cell_centres(g)
    d = w["dir"]
    s = d[0] * (X - w["vel"][0] * t) + d[1] * (Y - w["vel"][1] * t)
    prim = np.empty((4, g["ny"], g["nx"]))
    prim[0] = 1.0 + w["amp"] * np.exp(-(s / w["sigma"]) ** 2)
    prim[1], prim[2], prim[3] = w["vel"][0], w["vel"][1], 1.0
    return prim


def channel_inside(w, t, margin=0.0):
    """Cells whose centre lies inside the channel at time t, at least `margin` from both walls."""
    g = w["grid"]
    X, Y = cell_centres(g)
    n = w["normal"]
    d = n[0] * (X - w["speed"] * t) + n[1] * Y
    return np.abs(d) < 0.5 * w["width"] - margin


def uniform_expansion(ny=32, nx=8):
    """The gas spreading away from the axis of an axisymmetric domain (x, r) in [0, nx/ny] x
    [0, 1], reflective axis: rho = 1, u = 0, v = r, p = 1 at t = 0; the exact solution of the
    axisymmetric equations is rho = 1/(1+t)^2, u = 0, v = r/(1+t), p = (1+t)^(-2 gamma)."""
    g = grid(nx, ny, 0.0, nx / ny, 0.0, 1.0, bc=(0, 0, 1, 0))
    g["axisymmetric"] = True
    _, Y = cell_centres(g)
    prim = np.empty((4, ny, nx))
    prim[0], prim[1], prim[2], prim[3] = 1.0, 0.0, Y, 1.0
    return {"name": "uniform_expansion", "grid": g, "body": None, "prim": prim, "cfl": 0.5}


def piston_tube(ny=128, mach_s=1.76, gap=1.0 / 16.0, wall=0.125, axisymmetric=False):
    """Two bodies in relative motion, the planar form of the open-ended shock tube of
    Sec. 3.5 (the axisymmetric source terms are not modelled): lengths in tube diameters D,
    the half-tube above the reflective centre line y = 0.  Domain [0, 10] x [0, 4]
    (2.5 ny x ny cells); a static tube wall [-1, 6] x [0.5, 0.5 + wall] (its open end at
    x = 6); a rectangular piston [0.25, 0.5] x [-1, 0.5 - gap] moving along +x at the speed
    that drives a shock of Mach `mach_s` into gas at rest (rho = 1, p = 1).  The piston
    clears the tube wall by `gap` (reading: no cell may hold both bodies).  axisymmetric: the
    domain is the half plane (x, r) of the axisymmetric equations (the tube a cylinder, the
    piston a disc)."""
    g = grid(int(2.5 * ny), ny, 0.0, 10.0, 0.0, 4.0, bc=(0, 0, 1, 0))
    g["axisymmetric"] = bool(axisymmetric)
    a0 = math.sqrt(GAMMA)
    S = mach_s * a0
    k = (S * S - a0 * a0) / (2.0 * S)
    up = 4.0 * k / (GAMMA + 1.0)
    tube = body(rectangle(-1.0, 6.0, 0.5, 0.5 + wall))
    piston_b = body(rectangle(0.25, 0.5, -1.0, 0.5 - gap), vel=(up, 0.0))
    return {"name": "piston_tube", "grid": g, "bodies": [tube, piston_b],
            "prim": uniform_prim(g, 1.0, 0.0, 0.0, 1.0), "cfl": 0.8, "piston_speed": up,
            "shock_speed": S}
