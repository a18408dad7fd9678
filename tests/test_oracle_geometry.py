"""Pins of the oracle's cut-cell geometry (volume fractions, face apertures, classes).

Against: a hand-worked cell, brute-force point sampling on tiny grids, exact global
identities (total solid area = polygon area, effective wall normals telescope to zero,
column sums of face apertures = chord lengths), and the closed-polygon rule for vertices.
"""
import math

import numpy as np
import pytest

from oracle import ref
from paper_1711_11361_amd import workloads as W


def oracle_for_poly(nx, ny, box, poly):
    g = W.grid(nx, ny, *box)
    o = ref.Oracle(g, W.body(np.array(poly)))
    o.geometry_poly(np.array(poly).reshape(-1), 0)
    return o, o.geometry_dump(0)


def shoelace(p):
    p = np.asarray(p)
    x, y = p[:, 0], p[:, 1]
    return 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)


def inside(poly, X, Y):
    """Closed convex-polygon membership, vectorised (test-side brute force)."""
    poly = np.asarray(poly)
    ok = np.ones_like(X, dtype=bool)
    for k in range(len(poly)):
        a, b = poly[k], poly[(k + 1) % len(poly)]
        ok &= (b[0] - a[0]) * (Y - a[1]) - (b[1] - a[1]) * (X - a[0]) >= 0
    return ok


def test_hand_worked_cell():
    # unit cell, solid {x + y <= 0.5}: alpha 0.875, W and S half open, E and N open
    tri = [(-3.0, -3.0), (3.5, -3.0), (-3.0, 3.5)]
    o, G = oracle_for_poly(1, 1, (0.0, 1.0, 0.0, 1.0), tri)
    assert abs(G["alpha"][0, 0] - 0.875) < 1e-15
    assert abs(G["bx"][0, 0] - 0.5) < 1e-15 and G["bx"][0, 1] == 1.0
    assert abs(G["by"][0, 0] - 0.5) < 1e-15 and G["by"][1, 0] == 1.0
    assert list(G["vcls"].ravel()) == [1, 0, 0, 0]
    # shielded volume of the x-sweep: alpha - min(beta_W, beta_E) = 0.375; d = 0.375/0.5
    ahat = G["alpha"][0, 0] - min(G["bx"][0, 0], G["bx"][0, 1])
    assert abs(ahat - 0.375) < 1e-15
    # mean distance from the E face to the wall over the shielded part y in [0, 0.5]
    ys = (np.arange(100000) + 0.5) / 100000 * 0.5
    assert abs(np.mean(1.0 - (0.5 - ys)) - ahat / 0.5) < 1e-9
    wp = o.wall_point(0, 0, 0)
    assert np.allclose(wp, [0.25, 0.25], atol=1e-15)


def test_vertex_on_boundary_is_solid():
    tri = [(-3.0, -3.0), (3.5, -3.0), (-3.0, 3.5)]  # edge passes through (0.5, 0) and (0, 0.5)
    o, G = oracle_for_poly(2, 2, (0.0, 1.0, 0.0, 1.0), tri)
    assert G["vcls"][0, 1] == 1 and G["vcls"][1, 0] == 1  # (0.5,0) and (0,0.5) lie on the edge
    assert G["vcls"][1, 1] == 0


@pytest.mark.parametrize("shape", ["circle", "triangle", "naca", "square45"])
def test_volume_fractions_brute_force(shape):
    if shape == "circle":
        poly = W.circle(0.31, 48) + [0.52, 0.47]
    elif shape == "triangle":
        poly = W.triangle(0.6) @ np.array([[math.cos(0.3), math.sin(0.3)], [-math.sin(0.3), math.cos(0.3)]]) + [0.5, 0.5]
    elif shape == "naca":
        poly = W.naca00(0.3, 0.8, 40, 0.0) + [0.1, 0.5]
    else:
        poly = np.array([[0.5, 0.1], [0.9, 0.5], [0.5, 0.9], [0.1, 0.5]])
    n = 7
    o, G = oracle_for_poly(n, n, (0.0, 1.0, 0.0, 1.0), poly)
    N = 240  # samples per cell edge
    s = (np.arange(N * n) + 0.5) / (N * n)
    X, Y = np.meshgrid(s, s)
    solid = inside(poly, X, Y).reshape(n, N, n, N)
    frac = 1.0 - solid.mean(axis=(1, 3))
    assert np.abs(frac - G["alpha"]).max() < 6.0 / N
    # exact identity: total solid area equals the polygon area
    assert abs((1.0 - G["alpha"]).sum() / n ** 2 - shoelace(poly)) < 1e-13
    # classes of vertices by brute-force membership
    v = np.linspace(0.0, 1.0, n + 1)
    VX, VY = np.meshgrid(v, v)
    assert np.array_equal(G["vcls"].astype(bool), inside(poly, VX, VY))


def test_face_apertures_are_chords():
    poly = W.circle(0.3, 64) + [0.5, 0.5]
    n = 10
    o, G = oracle_for_poly(n, n, (0.0, 1.0, 0.0, 1.0), poly)
    h = 1.0 / n
    for i in range(n + 1):
        x = i * h
        # length of the vertical line x inside the polygon, by half-plane clipping
        lo, hi = -1.0, 2.0
        for k in range(len(poly)):
            a, b = poly[k], poly[(k + 1) % len(poly)]
            # g(y) = (b-a)x (y - a_y) - (b-a)y (x - a_x) >= 0
            c1 = b[0] - a[0]
            c0 = -c1 * a[1] - (b[1] - a[1]) * (x - a[0])
            if c1 > 0:
                lo = max(lo, -c0 / c1)
            elif c1 < 0:
                hi = min(hi, -c0 / c1)
            elif c0 < 0:
                lo, hi = 1, 0
        chord = max(0.0, min(hi, 1.0) - max(lo, 0.0))
        assert abs((1.0 - G["bx"][:, i]).sum() * h - chord) < 1e-13


def test_effective_wall_normals_telescope():
    for poly in (W.circle(0.27, 1024) + [0.45, 0.55], W.naca00(0.12, 0.6, 200, 0.25) + [0.5, 0.5]):
        o, G = oracle_for_poly(23, 19, (0.0, 1.0, 0.0, 1.0), poly)
        hx, hy = 1 / 23, 1 / 19
        Nx = (G["bx"][:, :-1] - G["bx"][:, 1:]) * hy
        Ny = (G["by"][:-1, :] - G["by"][1:, :]) * hx
        assert abs(Nx.sum()) < 1e-13 and abs(Ny.sum()) < 1e-13
        # and it is the integral of the outward (into-solid) normal: |N| sums to >= perimeter proxy
        assert np.hypot(Nx, Ny).sum() > 0


def test_cut_cells_classification_consistent():
    poly = W.circle(0.2, 256) + [0.5, 0.5]
    o, G = oracle_for_poly(32, 32, (0.0, 1.0, 0.0, 1.0), poly)
    v = G["vcls"]
    allsolid = (v[:-1, :-1] & v[1:, :-1] & v[:-1, 1:] & v[1:, 1:]).astype(bool)
    allfluid = ~(v[:-1, :-1] | v[1:, :-1] | v[:-1, 1:] | v[1:, 1:]).astype(bool)
    assert (G["alpha"][allsolid] == 0.0).all()
    assert (G["alpha"][allfluid] == 1.0).all()
    mixed = ~allsolid & ~allfluid
    assert ((G["alpha"][mixed] > 0.0) & (G["alpha"][mixed] < 1.0)).all()
