"""Pins of the oracle's gas dynamics against closed forms and values printed in the paper.

Closed forms: piston-driven shock and stationary normal shock (Rankine-Hugoniot), the
exact Riemann solution in cases that reduce to them, HLLC consistency and symmetry,
van Leer limiter properties.  Printed values: tests/golden/paper_states.json.
"""
import math

import numpy as np
import pytest

from oracle import exact, ref


def cons(rho, u, v, p, g=1.4):
    return np.array([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])


# ------------------------------------------------------------------ printed states (P1)
def test_piston_shock_matches_printed_state(golden):
    d = golden["piston_mach_1_76"]
    S, rho1, p1 = exact.piston_shock(d["gamma"], d["rho0"], d["p0"], d["u_piston"])
    a0 = math.sqrt(d["gamma"] * d["p0"] / d["rho0"])
    assert abs(S / a0 - d["mach_shock"]) < 5e-4
    assert abs(rho1 - d["rho1"]) < 5e-4 * d["rho1"]
    assert abs(p1 - d["p1"]) < 1.0  # printed to the pascal
    # and the inverse relation: the Mach number gives back the printed piston speed
    up = exact.piston_from_shock_mach(d["gamma"], d["rho0"], d["p0"], d["mach_shock"])
    assert abs(up - d["u_piston"]) < 0.5


def test_stationary_shock_matches_printed_states(golden):
    d = golden["stationary_shock_mach_1_34"]
    r, u, p = exact.stationary_shock_downstream(d["gamma"], d["rho_l"], d["u_l"], d["p_l"])
    assert abs(r - d["rho_r"]) < 1e-3
    # rho_l is printed to 3 digits (+-0.08 %), which moves u_r by up to +-0.25 m/s
    assert abs(u - d["u_r"]) < 0.3
    assert abs(p - d["p_r"]) < 0.5e3 and abs(p - d["p_r_sec33"]) < 0.05e3
    M = d["u_l"] / math.sqrt(d["gamma"] * d["p_l"] / d["rho_l"])
    assert abs(M - 1.34) < 5e-3


def test_mach_2_82_ratios_are_those_of_mach_2_81(golden):
    d = golden["mach_2_82_ratios"]
    r, pr = exact.normal_shock(d["gamma"], d["mach_consistent"])
    assert abs(pr - d["p_ratio"]) < 1e-3 and abs(r - d["rho_ratio"]) < 1e-3
    r2, pr2 = exact.normal_shock(d["gamma"], d["mach_quoted"])
    assert abs(pr2 - d["p_ratio"]) > 0.05  # the quoted Mach number does not give them


def test_naca_freestream_mach(golden):
    d = golden["naca_freestream"]
    M = d["u"] / math.sqrt(d["gamma"] * d["p"] / d["rho"])
    assert abs(M - d["mach"]) < 5e-4


def test_piston_relation_satisfies_jump_conditions():
    g, r0, p0, up = 1.4, 1.0, 1.0, 0.3
    S, r1, p1 = exact.piston_shock(g, r0, p0, up)
    # mass, momentum, energy fluxes in the shock frame
    w0, w1 = -S, up - S
    e0 = p0 / ((g - 1) * r0) + 0.5 * w0 * w0 + p0 / r0
    e1 = p1 / ((g - 1) * r1) + 0.5 * w1 * w1 + p1 / r1
    assert abs(r0 * w0 - r1 * w1) < 1e-13
    assert abs(r0 * w0 * w0 + p0 - (r1 * w1 * w1 + p1)) < 1e-12
    assert abs(e0 - e1) < 1e-12


# ------------------------------------------------------------------ exact Riemann solver
def test_exact_riemann_symmetric_collision_is_piston():
    g, r0, p0, up = 1.4, 1.0, 1.0, 0.3
    S, r1, p1 = exact.piston_shock(g, r0, p0, up)
    ps, us = exact.riemann_star((r0, up, p0), (r0, -up, p0), g)
    assert abs(ps - p1) < 1e-11 and abs(us) < 1e-13
    w = exact.riemann_sample((r0, up, p0), (r0, -up, p0), np.array([0.0, 0.5 * S]), g)
    assert abs(w[0, 0] - r1) < 1e-11


def test_exact_riemann_symmetric_expansion_is_isentropic():
    g, r0, p0, u = 1.4, 1.0, 1.0, 0.4
    ps, us = exact.riemann_star((r0, -u, p0), (r0, u, p0), g)
    a0 = math.sqrt(g * p0 / r0)
    # isentrope + Riemann invariant u + 2a/(g-1) = const gives the star pressure
    a_star = a0 - 0.5 * (g - 1) * u
    assert abs(ps - p0 * (a_star / a0) ** (2 * g / (g - 1))) < 1e-12
    assert abs(us) < 1e-14


def test_exact_riemann_single_shock():
    # right state at rest, left state the post-shock state of a right-moving shock
    g, r0, p0 = 1.4, 1.0, 1.0
    S, r1, p1 = exact.piston_shock(g, r0, p0, 0.5)
    ps, us = exact.riemann_star((r1, 0.5, p1), (r0, 0.0, p0), g)
    assert abs(ps - p1) < 1e-10 and abs(us - 0.5) < 1e-10
    w = exact.riemann_sample((r1, 0.5, p1), (r0, 0.0, p0), np.array([S - 1e-9, S + 1e-9]), g)
    assert abs(w[0, 0] - r1) < 1e-10 and abs(w[0, 1] - r0) < 1e-12


# ------------------------------------------------------------------ numerical flux
@pytest.mark.parametrize("d", [0, 1])
def test_hllc_consistency(d):
    rng = np.random.default_rng(1)
    for _ in range(50):
        q = cons(rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.2, 3))
        assert np.allclose(ref.hllc(q, q, d), ref.flux(q, d), rtol=1e-14, atol=1e-14)


def test_hllc_mirror_symmetry():
    rng = np.random.default_rng(2)
    for _ in range(50):
        a = (rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.2, 3))
        b = (rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(0.2, 3))
        f = ref.hllc(cons(*a), cons(*b), 0)
        # mirror x -> -x: swap sides and negate normal velocities; flux components flip
        fm = ref.hllc(cons(b[0], -b[1], b[2], b[3]), cons(a[0], -a[1], a[2], a[3]), 0)
        assert np.allclose(fm, [-f[0], f[1], -f[2], -f[3]], rtol=1e-12, atol=1e-13)
        # rotation x <-> y
        fy = ref.hllc(cons(a[0], a[2], a[1], a[3]), cons(b[0], b[2], b[1], b[3]), 1)
        assert np.allclose(fy, [f[0], f[2], f[1], f[3]], rtol=1e-14, atol=1e-14)


def test_hllc_resolves_stationary_contact():
    ql, qr = cons(1.0, 0.0, 0.3, 1.0), cons(0.25, 0.0, -0.7, 1.0)
    f = ref.hllc(ql, qr, 0)
    assert np.allclose(f, [0.0, 1.0, 0.0, 0.0], atol=1e-14)


def test_hllc_supersonic_upwinding():
    ql, qr = cons(1.0, 3.0, 0.0, 1.0), cons(0.5, 2.5, 0.1, 0.8)
    assert np.allclose(ref.hllc(ql, qr, 0), ref.flux(ql, 0), rtol=1e-15)
    assert np.allclose(ref.hllc(cons(1.0, -3.0, 0, 1.0), cons(0.5, -3.5, 0.1, 0.8), 0),
                       ref.flux(cons(0.5, -3.5, 0.1, 0.8), 0), rtol=1e-15)


def test_vanleer_properties():
    assert ref.vanleer(1.0, 1.0) == 1.0
    assert ref.vanleer(1.0, -1.0) == 0.0 and ref.vanleer(0.0, 2.0) == 0.0
    assert abs(ref.vanleer(1.0, 3.0) - 1.5) < 1e-15  # harmonic mean 2ab/(a+b)
    rng = np.random.default_rng(3)
    for _ in range(100):
        a, b = rng.normal(size=2)
        v = ref.vanleer(a, b)
        if a * b > 0:
            m = min(abs(a), abs(b))
            assert m * (1 - 1e-15) <= abs(v) <= 2 * m * (1 + 1e-15)  # between min and TVD bound
            assert np.sign(v) == np.sign(a)
        else:
            assert v == 0.0


def test_muscl_flat_profile_is_unchanged():
    q = cons(1.3, 0.2, -0.1, 2.0)
    el, er = ref.muscl(q, q, q, True, 0.4, 0)
    assert np.array_equal(el, q) and np.array_equal(er, q)


def test_wall_riemann_limits():
    q = cons(1.0, 0.0, 0.0, 1.0)
    # wall at rest, gas at rest: wall pressure equals the gas pressure
    p, r = ref.wall_riemann(q, (1.0, 0.0), (0.0, 0.0))
    assert abs(p - 1.0) < 1e-15 and abs(r - 1.0) < 1e-15
    # wall moving with the gas (consistency): no disturbance
    q2 = cons(1.0, 0.4, 0.3, 1.0)
    p, r = ref.wall_riemann(q2, (0.6, 0.8), (0.4, 0.3))
    assert abs(p - 1.0) < 1e-14 and abs(r - 1.0) < 1e-14
    # advancing wall compresses, retreating wall expands
    p_in, _ = ref.wall_riemann(q, (-1.0, 0.0), (0.3, 0.0))
    p_out, _ = ref.wall_riemann(q, (-1.0, 0.0), (-0.3, 0.0))
    assert p_in > 1.0 > p_out
