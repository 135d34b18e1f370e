"""Pins of every field of the oracle's diagnostics (CPU only).

Section "Energy Conservation Tests" tracks the kinetic, gravitational and elastic energy of
the system; with the contact plane on, its penalty spring stores energy too.  Each test below
fixes one or more fields of ``oracle.diagnostics.Diag`` against something other than the
oracle itself -- a closed form of the discrete step, a hand value, or an invariant of the
mechanics (pairwise-cancelling internal forces, conserved energy without damping) -- chosen so
that a perturbed formula (a flipped sign, a dropped 1/2, a wrong weight or axis) fails.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import diagnostics as D
from oracle import lattice as L
from oracle import physics as P


def _free_masses(m, g=(0.0, 0.0, -9.81), dt=1e-4, d=0.0, ground=False, kg=0.0, mu=0.0):
    n = len(m)
    return P.System(mass=np.asarray(m, float), pinned=np.zeros(n, bool), ends=np.zeros((0, 2), np.int64),
                    k=np.zeros(0), rest=np.zeros(0), gidx=np.zeros(0, np.int64), gravity=np.asarray(g, float),
                    damping=d, dt=dt, ground=ground, ground_z=0.0, ground_k=kg, ground_mu=mu)


def test_ke_and_pe_grav_free_fall_closed_form():
    """One mass falling from rest under a gravity vector with all three components, symplectic
    Euler without damping: v_n = g n dt and x_n = x_0 + g dt^2 n (n + 1) / 2, so
    KE_n = m |g|^2 n^2 dt^2 / 2 and PE_n = -m g . x_n (zero at the origin) exactly; their sum
    drops by m |g|^2 dt^2 / 2 per step (the integrator's O(dt) energy error in free fall)."""
    m, dt = 0.37, 2e-4
    g = np.array([0.5, -1.25, -9.81])
    sys = _free_masses([m], g=g, dt=dt)
    x0 = np.array([[0.3, -0.2, 1.7]])
    x, v = x0.copy(), np.zeros((1, 3))
    g2 = float(g @ g)
    e0 = D.diagnostics(sys, x, v, 0.0)[0]
    assert e0.ke == 0.0
    assert e0.pe_grav == pytest.approx(-m * float(g @ x0[0]), rel=1e-15)
    for n in range(1, 1501):
        x, v = P.step(sys, x, v, n - 1)
        if n % 250 == 0:
            d = D.diagnostics(sys, x, v, n * dt)[0]
            assert d.ke == pytest.approx(0.5 * m * g2 * (n * dt) ** 2, rel=1e-11)
            xn = x0[0] + g * dt * dt * n * (n + 1) / 2
            assert d.pe_grav == pytest.approx(-m * float(g @ xn), rel=1e-11)
            assert d.ke + d.pe_grav - (e0.ke + e0.pe_grav) == pytest.approx(-0.5 * m * g2 * dt * dt * n, rel=1e-6)
            assert d.pe_spring == 0.0 and d.pe_contact == 0.0


def _bounce_energy(dt, steps=40000):
    """A 0.1 kg mass dropped from 5 cm onto the plane (k_g = 1e4 N/m, no damping, no
    tangential motion): total energy KE + PE_grav + PE_contact every 10 steps."""
    sys = _free_masses([0.1], dt=dt, ground=True, kg=1e4, mu=0.8)
    x, v = np.array([[0.0, 0.0, 0.05]]), np.zeros((1, 3))
    E, pc = [], []
    for n in range(int(steps * 1e-4 / dt)):
        if n % 10 == 0:
            d = D.diagnostics(sys, x, v, n * dt)[0]
            E.append(d.ke + d.pe_grav + d.pe_contact)
            pc.append(d.pe_contact)
        x, v = P.step(sys, x, v, n)
    return np.array(E), np.array(pc)


def test_pe_contact_bounce_energy_conserved():
    """Several bounces on the penalty plane without damping: KE + PE_grav + PE_contact stays in
    a band proportional to dt (halving dt halves it) that is small against the contact energy
    stored at the deepest point, which equals the drop energy m g h plus m g p_max.  A missing
    1/2, or PE_contact left out, moves the total by that much during every contact."""
    E1, pc1 = _bounce_energy(1e-4)
    E2, _ = _bounce_energy(5e-5)
    m, g, h, kg = 0.1, 9.81, 0.05, 1e4
    assert (pc1 > 0).any() and (pc1 == 0).any()   # in and out of contact, several times
    p_max = (m * g + math.sqrt((m * g) ** 2 + 2 * kg * m * g * h)) / kg
    assert pc1.max() == pytest.approx(0.5 * kg * p_max ** 2, rel=2e-2)
    band1, band2 = np.ptp(E1), np.ptp(E2)
    assert band1 < 0.1 * pc1.max()
    assert 0.35 < band2 / band1 < 0.65


def test_pe_contact_at_rest_closed_form():
    """A 0.1 kg mass settled on the plane with damping: penetration m g / k_g, so the penalty
    spring holds (m g)^2 / (2 k_g)."""
    m, kg = 0.1, 1e5
    sys = _free_masses([m], d=0.01, ground=True, kg=kg, mu=0.8)
    x, v = np.array([[0.0, 0.0, 0.0]]), np.zeros((1, 3))
    for n in range(6000):
        x, v = P.step(sys, x, v, n)
    d = D.diagnostics(sys, x, v, 0.6)[0]
    assert d.pe_contact == pytest.approx((m * 9.81) ** 2 / (2 * kg), rel=1e-5)


def _clamped_beam(dt):
    """A 12 x 3 x 3-node cantilever of the cantilever workload's kind, fixed at x = 0, gravity
    on, no ground, no damping, released straight: total energy every 20 steps."""
    w = W.cantilever(12, 3, 3)
    lat = L.build(w)
    sys = P.system_from(lat, w, damping=0.0, dt=dt)
    x, v = lat.x.copy(), np.zeros_like(lat.x)
    E, pg = [], []
    for n in range(int(0.12 / dt)):
        if n % 20 == 0:
            d = D.diagnostics(sys, x, v, n * dt)[0]
            E.append(d.total)
            pg.append(d.pe_grav)
        x, v = P.step(sys, x, v, n)
    return np.array(E), np.array(pg)


def test_total_energy_with_gravity_bounded_no_drift():
    """The paper's beam energy test with gravity on: a clamped beam sagging and oscillating
    under its weight converts gravitational into elastic and kinetic energy and back; with
    damping and contact off the total stays in an O(dt) band (halving dt halves it) far below
    the gravitational energy exchanged, with no secular drift.  A flipped sign of PE_grav
    would swing the total by twice that exchange."""
    E1, pg1 = _clamped_beam(4e-5)
    E2, _ = _clamped_beam(2e-5)
    swing = np.ptp(pg1)
    assert swing > 0
    band1, band2 = np.ptp(E1), np.ptp(E2)
    assert band1 < 0.05 * swing
    assert 0.3 < band2 / band1 < 0.7
    third = len(E1) // 3
    assert abs(E1[-third:].mean() - E1[:third].mean()) < 0.2 * band1


def test_momentum_through_diagnostics_decays_geometrically():
    """No gravity, ground or fixed masses: internal spring forces cancel pairwise, so
    P_n = (1 - d)^n P_0.  The initial velocity is a uniform drift u plus mirror-antisymmetric
    internal motion (zero momentum by construction), so P_0 = M u."""
    w = W.cube_drop(5)
    lat = L.build(w)
    sys = P.system_from(lat, w, gravity=np.zeros(3), ground=False, damping=0.003)
    rng = np.random.default_rng(5)
    c = lat.coords
    mirror = np.lexsort((4 - c[:, 0], c[:, 1], c[:, 2]))   # node of the x-mirrored coordinate
    assert np.array_equal(c[mirror][:, 0], 4 - c[:, 0])
    s = rng.normal(0, 0.01, lat.x.shape)
    u = np.array([0.02, -0.03, 0.015])
    v = u + (s - s[mirror])
    x = lat.x + rng.uniform(-1e-4, 1e-4, lat.x.shape)
    M = float(lat.mass.sum())
    assert M == pytest.approx(125 * 0.001, rel=1e-14)
    p0 = D.diagnostics(sys, x, v, 0.0)[0].p
    np.testing.assert_allclose(p0, M * u, rtol=1e-12, atol=1e-15)
    for n in range(1, 201):
        x, v = P.step(sys, x, v, n - 1)
    p = D.diagnostics(sys, x, v, 200 * sys.dt)[0].p
    np.testing.assert_allclose(p, M * u * (1 - 0.003) ** 200, rtol=1e-10, atol=1e-15)


def test_com_free_fall_of_an_elastic_body():
    """A 5x5x5-node cube (uniform masses) on the unjittered grid: COM_0 is the grid centre
    (origin + 2a per axis).  Thrown with drift u, internal motion of zero momentum and gravity
    on, no ground or damping: internal forces cancel, so COM_n = COM_0 + u n dt +
    g dt^2 n (n + 1) / 2 exactly (to rounding) while the body vibrates."""
    w = W.cube_drop(5)
    lat = L.build(w)
    sys = P.system_from(lat, w, ground=False, damping=0.0)
    a = w.spacing
    com_hand = np.asarray(w.origin, float) + 2 * a
    rng = np.random.default_rng(6)
    c = lat.coords
    mirror = np.lexsort((c[:, 0], 4 - c[:, 1], c[:, 2]))
    u = np.array([0.1, 0.05, 0.2])
    s = rng.normal(0, 0.02, lat.x.shape)
    x, v = lat.x.copy(), u + (s - s[mirror])
    d0 = D.diagnostics(sys, x, v, 0.0)[0]
    np.testing.assert_allclose(d0.com, com_hand, rtol=0, atol=1e-15)
    g, dt = sys.gravity, sys.dt
    for n in range(1, 801):
        x, v = P.step(sys, x, v, n - 1)
    com = D.diagnostics(sys, x, v, 800 * dt)[0].com
    expect = com_hand + u * 800 * dt + g * dt * dt * 800 * 801 / 2
    np.testing.assert_allclose(com, expect, rtol=0, atol=1e-12)


def test_bbox_and_per_body_split_hand_values():
    """Two bodies side by side: each body's bounding box is its own node range; moving one node
    of the second body moves only that body's box, and only on the axes it crosses."""
    w = W.cube_drop(3)
    lat = L.build(w)
    n = len(lat.mass)
    a = w.spacing
    o = np.asarray(w.origin, float)
    x = np.concatenate([lat.x, lat.x + np.array([1.0, 0.0, 0.0])])
    v = np.zeros_like(x)
    sys = P.System(mass=np.concatenate([lat.mass, 2 * lat.mass]), pinned=np.zeros(2 * n, bool),
                   ends=np.zeros((0, 2), np.int64), k=np.zeros(0), rest=np.zeros(0), gidx=np.zeros(0, np.int64),
                   gravity=np.zeros(3), damping=0.0, dt=1e-4, body_offset=np.array([0, n, 2 * n]))
    b0, b1 = D.diagnostics(sys, x, v, 0.0)
    np.testing.assert_array_equal(b0.bbox_min, o)
    np.testing.assert_allclose(b0.bbox_max, o + 2 * a, rtol=0, atol=1e-15)
    np.testing.assert_allclose(b1.bbox_min, o + [1.0, 0.0, 0.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(b1.bbox_max, o + [1.0 + 2 * a, 2 * a, 2 * a], rtol=0, atol=1e-15)
    x[n + 4] = [5.0, -3.0, o[2] + a]
    c0, c1 = D.diagnostics(sys, x, v, 0.0)
    np.testing.assert_array_equal(c0.bbox_min, b0.bbox_min)
    np.testing.assert_array_equal(c0.bbox_max, b0.bbox_max)
    np.testing.assert_array_equal(c1.bbox_min, [b1.bbox_min[0], -3.0, b1.bbox_min[2]])
    np.testing.assert_array_equal(c1.bbox_max, [5.0, b1.bbox_max[1], b1.bbox_max[2]])
    # the second body's mass is twice the first's, and its COM is its own
    np.testing.assert_allclose(b1.com, o + [1.0 + a, a, a], rtol=0, atol=1e-14)


def test_ke_pe_spring_hand_values_and_nonfinite_flag():
    """Two masses on one spring: KE = sum m v^2 / 2, PE = k (l - l0)^2 / 2, P = sum m v and the
    mass-weighted centre by hand, PE also with an actuated rest length l0 (1 + A sin(2 pi f t +
    phi)); a NaN velocity or an infinite position sets the flag."""
    k, l0, u = 300.0, 0.02, 1.5e-3
    sys = P.System(mass=np.array([0.2, 0.5]), pinned=np.zeros(2, bool), ends=np.array([[0, 1]]),
                   k=np.array([k]), rest=np.array([l0]), gidx=np.array([0]), gravity=np.zeros(3),
                   damping=0.0, dt=1e-4, phase=np.array([0.3]), amp=np.array([0.1]), freq=2.0)
    x = np.array([[0.0, 0.0, 0.0], [0.0, l0 + u, 0.0]])
    v = np.array([[1.0, 2.0, -2.0], [0.0, 0.5, 0.0]])
    d = D.diagnostics(sys, x, v, 0.0)[0]
    assert d.ke == pytest.approx(0.5 * 0.2 * 9.0 + 0.5 * 0.5 * 0.25, rel=1e-15)
    # unequal masses: the mass-weighted centre, not the midpoint
    np.testing.assert_allclose(d.com, [0.0, 0.5 * (l0 + u) / 0.7, 0.0], rtol=1e-15, atol=0)
    np.testing.assert_allclose(d.p, [0.2, 0.4 + 0.25, -0.4], rtol=1e-15, atol=0)
    l0t = l0 * (1 + 0.1 * math.sin(0.3))
    assert d.pe_spring == pytest.approx(0.5 * k * (l0 + u - l0t) ** 2, rel=1e-12)
    t = 0.125   # a quarter period later: sin(pi/2 + 0.3) = cos(0.3)
    l0t = l0 * (1 + 0.1 * math.cos(0.3))
    assert D.diagnostics(sys, x, v, t)[0].pe_spring == pytest.approx(0.5 * k * (l0 + u - l0t) ** 2, rel=1e-12)
    assert not d.nonfinite
    v[1, 2] = np.nan
    assert D.diagnostics(sys, x, v, 0.0)[0].nonfinite
    x[0, 0] = np.inf
    v[1, 2] = 0.0
    assert D.diagnostics(sys, x, v, 0.0)[0].nonfinite
