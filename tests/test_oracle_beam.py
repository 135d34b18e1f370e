"""Euler-Bernoulli and natural-frequency pins of the oracle (section "Results": the
cantilever beam tests and the natural frequency analysis).  CPU only.

The lattice's Young's modulus along a lattice axis is E = 2.7 k_v / a for per-voxel stiffness
k_v (Cauchy-Born on the 26-neighbour cell: C11 = 13k/3a, C12 = 7k/3a), so a beam built with
k_v = E a / 2.7 should approach Euler-Bernoulli theory as the cross-section is refined.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import lattice as L
from oracle import linear as LN
from oracle import physics as P

K1 = 1.8751040687  # first root of cos(b) cosh(b) = -1 (clamped-free beam)


def _beam(nx, ny, nz, E=1.0e6, a=0.005):
    w = W.cantilever(nx, ny, nz, youngs=E, spacing=a)
    lat = L.build(w)
    Lb, Wd, H = (nx - 1) * a, (ny - 1) * a, (nz - 1) * a
    I = Wd * H ** 3 / 12.0
    return w, lat, E, Lb, Wd, H, I


def test_lattice_modulus_cauchy_born():
    """Lattice E[100] from C11, C12 of the 26-neighbour cell equals 2.7 k / a."""
    k, a = 1.0, 1.0
    c11, c12 = 13.0 / 3.0 * k / a, 7.0 / 3.0 * k / a
    e100 = (c11 - c12) * (c11 + 2 * c12) / (c11 + c12)
    assert e100 == pytest.approx(2.7 * k / a, rel=1e-14)


def test_euler_bernoulli_static_tip_deflection():
    """Tip load P on an 80x8x8-voxel cantilever: deflection P L^3 / (3 E I) within 4%
    (the lattice is slightly stiffer than the continuum: shear and end effects)."""
    w, lat, E, Lb, Wd, H, I = _beam(81, 9, 9)
    tip = lat.coords[:, 0] == 80
    Ptot = 1.0e-3
    f = np.zeros_like(lat.x)
    f[tip, 2] = -Ptot / tip.sum()
    u = LN.static_displacement(lat.x, lat.ends, lat.k, lat.rest, lat.pinned, f)
    ratio = -u[tip, 2].mean() / (Ptot * Lb ** 3 / (3 * E * I))
    assert 0.96 < ratio <= 1.0


def test_euler_bernoulli_first_frequency_and_refinement():
    """f1 = K^2/(2 pi) sqrt(E I / (rho A L^4)) with K = 1.8751: within 2.5% at 80x8x8 and
    closer than at 40x4x4 (the paper's f proportional to H / L^2 scaling)."""
    ratios = []
    for n in ((41, 5, 5), (81, 9, 9)):
        w, lat, E, Lb, Wd, H, I = _beam(*n)
        om, _ = LN.natural_frequencies(lat.x, lat.ends, lat.k, lat.rest, lat.mass, lat.pinned, 1)
        f1 = K1 ** 2 / (2 * math.pi) * math.sqrt(E * I / (1000.0 * Wd * H * Lb ** 4))
        ratios.append(om[0] / (2 * math.pi) / f1)
    assert abs(ratios[1] - 1) < 0.025
    assert abs(ratios[1] - 1) < abs(ratios[0] - 1)


def test_frequency_scaling_with_height_and_width():
    """Section "Euler-Bernoulli Beam Tests": f independent of width, affine in height."""
    def f_of(ny, nz):
        _, lat, *_ = _beam(41, ny, nz)
        om, _ = LN.natural_frequencies(lat.x, lat.ends, lat.k, lat.rest, lat.mass, lat.pinned, 2)
        return om / (2 * math.pi)
    f_w1, f_w2 = f_of(5, 5), f_of(9, 5)
    # bending in z (the lower mode of the wide beam) does not depend on the width
    assert min(f_w2) == pytest.approx(min(f_w1), rel=0.03)
    f_h2 = f_of(5, 9)
    assert min(f_h2) == pytest.approx(min(f_w1), rel=0.03)      # the other axis now is the thin one
    assert max(f_h2) / min(f_h2) == pytest.approx(2.0, rel=0.08)  # H doubled -> f doubled


def test_simulated_frequency_matches_eigen_prediction():
    """Section "Natural Frequency Analysis": the frequency of the simulated motion matches the
    smallest eigenvalue of K v = w^2 M v.  The beam is started along its first mode with a
    small amplitude (no gravity, no damping); the tip's zero crossings give the period."""
    w, lat, E, Lb, Wd, H, I = _beam(21, 3, 3)
    om, modes = LN.natural_frequencies(lat.x, lat.ends, lat.k, lat.rest, lat.mass, lat.pinned, 1)
    sys = P.system_from(lat, w, gravity=np.zeros(3), damping=0.0)
    dt = sys.dt
    w_d = math.acos(1.0 - (om[0] * dt) ** 2 / 2.0) / dt        # discrete-time frequency
    tip = np.nonzero((lat.coords[:, 0] == 20) & (lat.coords[:, 1] == 1) & (lat.coords[:, 2] == 1))[0][0]
    mode = modes[0] / np.abs(modes[0]).max()
    x = lat.x + 1.0e-6 * mode
    v = np.zeros_like(x)
    axis = int(np.argmax(np.abs(mode[tip])))
    period_steps = 2 * math.pi / w_d / dt
    n_steps = int(3.3 * period_steps)
    trace = np.empty(n_steps)
    for n in range(n_steps):
        x, v = P.step(sys, x, v, n)
        trace[n] = x[tip, axis] - lat.x[tip, axis]
    s = np.sign(trace)
    idx = np.nonzero(s[:-1] * s[1:] < 0)[0]
    cross = idx + trace[idx] / (trace[idx] - trace[idx + 1])       # linear interpolation
    period = 2.0 * np.mean(np.diff(cross)) * dt
    assert 2 * math.pi / period == pytest.approx(w_d, rel=2e-3)


def test_stiffness_matches_force_derivative():
    w = W.cube_drop(3)
    lat = L.build(w)
    rng = np.random.default_rng(7)
    x = lat.x + rng.uniform(-1e-3, 1e-3, lat.x.shape)
    l0 = lat.rest * (1 + rng.uniform(-0.1, 0.1, lat.n_springs))
    K = LN.stiffness(x, lat.ends, lat.k, l0).toarray()
    du = rng.normal(size=x.shape)
    h = 1e-7
    fp = P.spring_forces(x + h * du, lat.ends, lat.k, l0)
    fm = P.spring_forces(x - h * du, lat.ends, lat.k, l0)
    np.testing.assert_allclose(-(fp - fm).ravel() / (2 * h), K @ du.ravel(), rtol=1e-5, atol=1e-6)


def test_contact_stiffness_matches_force_derivative():
    """The contact plane's tangent stiffness is the derivative of the penalty normal force:
    central differences of the oracle's total force with the plane on, at a state where part
    of the body is below the plane (kept away from the kink at z = z_g)."""
    w = W.cube_drop(3)
    lat = L.build(w)
    sys_ = P.system_from(lat, w, gravity=np.zeros(3))
    rng = np.random.default_rng(9)
    x = lat.x.copy()
    x[:, 2] += sys_.ground_z - x[:, 2].min() - 0.5 * lat.rest.min()     # the bottom layer 1/2 spacing under
    x += rng.uniform(-1e-4, 1e-4, x.shape)
    below = x[:, 2] < sys_.ground_z
    assert 0 < below.sum() < len(x)
    K = (LN.stiffness(x, lat.ends, lat.k, lat.rest) + LN.contact_stiffness(x, sys_.ground_z, sys_.ground_k)).toarray()
    du = rng.normal(size=x.shape)
    h = 1e-7
    fp, fm = P.forces(sys_, x + h * du, 0.0), P.forces(sys_, x - h * du, 0.0)
    np.testing.assert_allclose(-(fp - fm).ravel() / (2 * h), K @ du.ravel(), rtol=1e-5, atol=1e-5)
