"""GPU natural frequencies (section "Natural Frequency Analysis": K v = w^2 M v) from the
device's FP64 Lanczos iterations, against the oracle's shift-invert eigen-solver of the same
tangent stiffness at the device's own FP32 positions, stiffnesses, rest lengths and masses
(run on an MI355X)."""
import numpy as np
import pytest

import workloads as W
from oracle import lattice as L
from oracle import linear as LN
from paper_2207_09334_amd import cronos as CR
from paper_2207_09334_amd import problem as PR
from tests.gpu_common import say

pytestmark = pytest.mark.gpu

F32 = lambda a: np.asarray(a, np.float32).astype(np.float64)


def oracle_omegas(lat, x, count):
    om, _ = LN.natural_frequencies(x, lat.ends, F32(lat.k), F32(lat.rest), F32(lat.mass), lat.pinned, count)
    return om


def distinct(values, rel=1e-7):
    out = []
    for v in values:
        if not out or v - out[-1] > rel * v:
            out.append(v)
    return np.array(out)


def test_rest_beam_lowest_three():
    """A 61x7x5 cantilever at rest: bending in z, bending in y, then the next mode."""
    w = W.cantilever(61, 7, 5)
    lat = L.build(w)
    sim, _, _ = PR.create(w, x0=lat.x, gravity=(0.0, 0.0, 0.0))
    xg, _, _ = CR.cronos_read_state(sim)
    ref = oracle_omegas(lat, xg, 3)
    om, iters = CR.cronos_natural_frequencies(sim, n_modes=3, tol=1e-10)
    say(f"  61x7x5 at rest: device {om} after {iters} Lanczos steps; oracle {ref}")
    assert len(om) == 3
    assert om == pytest.approx(ref, rel=1e-7)


def test_square_beam_reports_the_double_bending_mode_once():
    """61x7x7: the two bending modes share one frequency; the solver gives it once and then
    the next distinct frequency."""
    w = W.cantilever(61, 7, 7)
    lat = L.build(w)
    sim, _, _ = PR.create(w, x0=lat.x, gravity=(0.0, 0.0, 0.0))
    xg, _, _ = CR.cronos_read_state(sim)
    ref = distinct(oracle_omegas(lat, xg, 6), rel=1e-6)
    om, iters = CR.cronos_natural_frequencies(sim, n_modes=2, tol=1e-10)
    say(f"  61x7x7: device {om} after {iters} steps; oracle distinct {ref}")
    assert len(om) == 2
    assert om == pytest.approx(ref[:2], rel=1e-6)


def test_prestressed_state_uses_the_geometric_stiffness():
    """After 3000 steps under a weak gravity the springs carry tension and compression: the
    (1 - l0 / l)(I - n n^T) part of the tangent stiffness enters; the oracle takes K at the
    device's positions."""
    w = W.cantilever(61, 7, 5)
    lat = L.build(w)
    sim, _, _ = PR.create(w, x0=lat.x, gravity=(0.0, 0.0, -0.5))
    CR.cronos_step(sim, 3000)
    xg, _, _ = CR.cronos_read_state(sim)
    ref = oracle_omegas(lat, xg, 2)
    rest_ref = oracle_omegas(lat, F32(lat.x), 2)
    om, iters = CR.cronos_natural_frequencies(sim, n_modes=2, tol=1e-10)
    say(f"  61x7x5 sagged: device {om} ({iters} steps); oracle {ref}; at rest {rest_ref}")
    assert om == pytest.approx(ref, rel=1e-7)
    assert abs(ref[0] / rest_ref[0] - 1.0) > 1e-5      # the prestress does move the frequency


def test_repeatable_and_state_untouched():
    w = W.cantilever(31, 5, 5)
    lat = L.build(w)
    sim, _, _ = PR.create(w, x0=lat.x)
    CR.cronos_step(sim, 100)
    x0, v0, n0 = CR.cronos_read_state(sim)
    a = CR.cronos_natural_frequencies(sim, n_modes=2, seed=7)
    b = CR.cronos_natural_frequencies(sim, n_modes=2, seed=7)
    x1, v1, n1 = CR.cronos_read_state(sim)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1) and n0 == n1


def test_bad_arguments():
    w = W.cantilever(31, 5, 5)
    sim, _, _ = PR.create(w)
    for kw in (dict(n_modes=0), dict(n_modes=33), dict(tol=0.0), dict(tol=1.5), dict(n_modes=4, max_iter=10)):
        with pytest.raises(CR.CronosError):
            CR.cronos_natural_frequencies(sim, **kw)


def test_contact_plane_stiffness_enters():
    """A 61x7x5 cantilever whose bottom layer sits 2 mm below a contact plane: the plane's
    penalty stiffness k_g on those masses' z enters K (the oracle's K + contact term at the
    device's positions), and raises the frequencies above the free beam's."""
    w = W.cantilever(61, 7, 5)
    lat = L.build(w)
    over = dict(gravity=(0.0, 0.0, 0.0), ground=True, ground_z=0.002, ground_k=2.0e3, ground_mu=0.0)
    sim, _, _ = PR.create(w, x0=lat.x, **over)
    xg, _, _ = CR.cronos_read_state(sim)
    assert (xg[:, 2] < 0.002).sum() > 0
    om, _ = LN.natural_frequencies(xg, lat.ends, F32(lat.k), F32(lat.rest), F32(lat.mass), lat.pinned, 3,
                                   ground=(float(np.float32(0.002)), float(np.float32(2.0e3))))
    free = oracle_omegas(lat, xg, 3)
    dev, iters = CR.cronos_natural_frequencies(sim, n_modes=3, tol=1e-10)
    say(f"  on the plane: device {dev} ({iters} steps); oracle {om}; without the plane {free}")
    assert dev == pytest.approx(om, rel=1e-7)
    assert om[0] > 1.01 * free[0]


def test_structured_box_apply_matches_the_general_one():
    """A full box in the structured-box layout (512-mass cubes, neighbours at fixed tile
    offsets, no incidence data) gives the frequencies of the general incidence-list operator on
    the same system to FP64 rounding (the springs are summed in another order), at rest and
    deformed (the geometric term), with and without the contact plane."""
    for w, over in ((W.cantilever(64, 16, 16), dict(gravity=(0.0, 0.0, 0.0))),
                    (W.cube_drop(24), dict(ground_z=0.12))):
        lat = L.build(w)
        rng = np.random.default_rng(3)
        x0 = lat.x + rng.normal(0.0, 2e-4, lat.x.shape) * (~np.asarray(lat.pinned, bool))[:, None]
        sims = [PR.create(w, x0=x0, block_masses=512, flags=f, **over)[0] for f in (0, CR.NO_GRID)]
        forms = [CR.cronos_launch_config(s)["step_form"] for s in sims]
        assert forms == ["grid", "narrow"]
        (og, ig), (on, inn) = [CR.cronos_natural_frequencies(s, n_modes=2, tol=1e-10) for s in sims]
        say(f"  {w.name}: grid {og} ({ig} steps), general {on} ({inn} steps)")
        assert len(og) == len(on) == 2
        np.testing.assert_allclose(og, on, rtol=1e-8)
        for s in sims:
            s.close()
