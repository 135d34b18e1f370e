"""Natural frequency on the GPU (sections "Natural Frequency Analysis" and "Euler-Bernoulli Beam
Tests"): the device's motion of a cantilever started along its first mode oscillates at the
frequency the oracle's eigenproblem K v = w^2 M v predicts (run on an MI355X)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import lattice as L
from oracle import linear as LN
from paper_2207_09334_amd import cronos as CR
from paper_2207_09334_amd import problem as PR
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


def test_simulated_first_frequency_matches_eigen_prediction():
    """A 61x7x5 cantilever (its first mode, bending in the thinner direction, is simple, so the
    start shape is unique up to sign) started along that mode at 2e-4 m."""
    w = W.cantilever(61, 7, 5)
    lat = L.build(w)
    om, modes = LN.natural_frequencies(lat.x, lat.ends, lat.k, lat.rest, lat.mass, lat.pinned, 1)
    dt = w.dt
    w_d = math.acos(1.0 - (om[0] * dt) ** 2 / 2.0) / dt           # symplectic Euler's discrete frequency
    mode = modes[0] / np.abs(modes[0]).max()
    x0 = lat.x + 2.0e-4 * mode
    sim, nlat, _ = PR.create(w, x0=x0, gravity=(0.0, 0.0, 0.0))
    tip = int(np.argmax(np.abs(mode).sum(axis=1)))
    axis = int(np.argmax(np.abs(mode[tip])))
    period_steps = 2 * math.pi / w_d / dt
    every = 16
    n = int(3.3 * period_steps / every)
    trace = np.empty(n)
    for q in range(n):
        CR.cronos_step(sim, every)
        xg, _, _ = CR.cronos_read_state(sim)
        trace[q] = xg[tip, axis] - lat.x[tip, axis]
    s = np.sign(trace)
    idx = np.nonzero(s[:-1] * s[1:] < 0)[0]
    cross = idx + trace[idx] / (trace[idx] - trace[idx + 1])
    period = 2.0 * np.mean(np.diff(cross)) * every * dt
    say(f"  61x7x5 beam: simulated {1 / period:.5f} Hz, eigen {w_d / (2 * math.pi):.5f} Hz, "
        f"{len(cross)} crossings")
    assert len(cross) >= 5
    assert 2 * math.pi / period == pytest.approx(w_d, rel=2e-3)
