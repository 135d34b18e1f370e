"""The allocation-free natural-frequency entry point (its Lanczos buffers carved from the
library's fixed per-GPU workspace) against the allocating one: the same kernels on the same
state, so the frequencies and step counts agree bit for bit; and against the oracle's
eigen-solver within the bar of the allocating entry point's own test (run on an MI355X)."""
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


def _beam(nx, ny, nz):
    w = W.cantilever(nx, ny, nz)
    lat = L.build(w)
    sim, _, _ = PR.create(w, x0=lat.x, gravity=(0.0, 0.0, 0.0))
    return lat, sim


def _check(lat, sim, n_modes):
    xg, _, _ = CR.cronos_read_state(sim)
    ref, _ = LN.natural_frequencies(xg, lat.ends, F32(lat.k), F32(lat.rest), F32(lat.mass), lat.pinned, n_modes)
    om_a, it_a = CR.cronos_natural_frequencies(sim, n_modes=n_modes, tol=1e-10)
    om_n, it_n = CR.cronos_natural_frequencies_noalloc(sim, n_modes=n_modes, tol=1e-10)
    say(f"  {lat.n_masses} masses: allocating {om_a} ({it_a} steps), fixed workspace {om_n} ({it_n} steps), "
        f"oracle {ref}")
    assert it_n == it_a and np.array_equal(om_n, om_a)
    assert len(om_n) == n_modes and om_n == pytest.approx(ref, rel=1e-7)
    # the state is left alone
    x2, _, _ = CR.cronos_read_state(sim)
    assert np.array_equal(x2, xg)


def test_noalloc_frequencies_two_calls_second_smaller():
    lat, sim = _beam(61, 7, 5)
    _check(lat, sim, 3)
    sim.close()
    lat2, sim2 = _beam(31, 5, 4)      # a smaller system reuses the same workspace
    _check(lat2, sim2, 2)
    sim2.close()


def test_noalloc_rejects_what_the_workspace_cannot_hold():
    lat, sim = _beam(21, 4, 4)
    with pytest.raises(CR.CronosError, match="EINVAL.*workspace"):
        CR.cronos_natural_frequencies_noalloc(sim, n_modes=2, max_iter=1 << 24)
    # a failed call leaves the entry point usable
    om, _ = CR.cronos_natural_frequencies_noalloc(sim, n_modes=2, tol=1e-10)
    om_a, _ = CR.cronos_natural_frequencies(sim, n_modes=2, tol=1e-10)
    assert np.array_equal(om, om_a)
    sim.close()
