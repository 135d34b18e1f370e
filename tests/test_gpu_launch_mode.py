"""How cronos_step enqueues its steps: HIP graphs of 2^j steps (both buffer parities, a call's
step count taken from the largest power of two down) or plain launches, chosen at creation
from the measured step time unless a flag decides (run on an MI355X).  Either way a sequence
of step calls must give the same state bit for bit."""
import numpy as np
import pytest

import workloads as W
from paper_2207_09334_amd import cronos as CR
from paper_2207_09334_amd import problem as PR
from tests.gpu_common import say

pytestmark = pytest.mark.gpu

# call lengths that use every graph level, odd counts (a parity flip) and counts above 128
CALLS = (1, 3, 37, 130, 256, 5, 300)


def _run(w, flags, calls=CALLS, actuation=None):
    sim, lat, x0 = PR.create(w, flags=flags)
    mode = CR.cronos_launch_mode(sim)
    states = []
    total = 0
    for i, n in enumerate(calls):
        if actuation is not None and i == 3:
            CR.cronos_set_actuation(sim, *actuation)   # drops the captured graphs mid-sequence
        CR.cronos_step(sim, n)
        total += n
        x, v, step = CR.cronos_read_state(sim)
        assert step == total and np.isfinite(x).all()
        states.append((x, v))
    form = CR.cronos_launch_config(sim)["step_form"]
    sim.close()
    return states, mode, form


@pytest.mark.parametrize("name", ["grid", "quadruped", "quadruped_explicit", "cube_narrow"])
def test_graphs_and_plain_launches_give_the_same_state(name):
    flags, actuation = 0, None
    if name == "grid":
        w = W.cantilever(64, 16, 16)
    elif name == "cube_narrow":
        w = W.cube_drop(10)
    else:
        w = W.quadruped()
        ph = np.asarray(w.phase, float) + 0.5
        actuation = (ph, np.asarray(w.amp, float) * 0.5, w.freq_hz)
        if name == "quadruped_explicit":
            flags = CR.NO_TABLE                     # actuation as its own launch before each step
    say(f"case: launch modes on {w.name} ({name}), calls {CALLS}")
    sg, mg, form = _run(w, flags | CR.GRAPH, actuation=actuation)
    sp, mp, _ = _run(w, flags | CR.NO_GRAPH, actuation=actuation)
    say(f"  form {form}; forced graphs {mg}; plain {mp}")
    assert mg["hip_graph"] and mg["plain_step_us"] > 0
    assert not mp["hip_graph"]
    for (xg, vg), (xp, vp) in zip(sg, sp):
        assert np.array_equal(xg, xp) and np.array_equal(vg, vp)


def test_default_mode_follows_the_measured_step_time():
    for w in (W.cantilever(64, 16, 16), W.quadruped(), W.cantilever(400, 40, 40)):
        sim, _, _ = PR.create(w)
        m = CR.cronos_launch_mode(sim)
        say(f"  {w.name}: plain step {m['plain_step_us']:.2f} us -> graphs {m['hip_graph']}")
        assert m["plain_step_us"] > 0
        assert m["hip_graph"] == (m["plain_step_us"] < 12.0)
        sim.close()


def test_graph_flags_together_are_rejected():
    with pytest.raises(CR.CronosError):
        PR.create(W.cube_drop(4), flags=CR.GRAPH | CR.NO_GRAPH)


@pytest.mark.parametrize("name", ["population", "quadruped"])
def test_staged_and_direct_state_io_give_the_same_state(name):
    """The actuated one-lane table form reads velocities and writes the new state either where
    each lane's mass lies or through LDS in mass order: bitwise the same states over a sequence
    of calls, under plain launches and graphs."""
    w = W.population(6, lo=2000, hi=6000) if name == "population" else W.quadruped()
    say(f"case: staged vs direct state I/O on {w.name}, calls {CALLS}")
    outs = []
    for flags in (CR.DIRECT_IO, CR.STAGED_IO, CR.STAGED_IO | CR.NO_GRAPH):
        sim, _, _ = PR.create(w, flags=flags, block_masses=256, lanes_per_mass=1)
        m = CR.cronos_launch_mode(sim)
        assert m["staged_io"] == bool(flags & CR.STAGED_IO)
        states = []
        for n in CALLS:
            CR.cronos_step(sim, n)
            x, v, _ = CR.cronos_read_state(sim)
            assert np.isfinite(x).all()
            states.append((x, v))
        outs.append(states)
        sim.close()
    for other in outs[1:]:
        for (xa, va), (xb, vb) in zip(outs[0], other):
            assert np.array_equal(xa, xb) and np.array_equal(va, vb)


def test_state_io_flags_together_are_rejected():
    with pytest.raises(CR.CronosError):
        PR.create(W.cube_drop(4), flags=CR.STAGED_IO | CR.DIRECT_IO)


def test_staged_state_io_is_only_taken_by_the_actuated_table_form():
    w = W.cantilever(60, 10, 10)
    sim, _, _ = PR.create(w, flags=CR.STAGED_IO, block_masses=256, lanes_per_mass=1)
    assert CR.cronos_launch_config(sim)["step_form"] == "narrow"
    assert not CR.cronos_launch_mode(sim)["staged_io"]
    sim.close()
