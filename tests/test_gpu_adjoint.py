"""GPU adjoint (cronos_rollout / cronos_rollout_backward) against the FP64 oracle adjoint and
central finite differences of the FP64 oracle forward.  Bar: normwise relative error
<= 1e-3 on the gradient with respect to the actuation phases and amplitudes."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as A
from oracle import lattice as L
from oracle import physics as P
from paper_2207_09334_amd import cronos as CR
from paper_2207_09334_amd import problem as PR
from tests.gpu_common import oracle_problem, say

pytestmark = pytest.mark.gpu

G_TOL = 1e-3


def _actuated_cube(ground: bool, groups=3, n=5, seed=11):
    vox = W.box_voxels(n - 1, n - 1, n - 1)
    rng = np.random.default_rng(seed)
    mat = rng.integers(0, 3, len(vox)).astype(np.int32)
    grp = (np.arange(len(vox)) % groups).astype(np.int32)
    return W.Workload(
        name="adj", bodies=[W.Body(vox, mat, grp)], spacing=0.01, origin=(0.0, 0.0, 0.0 if ground else 0.05),
        mass_mode="uniform", mass_value=0.1, density=0.0, k_mode="assembly", k_uniform=0.0,
        material_k=(1e3, 3e3, 1e4), jitter=0.0, pin_axis=-1, pin_index=0, gravity=(0.0, 0.0, -9.81),
        damping=1e-3, dt=1e-4, ground=ground, ground_z=0.0, ground_k=1e5, ground_mu=0.8, steps=0,
        n_groups=groups, freq_hz=20.0, phase=rng.uniform(0, 2 * np.pi, groups), amp=np.full(groups, 0.15))


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _compare(w, T, K, loss_w, fd_h=None, **create):
    lat, sys_, x0 = oracle_problem(w)
    sim, _, _ = PR.create(w, x0=x0, **create)
    loss_g = CR.cronos_rollout(sim, T, K, loss_w)
    dp, da, dx, dv = CR.cronos_rollout_backward(sim, want_state=True)
    loss_o, op, oa, ox, ov = A.rollout_grad(sys_, x0, np.zeros_like(x0), 0, T, loss_w)
    g_dev, g_ora = np.concatenate([dp, da]), np.concatenate([op, oa])
    e = _rel(g_dev, g_ora)
    say(f"  loss dev {loss_g:.9e} oracle {loss_o:.9e}; gradient rel err vs oracle adjoint {e:.2e}")
    assert loss_g == pytest.approx(loss_o, rel=1e-5, abs=1e-9)
    assert e <= G_TOL
    if fd_h:
        G = len(op)
        fd = []
        for which in ("phase", "amp"):
            for g in range(G):
                def s_(delta):
                    ph, am = sys_.phase.copy(), sys_.amp.copy()
                    (ph if which == "phase" else am)[g] += delta
                    return dataclasses.replace(sys_, phase=ph, amp=am)
                fd.append((A.rollout_loss(s_(fd_h), x0, np.zeros_like(x0), 0, T, loss_w) -
                           A.rollout_loss(s_(-fd_h), x0, np.zeros_like(x0), 0, T, loss_w)) / (2 * fd_h))
        e_fd = _rel(g_dev, fd)
        say(f"  gradient rel err vs central differences {e_fd:.2e}")
        assert e_fd <= G_TOL
    return sim, dx, ox


def test_adjoint_smooth_vs_oracle_and_fd():
    w = _actuated_cube(ground=False)
    say("case: adjoint, free actuated cube, 150 steps, checkpoints every 40")
    lat = L.build(w)
    loss_w = np.random.default_rng(3).normal(size=lat.x.shape) / lat.n_masses
    sim, dx, ox = _compare(w, 150, 40, loss_w, fd_h=1e-6)
    assert _rel(dx, ox) <= G_TOL


def test_adjoint_contact_friction_vs_oracle_and_fd():
    w = _actuated_cube(ground=True)
    say("case: adjoint, actuated cube on the plane, 200 steps, checkpoints every 100")
    lat = L.build(w)
    loss_w = np.zeros_like(lat.x)
    loss_w[:, 0] = lat.mass / lat.mass.sum()
    _compare(w, 200, 100, loss_w, fd_h=1e-7)


def test_adjoint_four_lanes_per_mass_vs_oracle_and_fd():
    """The same bar with 4 lanes per mass in 64-mass workgroups (the autotuner's pick for the
    quadruped) in both the forward steps and the adjoint gather: the actuated cube on the plane
    against the oracle's adjoint and central differences, and the quadruped against the
    oracle's adjoint."""
    w = _actuated_cube(ground=True)
    say("case: adjoint with 4 lanes per mass: actuated cube 200 steps, quadruped 300 steps")
    lat = L.build(w)
    loss_w = np.zeros_like(lat.x)
    loss_w[:, 0] = lat.mass / lat.mass.sum()
    sim, _, _ = _compare(w, 200, 100, loss_w, fd_h=1e-7, lanes_per_mass=4, block_masses=64)
    assert CR.cronos_launch_config(sim)["lanes_per_mass"] == 4
    w = W.quadruped()
    lat = L.build(w)
    loss_w = np.zeros_like(lat.x)
    loss_w[:, 0] = lat.mass / lat.mass.sum()
    _compare(w, 300, 100, loss_w, lanes_per_mass=4, block_masses=64)


def test_adjoint_quadruped_vs_oracle():
    """The quadruped (16 groups, 12,711 masses), forward-displacement loss, 300 steps in 3
    checkpointed segments."""
    w = W.quadruped()
    say("case: adjoint, quadruped 300 steps, checkpoints every 100")
    lat = L.build(w)
    loss_w = np.zeros_like(lat.x)
    loss_w[:, 0] = lat.mass / lat.mass.sum()
    _compare(w, 300, 100, loss_w)


def test_adjoint_quadruped_full_rollout_runs():
    """The full 2000-step quadruped gradient with 20 checkpoints: finite, non-zero, and
    repeatable bit for bit."""
    w = W.quadruped()
    say("case: adjoint, quadruped 2000 steps, checkpoints every 100")
    sim, lat, x0 = PR.create(w)
    lw = np.zeros_like(lat.x)
    lw[:, 0] = lat.mass / lat.mass.sum()
    out = []
    for _ in range(2):
        CR.cronos_set_state(sim, x0, np.zeros_like(x0), 0)
        loss = CR.cronos_rollout(sim, 2000, 100, lw)
        dp, da = CR.cronos_rollout_backward(sim)
        out.append((loss, dp, da))
    assert np.isfinite(out[0][1]).all() and np.isfinite(out[0][2]).all()
    assert np.abs(out[0][1]).max() > 0 and np.abs(out[0][2]).max() > 0
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])


def _golden_gradients():
    import os
    rows = {}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "quadruped_gradient_2000.txt")
    for line in open(path):
        if line.startswith("#"):
            continue
        p = line.split()
        rows[p[0]] = (float(p[1]), np.array([float(v) for v in p[2:]]))
    return rows


@pytest.mark.parametrize("ground", [True, False])
def test_adjoint_quadruped_2000_steps_vs_oracle_within_fp32_state_floor(ground):
    """The configured quadruped gradient: 2000 steps, a checkpoint every 100 (20 segments),
    against the FP64 oracle's gradients stored by tests/golden/make_quadruped_gradient.py.  Over
    2000 steps the actuated body is chaotic, on its contact plane and off it: the oracle with
    its state merely rounded to FP32 after every step moves the gradient by 3.7x its norm with
    contact (0.24x without) and the loss by 2.6e-4 (4.5e-3), so no FP32-state implementation
    can hold the 1e-3 bar at this length (it is held over 300 steps above).  As for the chaotic
    positions, the device must stay within 10x that FP32-state floor of the exact gradient, and
    its loss within 10x the loss floor."""
    rows = _golden_gradients()
    key = "" if ground else "noground_"
    l64, g64 = rows[key + "fp64"]
    l32, g32 = rows[key + "fp32_state"]
    w = W.quadruped()
    say(f"case: adjoint, quadruped 2000 steps, 20 checkpoints, {'contact' if ground else 'no contact plane'}")
    lat = L.build(w)
    if ground:
        lw = np.zeros_like(lat.x)
        lw[:, 0] = lat.mass / lat.mass.sum()
        sim, _, x0 = PR.create(w)
    else:
        lw = np.random.default_rng(2000).normal(size=lat.x.shape) / lat.n_masses
        sim, _, x0 = PR.create(w, ground=False)
    assert np.array_equal(x0, lat.x)
    loss = CR.cronos_rollout(sim, 2000, 100, lw)
    dp, da = CR.cronos_rollout_backward(sim)
    g = np.concatenate([dp, da])
    e_g, f_g = _rel(g, g64), _rel(g32, g64)
    e_l, f_l = abs(loss - l64) / abs(l64), abs(l32 - l64) / abs(l64)
    say(f"  loss dev {loss:.9e} oracle {l64:.9e}: err {e_l:.2e} (FP32-state floor {f_l:.2e}); "
        f"gradient err {e_g:.2e} (floor {f_g:.2e})")
    assert np.isfinite(g).all()
    assert e_l <= 10.0 * f_l
    assert e_g <= 10.0 * f_g


def test_autograd_function_drives_torch():
    torch = pytest.importorskip("torch")
    from paper_2207_09334_amd.autograd import RolloutGrad, forward_displacement_weights
    w = _actuated_cube(ground=True)
    sim, lat, x0 = PR.create(w)
    lw = forward_displacement_weights(lat.mass)
    phase = torch.tensor(w.phase, dtype=torch.float64, requires_grad=True)
    amp = torch.tensor(w.amp, dtype=torch.float64, requires_grad=True)
    loss = RolloutGrad.apply(phase, amp, sim, x0, np.zeros_like(x0), 0, 200, 50, lw, w.freq_hz)
    loss.backward()
    CR.cronos_set_state(sim, x0, np.zeros_like(x0), 0)
    CR.cronos_set_actuation(sim, w.phase, w.amp, w.freq_hz)
    CR.cronos_rollout(sim, 200, 50, lw)
    dp, da = CR.cronos_rollout_backward(sim)
    assert np.array_equal(phase.grad.numpy(), dp) and np.array_equal(amp.grad.numpy(), da)


def test_repeated_sweeps_follow_amplitude_increases_in_the_shifted_frame():
    """Without the contact plane the device frame is shifted, so wavefronts take the plain
    coordinate difference when all their masses lie beyond the safe distance, which grows with
    the largest amplitude.  Raising the amplitudes between calls (0.02 -> 0.1 -> 0.25) must
    reach every launch that depends on it (the forward's step graphs are captured again): every
    call's gradients equal those of a simulation on plain launches bit for bit."""
    w = _actuated_cube(ground=False)
    say("case: adjoint sweeps, default launches vs plain launches in the shifted frame, amplitudes raised per call")
    sim_g, lat, x0 = PR.create(w)
    sim_p, _, _ = PR.create(w, flags=CR.NO_GRAPH)
    # not the centre of mass: with no contact plane its motion ignores the internal forces, so
    # its gradient with respect to the actuation is zero; seeded per-mass weights see the springs
    lw = np.random.default_rng(5).normal(0.0, 1.0, lat.x.shape) / len(lat.x)
    for amp in (0.02, 0.1, 0.25):
        am = np.full(len(w.amp), amp)
        out = []
        for sim in (sim_g, sim_p):
            CR.cronos_set_state(sim, x0, np.zeros_like(x0), 0)
            CR.cronos_set_actuation(sim, w.phase, am, w.freq_hz)
            loss = CR.cronos_rollout(sim, 200, 50, lw)
            dp, da = CR.cronos_rollout_backward(sim)
            out.append((loss, dp, da))
        say(f"  amplitude {amp}: loss {out[0][0]:.9e}, |dphase| {np.abs(out[0][1]).max():.3e}")
        assert out[0][0] == out[1][0]
        assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])
        assert np.abs(out[0][1]).max() > 0
    sim_g.close()
    sim_p.close()


def test_repeated_sweeps_match_plain_launches():
    """Repeated rollouts and reverse sweeps on one simulation, with new phases and amplitudes
    between them (and other work on the stream in between), give bitwise the gradients of a
    simulation on plain launches."""
    w = _actuated_cube(ground=True)
    say("case: adjoint reverse sweeps, default launches vs plain launches, 3 calls")
    sim_g, lat, x0 = PR.create(w)
    sim_p, _, _ = PR.create(w, flags=CR.NO_GRAPH)
    lw = np.zeros_like(lat.x)
    lw[:, 0] = lat.mass / lat.mass.sum()
    rng = np.random.default_rng(3)
    for rep in range(3):
        ph = w.phase + rng.normal(0.0, 0.3, len(w.phase))
        am = np.clip(w.amp + rng.normal(0.0, 0.02, len(w.amp)), 0.0, 0.25)
        out = []
        for sim in (sim_g, sim_p):
            CR.cronos_set_state(sim, x0, np.zeros_like(x0), 0)
            CR.cronos_set_actuation(sim, ph, am, w.freq_hz)
            loss = CR.cronos_rollout(sim, 300, 50, lw)
            dp, da, dx, dv = CR.cronos_rollout_backward(sim, want_state=True)
            out.append((loss, dp, da, dx, dv))
        CR.cronos_step(sim_g, 7)
        CR.cronos_diagnostics(sim_g)
        assert out[0][0] == out[1][0]
        for a, b in zip(out[0][1:], out[1][1:]):
            assert np.array_equal(a, b)
        assert np.abs(out[0][1]).max() > 0
