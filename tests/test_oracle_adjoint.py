"""Pins of the FP64 adjoint against central finite differences of the FP64 forward (CPU)."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as A
from oracle import lattice as L
from oracle import physics as P


def _small_actuated(ground: bool, n=4, groups=3, damping=1e-3, T=150, seed=11):
    """A small multi-material cube whose voxels drive 3 actuation groups."""
    vox = W.box_voxels(n - 1, n - 1, n - 1)
    rng = np.random.default_rng(seed)
    mat = rng.integers(0, 3, len(vox)).astype(np.int32)
    grp = (np.arange(len(vox)) % groups).astype(np.int32)
    w = W.Workload(
        name="adj", bodies=[W.Body(vox, mat, grp)], spacing=0.01, origin=(0.0, 0.0, 0.0 if ground else 0.05),
        mass_mode="uniform", mass_value=0.1, density=0.0, k_mode="assembly", k_uniform=0.0,
        material_k=(1e3, 3e3, 1e4), jitter=0.0, pin_axis=-1, pin_index=0, gravity=(0.0, 0.0, -9.81),
        damping=damping, dt=1e-4, ground=ground, ground_z=0.0, ground_k=1e5, ground_mu=0.8, steps=T,
        n_groups=groups, freq_hz=20.0, phase=rng.uniform(0, 2 * np.pi, groups), amp=np.full(groups, 0.15))
    lat = L.build(w)
    sys_ = P.system_from(lat, w)
    if ground:
        # forward displacement: x of the centre of mass (friction lets actuation move it)
        loss_w = np.zeros_like(lat.x)
        loss_w[:, 0] = lat.mass / lat.mass.sum()
    else:
        # without contact the centre of mass ignores internal forces, so weigh the shape
        loss_w = rng.normal(size=lat.x.shape) / lat.n_masses
    return sys_, lat.x.copy(), np.zeros_like(lat.x), loss_w, T


def _fd(sys_, x0, v0, T, lw, which, g, h):
    def with_param(delta):
        ph, am = sys_.phase.copy(), sys_.amp.copy()
        (ph if which == "phase" else am)[g] += delta
        return dataclasses.replace(sys_, phase=ph, amp=am)
    lp = A.rollout_loss(with_param(h), x0, v0, 0, T, lw)
    lm = A.rollout_loss(with_param(-h), x0, v0, 0, T, lw)
    return (lp - lm) / (2 * h)


def test_adjoint_matches_finite_differences_smooth():
    """No contact: the rollout is smooth; central differences agree to ~1e-7."""
    sys_, x0, v0, lw, T = _small_actuated(ground=False)
    loss, dph, dam, _, _ = A.rollout_grad(sys_, x0, v0, 0, T, lw)
    assert loss == pytest.approx(A.rollout_loss(sys_, x0, v0, 0, T, lw), rel=1e-14)
    g_fd = np.array([_fd(sys_, x0, v0, T, lw, "phase", g, 1e-6) for g in range(3)] +
                    [_fd(sys_, x0, v0, T, lw, "amp", g, 1e-6) for g in range(3)])
    g_ad = np.concatenate([dph, dam])
    assert np.linalg.norm(g_ad - g_fd) <= 1e-6 * np.linalg.norm(g_fd)


def test_adjoint_initial_state_gradient_smooth():
    sys_, x0, v0, lw, T = _small_actuated(ground=False, T=60)
    _, _, _, gx, gv = A.rollout_grad(sys_, x0, v0, 0, T, lw)
    rng = np.random.default_rng(1)
    dx = rng.normal(size=x0.shape)
    h = 1e-7
    fd = (A.rollout_loss(sys_, x0 + h * dx, v0, 0, T, lw) - A.rollout_loss(sys_, x0 - h * dx, v0, 0, T, lw)) / (2 * h)
    assert (gx * dx).sum() == pytest.approx(fd, rel=1e-6)
    dv = rng.normal(size=v0.shape)
    fdv = (A.rollout_loss(sys_, x0, v0 + h * dv, 0, T, lw) - A.rollout_loss(sys_, x0, v0 - h * dv, 0, T, lw)) / (2 * h)
    assert (gv * dv).sum() == pytest.approx(fdv, rel=1e-6)


def test_adjoint_with_contact_and_friction():
    """With the contact plane and the friction clamp the rollout is piecewise smooth; at a
    step size small enough not to cross a stick/slip switch the central differences still
    agree (checked normwise to 1e-4)."""
    sys_, x0, v0, lw, T = _small_actuated(ground=True, T=120)
    _, dph, dam, _, _ = A.rollout_grad(sys_, x0, v0, 0, T, lw)
    g_ad = np.concatenate([dph, dam])
    g_fd = np.array([_fd(sys_, x0, v0, T, lw, "phase", g, 1e-7) for g in range(3)] +
                    [_fd(sys_, x0, v0, T, lw, "amp", g, 1e-7) for g in range(3)])
    assert np.linalg.norm(g_ad - g_fd) <= 1e-4 * np.linalg.norm(g_fd)


def test_adjoint_fixed_masses_and_linearity_in_weights():
    """Fixed masses carry no velocity adjoint; the gradient is linear in the loss weights."""
    sys_, x0, v0, lw, T = _small_actuated(ground=False, T=40)
    pinned = sys_.pinned.copy()
    pinned[:5] = True
    s2 = dataclasses.replace(sys_, pinned=pinned)
    _, a1, b1, _, gv = A.rollout_grad(s2, x0, v0, 0, T, lw)
    assert (gv[:5] == 0).all()
    _, a2, b2, _, _ = A.rollout_grad(s2, x0, v0, 0, T, 2.5 * lw)
    np.testing.assert_allclose(a2, 2.5 * a1, rtol=1e-12)
    np.testing.assert_allclose(b2, 2.5 * b1, rtol=1e-12)
