"""torch.autograd bridge for gait gradients: loss of a rollout as a differentiable function of
the actuation phases and amplitudes.  The forward pass is ``cronos_rollout`` and the backward
pass ``cronos_rollout_backward`` (the library's adjoint kernels); torch only carries the
tensors.  Marshalling only."""
from __future__ import annotations

import numpy as np
import torch

from . import cronos as CR


class RolloutGrad(torch.autograd.Function):
    """loss = RolloutGrad.apply(phase, amp, sim, x0, v0, n0, n_steps, ckpt_every, loss_w, freq_hz)

    phase, amp: 1-D float64 tensors [n_bodies * n_groups].  The simulation is reset to
    (x0, v0, step n0) before the rollout, so repeated calls are independent."""

    @staticmethod
    def forward(ctx, phase, amp, sim, x0, v0, n0, n_steps, ckpt_every, loss_w, freq_hz):
        ph = phase.detach().cpu().double().numpy()
        am = amp.detach().cpu().double().numpy()
        CR.cronos_set_state(sim, x0, v0, n0)
        CR.cronos_set_actuation(sim, ph, am, freq_hz)
        loss = CR.cronos_rollout(sim, n_steps, ckpt_every, loss_w)
        ctx.sim = sim
        ctx.dtype, ctx.device = phase.dtype, phase.device
        return torch.tensor(loss, dtype=phase.dtype, device=phase.device)

    @staticmethod
    def backward(ctx, grad_out):
        dp, da = CR.cronos_rollout_backward(ctx.sim)
        g = grad_out.detach().cpu().double().item()
        to = lambda a: torch.as_tensor(g * np.asarray(a), dtype=ctx.dtype, device=ctx.device)
        return to(dp), to(da), None, None, None, None, None, None, None, None


def forward_displacement_weights(mass: np.ndarray, body_offset=None, axis: int = 0) -> np.ndarray:
    """Loss weights of the mass-weighted centre-of-mass coordinate along `axis` (summed over
    bodies): sum_i w_i . x_i = sum_bodies COM_axis."""
    mass = np.asarray(mass, float)
    w = np.zeros((len(mass), 3))
    bo = [0, len(mass)] if body_offset is None else list(body_offset)
    for b in range(len(bo) - 1):
        s, e = bo[b], bo[b + 1]
        w[s:e, axis] = mass[s:e] / mass[s:e].sum()
    return w
