"""Reverse-mode derivative of the discrete step, FP64 (test infrastructure).

The paper says differentiation is enabled by its system but does not describe it; this is
the plain adjoint of the step of ``physics.step`` (symplectic Euler with contact, Coulomb
clamp, damping, fixed masses and actuated rest lengths) for a loss L = sum_i w_i . x_i(T).
It stores every state of the rollout (no checkpointing) and runs the recurrences backwards:

  x' = x + dt v'             ->  x_bar += x'_bar ;  v'_bar_tot = v'_bar + dt x'_bar
  v' = (1 - d) v**           ->  v**_bar = (1 - d) v'_bar_tot
  v** = clamp(v*) (contact)  ->  v*_bar = J^T v**_bar,  J = I - (c/|v_t|)(I - u u^T) when
                                 sliding, 0 when stuck; c = mu F_n dt / m depends on z
  v* = v + dt f(x, theta)/m  ->  v_bar = v*_bar ;  w = dt v*_bar / m is the adjoint of f
  f(x)                        ->  x_bar_i += sum_springs K_s (w_j - w_i) - k_g w_z (contact),
                                 K_s = k [n n^T + (1 - l0/l)(I - n n^T)]
  l0(theta)                   ->  theta_bar += (dl0/dtheta) k n . (w_j - w_i)
  fixed masses: x' = x, v' = 0 (their w is zero).

Pinned by central finite differences of the forward rollout (tests/test_oracle_adjoint.py).
"""
from __future__ import annotations

import numpy as np

from . import physics as P


def rollout_loss(sys: P.System, x0, v0, n0: int, T: int, loss_w) -> float:
    x, v = P.run(sys, np.array(x0, float), np.array(v0, float), n0, T)
    return float((loss_w * x).sum())


def rollout_grad(sys: P.System, x0, v0, n0: int, T: int, loss_w, state_round=None):
    """Returns (loss, dL/dphase, dL/damp, dL/dx0, dL/dv0).  state_round (optional) is applied to
    every state of the forward rollout before it is stored and stepped on (e.g. rounding to
    FP32, to measure how far a trajectory stored in FP32 moves the gradient)."""
    rnd = state_round if state_round is not None else (lambda a: a)
    xs, vs = [np.array(x0, float)], [np.array(v0, float)]
    for n in range(T):
        x, v = P.step(sys, xs[-1], vs[-1], n0 + n)
        xs.append(rnd(x))
        vs.append(rnd(v))
    loss = float((loss_w * xs[-1]).sum())

    N = sys.n
    m = sys.mass
    free = ~sys.pinned
    i, j = sys.ends[:, 0], sys.ends[:, 1]
    act = sys.gidx >= 0
    G = 0 if sys.phase is None else len(sys.phase)
    dphase, damp = np.zeros(G), np.zeros(G)
    omega = 2.0 * np.pi * sys.freq

    xb = np.array(loss_w, float)
    vb = np.zeros((N, 3))
    for n in reversed(range(T)):
        x, v = xs[n], vs[n]
        t = (n0 + n) * sys.dt
        l0 = P.rest_lengths(sys, t)
        f = P.forces(sys, x, t)
        vstar = v + sys.dt * f / m[:, None]
        fn = P.contact_normal(sys, x)

        vtot = vb + sys.dt * xb
        vbb = (1.0 - sys.damping) * vtot
        vsb = vbb.copy()
        zb = np.zeros(N)
        touching = fn > 0
        if touching.any():
            c = sys.ground_mu * fn * sys.dt / m
            vt = vstar[:, :2]
            sp = np.sqrt((vt * vt).sum(axis=1))
            slide = touching & (sp > c)
            stick = touching & ~slide
            g = vbb[:, :2]
            if slide.any():
                u = vt[slide] / sp[slide, None]
                gs = g[slide]
                ug = (u * gs).sum(axis=1)
                vsb[slide, :2] = gs - (c[slide] / sp[slide])[:, None] * (gs - u * ug[:, None])
                cb = -ug
                zb[slide] += cb * (-sys.ground_mu * sys.dt * sys.ground_k / m[slide])
            vsb[stick, :2] = 0.0
        w = np.where(free[:, None], sys.dt * vsb / m[:, None], 0.0)

        # spring terms K_s (w_j - w_i)
        d = x[j] - x[i]
        length = np.sqrt((d * d).sum(axis=1))
        nvec = d / length[:, None]
        dw = w[j] - w[i]
        ndw = (nvec * dw).sum(axis=1)
        k = sys.k
        Kdw = k[:, None] * (nvec * ndw[:, None] + (1.0 - l0 / length)[:, None] * (dw - nvec * ndw[:, None]))
        xbn = xb.copy()
        np.add.at(xbn, i, Kdw)
        np.add.at(xbn, j, -Kdw)
        if sys.ground:
            xbn[:, 2] += np.where(touching, -sys.ground_k * w[:, 2], 0.0) + zb * free

        if G and act.any():
            q = k[act] * ndw[act]
            ga = sys.gidx[act]
            arg = omega * t + sys.phase[ga]
            np.add.at(dphase, ga, sys.rest[act] * sys.amp[ga] * np.cos(arg) * q)
            np.add.at(damp, ga, sys.rest[act] * np.sin(arg) * q)

        vb = np.where(free[:, None], vsb, 0.0)
        xb = xbn
    return loss, dphase, damp, xb, vb
