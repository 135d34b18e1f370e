"""Writes quadruped_gradient_2000.txt: the FP64 oracle's gradient of a quadruped rollout loss
after 2000 steps with respect to its 16 actuation phases and 16 amplitudes.

Two problems, each twice (along the exact FP64 trajectory, and along the same trajectory with
the state rounded to FP32 after every step: how far storing the state in FP32 alone moves the
gradient):
  contact   -- the configured quadruped on its contact plane, loss = forward displacement (x of
               the mass-weighted centre of mass after 2000 steps);
  noground  -- the same body with the contact plane off (gravity on), loss = sum_i w_i . x_i
               with w drawn from numpy's default_rng(2000) standard normal, divided by the mass
               count: smooth dynamics, where the gradient is well defined at the 1e-3 bar.
Calls only the oracle and the input generators.  Run from the repository root:
    python tests/golden/make_quadruped_gradient.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import adjoint as A  # noqa: E402
from oracle import lattice as L  # noqa: E402
from oracle import physics as P  # noqa: E402

T = 2000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "quadruped_gradient_2000.txt")


def noground_weights(n_masses: int) -> np.ndarray:
    return np.random.default_rng(2000).normal(size=(n_masses, 3)) / n_masses


def main():
    w = W.quadruped()
    lat = L.build(w)
    assert w.jitter == 0.0 or all(b.jitter_seed is None for b in w.bodies)
    x0, v0 = lat.x.copy(), np.zeros_like(lat.x)
    lw_contact = np.zeros_like(lat.x)
    lw_contact[:, 0] = lat.mass / lat.mass.sum()
    problems = (("", P.system_from(lat, w), lw_contact),
                ("noground_", P.system_from(lat, w, ground=False), noground_weights(lat.n_masses)))
    fp32 = lambda a: a.astype(np.float32).astype(np.float64)
    rows = []
    for prefix, sys_, lw in problems:
        for name, rnd in (("fp64", None), ("fp32_state", fp32)):
            t0 = time.time()
            loss, dp, da, _, _ = A.rollout_grad(sys_, x0, v0, 0, T, lw, state_round=rnd)
            print(f"{prefix}{name}: loss {loss:.12e}, |g| {np.linalg.norm(np.concatenate([dp, da])):.6e}, "
                  f"{time.time() - t0:.0f} s", flush=True)
            rows.append((prefix + name, loss, dp, da))
    with open(OUT, "w") as f:
        f.write("# FP64 oracle gradients of quadruped rollout losses after 2000 steps (seed 2, dt 1e-4,\n")
        f.write("# 16 groups): written by make_quadruped_gradient.py.  Rows fp64 / fp32_state: the\n")
        f.write("# configured body on its contact plane, forward displacement; rows noground_*: no contact\n")
        f.write("# plane, loss weights default_rng(2000).normal / n_masses.\n")
        f.write("# row: trajectory loss dphase[0..15] damp[0..15]\n")
        for name, loss, dp, da in rows:
            f.write(" ".join([name, repr(float(loss))] + [repr(float(v)) for v in np.concatenate([dp, da])]) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
