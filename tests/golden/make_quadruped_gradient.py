"""Writes quadruped_gradient_2000.txt: the FP64 oracle's gradient of the quadruped's forward
displacement (x of the mass-weighted centre of mass after 2000 steps) with respect to its 16
actuation phases and 16 amplitudes, twice: along the exact FP64 trajectory, and along the same
trajectory with the state rounded to FP32 after every step (how far storing the state in FP32
alone moves the gradient of this chaotic contact problem).  Calls only the oracle and the
input generators.  Run from the repository root: python tests/golden/make_quadruped_gradient.py
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


def main():
    w = W.quadruped()
    lat = L.build(w)
    assert w.jitter == 0.0 or all(b.jitter_seed is None for b in w.bodies)
    sys_ = P.system_from(lat, w)
    x0, v0 = lat.x.copy(), np.zeros_like(lat.x)
    lw = np.zeros_like(lat.x)
    lw[:, 0] = lat.mass / lat.mass.sum()
    rows = []
    for name, rnd in (("fp64", None), ("fp32_state", lambda a: a.astype(np.float32).astype(np.float64))):
        t0 = time.time()
        loss, dp, da, _, _ = A.rollout_grad(sys_, x0, v0, 0, T, lw, state_round=rnd)
        print(f"{name}: loss {loss:.12e}, |g| {np.linalg.norm(np.concatenate([dp, da])):.6e}, {time.time() - t0:.0f} s",
              flush=True)
        rows.append((name, loss, dp, da))
    with open(OUT, "w") as f:
        f.write("# FP64 oracle gradient of the quadruped's forward displacement after 2000 steps (seed 2,\n")
        f.write("# dt 1e-4, contact plane, 16 groups): written by make_quadruped_gradient.py.\n")
        f.write("# row: trajectory loss dphase[0..15] damp[0..15]\n")
        for name, loss, dp, da in rows:
            f.write(" ".join([name, repr(float(loss))] + [repr(float(v)) for v in np.concatenate([dp, da])]) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
