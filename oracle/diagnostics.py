"""Energy and momentum diagnostics, FP64 (test infrastructure; see package docstring).

Section "Energy Conservation Tests" tracks the elastic potential energy of the springs, the
gravitational potential energy and the kinetic energy of the masses (the paper's phrase
"of each spring" is read as: elastic energy per spring, the other two per mass).  With the
contact plane on, the penalty spring of the plane stores 1/2 k_g p^2 per penetrating mass.
Everything is evaluated per body (bodies = contiguous node ranges).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import physics


@dataclasses.dataclass
class Diag:
    ke: float
    pe_spring: float
    pe_grav: float
    pe_contact: float
    p: np.ndarray
    com: np.ndarray
    bbox_min: np.ndarray
    bbox_max: np.ndarray
    nonfinite: bool

    @property
    def total(self) -> float:
        return self.ke + self.pe_spring + self.pe_grav + self.pe_contact


def diagnostics(sys: physics.System, x: np.ndarray, v: np.ndarray, t: float) -> list:
    """List of Diag, one per body.  PE_grav = -sum m g.x (zero at the origin)."""
    l0 = physics.rest_lengths(sys, t)
    _, length = physics.spring_vectors(x, sys.ends)
    e_spring = 0.5 * sys.k * (length - l0) ** 2
    pen = np.maximum(0.0, sys.ground_z - x[:, 2]) if sys.ground else np.zeros(len(x))
    bo = sys.body_offset if sys.body_offset is not None else np.array([0, len(x)])
    out = []
    for b in range(len(bo) - 1):
        s, e = int(bo[b]), int(bo[b + 1])
        m = sys.mass[s:e]
        xb, vb = x[s:e], v[s:e]
        in_body = (sys.ends[:, 0] >= s) & (sys.ends[:, 0] < e)
        out.append(Diag(
            ke=float(0.5 * (m * (vb * vb).sum(axis=1)).sum()),
            pe_spring=float(e_spring[in_body].sum()),
            pe_grav=float(-(m * (xb @ sys.gravity)).sum()),
            pe_contact=float((0.5 * sys.ground_k * pen[s:e] ** 2).sum()),
            p=(m[:, None] * vb).sum(axis=0),
            com=(m[:, None] * xb).sum(axis=0) / m.sum(),
            bbox_min=xb.min(axis=0), bbox_max=xb.max(axis=0),
            nonfinite=bool(~np.isfinite(xb).all() or ~np.isfinite(vb).all())))
    return out
