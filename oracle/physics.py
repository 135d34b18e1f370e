"""FP64 step of the Hookean mass-spring system (test infrastructure; see package docstring).

What one time step computes, in the paper's order:

1. actuated rest lengths l0_s(t_n) = L0_s (1 + A_g sin(2 pi f t_n + phi_g)), t_n = n dt
   (springs "individually rigid, actuated, or functionally parameterized", section "Method",
   figure of a mass and its springs; volumetric actuation, section "Applications");
2. eq. (2): f_i = m_i g + f_ext_i + sum_j k_ij (|l_ij| - l0_ij) l_ij / |l_ij|, l_ij = x_j - x_i;
   Algorithm 1 applies each spring's force +F to one end and -F to the other, and every mass
   sums what it received (the algorithm's "<-" is read as "+=");
3. contact plane z = z_g (section "Generating a Lattice": planes as constraints; Appendix A:
   contact planes with friction): penetration p_i = z_g - z_i > 0 adds F_n = k_g p_i along +z;
4. velocity update v* = v + dt f / m (eqs. (3)-(4));
5. Coulomb friction on contacting masses, as a velocity clamp: c = mu F_n dt / m; the
   tangential velocity loses c of its magnitude, or stops if it is smaller than c;
6. velocity damping v' = (1 - d) v* ("simple velocity damping", Euler-Bernoulli section);
7. position update x' = x + dt v'  -- the semi-implicit (symplectic) form of eq. (4): eq. (4)
   as printed advances x with v_n, which is not energy-stable; the paper reports energy
   conservation, which the symplectic variant gives;
8. pinned (fixed) masses keep x and get v' = 0.

The Verlet integrator of eqs. (5)-(6) is ``verlet_start`` / ``verlet_step``.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class System:
    mass: np.ndarray            # (N,)
    pinned: np.ndarray          # (N,) bool
    ends: np.ndarray            # (S, 2)
    k: np.ndarray               # (S,)
    rest: np.ndarray            # (S,) nominal L0
    gidx: np.ndarray            # (S,) global actuation index body*G + g, or -1
    gravity: np.ndarray         # (3,)
    damping: float
    dt: float
    ground: bool = False
    ground_z: float = 0.0
    ground_k: float = 0.0
    ground_mu: float = 0.0
    fext: Optional[np.ndarray] = None   # (N, 3)
    phase: Optional[np.ndarray] = None  # (B*G,)
    amp: Optional[np.ndarray] = None
    freq: float = 0.0
    body_offset: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return len(self.mass)


def system_from(lat, workload, **over) -> System:
    """System for a lattice built from a workload (input order)."""
    spring_body = np.repeat(np.arange(len(lat.spring_offset) - 1), np.diff(lat.spring_offset))
    G = workload.n_groups
    gidx = np.where(lat.group >= 0, spring_body * G + lat.group, -1)
    kw = dict(mass=lat.mass.copy(), pinned=lat.pinned.copy(), ends=lat.ends.copy(), k=lat.k.copy(),
              rest=lat.rest.copy(), gidx=gidx, gravity=np.asarray(workload.gravity, float),
              damping=workload.damping, dt=workload.dt, ground=workload.ground,
              ground_z=workload.ground_z, ground_k=workload.ground_k, ground_mu=workload.ground_mu,
              phase=None if workload.phase is None else np.asarray(workload.phase, float),
              amp=None if workload.amp is None else np.asarray(workload.amp, float),
              freq=workload.freq_hz, body_offset=lat.body_offset)
    kw.update(over)
    return System(**kw)


def actuation(sys: System, t: float) -> np.ndarray:
    """alpha_g(t) = A_g sin(2 pi f t + phi_g) for every (body, group)."""
    if sys.phase is None:
        return np.zeros(0)
    return sys.amp * np.sin(2.0 * np.pi * sys.freq * t + sys.phase)


def rest_lengths(sys: System, t: float) -> np.ndarray:
    l0 = sys.rest.copy()
    act = sys.gidx >= 0
    if act.any():
        alpha = actuation(sys, t)
        l0[act] = sys.rest[act] * (1.0 + alpha[sys.gidx[act]])
    return l0


def spring_vectors(x: np.ndarray, ends: np.ndarray):
    d = x[ends[:, 1]] - x[ends[:, 0]]
    length = np.sqrt((d * d).sum(axis=1))
    return d, length


def spring_forces(x: np.ndarray, ends: np.ndarray, k: np.ndarray, l0: np.ndarray) -> np.ndarray:
    """Hooke term of eq. (2) summed per mass; F on end 0 is k (l - l0) d / l, on end 1 it is -F."""
    d, length = spring_vectors(x, ends)
    safe = np.where(length > 0, length, 1.0)
    scale = np.where(length > 0, k * (length - l0) / safe, 0.0)
    F = scale[:, None] * d
    f = np.zeros_like(x)
    np.add.at(f, ends[:, 0], F)
    np.add.at(f, ends[:, 1], -F)
    return f


def contact_normal(sys: System, x: np.ndarray) -> np.ndarray:
    """Penalty normal force magnitude k_g max(0, z_g - z) per mass."""
    if not sys.ground:
        return np.zeros(len(x))
    return sys.ground_k * np.maximum(0.0, sys.ground_z - x[:, 2])


def forces(sys: System, x: np.ndarray, t: float) -> np.ndarray:
    """Total force of eq. (2) plus the contact normal force, per mass."""
    f = spring_forces(x, sys.ends, sys.k, rest_lengths(sys, t))
    f += sys.mass[:, None] * sys.gravity[None, :]
    if sys.fext is not None:
        f += sys.fext
    f[:, 2] += contact_normal(sys, x)
    return f


def friction(sys: System, x: np.ndarray, vs: np.ndarray, h: float) -> np.ndarray:
    """Coulomb clamp of the tangential velocity of contacting masses for a kick of length h:
    it loses c = mu F_n h / m of its magnitude, or stops if it is smaller (in place)."""
    if sys.ground:
        fn = contact_normal(sys, x)
        touching = fn > 0
        if touching.any():
            c = sys.ground_mu * fn[touching] * h / sys.mass[touching]
            vt = vs[touching, :2]
            speed = np.sqrt((vt * vt).sum(axis=1))
            slide = speed > c
            scale = np.zeros_like(speed)
            scale[slide] = (speed[slide] - c[slide]) / speed[slide]
            vs[touching, :2] = vt * scale[:, None]
    return vs


def step(sys: System, x: np.ndarray, v: np.ndarray, n: int):
    """One time step from t_n = n dt; returns (x_{n+1}, v_{n+1})."""
    t = n * sys.dt
    f = forces(sys, x, t)
    vs = friction(sys, x, v + sys.dt * f / sys.mass[:, None], sys.dt)
    vn = (1.0 - sys.damping) * vs
    xn = x + sys.dt * vn
    xn[sys.pinned] = x[sys.pinned]
    vn[sys.pinned] = 0.0
    return xn, vn


# ---------------------------------------------------------------- Verlet (eqs. (5)-(6))
#
# Eq. (5) starts from (x_0, v_0): x_1 = x_0 + dt v_0 + dt^2 / (2 m) f(0, x_0); eq. (6) then
# advances x_{n+1} = 2 x_n - x_{n-1} + dt^2 / m f(t_n, x_n).  The paper does not say how
# contact friction and damping enter; they act, as in the Euler step, on the velocity of the
# interval, w = (x_{n+1} - x_n) / dt (before them: w = (x_n - x_{n-1}) / dt + dt f / m, which
# is eq. (6) itself), with a kick of dt / 2 in the first step.  Without contact and damping
# both functions reduce to eqs. (5) and (6).

def verlet_start(sys: System, x0: np.ndarray, v0: np.ndarray, n0: int = 0) -> np.ndarray:
    """Eq. (5): x_1 from (x_0, v_0) at t_{n0}."""
    h = 0.5 * sys.dt
    f = forces(sys, x0, n0 * sys.dt)
    w = friction(sys, x0, v0 + h * f / sys.mass[:, None], h)
    w = (1.0 - sys.damping) * w
    x1 = x0 + sys.dt * w
    x1[sys.pinned] = x0[sys.pinned]
    return x1


def verlet_step(sys: System, x_prev: np.ndarray, x: np.ndarray, n: int) -> np.ndarray:
    """Eq. (6): x_{n+1} from x_{n-1} and x_n at t_n = n dt."""
    f = forces(sys, x, n * sys.dt)
    if not sys.ground and sys.damping == 0.0:
        xn = 2.0 * x - x_prev + sys.dt ** 2 * f / sys.mass[:, None]
    else:
        w = friction(sys, x, (x - x_prev) / sys.dt + sys.dt * f / sys.mass[:, None], sys.dt)
        xn = x + sys.dt * (1.0 - sys.damping) * w
    xn[sys.pinned] = x[sys.pinned]
    return xn


def run_verlet(sys: System, x0: np.ndarray, v0: np.ndarray, n0: int, steps: int):
    """Positions after ``steps`` Verlet steps from (x_0, v_0) at step n0; returns (x_n, x_{n-1})."""
    x_prev, x = x0, verlet_start(sys, x0, v0, n0)
    for s in range(1, steps):
        x_prev, x = x, verlet_step(sys, x_prev, x, n0 + s)
    return (x, x_prev) if steps > 0 else (x0, x0)


def run(sys: System, x: np.ndarray, v: np.ndarray, n0: int, steps: int, every: int = 0):
    """Advance ``steps`` steps from step index n0; optionally record states every ``every``."""
    rec = []
    for s in range(steps):
        x, v = step(sys, x, v, n0 + s)
        if every and (s + 1) % every == 0:
            rec.append((n0 + s + 1, x.copy(), v.copy()))
    return (x, v, rec) if every else (x, v)
