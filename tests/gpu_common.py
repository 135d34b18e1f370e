"""Shared set-up for the GPU parity tests: the same workload built twice, once by the oracle
(FP64, test infrastructure) and once by the native library, plus the error metrics."""
import dataclasses
import sys

import numpy as np

import workloads as W
from oracle import lattice as L
from oracle import physics as P


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_problem(w):
    lat = L.build(w)
    x0 = lat.x.copy()
    if w.jitter > 0:
        for b, body in enumerate(w.bodies):
            if body.jitter_seed is not None:
                s, e = lat.body_offset[b], lat.body_offset[b + 1]
                x0[s:e] += W.node_jitter(body.jitter_seed, lat.coords[s:e], w.jitter, body=b)
    return lat, P.system_from(lat, w), x0


def as_f32(sys_: P.System) -> P.System:
    """The same system with every parameter the device holds rounded to FP32."""
    r = lambda a: None if a is None else np.asarray(a, np.float32).astype(np.float64)
    return dataclasses.replace(sys_, mass=r(sys_.mass), k=r(sys_.k), rest=r(sys_.rest), gravity=r(sys_.gravity),
                               ground_z=float(np.float32(sys_.ground_z)), ground_k=float(np.float32(sys_.ground_k)),
                               fext=r(sys_.fext))


def force_scale(sys_: P.System, x: np.ndarray, t: float) -> np.ndarray:
    """S_i = sum over springs of |k (l - l0)| + m |g| + F_n: the size of what is summed at i."""
    l0 = P.rest_lengths(sys_, t)
    _, length = P.spring_vectors(x, sys_.ends)
    mag = np.abs(sys_.k * (length - l0))
    S = np.zeros(len(x))
    np.add.at(S, sys_.ends[:, 0], mag)
    np.add.at(S, sys_.ends[:, 1], mag)
    S += sys_.mass * np.linalg.norm(sys_.gravity) + P.contact_normal(sys_, x)
    if sys_.fext is not None:
        S += np.linalg.norm(sys_.fext, axis=1)
    return S


def force_error(f_gpu, sys_, x, t):
    """max_i |f_gpu - f_ref| / S_i with the oracle fed the device's FP32 state and parameters."""
    s32 = as_f32(sys_)
    f_ref = P.forces(s32, x, t)
    S = force_scale(s32, x, t)
    err = np.linalg.norm(f_gpu - f_ref, axis=1) / np.maximum(S, 1e-300)
    return float(err.max()), float(np.abs(f_gpu - f_ref).max() / max(np.abs(f_ref).max(), 1e-300))


def position_error(x_gpu, x_ref):
    ext = float((x_ref.max(axis=0) - x_ref.min(axis=0)).max())
    return float(np.linalg.norm(x_gpu - x_ref, axis=1).max() / ext)
