"""Best-candidate lattices, brute force, FP64 (test infrastructure; see package docstring).

Section "Generating a Lattice", second method: a quasi-uniform point set is grown one vertex at
a time; the first vertex is random, and each following vertex is the best of 100 random
candidates, best meaning the one whose distances to its k nearest already-placed vertices are
largest (here: the largest sum of those k distances, summed in ascending order; ties go to the
lowest candidate index), until the requested number of vertices is placed.  Springs join every
pair of vertices no farther apart than a cutoff distance.

The random candidates come from ``workloads.uniform01(seed, 8, p, c, axis)`` (the counter hash
of the input generators), scaled by the box size.
"""
from __future__ import annotations

import numpy as np

import workloads as W

S_CANDIDATE = W.S_CANDIDATE


def best_candidate_points(size, n_points: int, n_candidates: int = 100, k_nn: int = 4, seed: int = 0) -> np.ndarray:
    size = np.asarray(size, float)
    pts = np.empty((n_points, 3))
    pts[0] = size * W.uniform01(seed, S_CANDIDATE, 0, 0, np.arange(3))
    c = np.arange(n_candidates)[:, None]
    a = np.arange(3)[None, :]
    for p in range(1, n_points):
        cand = size[None, :] * W.uniform01(seed, S_CANDIDATE, p, c, a)          # (C, 3)
        d = cand[:, None, :] - pts[None, :p, :]                                  # (C, p, 3)
        dist = np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2])
        k = min(k_nn, p)
        near = np.sort(dist, axis=1)[:, :k]
        score = near[:, 0].copy()
        for j in range(1, k):                                                    # ascending order
            score = score + near[:, j]
        pts[p] = cand[int(np.argmax(score))]
    return pts


def cutoff_springs(points: np.ndarray, cutoff: float) -> np.ndarray:
    """All pairs i < j with |p_i - p_j|^2 <= cutoff^2, sorted by (i, j)."""
    d = points[:, None, :] - points[None, :, :]
    d2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]
    i, j = np.nonzero(np.triu(d2 <= cutoff * cutoff, k=1))
    return np.stack([i, j], axis=1)


def system(pw, points: np.ndarray, ends: np.ndarray):
    """The oracle System of a best-candidate lattice: rest length = initial length,
    k = k_ref * length_ref / length, uniform mass, points with x < pin_x fixed."""
    from . import physics as P
    d = points[ends[:, 1]] - points[ends[:, 0]]
    rest = np.sqrt((d * d).sum(axis=1))
    return P.System(mass=np.full(len(points), pw.mass), pinned=points[:, 0] < pw.pin_x, ends=np.asarray(ends, np.int64),
                    k=pw.k_ref * pw.length_ref / rest, rest=rest, gidx=np.full(len(ends), -1),
                    gravity=np.asarray(pw.gravity, float), damping=pw.damping, dt=pw.dt, ground=pw.ground,
                    ground_z=pw.ground_z, ground_k=pw.ground_k, ground_mu=pw.ground_mu)
