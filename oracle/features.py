"""Surrogate input features of a voxel robot, FP64 (test infrastructure).

32 morphology descriptors (lengths in metres; voxel centres c = (v - min + 1/2) a):
  0 log(node count), 1 log(voxel count), 2-4 extent per axis, 5-7 fraction of materials 0/1/2,
  8-10 mean voxel centre minus bbox centre, 11-16 second moments about the mean centre
  (xx, yy, zz, xy, xz, yz), 17 bottom-layer fraction, 18-25 8-bin histogram of voxel height
  (bin = min(7, floor(8 (z - zmin) / nz))), 26 actuated fraction, 27 mean log10 voxel
  stiffness, 28-30 stiffness-weighted mean centre minus mean centre, 31 fraction of voxel
  faces without a neighbouring voxel;
then (A_g cos phi_g, A_g sin phi_g) for every actuation group g.
Pinned by hand-computed values: every field of a single voxel and of a three-voxel L (two arms,
three materials, one passive voxel), in tests/test_native_features.py.
"""
from __future__ import annotations

import numpy as np


def morphology(voxels, material, group, material_k, spacing) -> np.ndarray:
    v = np.asarray(voxels, dtype=np.int64)
    mn, mx = v.min(axis=0), v.max(axis=0)
    nv = len(v)
    mat = np.zeros(nv, np.int64) if material is None else np.asarray(material, np.int64)
    grp = np.full(nv, -1) if group is None else np.asarray(group)
    corners = {(int(a + dx), int(b + dy), int(c + dz)) for a, b, c in v.tolist()
               for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)}
    ext = (mx - mn + 1).astype(float) * spacing
    ctr = ((v - mn).astype(float) + 0.5) * spacing
    com = ctr.mean(axis=0)
    d = ctr - com
    k = np.asarray(material_k, float)[mat] if material_k is not None else np.ones(nv)
    nz = mx[2] - mn[2] + 1
    hist = np.bincount(np.minimum(7, (8 * (v[:, 2] - mn[2])) // nz), minlength=8) / nv
    occupied = {tuple(x) for x in v.tolist()}
    exposed = sum((a + dx, b + dy, c + dz) not in occupied for a, b, c in v.tolist()
                  for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)))
    f = np.empty(32)
    f[0] = np.log(len(corners))
    f[1] = np.log(nv)
    f[2:5] = ext
    f[5:8] = [np.mean(mat == m) for m in range(3)]
    f[8:11] = com - 0.5 * ext
    f[11:17] = [(d[:, 0] ** 2).mean(), (d[:, 1] ** 2).mean(), (d[:, 2] ** 2).mean(),
                (d[:, 0] * d[:, 1]).mean(), (d[:, 0] * d[:, 2]).mean(), (d[:, 1] * d[:, 2]).mean()]
    f[17] = np.mean(v[:, 2] == mn[2])
    f[18:26] = hist
    f[26] = np.mean(grp >= 0)
    f[27] = np.log10(k).mean()
    f[28:31] = (k[:, None] * ctr).sum(axis=0) / k.sum() - com
    f[31] = exposed / (6.0 * nv)
    return f


def features(body, material_k, spacing, phase, amp) -> np.ndarray:
    """Full feature vector of one robot (workloads.Body) with its actuation parameters."""
    act = np.stack([np.asarray(amp) * np.cos(phase), np.asarray(amp) * np.sin(phase)], axis=1).ravel()
    return np.concatenate([morphology(body.voxels, body.material, body.group, material_k, spacing), act])
