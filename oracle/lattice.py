"""Voxel lattice -> masses and springs, FP64 (test infrastructure; see package docstring).

Follows section "Generating a Lattice" and its figure of the voxel cell: a voxel grid is laid
over the object; masses sit at the voxel corners; each voxel links its corners along the cube
edges, the face diagonals (duplicates merged between neighbouring voxels) and the long (body)
diagonals.  Parameter choices (mass per node, spring constant per spring) follow the same
section: uniform mass or mass lumped from material density, and spring constants either
uniform or assembled from per-voxel material stiffness.

Conventions (readings where the paper is silent):
* canonical node order: sorted by (z, y, x) of the integer corner coordinate, x fastest;
* canonical voxel order: the same, on voxel coordinates;
* springs are listed once as (i, j), i < j in canonical node order, sorted by (i, j);
* a node pair is linked iff both lie on one occupied voxel (so a concave shape has no
  spring across a gap), which for a full box gives all 26 neighbours;
* per-voxel assembly: voxel stiffness k_v adds k_v/4 to each of its 12 edges (an edge is
  shared by up to 4 voxels), k_v/2 to each of its 12 face diagonals (shared by up to 2)
  and k_v to each of its 4 body diagonals, so a uniform box interior has k = k_v;
* rest lengths are nominal: a, a*sqrt(2), a*sqrt(3);
* lumped mass: every voxel adds density*a^3/8 to each of its 8 corners;
* an actuated spring takes the group of the lowest-index actuated voxel containing it.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# corner c of a voxel has offset (c & 1, (c >> 1) & 1, (c >> 2) & 1)
CORNERS = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.int64)
# the 28 corner pairs (c1 < c2) of one voxel in loop order
PAIRS = np.array([(c1, c2) for c1 in range(8) for c2 in range(c1 + 1, 8)], dtype=np.int64)
# link type = number of differing coordinates: 1 edge, 2 face diagonal, 3 body diagonal
PAIR_TYPE = np.abs(CORNERS[PAIRS[:, 0]] - CORNERS[PAIRS[:, 1]]).sum(axis=1)
# fraction of voxel stiffness each link type receives in the per-voxel assembly
TYPE_WEIGHT = {1: 0.25, 2: 0.5, 3: 1.0}


@dataclasses.dataclass
class Lattice:
    """Masses and springs of one or more bodies, in canonical (input) order."""
    coords: np.ndarray        # (N, 3) int64 integer lattice coordinate of each node
    x: np.ndarray             # (N, 3) float64 positions
    mass: np.ndarray          # (N,) float64
    pinned: np.ndarray        # (N,) bool
    ends: np.ndarray          # (S, 2) int64, i < j, within one body
    k: np.ndarray             # (S,) float64
    rest: np.ndarray          # (S,) float64 nominal rest length
    group: np.ndarray         # (S,) int64 actuation group within its body, -1 passive
    body_offset: np.ndarray   # (B+1,) int64 node offsets
    spring_offset: np.ndarray  # (B+1,) int64 spring offsets

    @property
    def n_masses(self) -> int:
        return len(self.mass)

    @property
    def n_springs(self) -> int:
        return len(self.k)


def _canonical_order(c: np.ndarray) -> np.ndarray:
    return np.lexsort((c[:, 0], c[:, 1], c[:, 2]))


def _key(c: np.ndarray) -> np.ndarray:
    """Injective int64 key of integer coordinates in [-2^20, 2^20), ordered by (z, y, x)."""
    off = 1 << 20
    return ((c[..., 2] + off) << 42) | ((c[..., 1] + off) << 21) | (c[..., 0] + off)


def build_body(voxels, spacing, origin, mass_mode, mass_value, density, k_mode, k_uniform,
               material_k, material=None, voxel_group=None, pin_axis=-1, pin_index=0):
    """One body: returns (coords, x, mass, pinned, ends, k, rest, group)."""
    vox = np.asarray(voxels, dtype=np.int64)
    if len(vox) == 0:
        raise ValueError("empty voxel set")
    vorder = _canonical_order(vox)
    vox = vox[vorder]
    mat = None if material is None else np.asarray(material)[vorder]
    vgrp = None if voxel_group is None else np.asarray(voxel_group)[vorder]
    if np.abs(vox).max() >= (1 << 20) - 1:
        raise ValueError("voxel coordinates out of range")
    if len(np.unique(_key(vox))) != len(vox):
        raise ValueError("duplicate voxels")

    # nodes = distinct voxel corners; sorting the (z, y, x) key gives canonical order
    corner_pos = (vox[:, None, :] + CORNERS[None, :, :]).reshape(-1, 3)
    ukeys, first, corner_node = np.unique(_key(corner_pos), return_index=True, return_inverse=True)
    coords = corner_pos[first]
    corner_node = corner_node.reshape(len(vox), 8)       # (V, 8) canonical node indices

    # links of every voxel, in (voxel, pair) loop order
    li = corner_node[:, PAIRS[:, 0]]
    lj = corner_node[:, PAIRS[:, 1]]
    lo = np.minimum(li, lj).ravel()
    hi = np.maximum(li, lj).ravel()
    ltype = np.broadcast_to(PAIR_TYPE, li.shape).ravel()
    lvox = np.repeat(np.arange(len(vox)), len(PAIRS))
    key = lo * len(coords) + hi
    ukey, sidx = np.unique(key, return_inverse=True)
    ends = np.stack([ukey // len(coords), ukey % len(coords)], axis=1)
    S = len(ukey)
    stype = np.zeros(S, dtype=np.int64)
    stype[sidx] = ltype

    if k_mode == "uniform":
        k = np.full(S, float(k_uniform))
    elif k_mode == "assembly":
        kv = np.asarray(material_k, dtype=np.float64)[mat if mat is not None else np.zeros(len(vox), np.int64)]
        contrib = kv[lvox] * np.array([0.0, 0.25, 0.5, 1.0])[ltype]
        k = np.zeros(S)
        np.add.at(k, sidx, contrib)        # sequential: canonical voxel order, then pair order
    else:
        raise ValueError(k_mode)
    rest = spacing * np.sqrt(stype.astype(np.float64))

    group = np.full(S, -1, dtype=np.int64)
    if vgrp is not None:
        act = vgrp[lvox] >= 0
        # first (lowest canonical voxel index) actuated voxel of each spring
        first = np.full(S, len(vox), dtype=np.int64)
        np.minimum.at(first, sidx[act], lvox[act])
        has = first < len(vox)
        group[has] = vgrp[first[has]]

    if mass_mode == "uniform":
        mass = np.full(len(coords), float(mass_value))
    elif mass_mode == "lumped":
        m_corner = density * spacing * spacing * spacing / 8.0
        count = np.bincount(corner_node.ravel(), minlength=len(coords))
        mass = count.astype(np.float64) * m_corner
    else:
        raise ValueError(mass_mode)

    x = np.empty((len(coords), 3))
    for c in range(3):
        x[:, c] = origin[c] + spacing * coords[:, c].astype(np.float64)
    pinned = np.zeros(len(coords), dtype=bool)
    if pin_axis >= 0:
        pinned = (coords[:, pin_axis] - coords[:, pin_axis].min()) == pin_index
    return coords, x, mass, pinned, ends, k, rest, group


def build(workload) -> Lattice:
    """All bodies of a workload, concatenated (body b's nodes and springs contiguous)."""
    parts = []
    for b in workload.bodies:
        parts.append(build_body(b.voxels, workload.spacing, workload.origin, workload.mass_mode,
                                workload.mass_value, workload.density, workload.k_mode,
                                workload.k_uniform, workload.material_k, b.material, b.group,
                                workload.pin_axis, workload.pin_index))
    noff = np.cumsum([0] + [len(p[2]) for p in parts])
    soff = np.cumsum([0] + [len(p[5]) for p in parts])
    return Lattice(
        coords=np.concatenate([p[0] for p in parts]),
        x=np.concatenate([p[1] for p in parts]),
        mass=np.concatenate([p[2] for p in parts]),
        pinned=np.concatenate([p[3] for p in parts]),
        ends=np.concatenate([p[4] + noff[i] for i, p in enumerate(parts)]),
        k=np.concatenate([p[5] for p in parts]),
        rest=np.concatenate([p[6] for p in parts]),
        group=np.concatenate([p[7] for p in parts]),
        body_offset=noff.astype(np.int64), spring_offset=soff.astype(np.int64))


def spring_count_box(nx: int, ny: int, nz: int) -> int:
    """Closed-form spring count of an nx x ny x nz node box with all 26-neighbour links:
    axis links + 2 per face-diagonal cell + 4 body diagonals per cell."""
    ax = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    fd = 2 * ((nx - 1) * (ny - 1) * nz + (nx - 1) * ny * (nz - 1) + nx * (ny - 1) * (nz - 1))
    bd = 4 * (nx - 1) * (ny - 1) * (nz - 1)
    return ax + fd + bd
