"""Seeded synthetic inputs shared by the oracle-side tests and the HIP-side tests/bench.

This module holds no arithmetic of the simulation method itself: it produces voxel
occupancy sets, per-voxel material and actuation-group labels, random jitter draws,
actuation phases/amplitudes and the physical constants of each workload.  Turning
voxels into masses and springs, reordering, forces and integration are done separately
by the oracle (``oracle/``) and by the native library, which never import each other.

Randomness comes from a counter-based hash built on SplitMix64 (Steele, Lea & Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): every draw is a pure
function of (seed, stream, key...), so any consumer can regenerate the same value
independent of iteration order.

Workload shapes follow the paper's test objects: a voxelised cube dropped on a
frictional contact plane, a fixed-end cantilever beam (section "Euler-Bernoulli Beam
Tests"), a multi-material soft-legged quadruped (section "Applications of the
Simulation Method"), a batched population of random robots and the surrogate's
training set.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Optional

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)

# stream identifiers of the counter hash
S_JITTER = 1
S_MATERIAL = 2
S_PHASE = 3
S_AMP = 4
S_WALK = 5
S_SIZE = 6
S_STATE = 7
S_CANDIDATE = 8


def _splitmix64(x):
    """SplitMix64 output function applied to uint64 array(s) (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = (np.asarray(x, dtype=np.uint64) + _GAMMA)
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
        return z ^ (z >> np.uint64(31))


def _as_u64(k):
    a = np.asarray(k)
    if a.dtype.kind == "i":
        return a.astype(np.int64).view(np.uint64) if a.ndim else np.uint64(np.int64(a).view(np.uint64))
    return a.astype(np.uint64)


def hash_u64(seed: int, stream: int, *keys) -> np.ndarray:
    """h(seed, stream, k0, k1, ...) -> uint64, chaining SplitMix64 over each key (broadcasting)."""
    z = _splitmix64(np.uint64(seed))
    z = _splitmix64(z ^ np.uint64(stream))
    for k in keys:
        z = _splitmix64(z ^ _as_u64(k))
    return z


def uniform01(seed: int, stream: int, *keys) -> np.ndarray:
    """Uniform double in [0, 1) from the top 53 bits of the hash."""
    return (hash_u64(seed, stream, *keys) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ----------------------------------------------------------------------------------------
# voxel shapes
# ----------------------------------------------------------------------------------------

def box_voxels(nx: int, ny: int, nz: int, x0: int = 0, y0: int = 0, z0: int = 0) -> np.ndarray:
    """All voxels of an nx x ny x nz voxel box, as int64 (n, 3) [vx, vy, vz], x fastest."""
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel() + x0, y.ravel() + y0, z.ravel() + z0], axis=1).astype(np.int64)


def box_voxels_for_nodes(nx_nodes: int, ny_nodes: int, nz_nodes: int) -> np.ndarray:
    """Voxels whose corners form an nx x ny x nz node lattice."""
    return box_voxels(nx_nodes - 1, ny_nodes - 1, nz_nodes - 1)


QUADRUPED_GROUPS = 16


def quadruped_voxels() -> tuple[np.ndarray, np.ndarray]:
    """Soft-legged quadruped: a 40x20x10 voxel body on four 8x8x10 legs.

    Body voxels x in [0,40), y in [0,20), z in [10,20); legs x in [0,8) or [32,40),
    y in [0,8) or [12,20), z in [0,10).  Returns (voxels, region_group) where
    region_group is the actuation group a voxel would drive if actuated: legs give
    4 legs x {z < 5, z >= 5} = groups 0..7, the body gives 2 (y halves) x 4 (x quarters)
    = groups 8..15.
    """
    body = box_voxels(40, 20, 10, 0, 0, 10)
    legs = [box_voxels(8, 8, 10, lx, ly, 0) for lx in (0, 32) for ly in (0, 12)]
    vox = np.concatenate([body] + legs, axis=0)
    grp = np.empty(len(vox), dtype=np.int64)
    nb = len(body)
    bx, by = body[:, 0], body[:, 1]
    grp[:nb] = 8 + (by // 10) * 4 + (bx // 10)
    off = nb
    for leg_id, leg in enumerate(legs):
        grp[off:off + len(leg)] = leg_id * 2 + (leg[:, 2] >= 5)
        off += len(leg)
    return vox, grp


def _corner_offsets() -> np.ndarray:
    return np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=np.int64)


def _pack(p: np.ndarray) -> np.ndarray:
    off = np.int64(1 << 20)
    return ((p[..., 0] + off) | ((p[..., 1] + off) << np.int64(21)) | ((p[..., 2] + off) << np.int64(42)))


def random_walk_voxels(seed: int, robot: int, target_nodes: int) -> np.ndarray:
    """Voxel shape grown by a seeded random walk on the cubic grid.

    The walk starts at (0,0,0) and moves to a uniformly chosen face neighbour each step;
    each voxel is added when first visited, until the shape's corner count reaches
    ``target_nodes``.  Returned voxels are in order of first visit, shifted so that the
    minimum coordinate on each axis is 0.
    """
    dirs = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                    dtype=np.int64)
    corners = _corner_offsets()
    n_steps = max(64, 4 * target_nodes)
    while True:
        if n_steps >= (1 << 20):
            raise ValueError("random walk too long")
        step_idx = np.arange(n_steps, dtype=np.int64)
        d = (hash_u64(seed, S_WALK, robot, step_idx) % np.uint64(6)).astype(np.int64)
        pos = np.concatenate([np.zeros((1, 3), np.int64), np.cumsum(dirs[d], axis=0)], axis=0)
        _, first = np.unique(_pack(pos), return_index=True)
        vox = pos[np.sort(first)]                          # distinct voxels in visit order
        # corner count after the first v voxels
        ckey = _pack(vox[:, None, :] + corners[None, :, :]).ravel()
        cvox = np.repeat(np.arange(len(vox), dtype=np.int64), 8)
        ukey, cinv = np.unique(ckey, return_inverse=True)
        cfirst = np.full(len(ukey), len(vox), dtype=np.int64)
        np.minimum.at(cfirst, cinv.ravel(), cvox)
        count = np.cumsum(np.bincount(cfirst, minlength=len(vox) + 1)[:len(vox)])
        hit = np.nonzero(count >= target_nodes)[0]
        if len(hit):
            vox = vox[: hit[0] + 1]
            return vox - vox.min(axis=0)
        n_steps *= 2


# ----------------------------------------------------------------------------------------
# per-voxel labels and per-node draws
# ----------------------------------------------------------------------------------------

def voxel_materials(seed: int, voxels: np.ndarray, n_materials: int = 3, body: int = 0) -> np.ndarray:
    """I.i.d. uniform material index per voxel, keyed by (body, voxel coordinates)."""
    v = np.asarray(voxels, dtype=np.int64)
    h = hash_u64(seed, S_MATERIAL, body, v[:, 0], v[:, 1], v[:, 2])
    return (h % np.uint64(n_materials)).astype(np.int32)


def node_jitter(seed: int, node_coords: np.ndarray, amplitude: float, body: int = 0) -> np.ndarray:
    """Uniform jitter in [-amplitude, amplitude) per node and component, keyed by the node's
    integer lattice coordinates (so it does not depend on any node numbering)."""
    c = np.asarray(node_coords, dtype=np.int64)
    comp = np.arange(3, dtype=np.int64)[None, :]
    u = uniform01(seed, S_JITTER, body, c[:, 0:1], c[:, 1:2], c[:, 2:3], comp)
    return amplitude * (2.0 * u - 1.0)


def group_phases(seed: int, n_groups: int, body: int = 0) -> np.ndarray:
    return 2.0 * math.pi * uniform01(seed, S_PHASE, body, np.arange(n_groups))


def group_amplitudes(seed: int, n_groups: int, lo: float, hi: float, body: int = 0) -> np.ndarray:
    return lo + (hi - lo) * uniform01(seed, S_AMP, body, np.arange(n_groups))


# ----------------------------------------------------------------------------------------
# workload descriptions
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class Body:
    """One voxel body: its voxels plus per-voxel material and actuation group (-1 = passive)."""
    voxels: np.ndarray
    material: Optional[np.ndarray] = None
    group: Optional[np.ndarray] = None
    jitter_seed: Optional[int] = None


@dataclasses.dataclass
class Workload:
    name: str
    bodies: list
    spacing: float
    origin: tuple
    mass_mode: str               # "uniform": mass_value per node; "lumped": density*a^3/8 per voxel corner
    mass_value: float
    density: float
    k_mode: str                  # "uniform": k_uniform per spring; "assembly": per-voxel material stiffness
    k_uniform: float
    material_k: tuple
    jitter: float
    pin_axis: int                # -1: none; else nodes with lattice index pin_index on that axis are fixed
    pin_index: int
    gravity: tuple
    damping: float
    dt: float
    ground: bool
    ground_z: float
    ground_k: float
    ground_mu: float
    steps: int
    n_groups: int = 0
    freq_hz: float = 0.0
    phase: Optional[np.ndarray] = None   # [n_bodies * n_groups]
    amp: Optional[np.ndarray] = None


def cube_drop(n: int = 10, seed: int = 0) -> Workload:
    """Cube drop: n^3 nodes, 1 g each, 1 cm spacing, uniform k = 1e4 N/m, released 5 cm
    above a frictional plane; positions jittered by up to 1e-4 m."""
    return Workload(
        name=f"cube_drop_{n}x{n}x{n}", bodies=[Body(box_voxels_for_nodes(n, n, n), jitter_seed=seed)],
        spacing=0.01, origin=(0.0, 0.0, 0.05), mass_mode="uniform", mass_value=0.001,
        density=0.0, k_mode="uniform", k_uniform=1.0e4, material_k=(), jitter=1.0e-4,
        pin_axis=-1, pin_index=0, gravity=(0.0, 0.0, -9.81), damping=0.01, dt=1.0e-4,
        ground=True, ground_z=0.0, ground_k=1.0e5, ground_mu=0.8, steps=10_000)


def cantilever(nx: int = 400, ny: int = 40, nz: int = 40, gravity: float = 9.81,
               youngs: float = 1.0e6, spacing: float = 0.005) -> Workload:
    """Cantilever beam of nx x ny x nz nodes, end face x = 0 fixed, gravity on, no ground.

    Springs take per-voxel stiffness k_v = E a / 2.7, the value for which the lattice's
    [100] Young's modulus equals E."""
    k_v = youngs * spacing / 2.7
    return Workload(
        name=f"cantilever_{nx}x{ny}x{nz}", bodies=[Body(box_voxels_for_nodes(nx, ny, nz))],
        spacing=spacing, origin=(0.0, 0.0, 0.0), mass_mode="lumped", mass_value=0.0,
        density=1000.0, k_mode="assembly", k_uniform=0.0, material_k=(k_v,), jitter=0.0,
        pin_axis=0, pin_index=0, gravity=(0.0, 0.0, -gravity), damping=0.0, dt=5.0e-5,
        ground=False, ground_z=0.0, ground_k=0.0, ground_mu=0.0, steps=100_000)


MATERIAL_K = (1.0e3, 1.0e4, 1.0e5)


def quadruped(seed: int = 2) -> Workload:
    """Actuated multi-material quadruped: 3 materials per voxel, materials 0 and 1 actuated
    in 16 phase groups with rest length L0 (1 + A_g sin(2 pi 2Hz t + phi_g)), A_g = 0.2."""
    vox, region = quadruped_voxels()
    mat = voxel_materials(seed, vox)
    grp = np.where(mat < 2, region, -1).astype(np.int32)
    G = QUADRUPED_GROUPS
    return Workload(
        name="quadruped_40x20x10_legs4", bodies=[Body(vox, mat, grp)],
        spacing=0.01, origin=(0.0, 0.0, 0.0), mass_mode="uniform", mass_value=0.1,
        density=0.0, k_mode="assembly", k_uniform=0.0, material_k=MATERIAL_K, jitter=0.0,
        pin_axis=-1, pin_index=0, gravity=(0.0, 0.0, -9.81), damping=1.0e-4, dt=1.0e-4,
        ground=True, ground_z=0.0, ground_k=1.0e5, ground_mu=0.8, steps=2000,
        n_groups=G, freq_hz=2.0, phase=group_phases(seed, G), amp=np.full(G, 0.2))


POP_GROUPS = 32


def population_robot(seed: int, robot: int, lo: int = 500, hi: int = 50_000) -> Body:
    """One random-walk robot: log-uniform node target in [lo, hi], 3 materials, 32 actuation
    groups = 32 contiguous chunks of the walk's visit order (materials 0/1 actuated)."""
    u = float(uniform01(seed, S_SIZE, robot))
    target = int(round(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))
    vox = random_walk_voxels(seed, robot, target)
    mat = voxel_materials(seed, vox, body=robot)
    chunk = (np.arange(len(vox)) * POP_GROUPS) // len(vox)
    grp = np.where(mat < 2, chunk, -1).astype(np.int32)
    return Body(vox, mat, grp)


def _robots(args):
    seed, first, count, lo, hi = args
    return [population_robot(seed, first + r, lo, hi) for r in range(count)]


def population(n_robots: int = 1024, seed: int = 3, lo: int = 500, hi: int = 50_000,
               first_robot: int = 0, workers: Optional[int] = None) -> Workload:
    """Population of independent random-walk robots.  Robots are generated in parallel
    processes (spawned, so no state of the caller is inherited) when there are many."""
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if n_robots >= 64 else 1
    if workers > 1:
        import concurrent.futures as cf
        import multiprocessing as mp
        per = (n_robots + workers - 1) // workers
        jobs = [(seed, first_robot + k, min(per, n_robots - k), lo, hi) for k in range(0, n_robots, per)]
        with cf.ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
            bodies = [b for part in ex.map(_robots, jobs) for b in part]
    else:
        bodies = _robots((seed, first_robot, n_robots, lo, hi))
    G = POP_GROUPS
    ph = np.concatenate([group_phases(seed, G, body=first_robot + r) for r in range(n_robots)])
    am = np.concatenate([group_amplitudes(seed, G, 0.0, 0.25, body=first_robot + r)
                         for r in range(n_robots)])
    return Workload(
        name=f"population_{n_robots}", bodies=bodies, spacing=0.01, origin=(0.0, 0.0, 0.0),
        mass_mode="uniform", mass_value=0.1, density=0.0, k_mode="assembly", k_uniform=0.0,
        material_k=MATERIAL_K, jitter=0.0, pin_axis=-1, pin_index=0,
        gravity=(0.0, 0.0, -9.81), damping=1.0e-4, dt=1.0e-4, ground=True, ground_z=0.0,
        ground_k=1.0e5, ground_mu=0.8, steps=5000, n_groups=G, freq_hz=2.0, phase=ph, amp=am)


# ----------------------------------------------------------------------------------------
# surrogate network inputs
# ----------------------------------------------------------------------------------------

S_MLP = 8
MLP_SIZES = (96, 256, 256, 256, 3)


def mlp_init(seed: int = 4, sizes=MLP_SIZES) -> list:
    """Initial weights [W1, b1, ..., W4, b4]: W_l uniform in +-sqrt(6 / (fan_in + fan_out))
    (Glorot & Bengio 2010), keyed by (layer, row, column); biases zero."""
    params = []
    for l in range(len(sizes) - 1):
        fi, fo = sizes[l], sizes[l + 1]
        lim = math.sqrt(6.0 / (fi + fo))
        r = np.arange(fi)[:, None]
        c = np.arange(fo)[None, :]
        params.append(lim * (2.0 * uniform01(seed, S_MLP, l, r, c) - 1.0))
        params.append(np.zeros(fo))
    return params


def population_actuation(seed: int, n_robots: int, n_groups: int = 32, draw: int = 0, first_robot: int = 0):
    """Phases in [0, 2 pi) and amplitudes in [0, 0.25] for every (robot, group); `draw` selects
    an independent set for the same robots (training rollouts re-use morphologies)."""
    r = np.arange(first_robot, first_robot + n_robots)[:, None]
    g = np.arange(n_groups)[None, :]
    ph = 2.0 * math.pi * uniform01(seed, S_PHASE, draw, r, g)
    am = 0.25 * uniform01(seed, S_AMP, draw, r, g)
    return ph.ravel(), am.ravel()


# ----------------------------------------------------------------------------------------
# best-candidate point lattices (section "Generating a Lattice", second method)
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class PointWorkload:
    """A quasi-uniform lattice grown by best-candidate sampling in a box: the sampling
    parameters (candidate coordinates are uniform01(seed, S_CANDIDATE, point, candidate, axis)
    times the box size), the spring cutoff, and the physical constants.  Springs get
    k = k_ref * length_ref / length (the paper's default spring constant, scaled inversely to
    the spring's length) and rest length = initial length; every point has the same mass."""
    name: str
    size: tuple
    n_points: int
    n_candidates: int
    k_nn: int
    seed: int
    cutoff: float
    k_ref: float
    length_ref: float
    mass: float
    pin_x: float            # points with x < pin_x are fixed (the x = 0 end of the bar)
    gravity: tuple
    damping: float
    dt: float
    ground: bool = False
    ground_z: float = 0.0
    ground_k: float = 0.0
    ground_mu: float = 0.0
    steps: int = 1000


def candidate_bar(n_points: int = 200_000, size=(0.4, 0.04, 0.04), seed: int = 5) -> PointWorkload:
    """A bar of best-candidate points (100 candidates, nearest-neighbour criterion), springs up
    to 1.6 mean spacings, 0.1 kg per point, k = 1e4 N/m at the mean spacing, fixed at x = 0,
    sagging under gravity."""
    spacing = (size[0] * size[1] * size[2] / n_points) ** (1.0 / 3.0)
    return PointWorkload(name=f"candidate_bar_{n_points}", size=tuple(size), n_points=n_points, n_candidates=100,
                         k_nn=1, seed=seed, cutoff=1.6 * spacing, k_ref=1.0e4, length_ref=spacing, mass=0.1,
                         pin_x=0.75 * spacing, gravity=(0.0, 0.0, -9.81), damping=0.0, dt=1.0e-4)
