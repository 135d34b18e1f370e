"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test pins one part of the oracle against something other than itself: closed forms,
hand-derived counts (tests/golden), brute force on tiny inputs, invariants, and the
Euler-Bernoulli / natural-frequency validations of the paper's Results section.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import diagnostics as D
from oracle import lattice as L
from oracle import layout as LY
from oracle import physics as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _wl(voxels, **kw):
    base = W.cube_drop().__dict__.copy()
    base.update(bodies=[W.Body(np.asarray(voxels))], jitter=0.0)
    base.update(kw)
    return W.Workload(**base)


def _read_table(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


SHAPES = {
    "box_2x2x2": W.box_voxels(1, 1, 1),
    "box_3x3x3": W.box_voxels(2, 2, 2),
    "box_4x3x5": W.box_voxels(3, 2, 4),
    "box_10x10x10": W.box_voxels(9, 9, 9),
    "pair_face": np.array([[0, 0, 0], [1, 0, 0]]),
    "pair_edge": np.array([[0, 0, 0], [1, 0, 1]]),
}


# ---------------------------------------------------------------- P1: lattice counts

@pytest.mark.parametrize("row", _read_table("lattice_counts.txt"), ids=lambda r: r[0])
def test_lattice_counts_golden(row):
    name, nodes, springs, maxdeg = row[0], int(row[1]), int(row[2]), int(row[3])
    lat = L.build(_wl(SHAPES[name]))
    assert lat.n_masses == nodes
    assert lat.n_springs == springs
    deg = np.bincount(lat.ends.ravel(), minlength=lat.n_masses)
    assert deg.max() == maxdeg
    assert deg.max() <= 26


@pytest.mark.parametrize("n", [(2, 2, 2), (3, 4, 2), (5, 3, 4), (10, 10, 10), (7, 2, 3)])
def test_spring_count_closed_form(n):
    lat = L.build(_wl(W.box_voxels_for_nodes(*n)))
    assert lat.n_masses == n[0] * n[1] * n[2]
    assert lat.n_springs == L.spring_count_box(*n)


def _brute_force(vox, a, k_v_of_voxel):
    """O(V * N^2) definition: two nodes are linked iff some occupied voxel has both as
    corners; k = sum over such voxels of k_v * (1/4 edge, 1/2 face diagonal, 1 long)."""
    vox = [tuple(v) for v in vox]
    nodes = sorted({(v[0] + dx, v[1] + dy, v[2] + dz) for v in vox
                    for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)},
                   key=lambda c: (c[2], c[1], c[0]))
    springs = {}
    for i in range(len(nodes)):
        for j in range(i + 1, len(nodes)):
            p, q = nodes[i], nodes[j]
            diff = [abs(p[c] - q[c]) for c in range(3)]
            if max(diff) != 1:
                continue
            kk = 0.0
            for vi, v in enumerate(vox):
                inside = all(v[c] <= p[c] <= v[c] + 1 and v[c] <= q[c] <= v[c] + 1 for c in range(3))
                if inside:
                    kk += k_v_of_voxel[vi] * {1: 0.25, 2: 0.5, 3: 1.0}[sum(diff)]
            if kk > 0:
                springs[(i, j)] = (kk, a * math.sqrt(sum(diff)))
    return nodes, springs


def test_lattice_brute_force_concave_multimaterial():
    rng = np.random.default_rng(5)
    # an irregular concave voxel set (random subset of a 4x3x3 box)
    vox = W.box_voxels(4, 3, 3)
    vox = vox[rng.random(len(vox)) < 0.55]
    mat = rng.integers(0, 3, len(vox))
    kvals = (1.0e3, 1.0e4, 1.0e5)
    lat = L.build(_wl(vox, k_mode="assembly", material_k=kvals,
                      bodies=[W.Body(vox, mat.astype(np.int32))]))
    nodes, springs = _brute_force(vox, 0.01, [kvals[m] for m in mat])
    assert [tuple(c) for c in lat.coords] == nodes
    got = {(int(i), int(j)): (k, r) for (i, j), k, r in zip(lat.ends, lat.k, lat.rest)}
    assert set(got) == set(springs)
    for key, (k, r) in springs.items():
        assert got[key][0] == pytest.approx(k, rel=1e-15)
        assert got[key][1] == pytest.approx(r, rel=1e-15)


def test_lumped_mass_and_total():
    w = W.cantilever(6, 3, 4)
    lat = L.build(w)
    vox = w.bodies[0].voxels
    total = len(vox) * 1000.0 * 0.005 ** 3
    assert lat.mass.sum() == pytest.approx(total, rel=1e-13)
    # a corner node of the box touches exactly one voxel
    corner = np.all(lat.coords == 0, axis=1)
    assert lat.mass[corner][0] == pytest.approx(1000.0 * 0.005 ** 3 / 8, rel=1e-15)
    assert lat.pinned.sum() == 3 * 4


def test_actuation_group_lowest_voxel():
    # two voxels sharing a face, in different groups: shared springs take the lower voxel's group
    vox = np.array([[0, 0, 0], [1, 0, 0]])
    lat = L.build(_wl(vox, bodies=[W.Body(vox, None, np.array([5, 7]))]))
    shared = np.all(lat.coords[lat.ends][:, :, 0] == 1, axis=1)
    assert (lat.group[shared] == 5).all()
    right = np.all(lat.coords[lat.ends][:, :, 0] >= 1, axis=1) & ~shared
    assert (lat.group[right] == 7).all()
    lat2 = L.build(_wl(vox, bodies=[W.Body(vox, None, np.array([-1, 7]))]))
    assert (lat2.group[shared] == 7).all()
    left_only = np.any(lat2.coords[lat2.ends][:, :, 0] == 0, axis=1)
    assert (lat2.group[left_only] == -1).all()


def test_quadruped_and_cube_sizes():
    assert L.build(W.cube_drop()).n_springs == 10476
    lat = L.build(W.quadruped())
    assert (lat.n_masses, lat.n_springs) == (12711, 145550)


# ---------------------------------------------------------------- P11: Morton / CSR

def test_morton_golden():
    rows = np.array(_read_table("morton_small.txt"), dtype=np.uint64)
    keys = LY.morton_key(rows[:, :3])
    assert (keys == rows[:, 3]).all()


def test_csr_invariants_and_locality():
    w = W.cube_drop(6)
    lat = L.build(w)
    lay = LY.reorder(lat.ends, lat.body_offset, coords=lat.coords)
    N, S = lat.n_masses, lat.n_springs
    assert sorted(lay.perm) == list(range(N))
    assert lay.row_ptr[-1] == 2 * S
    assert (np.bincount(lay.sid, minlength=S) == 2).all()
    rows = np.repeat(np.arange(N), np.diff(lay.row_ptr))
    pairs = set(zip(rows.tolist(), lay.col.tolist()))
    assert all((c, r) in pairs for r, c in pairs)                     # symmetric
    for i in range(N):
        seg = lay.col[lay.row_ptr[i]:lay.row_ptr[i + 1]]
        assert (np.diff(seg) > 0).all()
    # spring s of the new order joins its two incidences
    assert (lay.ends[lay.sid, 0] == np.minimum(rows, lay.col)).all()
    # renumbered springs are the input springs
    old = {tuple(sorted(e)) for e in lat.ends.tolist()}
    new = {tuple(sorted((int(lay.perm[a]), int(lay.perm[b])))) for a, b in lay.ends}
    assert old == new
    # Morton keys are non-decreasing along the new order
    keys = LY.morton_key(lat.coords[lay.perm] - lat.coords.min(axis=0))
    assert (np.diff(keys.astype(np.float64)) >= 0).all()


def test_morton_8cube_blocks():
    # an 8x8x8 node box in Morton order: consecutive 64-runs are 4x4x4 sub-cubes
    lat = L.build(_wl(W.box_voxels_for_nodes(8, 8, 8)))
    lay = LY.reorder(lat.ends, lat.body_offset, coords=lat.coords)
    c = lat.coords[lay.perm]
    for b in range(0, 512, 64):
        blk = c[b:b + 64]
        assert (blk.max(axis=0) - blk.min(axis=0) == 3).all()


def test_quantised_morton_matches_grid_order_for_unjittered_box():
    lat = L.build(_wl(W.box_voxels_for_nodes(8, 8, 8)))
    a = LY.reorder(lat.ends, lat.body_offset, coords=lat.coords)
    b = LY.reorder(lat.ends, lat.body_offset, x=lat.x)
    assert (a.perm == b.perm).all()


# ---------------------------------------------------------------- force model pins

def _energy(x, sys, l0):
    _, length = P.spring_vectors(x, sys.ends)
    return 0.5 * (sys.k * (length - l0) ** 2).sum()


def test_spring_force_is_minus_energy_gradient():
    w = W.cube_drop(3)
    lat = L.build(w)
    rng = np.random.default_rng(1)
    x = lat.x + rng.uniform(-1e-3, 1e-3, lat.x.shape)
    sys = P.system_from(lat, w)
    f = P.spring_forces(x, sys.ends, sys.k, sys.rest)
    h = 1e-7
    for i in range(lat.n_masses):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            g = (_energy(xp, sys, sys.rest) - _energy(xm, sys, sys.rest)) / (2 * h)
            assert f[i, c] == pytest.approx(-g, rel=1e-5, abs=1e-6)


def test_newton_third_law_sum_zero():
    w = W.cube_drop(5)
    lat = L.build(w)
    rng = np.random.default_rng(2)
    x = lat.x + rng.uniform(-1e-3, 1e-3, lat.x.shape)
    f = P.spring_forces(x, lat.ends, lat.k, lat.rest)
    scale = np.abs(f).max()
    assert np.abs(f.sum(axis=0)).max() <= 1e-12 * scale * lat.n_masses


def test_homogeneous_strain_interior_zero_and_plane_force():
    """Uniform axial strain eps of a per-voxel-assembled box: interior nodes carry no net
    force, and the force transmitted across a mid plane is C11 eps a^2 per voxel with
    C11 = 13 k_v / (3 a) (Cauchy-Born of the 26-neighbour cell)."""
    nx, ny, nz, a, kv = 9, 5, 6, 0.01, 1234.5
    w = _wl(W.box_voxels_for_nodes(nx, ny, nz), k_mode="assembly", material_k=(kv,), spacing=a,
            origin=(0.0, 0.0, 0.0))
    lat = L.build(w)
    eps = 1e-7
    x = lat.x.copy()
    x[:, 0] *= (1.0 + eps)
    f = P.spring_forces(x, lat.ends, lat.k, lat.rest)
    c = lat.coords
    interior = ((c > 0) & (c < np.array([nx - 1, ny - 1, nz - 1]))).all(axis=1)
    expected_plane = 13.0 / 3.0 * kv * a * eps * (ny - 1) * (nz - 1)
    assert np.abs(f[interior]).max() < 1e-6 * expected_plane
    right = c[:, 0] >= nx // 2
    assert -f[right, 0].sum() == pytest.approx(expected_plane, rel=1e-5)
    assert abs(f[right, 1].sum()) < 1e-6 * expected_plane


# ---------------------------------------------------------------- P2 / P3 / P4 / P5 dynamics

def _two_mass(k=50.0, m=0.2, l0=0.1, u0=1e-3, dt=1e-3, anchored=False):
    x = np.array([[0.0, 0.0, 0.0], [l0 + u0, 0.0, 0.0]])
    sys = P.System(mass=np.array([m, m]), pinned=np.array([anchored, False]),
                   ends=np.array([[0, 1]]), k=np.array([k]), rest=np.array([l0]),
                   gidx=np.array([-1]), gravity=np.zeros(3), damping=0.0, dt=dt)
    return sys, x, np.zeros_like(x)


@pytest.mark.parametrize("anchored", [False, True])
def test_two_mass_exact_discrete_trajectory(anchored):
    """Linear 1-D oscillator under symplectic Euler: u_{n+1} - 2u_n + u_{n-1} = -w^2 dt^2 u_n,
    so u_n = u0 cos(n th) + D sin(n th) with cos th = 1 - w^2 dt^2 / 2; w^2 = 2k/m for two free
    masses (relative coordinate), k/m for one mass against an anchor."""
    k, m, l0, u0, dt = 50.0, 0.2, 0.1, 1e-3, 1e-3
    sys, x, v = _two_mass(k, m, l0, u0, dt, anchored)
    w2 = (k / m) if anchored else (2 * k / m)
    th = math.acos(1 - w2 * dt * dt / 2)
    u1 = u0 * (1 - w2 * dt * dt)
    Dc = (u1 - u0 * math.cos(th)) / math.sin(th)
    for n in range(1, 3001):
        x, v = P.step(sys, x, v, n - 1)
        u = x[1, 0] - x[0, 0] - l0
        exact = u0 * math.cos(n * th) + Dc * math.sin(n * th)
        assert abs(u - exact) <= 1e-11 * u0 + 1e-15
    # the discrete frequency tends to sqrt(k/m) (anchored) / sqrt(2k/m) as dt -> 0
    assert th / dt == pytest.approx(math.sqrt(w2), rel=w2 * dt * dt / 20)


def test_free_fall_with_damping_closed_form():
    g, d, dt = -9.81, 0.01, 1e-4
    sys = P.System(mass=np.array([0.3]), pinned=np.array([False]), ends=np.zeros((0, 2), np.int64),
                   k=np.zeros(0), rest=np.zeros(0), gidx=np.zeros(0, np.int64),
                   gravity=np.array([0, 0, g]), damping=d, dt=dt)
    x, v = np.array([[0.0, 0.0, 1.0]]), np.array([[0.5, 0.0, 0.0]])
    vz, z = 0.0, 1.0
    for n in range(1, 2001):
        x, v = P.step(sys, x, v, n - 1)
        r = (1 - d) ** n
        vz_exact = g * dt * (1 - d) * (1 - r) / d
        vz = (1 - d) * (vz + dt * g)
        z += dt * vz
        assert v[0, 2] == pytest.approx(vz_exact, rel=1e-12)
        assert v[0, 0] == pytest.approx(0.5 * r, rel=1e-12)
    # position: sum of the closed-form velocities
    n = np.arange(1, 2001)
    vz_all = g * dt * (1 - d) * (1 - (1 - d) ** n) / d
    assert x[0, 2] == pytest.approx(1.0 + dt * vz_all.sum(), rel=1e-12)


def test_momentum_decay_no_gravity_no_ground():
    w = W.cube_drop(5)
    lat = L.build(w)
    rng = np.random.default_rng(3)
    x = lat.x + rng.uniform(-1e-4, 1e-4, lat.x.shape)
    v = rng.normal(0, 0.01, lat.x.shape)
    sys = P.system_from(lat, w, gravity=np.zeros(3), ground=False, damping=0.003)
    p0 = (sys.mass[:, None] * v).sum(axis=0)
    for n in range(200):
        x, v = P.step(sys, x, v, n)
    p = (sys.mass[:, None] * v).sum(axis=0)
    np.testing.assert_allclose(p, p0 * (1 - 0.003) ** 200, rtol=1e-10, atol=1e-14)


def test_one_dof_modified_energy_exact():
    """Symplectic Euler (v first, then x) on x'' = -w^2 x conserves
    H~ = v^2 + w^2 x^2 - dt w^2 x v exactly."""
    k, m, l0, u0, dt = 50.0, 0.2, 0.1, 1e-3, 2e-3
    sys, x, v = _two_mass(k, m, l0, u0, dt, anchored=True)
    w2 = k / m

    def H(x, v):
        u, vv = x[1, 0] - l0, v[1, 0]
        return vv * vv + w2 * u * u - dt * w2 * u * vv

    h0 = H(x, v)
    for n in range(2000):
        x, v = P.step(sys, x, v, n)
        assert H(x, v) == pytest.approx(h0, rel=1e-10)


def _energy_series(dt, steps, every):
    w = W.cube_drop(4)
    lat = L.build(w)
    rng = np.random.default_rng(4)
    x = lat.x + rng.uniform(-2e-4, 2e-4, lat.x.shape)
    v = np.zeros_like(x)
    sys = P.system_from(lat, w, ground=False, damping=0.0, gravity=np.zeros(3), dt=dt)
    E = []
    for n in range(steps):
        if n % every == 0:
            E.append(D.diagnostics(sys, x, v, n * dt)[0].total)
        x, v = P.step(sys, x, v, n)
    return np.array(E)


def test_lattice_energy_bounded_first_order_no_drift():
    """With damping and contact off, symplectic Euler keeps the energy within an O(dt) band
    (halving dt halves the band) and shows no secular drift (section "Energy Conservation
    Tests": constant total energy once damping is released)."""
    E1 = _energy_series(2e-5, 4000, 10)
    E2 = _energy_series(1e-5, 8000, 20)
    band1, band2 = np.ptp(E1), np.ptp(E2)
    assert band1 < 0.2 * E1.mean()
    assert 0.35 < band2 / band1 < 0.65
    third = len(E1) // 3
    drift = abs(E1[-third:].mean() - E1[:third].mean())
    assert drift < 0.1 * band1


# ---------------------------------------------------------------- P6 contact + friction

def _one_mass(z, vx=0.0, fx=0.0, m=0.1, kg=1e5, mu=0.8, dt=1e-4, d=0.0):
    sys = P.System(mass=np.array([m]), pinned=np.array([False]), ends=np.zeros((0, 2), np.int64),
                   k=np.zeros(0), rest=np.zeros(0), gidx=np.zeros(0, np.int64),
                   gravity=np.array([0, 0, -9.81]), damping=d, dt=dt, ground=True, ground_z=0.0,
                   ground_k=kg, ground_mu=mu,
                   fext=np.array([[fx, 0.0, 0.0]]))
    return sys, np.array([[0.0, 0.0, z]]), np.array([[vx, 0.0, 0.0]])


def test_contact_rest_penetration():
    m, kg = 0.1, 1e5
    sys, x, v = _one_mass(0.0, m=m, kg=kg, d=0.01)
    for n in range(5000):
        x, v = P.step(sys, x, v, n)
    assert -x[0, 2] == pytest.approx(m * 9.81 / kg, rel=1e-6)


def test_sliding_deceleration_and_stop():
    m, kg, mu, dt, v0 = 0.1, 1e5, 0.5, 1e-4, 0.2
    p_eq = m * 9.81 / kg
    sys, x, v = _one_mass(-p_eq, vx=v0, m=m, kg=kg, mu=mu, dt=dt)
    for n in range(100):
        x, v = P.step(sys, x, v, n)
    # at equilibrium penetration F_n = m g, so the speed drops by mu g dt per step
    assert v[0, 0] == pytest.approx(v0 - 100 * mu * 9.81 * dt, rel=1e-6)
    t_stop = v0 / (mu * 9.81)
    for n in range(100, int(1.2 * t_stop / dt)):
        x, v = P.step(sys, x, v, n)
    assert v[0, 0] == 0.0
    # distance: dt * sum of the positive post-update speeds v0 - n mu g dt, which tends to
    # v0^2 / (2 mu g) as dt -> 0
    speeds = v0 - np.arange(1, 100000) * mu * 9.81 * dt
    expected = dt * speeds[speeds > 0].sum()
    assert x[0, 0] == pytest.approx(expected, rel=1e-9)
    assert expected == pytest.approx(v0 * v0 / (2 * mu * 9.81), rel=5e-3)


def test_static_friction_holds_below_mu_mg():
    m, mu = 0.1, 0.8
    p_eq = m * 9.81 / 1e5
    sys, x, v = _one_mass(-p_eq, fx=0.9 * mu * m * 9.81, m=m, mu=mu)
    for n in range(2000):
        x, v = P.step(sys, x, v, n)
    assert x[0, 0] == 0.0
    sys2, x2, v2 = _one_mass(-p_eq, fx=1.2 * mu * m * 9.81, m=m, mu=mu)
    for n in range(2000):
        x2, v2 = P.step(sys2, x2, v2, n)
    assert x2[0, 0] > 0.0


# ---------------------------------------------------------------- actuation

def test_actuated_rest_length_formula_and_period():
    w = W.quadruped()
    lat = L.build(w)
    sys = P.system_from(lat, w)
    act = np.nonzero(sys.gidx >= 0)[0][:50]
    for t in (0.0, 0.1234, 0.5):
        l0 = P.rest_lengths(sys, t)
        for s in act:
            g = sys.gidx[s]
            assert l0[s] == pytest.approx(sys.rest[s] * (1 + 0.2 * math.sin(4 * math.pi * t + w.phase[g])),
                                          rel=1e-15)
    # 2 Hz: period 0.5 s
    np.testing.assert_allclose(P.rest_lengths(sys, 0.1), P.rest_lengths(sys, 0.6), rtol=1e-12)
    passive = sys.gidx < 0
    assert (P.rest_lengths(sys, 0.3)[passive] == sys.rest[passive]).all()


# ---------------------------------------------------------------- Verlet (eqs. (5)-(6))

@pytest.mark.parametrize("anchored", [False, True])
def test_verlet_two_mass_exact_discrete_trajectory(anchored):
    """Eq. (6) on the linear 1-D oscillator is u_{n+1} = (2 - w^2 dt^2) u_n - u_{n-1}, and eq. (5)
    from rest gives u_1 = u0 (1 - w^2 dt^2 / 2) = u0 cos th: so u_n = u0 cos(n th) exactly,
    cos th = 1 - w^2 dt^2 / 2 (Chebyshev recurrence)."""
    k, m, l0, u0, dt = 50.0, 0.2, 0.1, 1e-3, 1e-3
    sys, x0, v0 = _two_mass(k, m, l0, u0, dt, anchored)
    w2 = (k / m) if anchored else (2 * k / m)
    th = math.acos(1 - w2 * dt * dt / 2)
    x_prev, x = x0, P.verlet_start(sys, x0, v0)
    for n in range(1, 3001):
        # the position form carries u in coordinates of ~0.1 m: rounding of 2 x_n - x_{n-1}
        # accumulates to ~1e-14 over the run
        u = x[1, 0] - x[0, 0] - l0
        assert abs(u - u0 * math.cos(n * th)) <= 1e-10 * u0
        x_prev, x = x, P.verlet_step(sys, x_prev, x, n)


def test_verlet_free_fall_is_exact():
    """Constant acceleration: eqs. (5)-(6) reproduce x0 + v0 t + g t^2 / 2 at every step."""
    g, dt = np.array([0.0, 0.0, -9.81]), 1e-3
    sys = P.System(mass=np.array([0.3]), pinned=np.array([False]), ends=np.zeros((0, 2), np.int64),
                   k=np.zeros(0), rest=np.zeros(0), gidx=np.zeros(0, np.int64), gravity=g, damping=0.0, dt=dt)
    x0, v0 = np.array([[0.1, -0.2, 1.0]]), np.array([[0.5, 0.25, 3.0]])
    x, x_prev = P.run_verlet(sys, x0, v0, 0, 1000)
    # rounding of 2 x_n - x_{n-1} acts as a velocity error, so it grows like n^2 ulp (~1e-10)
    t = 1000 * dt
    np.testing.assert_allclose(x, x0 + v0 * t + 0.5 * g * t * t, rtol=0, atol=1e-9)
    t = 999 * dt
    np.testing.assert_allclose(x_prev, x0 + v0 * t + 0.5 * g * t * t, rtol=0, atol=1e-9)


def test_verlet_is_symplectic_euler_with_a_half_kick():
    """Without contact and damping, eq. (6) is the symplectic Euler recurrence for the
    positions; they coincide when Euler starts from v0 - dt/2 f(x0)/m (the first half kick of
    eq. (5)).  Jittered cube with gravity, 300 steps."""
    w = W.cube_drop(4)
    lat = L.build(w)
    sys = P.system_from(lat, w, ground=False, damping=0.0)
    rng = np.random.default_rng(11)
    x0 = lat.x + rng.uniform(-2e-4, 2e-4, lat.x.shape)
    v0 = rng.normal(0.0, 0.01, lat.x.shape)
    xv, _ = P.run_verlet(sys, x0, v0, 0, 300)
    ve = v0 - 0.5 * sys.dt * P.forces(sys, x0, 0.0) / sys.mass[:, None]
    xe, _ = P.run(sys, x0, ve, 0, 300)
    np.testing.assert_allclose(xv, xe, rtol=0, atol=1e-12)


def test_verlet_contact_and_damping_reading():
    """With the contact plane and damping the Verlet step acts on the interval velocity
    w = (x_{n+1} - x_n)/dt exactly as the Euler step acts on v (kick dt/2 in the first step):
    a mass resting on the plane settles at the same penetration m g / k_g, and one sliding at
    the equilibrium penetration loses mu g dt of speed per step."""
    m, kg, mu, dt = 0.1, 1e5, 0.5, 1e-4
    sys, x, v = _one_mass(0.0, m=m, kg=kg, d=0.01)
    x, _ = P.run_verlet(sys, x, v, 0, 5000)
    assert -x[0, 2] == pytest.approx(m * 9.81 / kg, rel=1e-6)
    p_eq = m * 9.81 / kg
    sys, x0, v0 = _one_mass(-p_eq, vx=0.2, m=m, kg=kg, mu=mu, dt=dt)
    x_prev, x = x0, P.verlet_start(sys, x0, v0)
    assert (x[0, 0] - x0[0, 0]) / dt == pytest.approx(0.2 - 0.5 * mu * 9.81 * dt, rel=1e-9)
    for n in range(1, 101):
        x_prev, x = x, P.verlet_step(sys, x_prev, x, n)
    assert (x[0, 0] - x_prev[0, 0]) / dt == pytest.approx(0.2 - 100.5 * mu * 9.81 * dt, rel=1e-6)
