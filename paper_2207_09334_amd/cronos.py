"""ctypes binding of libcronos.so: the same entry points as include/cronos.h, with NumPy
arrays marshalled to plain pointers.  Every computation happens in the native library; this
module only converts arguments, checks status codes and raises ``CronosError``.

The library is loaded from this package's directory; importing this module fails loudly if
it has not been built (``python -m paper_2207_09334_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcronos.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5
ALLOW_UNSTABLE, CHECK_LAYOUT, NO_GRAPH, FAST_DIFF, NO_TABLE, NO_SHIFT, SPLIT, VERLET, RESIDENT, WIDE_ENTRIES = (
    0x1, 0x2, 0x4, 0x8, 0x10, 0x20, 0x40, 0x80, 0x100, 0x200)
NO_GRID = 0x400
GRAPH = 0x800
DIRECT_IO, STAGED_IO = 0x1000, 0x2000
MASS_UNIFORM, MASS_LUMPED = 0, 1
K_UNIFORM, K_ASSEMBLY = 0, 1

_STATUS_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", EUNSTABLE: "EUNSTABLE",
                 ESTATE: "ESTATE"}


class CronosError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2207_09334_amd.build`")
_lib = C.CDLL(LIB_PATH)

_p = C.c_void_p
_i64, _i32, _u32, _f64 = C.c_int64, C.c_int32, C.c_uint32, C.c_double


class LatticeDesc(C.Structure):
    _fields_ = [("n_bodies", _i32), ("body_voxel_offset", _p), ("n_voxels", _i64), ("voxels", _p),
                ("material", _p), ("group", _p), ("spacing", _f64), ("origin", _f64 * 3),
                ("mass_mode", _i32), ("mass_value", _f64), ("density", _f64), ("k_mode", _i32),
                ("k_uniform", _f64), ("n_materials", _i32), ("material_k", _p), ("pin_axis", _i32),
                ("pin_index", _i32)]


class Desc(C.Structure):
    _fields_ = [("n_masses", _i64), ("n_springs", _i64), ("n_bodies", _i32), ("body_offset", _p),
                ("x0", _p), ("v0", _p), ("mass", _p), ("pinned", _p), ("grid", _p), ("fext", _p),
                ("ends", _p), ("k", _p), ("rest", _p), ("group", _p), ("n_groups", _i32),
                ("gravity", _f64 * 3), ("damping", _f64), ("dt", _f64), ("ground", _i32),
                ("ground_z", _f64), ("ground_k", _f64), ("ground_mu", _f64), ("device", _i32),
                ("stream", _p), ("flags", _u32), ("block_masses", _i32), ("batch", _i32),
                ("persistent", _i32), ("lanes_per_mass", _i32)]


class Tune(C.Structure):
    _fields_ = [("block_masses", _i32), ("batch", _i32), ("persistent", _i32), ("lanes_per_mass", _i32),
                ("us_per_step", _f64), ("us_default", _f64)]


class Diag(C.Structure):
    _fields_ = [("ke", _f64), ("pe_spring", _f64), ("pe_grav", _f64), ("pe_contact", _f64),
                ("p", _f64 * 3), ("com", _f64 * 3), ("bbox_min", _f64 * 3), ("bbox_max", _f64 * 3),
                ("mass", _f64), ("step", _i64), ("nonfinite", _i32), ("pad_", _i32)]

    def as_dict(self) -> dict:
        return {"ke": self.ke, "pe_spring": self.pe_spring, "pe_grav": self.pe_grav,
                "pe_contact": self.pe_contact, "p": np.array(self.p[:]), "com": np.array(self.com[:]),
                "bbox_min": np.array(self.bbox_min[:]), "bbox_max": np.array(self.bbox_max[:]),
                "mass": self.mass, "step": self.step, "nonfinite": bool(self.nonfinite)}


_SIGS = {
    "cronos_last_error": (C.c_char_p, []),
    "cronos_version": (C.c_char_p, []),
    "cronos_lattice_build": (C.c_int, [C.POINTER(LatticeDesc), C.POINTER(_p)]),
    "cronos_lattice_sizes": (C.c_int, [_p, C.POINTER(_i64), C.POINTER(_i64)]),
    "cronos_lattice_export": (C.c_int, [_p] + [_p] * 9),
    "cronos_lattice_destroy": (None, [_p]),
    "cronos_layout_build": (C.c_int, [_i64, _i32, _p, _p, _p, _i64, _p, _i32, C.POINTER(_p)]),
    "cronos_layout_get": (C.c_int, [_p] * 6),
    "cronos_layout_check": (C.c_int, [_p]),
    "cronos_layout_stats": (C.c_int, [_p, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i32)]),
    "cronos_layout_destroy": (None, [_p]),
    "cronos_create": (C.c_int, [C.POINTER(Desc), C.POINTER(_p)]),
    "cronos_destroy": (None, [_p]),
    "cronos_set_actuation": (C.c_int, [_p, _p, _p, _f64]),
    "cronos_step": (C.c_int, [_p, _i64]),
    "cronos_read_state": (C.c_int, [_p, _p, _p, C.POINTER(_i64)]),
    "cronos_set_state": (C.c_int, [_p, _p, _p, _i64]),
    "cronos_eval_forces": (C.c_int, [_p, _p]),
    "cronos_diagnostics": (C.c_int, [_p, C.POINTER(Diag)]),
    "cronos_natural_frequencies": (C.c_int, [_p, _i32, _i32, _f64, C.c_uint64, _p, C.POINTER(_i32),
                                             C.POINTER(_i32)]),
    "cronos_natural_frequencies_noalloc": (C.c_int, [_p, _i32, _i32, _f64, C.c_uint64, _p, C.POINTER(_i32),
                                                     C.POINTER(_i32)]),
    "cronos_tridiag_smallest": (C.c_int, [_i64, _p, _p, _i64, _p, _p]),
    "cronos_stream_bandwidth": (C.c_int, [_i32, _i64, _i32, C.POINTER(_f64), C.POINTER(_f64)]),
    "cronos_info": (C.c_int, [_p, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i32), C.POINTER(_i32),
                              C.POINTER(_i64)]),
    "cronos_get_layout": (C.c_int, [_p] * 6),
    "cronos_candidate_points": (C.c_int, [_p, _i64, _i32, _i32, C.c_uint64, _p]),
    "cronos_cutoff_springs": (C.c_int, [_i64, _p, _f64, _i64, _p, C.POINTER(_i64)]),
    "cronos_point_params": (C.c_int, [_i64, _p, _i64, _p, _f64, _f64, _f64, _i32, _f64, _p, _p, _p, _p]),
    "cronos_launch_mode": (C.c_int, [_p, C.POINTER(_i32), C.POINTER(_f64), C.POINTER(_i32)]),
    "cronos_launch_config": (C.c_int, [_p, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32),
                                       C.POINTER(_i32)]),
    "cronos_autotune": (C.c_int, [C.POINTER(Desc), _i32, C.POINTER(Tune)]),
    "cronos_rollout": (C.c_int, [_p, _i64, _i32, _p, C.POINTER(_f64)]),
    "cronos_rollout_backward": (C.c_int, [_p, _p, _p, _p, _p]),
    "cronos_features": (C.c_int, [_i32, _p, _p, _p, _p, _i32, _p, _f64, _i32, _p, _p, _p]),
    "cronos_candidate_features": (C.c_int, [_i64, _p, _i32, _p, _i32, _p, _p, _p]),
    "cronos_mlp_create": (C.c_int, [_p, _p, _i32, _i32, _p, C.POINTER(_p)]),
    "cronos_mlp_destroy": (None, [_p]),
    "cronos_mlp_get_params": (C.c_int, [_p, _p]),
    "cronos_mlp_forward": (C.c_int, [_p, _p, _i64, _p]),
    "cronos_mlp_loss_grad": (C.c_int, [_p, _p, _p, _i32, C.POINTER(_f64), _p]),
    "cronos_mlp_adam": (C.c_int, [_p, _f64, _f64, _f64, _f64]),
    "cronos_mlp_train": (C.c_int, [_p, _p, _p, _i64, _i32, _i32, _f64, _f64, C.c_uint64, C.POINTER(_f64)]),
}

for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)        # AttributeError = the library lacks a declared entry point
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_p)


def _arr(a, dtype, shape=None):
    if a is None:
        return None
    out = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None:
        out = out.reshape(shape)
    return out


def _check(st: int, allow=()):
    if st != OK and st not in allow:
        raise CronosError(st, _lib.cronos_last_error().decode())
    return st


def cronos_last_error() -> str:
    return _lib.cronos_last_error().decode()


def cronos_version() -> str:
    return _lib.cronos_version().decode()


# ------------------------------------------------------------------------------ lattice

class Lattice:
    """Result of cronos_lattice_build, exported to NumPy (input order)."""

    def __init__(self, **kw):
        self.__dict__.update(kw)

    @property
    def n_masses(self):
        return len(self.mass)

    @property
    def n_springs(self):
        return len(self.k)


def cronos_lattice_build(voxels, spacing, origin=(0.0, 0.0, 0.0), body_voxel_offset=None, material=None,
                         group=None, mass_mode=MASS_UNIFORM, mass_value=0.0, density=0.0, k_mode=K_UNIFORM,
                         k_uniform=0.0, material_k=None, pin_axis=-1, pin_index=0) -> Lattice:
    vox = _arr(voxels, np.int32, (-1, 3))
    bvo = _arr(body_voxel_offset, np.int64)
    mat = _arr(material, np.int32)
    grp = _arr(group, np.int32)
    mk = _arr(material_k, np.float64)
    d = LatticeDesc(n_bodies=1 if bvo is None else len(bvo) - 1, body_voxel_offset=_ptr(bvo),
                    n_voxels=len(vox), voxels=_ptr(vox), material=_ptr(mat), group=_ptr(grp),
                    spacing=spacing, origin=(_f64 * 3)(*origin), mass_mode=mass_mode, mass_value=mass_value,
                    density=density, k_mode=k_mode, k_uniform=k_uniform,
                    n_materials=0 if mk is None else len(mk), material_k=_ptr(mk), pin_axis=pin_axis,
                    pin_index=pin_index)
    h = _p()
    _check(_lib.cronos_lattice_build(C.byref(d), C.byref(h)))
    try:
        n, s = _i64(), _i64()
        _check(_lib.cronos_lattice_sizes(h, C.byref(n), C.byref(s)))
        n, s = n.value, s.value
        nb = d.n_bodies
        out = dict(coords=np.empty((n, 3), np.int32), x=np.empty((n, 3)), mass=np.empty(n),
                   pinned=np.empty(n, np.uint8), body_offset=np.empty(nb + 1, np.int64),
                   ends=np.empty((s, 2), np.int32), k=np.empty(s), rest=np.empty(s), group=np.empty(s, np.int16))
        _check(_lib.cronos_lattice_export(h, *[_ptr(out[f]) for f in
                                               ("coords", "x", "mass", "pinned", "body_offset", "ends", "k",
                                                "rest", "group")]))
    finally:
        _lib.cronos_lattice_destroy(h)
    return Lattice(**out)


# ------------------------------------------------------------------------------ layout

def cronos_layout_build(ends, n_masses, body_offset=None, x=None, grid=None, block_masses=0, check=False):
    """Returns dict(perm, row_ptr, col, sid, spring_perm, sell_entries, halo_entries, max_halo)."""
    e = _arr(ends, np.int32, (-1, 2))
    bo = _arr(body_offset, np.int64)
    xx = _arr(x, np.float64, (-1, 3))
    gg = _arr(grid, np.int32, (-1, 3))
    h = _p()
    _check(_lib.cronos_layout_build(n_masses, 1 if bo is None else len(bo) - 1, _ptr(bo), _ptr(xx), _ptr(gg),
                                    len(e), _ptr(e), block_masses, C.byref(h)))
    try:
        S = len(e)
        out = dict(perm=np.empty(n_masses, np.int32), row_ptr=np.empty(n_masses + 1, np.int64),
                   col=np.empty(2 * S, np.int32), sid=np.empty(2 * S, np.int32), spring_perm=np.empty(S, np.int32))
        _check(_lib.cronos_layout_get(h, *[_ptr(out[f]) for f in ("perm", "row_ptr", "col", "sid", "spring_perm")]))
        if check:
            _check(_lib.cronos_layout_check(h))
        a, b, c = _i64(), _i64(), _i32()
        _check(_lib.cronos_layout_stats(h, C.byref(a), C.byref(b), C.byref(c)))
        out.update(sell_entries=a.value, halo_entries=b.value, max_halo=c.value)
    finally:
        _lib.cronos_layout_destroy(h)
    return out


# ------------------------------------------------------------------------------ simulation

class Sim:
    """Owner of a cronos_sim handle (destroyed with the object)."""

    def __init__(self, handle, n_masses, n_springs, n_bodies, n_groups):
        self.handle = handle
        self.n_masses, self.n_springs, self.n_bodies, self.n_groups = n_masses, n_springs, n_bodies, n_groups

    def close(self):
        if self.handle:
            _lib.cronos_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cronos_create(x0, mass, ends, k, rest, *, v0=None, pinned=None, grid=None, fext=None, group=None,
                  n_groups=0, body_offset=None, gravity=(0.0, 0.0, -9.81), damping=0.0, dt=1e-4, ground=False,
                  ground_z=0.0, ground_k=0.0, ground_mu=0.0, device=0, stream=None, flags=0,
                  block_masses=0, batch=0, persistent=0, lanes_per_mass=0, _tune_steps=0):
    x0 = _arr(x0, np.float64, (-1, 3))
    n = len(x0)
    ends = _arr(ends, np.int32, (-1, 2))
    keep = dict(x0=x0, mass=_arr(mass, np.float64), ends=ends, k=_arr(k, np.float64), rest=_arr(rest, np.float64),
                v0=_arr(v0, np.float64, (-1, 3)), pinned=_arr(pinned, np.uint8), grid=_arr(grid, np.int32, (-1, 3)),
                fext=_arr(fext, np.float64, (-1, 3)), group=_arr(group, np.int16),
                body_offset=_arr(body_offset, np.int64))
    nb = 1 if keep["body_offset"] is None else len(keep["body_offset"]) - 1
    d = Desc(n_masses=n, n_springs=len(ends), n_bodies=nb, body_offset=_ptr(keep["body_offset"]),
             x0=_ptr(x0), v0=_ptr(keep["v0"]), mass=_ptr(keep["mass"]), pinned=_ptr(keep["pinned"]),
             grid=_ptr(keep["grid"]), fext=_ptr(keep["fext"]), ends=_ptr(ends), k=_ptr(keep["k"]),
             rest=_ptr(keep["rest"]), group=_ptr(keep["group"]), n_groups=n_groups,
             gravity=(_f64 * 3)(*gravity), damping=damping, dt=dt, ground=int(bool(ground)), ground_z=ground_z,
             ground_k=ground_k, ground_mu=ground_mu, device=device, stream=stream, flags=flags,
             block_masses=block_masses, batch=batch, persistent=persistent, lanes_per_mass=lanes_per_mass)
    if _tune_steps:
        t = Tune()
        _check(_lib.cronos_autotune(C.byref(d), int(_tune_steps), C.byref(t)))
        return {"block_masses": t.block_masses, "batch": t.batch, "persistent": t.persistent,
                "lanes_per_mass": t.lanes_per_mass, "us_per_step": t.us_per_step, "us_default": t.us_default}
    h = _p()
    _check(_lib.cronos_create(C.byref(d), C.byref(h)))
    return Sim(h, n, len(ends), nb, n_groups)


def cronos_autotune(x0, mass, ends, k, rest, n_steps=20, **kw) -> dict:
    """Same arguments as cronos_create; returns the tuned launch configuration (and caches it
    in the library for later creates of the same problem class)."""
    return cronos_create(x0, mass, ends, k, rest, _tune_steps=n_steps, **kw)


FORMS = ("explicit", "table", "split", "resident", "narrow", "grid")


def cronos_candidate_points(size, n_points: int, n_candidates: int = 100, k_nn: int = 4, seed: int = 0) -> np.ndarray:
    sz = _arr(size, np.float64)
    out = np.empty((int(n_points), 3))
    _check(_lib.cronos_candidate_points(_ptr(sz), int(n_points), int(n_candidates), int(k_nn), C.c_uint64(seed),
                                        _ptr(out)))
    return out


def cronos_cutoff_springs(points, cutoff: float) -> np.ndarray:
    pts = _arr(points, np.float64, (-1, 3))
    count = _i64()
    _check(_lib.cronos_cutoff_springs(len(pts), _ptr(pts), float(cutoff), 0, None, C.byref(count)))
    ends = np.empty((count.value, 2), np.int32)
    _check(_lib.cronos_cutoff_springs(len(pts), _ptr(pts), float(cutoff), len(ends), _ptr(ends), C.byref(count)))
    return ends


def cronos_point_params(points, ends, k_ref: float, length_ref: float, mass_per_point: float, pin_axis: int = -1,
                        pin_below: float = 0.0) -> tuple:
    """Returns (k [S], rest [S], mass [N], pinned [N] uint8) of a point lattice."""
    pts = _arr(points, np.float64, (-1, 3))
    e = _arr(ends, np.int32, (-1, 2))
    k, rest = np.empty(len(e)), np.empty(len(e))
    mass, pinned = np.empty(len(pts)), np.empty(len(pts), np.uint8)
    _check(_lib.cronos_point_params(len(pts), _ptr(pts), len(e), _ptr(e), float(k_ref), float(length_ref),
                                    float(mass_per_point), int(pin_axis), float(pin_below), _ptr(k), _ptr(rest),
                                    _ptr(mass), _ptr(pinned)))
    return k, rest, mass, pinned


def cronos_launch_config(sim: Sim) -> dict:
    b, bt, pg, fm, ln = _i32(), _i32(), _i32(), _i32(), _i32()
    _check(_lib.cronos_launch_config(sim.handle, C.byref(b), C.byref(bt), C.byref(pg), C.byref(fm), C.byref(ln)))
    return {"block_masses": b.value, "batch": bt.value, "persistent_groups": pg.value, "step_form": FORMS[fm.value],
            "lanes_per_mass": ln.value}


def cronos_launch_mode(sim: Sim) -> dict:
    """{"hip_graph": whether step calls launch HIP graphs, "plain_step_us": step time with
    plain launches measured at creation, "staged_io": whether the one-lane general forms pass
    velocities and the new state through LDS in mass order}."""
    g, t, io = _i32(), _f64(0.0), _i32()
    _check(_lib.cronos_launch_mode(sim.handle, C.byref(g), C.byref(t), C.byref(io)))
    return {"hip_graph": bool(g.value), "plain_step_us": t.value, "staged_io": bool(io.value)}


def cronos_destroy(sim: Sim):
    sim.close()


def cronos_set_actuation(sim: Sim, phase, amp, freq_hz: float):
    ph, am = _arr(phase, np.float64), _arr(amp, np.float64)
    if len(ph) != sim.n_bodies * sim.n_groups or len(am) != len(ph):
        raise CronosError(EINVAL, "phase/amp must have n_bodies * n_groups entries")
    _check(_lib.cronos_set_actuation(sim.handle, _ptr(ph), _ptr(am), freq_hz))


def cronos_step(sim: Sim, n_steps: int):
    _check(_lib.cronos_step(sim.handle, int(n_steps)))


def cronos_read_state(sim: Sim, want_x=True, want_v=True):
    x = np.empty((sim.n_masses, 3)) if want_x else None
    v = np.empty((sim.n_masses, 3)) if want_v else None
    step = _i64()
    _check(_lib.cronos_read_state(sim.handle, _ptr(x), _ptr(v), C.byref(step)))
    return x, v, step.value


def cronos_set_state(sim: Sim, x=None, v=None, step: int = 0):
    xx, vv = _arr(x, np.float64, (-1, 3)), _arr(v, np.float64, (-1, 3))
    for a in (xx, vv):
        if a is not None and len(a) != sim.n_masses:
            raise CronosError(EINVAL, "state arrays must have n_masses rows")
    _check(_lib.cronos_set_state(sim.handle, _ptr(xx), _ptr(vv), int(step)))


def cronos_eval_forces(sim: Sim) -> np.ndarray:
    f = np.empty((sim.n_masses, 3))
    _check(_lib.cronos_eval_forces(sim.handle, _ptr(f)))
    return f


def cronos_natural_frequencies(sim: Sim, n_modes: int = 2, max_iter: int = 200_000, tol: float = 1e-9,
                               seed: int = 1) -> tuple:
    """Lowest distinct angular frequencies (rad/s) of the system linearised about its current
    positions; returns (omega[:n_found], iterations)."""
    omega = np.zeros(n_modes)
    found, iters = _i32(0), _i32(0)
    _check(_lib.cronos_natural_frequencies(sim.handle, n_modes, max_iter, tol, seed, _ptr(omega), C.byref(found),
                                           C.byref(iters)))
    return omega[:found.value].copy(), iters.value


def cronos_natural_frequencies_noalloc(sim: Sim, n_modes: int = 2, max_iter: int = 200_000, tol: float = 1e-9,
                                       seed: int = 1) -> tuple:
    """cronos_natural_frequencies on the library's fixed device workspace (no device
    allocation); returns (omega[:n_found], iterations)."""
    omega = np.zeros(n_modes)
    found, iters = _i32(0), _i32(0)
    _check(_lib.cronos_natural_frequencies_noalloc(sim.handle, n_modes, max_iter, tol, seed, _ptr(omega),
                                                   C.byref(found), C.byref(iters)))
    return omega[:found.value].copy(), iters.value


def cronos_stream_bandwidth(bytes_: int = 2 << 30, reps: int = 5, device: int = 0) -> tuple:
    """(copy GB/s, read GB/s) of the library's plain streaming kernels over `bytes_`."""
    c, r = _f64(0.0), _f64(0.0)
    _check(_lib.cronos_stream_bandwidth(device, int(bytes_), int(reps), C.byref(c), C.byref(r)))
    return c.value, r.value


def cronos_tridiag_smallest(a, b, count: int) -> tuple:
    """Smallest `count` eigenvalues of the symmetric tridiagonal matrix (diagonal a,
    off-diagonal b) and |last entry| of their unit eigenvectors."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    theta, last = np.empty(count), np.empty(count)
    _check(_lib.cronos_tridiag_smallest(len(a), _ptr(a), _ptr(b) if len(b) else None, count, _ptr(theta),
                                        _ptr(last)))
    return theta, last


def cronos_diagnostics(sim: Sim, allow_nonfinite=False) -> list:
    out = (Diag * sim.n_bodies)()
    _check(_lib.cronos_diagnostics(sim.handle, out), allow=(ESTATE,) if allow_nonfinite else ())
    return [o.as_dict() for o in out]


def cronos_info(sim: Sim) -> dict:
    n, s, st = _i64(), _i64(), _i64()
    nb, blk = _i32(), _i32()
    _check(_lib.cronos_info(sim.handle, C.byref(n), C.byref(s), C.byref(nb), C.byref(blk), C.byref(st)))
    return dict(n_masses=n.value, n_springs=s.value, n_bodies=nb.value, block_masses=blk.value, step=st.value)


def cronos_get_layout(sim: Sim) -> dict:
    S = sim.n_springs
    out = dict(perm=np.empty(sim.n_masses, np.int32), row_ptr=np.empty(sim.n_masses + 1, np.int64),
               col=np.empty(2 * S, np.int32), sid=np.empty(2 * S, np.int32), spring_perm=np.empty(S, np.int32))
    _check(_lib.cronos_get_layout(sim.handle, *[_ptr(out[f]) for f in ("perm", "row_ptr", "col", "sid",
                                                                       "spring_perm")]))
    return out


def cronos_rollout(sim: Sim, n_steps: int, ckpt_every: int, loss_w) -> float:
    lw = _arr(loss_w, np.float64, (-1, 3))
    if len(lw) != sim.n_masses:
        raise CronosError(EINVAL, "loss_w must have n_masses rows")
    out = _f64()
    _check(_lib.cronos_rollout(sim.handle, int(n_steps), int(ckpt_every), _ptr(lw), C.byref(out)))
    return out.value


def cronos_rollout_backward(sim: Sim, want_state=False):
    """Returns (dphase, damp) or, with want_state, (dphase, damp, dx0, dv0)."""
    G = sim.n_bodies * sim.n_groups
    dp, da = np.zeros(G), np.zeros(G)
    dx = np.empty((sim.n_masses, 3)) if want_state else None
    dv = np.empty((sim.n_masses, 3)) if want_state else None
    _check(_lib.cronos_rollout_backward(sim.handle, _ptr(dp), _ptr(da), _ptr(dx), _ptr(dv)))
    return (dp, da, dx, dv) if want_state else (dp, da)


# ------------------------------------------------------------------------------ surrogate

def cronos_features(bodies, material_k, spacing, n_groups, phase, amp) -> np.ndarray:
    """bodies: sequence of objects with .voxels, .material, .group (workloads.Body)."""
    vox = _arr(np.concatenate([b.voxels for b in bodies]), np.int32, (-1, 3))
    off = _arr(np.cumsum([0] + [len(b.voxels) for b in bodies]), np.int64)
    mat = grp = None
    if any(b.material is not None for b in bodies):
        mat = _arr(np.concatenate([b.material if b.material is not None else np.zeros(len(b.voxels))
                                   for b in bodies]), np.int32)
    if any(b.group is not None for b in bodies):
        grp = _arr(np.concatenate([b.group if b.group is not None else np.full(len(b.voxels), -1)
                                   for b in bodies]), np.int32)
    mk = _arr(material_k, np.float64)
    ph, am = _arr(phase, np.float64), _arr(amp, np.float64)
    out = np.empty((len(bodies), 32 + 2 * n_groups))
    _check(_lib.cronos_features(len(bodies), _ptr(off), _ptr(vox), _ptr(mat), _ptr(grp),
                                0 if mk is None else len(mk), _ptr(mk), spacing, n_groups, _ptr(ph), _ptr(am),
                                _ptr(out)))
    return out


def cronos_candidate_features(body_of, morph, n_groups, phase, amp) -> np.ndarray:
    bo = _arr(body_of, np.int32)
    mo = _arr(morph, np.float64, (-1, 32))
    ph, am = _arr(phase, np.float64), _arr(amp, np.float64)
    out = np.empty((len(bo), 32 + 2 * n_groups))
    _check(_lib.cronos_candidate_features(len(bo), _ptr(bo), len(mo), _ptr(mo), n_groups, _ptr(ph), _ptr(am),
                                          _ptr(out)))
    return out


class MLP:
    def __init__(self, handle, sizes):
        self.handle, self.sizes = handle, tuple(sizes)

    def close(self):
        if self.handle:
            _lib.cronos_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_params(self):
        s = self.sizes
        return sum(s[l] * s[l + 1] + s[l + 1] for l in range(4))


def _flat(params) -> np.ndarray:
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in params])


def _unflat(flat, sizes):
    out, o = [], 0
    for l in range(4):
        fi, fo = sizes[l], sizes[l + 1]
        out.append(flat[o:o + fi * fo].reshape(fi, fo))
        o += fi * fo
        out.append(flat[o:o + fo].copy())
        o += fo
    return out


def cronos_mlp_create(params, sizes=(96, 256, 256, 256, 3), max_rows=4096, device=0, stream=None) -> MLP:
    sz = _arr(sizes, np.int32)
    fl = _flat(params)
    h = _p()
    _check(_lib.cronos_mlp_create(_ptr(sz), _ptr(fl), int(max_rows), device, stream, C.byref(h)))
    return MLP(h, sizes)


def cronos_mlp_get_params(mlp: MLP) -> list:
    fl = np.empty(mlp.n_params)
    _check(_lib.cronos_mlp_get_params(mlp.handle, _ptr(fl)))
    return _unflat(fl, mlp.sizes)


def cronos_mlp_forward(mlp: MLP, x) -> np.ndarray:
    xx = _arr(x, np.float32, (-1, mlp.sizes[0]))
    y = np.empty((len(xx), mlp.sizes[4]), np.float32)
    _check(_lib.cronos_mlp_forward(mlp.handle, _ptr(xx), len(xx), _ptr(y)))
    return y


def cronos_mlp_loss_grad(mlp: MLP, x, t):
    xx = _arr(x, np.float32, (-1, mlp.sizes[0]))
    tt = _arr(t, np.float32, (-1, mlp.sizes[4]))
    loss = _f64()
    g = np.empty(mlp.n_params)
    _check(_lib.cronos_mlp_loss_grad(mlp.handle, _ptr(xx), _ptr(tt), len(xx), C.byref(loss), _ptr(g)))
    return loss.value, _unflat(g, mlp.sizes)


def cronos_mlp_adam(mlp: MLP, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(_lib.cronos_mlp_adam(mlp.handle, lr, beta1, beta2, eps))


def cronos_mlp_train(mlp: MLP, x, t, batch=1024, epochs=1, lr=1e-3, seed=4, lr_final=None) -> float:
    xx = _arr(x, np.float32, (-1, mlp.sizes[0]))
    tt = _arr(t, np.float32, (-1, mlp.sizes[4]))
    out = _f64()
    _check(_lib.cronos_mlp_train(mlp.handle, _ptr(xx), _ptr(tt), len(xx), int(batch), int(epochs), float(lr),
                                 float(lr if lr_final is None else lr_final), C.c_uint64(seed), C.byref(out)))
    return out.value
