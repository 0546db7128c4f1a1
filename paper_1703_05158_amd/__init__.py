"""Python binding of liblbm (the gfx950 D3Q19 moving-boundary LBM step).

Argument marshalling only: every computation runs in the HIP library behind
the C ABI declared in ``include/lbm.h``.  The module-level functions carry
the C names (``lbm_create``, ``lbm_set_bodies``, ``lbm_step`` ...); host
arrays are numpy arrays (converted to contiguous float64/uint8), device
arrays are torch CUDA tensors or raw integer addresses, streams are
``torch.cuda.Stream.cuda_stream`` handles or integers.

Importing the package fails loudly if ``liblbm.so`` has not been built
(``python __graft_entry__.py build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

__all__ = [
    "LBMError", "LBMConfig", "LBMInfo", "config", "Lattice", "Batch", "TILE_SHAPES", "SphereDrag",
    "lbm_version", "lbm_create", "lbm_destroy", "lbm_last_error", "lbm_set_stream",
    "lbm_set_walls", "lbm_set_bodies", "lbm_set_bodies_device", "lbm_init_fields",
    "lbm_step", "lbm_step_noalloc", "lbm_get_forces", "lbm_get_forces_device", "lbm_get_populations",
    "lbm_set_populations", "lbm_get_macro", "lbm_get_owner", "lbm_get_state",
    "lbm_set_state", "lbm_get_info", "lbm_count_fluid", "lbm_profile", "lbm_profile_read",
    "lbm_profile_read_parts", "lbm_set_step_path", "lbm_get_step_path",
    "STORAGE", "BB_MODE", "STEP_PATH", "PROF_PARTS", "LIB_PATH",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbm.so")

STATUS = {0: "LBM_OK", 1: "LBM_ERR_ARG", 2: "LBM_ERR_OOM", 3: "LBM_ERR_HIP",
          4: "LBM_ERR_STATE", 5: "LBM_ERR_UNSTABLE", 6: "LBM_ERR_CAPACITY"}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
BB_MODE = {"bouzidi": 0, "halfway": 1}
STEP_PATH = {"fused": 0, "split": 1}
PROF_PARTS = ("geometry", "links", "step", "whole")


class LBMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class LBMConfig(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("storage", ct.c_int32), ("tau0", ct.c_double), ("smag_c", ct.c_double),
                ("rho0", ct.c_double), ("body_force", ct.c_double * 3),
                ("bb_mode", ct.c_int32), ("max_bodies", ct.c_int32), ("max_walls", ct.c_int32),
                ("nan_guard_every", ct.c_int32), ("stream", ct.c_void_p)]


class LBMInfo(ct.Structure):
    _fields_ = [("n_nodes", ct.c_int64), ("n_bodies", ct.c_int32),
                ("n_walls", ct.c_int32), ("storage_bytes", ct.c_int32),
                ("steps_done", ct.c_int32), ("device_bytes", ct.c_int64)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python __graft_entry__.py build` "
                      "(there is no non-HIP fallback)")
_L = ct.CDLL(LIB_PATH)

_H = ct.c_void_p
_dp = ct.POINTER(ct.c_double)
_sig = {
    "lbm_version": (ct.c_int32, []),
    "lbm_create": (ct.c_int, [ct.POINTER(LBMConfig), ct.POINTER(_H)]),
    "lbm_destroy": (None, [_H]),
    "lbm_last_error": (ct.c_char_p, [_H]),
    "lbm_set_stream": (ct.c_int, [_H, ct.c_void_p]),
    "lbm_set_walls": (ct.c_int, [_H, ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p]),
    "lbm_set_bodies": (ct.c_int, [_H, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "lbm_set_bodies_device": (ct.c_int, [_H, ct.c_int32, ct.c_void_p]),
    "lbm_init_fields": (ct.c_int, [_H, ct.c_void_p, ct.c_void_p]),
    "lbm_step": (ct.c_int, [_H, ct.c_int32]),
    "lbm_step_noalloc": (ct.c_int, [_H, ct.c_int32]),
    "lbm_get_forces": (ct.c_int, [_H, ct.c_void_p, ct.c_void_p]),
    "lbm_get_forces_device": (ct.c_int, [_H, ct.c_void_p]),
    "lbm_get_populations": (ct.c_int, [_H, ct.c_void_p]),
    "lbm_set_populations": (ct.c_int, [_H, ct.c_void_p]),
    "lbm_get_macro": (ct.c_int, [_H, ct.c_void_p, ct.c_void_p]),
    "lbm_get_owner": (ct.c_int, [_H, ct.c_void_p]),
    "lbm_get_state": (ct.c_int, [_H, ct.c_void_p, ct.POINTER(ct.c_size_t)]),
    "lbm_set_state": (ct.c_int, [_H, ct.c_void_p, ct.c_size_t]),
    "lbm_get_info": (ct.c_int, [_H, ct.POINTER(LBMInfo)]),
    "lbm_count_fluid": (ct.c_int, [_H, ct.POINTER(ct.c_int64)]),
    "lbm_profile": (ct.c_int, [_H, ct.c_int32]),
    "lbm_profile_read": (ct.c_int, [_H, _dp, ct.POINTER(ct.c_int64)]),
    "lbm_profile_read_parts": (ct.c_int, [_H, _dp, ct.POINTER(ct.c_int64)]),
    "lbm_set_step_path": (ct.c_int, [_H, ct.c_int32]),
    "lbm_get_step_path": (ct.c_int, [_H, ct.POINTER(ct.c_int32)]),
    "lbm_set_zieb": (ct.c_int, [_H, ct.c_int32, ct.c_double, ct.c_double, ct.c_double]),
    "lbm_get_zieb": (ct.c_int, [_H, _dp]),
    "lbm_set_body_force": (ct.c_int, [_H, ct.c_void_p]),
    "lbm_drag_gradient": (ct.c_int, [_H, ct.c_int32, ct.c_int32, _dp, ct.c_void_p, ct.c_void_p]),
    "lbm_set_tile": (ct.c_int, [_H, ct.c_int32]),
    "lbm_get_tile": (ct.c_int, [_H, ct.POINTER(ct.c_int32)]),
    "lbm_autotune_tile": (ct.c_int, [_H, ct.c_int32, ct.c_char_p, ct.POINTER(ct.c_int32), _dp]),
    "lbm_batch_create": (ct.c_int, [ct.POINTER(_H), ct.c_int32, ct.c_void_p, ct.POINTER(_H)]),
    "lbm_batch_step": (ct.c_int, [_H, ct.c_int32]),
    "lbm_batch_last_error": (ct.c_char_p, [_H]),
    "lbm_batch_destroy": (None, [_H]),
    "lbm_batch_set_tile": (ct.c_int, [_H, ct.c_int32]),
    "lbm_batch_get_tile": (ct.c_int, [_H, ct.POINTER(ct.c_int32)]),
    "lbm_batch_autotune": (ct.c_int, [_H, ct.c_int32, ct.POINTER(ct.c_int32), _dp]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_L, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sig)


def _check(h, st):
    if st != 0:
        msg = _L.lbm_last_error(h)
        raise LBMError(st, msg.decode() if msg else "")


def _host(a, dtype, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _dev_ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return ct.c_void_p(t)
    return ct.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ct.c_void_p(stream)
    return ct.c_void_p(stream.cuda_stream)


# ---- C functions, same names -------------------------------------------------

def lbm_version() -> int:
    return _L.lbm_version()


def config(nx, ny, nz, tau0, smag_c, rho0=1.0, body_force=(0.0, 0.0, 0.0), storage="f32",
           bb_mode="bouzidi", max_bodies=0, max_walls=0, nan_guard_every=0, stream=None) -> LBMConfig:
    c = LBMConfig()
    c.nx, c.ny, c.nz = int(nx), int(ny), int(nz)
    c.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.tau0, c.smag_c, c.rho0 = float(tau0), float(smag_c), float(rho0)
    c.body_force[:] = [float(v) for v in body_force]
    c.bb_mode = BB_MODE[bb_mode] if isinstance(bb_mode, str) else int(bb_mode)
    c.max_bodies, c.max_walls = int(max_bodies), int(max_walls)
    c.nan_guard_every = int(nan_guard_every)
    c.stream = _stream_ptr(stream)
    return c


def lbm_create(cfg: LBMConfig) -> int:
    h = _H()
    st = _L.lbm_create(ct.byref(cfg), ct.byref(h))
    if st != 0:
        raise LBMError(st, "lbm_create rejected the configuration or could not allocate")
    return h.value


def lbm_destroy(h) -> None:
    _L.lbm_destroy(h)


def lbm_last_error(h) -> str:
    r = _L.lbm_last_error(h)
    return r.decode() if r else ""


def lbm_set_stream(h, stream) -> None:
    _check(h, _L.lbm_set_stream(h, _stream_ptr(stream)))


def lbm_set_walls(h, wall_id, wall_vel, wall_ref=None) -> None:
    w = _host(wall_id, np.uint8)
    v = _host(wall_vel, np.float64).reshape(-1, 3) if wall_vel is not None else np.zeros((0, 3))
    r = _host(wall_ref, np.float64).reshape(-1, 3) if wall_ref is not None else None
    _check(h, _L.lbm_set_walls(h, _ptr(w), len(v), _ptr(v) if len(v) else None, _ptr(r)))


def lbm_set_bodies(h, X, V, Omega, R) -> None:
    R = _host(R, np.float64).reshape(-1)
    n = len(R)
    X, V, Om = (_host(a, np.float64, 3 * n) for a in (X, V, Omega))
    _check(h, _L.lbm_set_bodies(h, n, _ptr(X), _ptr(V), _ptr(Om), _ptr(R)))


def lbm_set_bodies_device(h, n, d_table) -> None:
    _check(h, _L.lbm_set_bodies_device(h, int(n), _dev_ptr(d_table)))


def lbm_init_fields(h, rho=None, u=None) -> None:
    r = _host(rho, np.float64) if rho is not None else None
    v = _host(u, np.float64) if u is not None else None
    _check(h, _L.lbm_init_fields(h, _ptr(r), _ptr(v)))


def lbm_step(h, nsteps=1) -> None:
    _check(h, _L.lbm_step(h, int(nsteps)))


def lbm_step_noalloc(h, nsteps=1) -> None:
    _check(h, _L.lbm_step_noalloc(h, int(nsteps)))


def lbm_get_info(h) -> dict:
    info = LBMInfo()
    _check(h, _L.lbm_get_info(h, ct.byref(info)))
    return {k: getattr(info, k) for k, _ in LBMInfo._fields_}


def lbm_count_fluid(h) -> int:
    n = ct.c_int64(0)
    _check(h, _L.lbm_count_fluid(h, ct.byref(n)))
    return n.value


def lbm_get_forces(h, nbt=None):
    if nbt is None:
        i = lbm_get_info(h)
        nbt = i["n_bodies"] + i["n_walls"]
    F = np.zeros((nbt, 3))
    T = np.zeros((nbt, 3))
    _check(h, _L.lbm_get_forces(h, _ptr(F), _ptr(T)))
    return F, T


def lbm_get_forces_device(h, d_out) -> None:
    _check(h, _L.lbm_get_forces_device(h, _dev_ptr(d_out)))


def lbm_get_populations(h, shape):
    nz, ny, nx = shape
    f = np.zeros((19, nz, ny, nx))
    _check(h, _L.lbm_get_populations(h, _ptr(f)))
    return f


def lbm_set_populations(h, f) -> None:
    f = _host(f, np.float64)
    _check(h, _L.lbm_set_populations(h, _ptr(f)))


def lbm_get_macro(h, shape):
    nz, ny, nx = shape
    rho = np.zeros((nz, ny, nx))
    u = np.zeros((3, nz, ny, nx))
    _check(h, _L.lbm_get_macro(h, _ptr(rho), _ptr(u)))
    return rho, u


def lbm_get_owner(h, shape):
    own = np.zeros(shape, np.int32)
    _check(h, _L.lbm_get_owner(h, _ptr(own)))
    return own


def lbm_get_state(h) -> bytes:
    n = ct.c_size_t(0)
    _check(h, _L.lbm_get_state(h, None, ct.byref(n)))
    buf = ct.create_string_buffer(n.value)
    _check(h, _L.lbm_get_state(h, buf, ct.byref(n)))
    return buf.raw[:n.value]


def lbm_set_state(h, state: bytes) -> None:
    _check(h, _L.lbm_set_state(h, state, len(state)))


def lbm_profile(h, every) -> None:
    """every: False/0 stops; True/1 records every step, n > 1 every n-th."""
    _check(h, _L.lbm_profile(h, int(every)))


def lbm_profile_read(h):
    ms = ct.c_double(0.0)
    n = ct.c_int64(0)
    _check(h, _L.lbm_profile_read(h, ct.byref(ms), ct.byref(n)))
    return ms.value, n.value


def lbm_profile_read_parts(h):
    """({part: summed milliseconds} for the parts of PROF_PARTS, steps recorded)."""
    ms = (ct.c_double * len(PROF_PARTS))()
    n = ct.c_int64(0)
    _check(h, _L.lbm_profile_read_parts(h, ms, ct.byref(n)))
    return dict(zip(PROF_PARTS, list(ms))), n.value


def lbm_set_step_path(h, path) -> None:
    _check(h, _L.lbm_set_step_path(h, STEP_PATH[path] if isinstance(path, str) else int(path)))


def lbm_get_step_path(h) -> str:
    p = ct.c_int32(0)
    _check(h, _L.lbm_get_step_path(h, ct.byref(p)))
    return {v: k for k, v in STEP_PATH.items()}[p.value]


def lbm_set_zieb(h, z_s, area, volume, v_piston) -> None:
    _check(h, _L.lbm_set_zieb(h, int(z_s), float(area), float(volume), float(v_piston)))


def lbm_get_zieb(h):
    """(cylinder density, piston displacement, mean inflow velocity) of the last step."""
    out = (ct.c_double * 3)()
    _check(h, _L.lbm_get_zieb(h, out))
    return tuple(out)


def lbm_set_body_force(h, F) -> None:
    _check(h, _L.lbm_set_body_force(h, _ptr(_host(F, np.float64, 3))))


def lbm_drag_gradient(h, nsteps, ckpt, n_bodies):
    """(J, dJ/dF [3], dJ/dV [n_bodies, 3])."""
    J = ct.c_double(0.0)
    dF = np.zeros(3)
    dV = np.zeros((max(n_bodies, 1), 3))
    _check(h, _L.lbm_drag_gradient(h, int(nsteps), int(ckpt), ct.byref(J), _ptr(dF), _ptr(dV)))
    return J.value, dF, dV[:n_bodies]


TILE_SHAPES = ("64x2x2", "32x4x2", "32x2x4", "16x8x2")


def lbm_set_tile(h, shape) -> None:
    _check(h, _L.lbm_set_tile(h, TILE_SHAPES.index(shape) if isinstance(shape, str) else int(shape)))


def lbm_get_tile(h) -> int:
    s = ct.c_int32(0)
    _check(h, _L.lbm_get_tile(h, ct.byref(s)))
    return s.value


def lbm_autotune_tile(h, trial_steps=10, cache_path=None):
    """(chosen shape, per-shape kernel microseconds, -1 where not timed)."""
    s = ct.c_int32(0)
    us = (ct.c_double * len(TILE_SHAPES))()
    path = None if cache_path is None else str(cache_path).encode()
    _check(h, _L.lbm_autotune_tile(h, int(trial_steps), path, ct.byref(s), us))
    return s.value, list(us)


def _bcheck(b, st):
    if st != 0:
        msg = _L.lbm_batch_last_error(b)
        raise LBMError(st, msg.decode() if msg else "")


def lbm_batch_create(handles, stream=None):
    arr = (_H * len(handles))(*handles)
    out = _H()
    st = _L.lbm_batch_create(arr, len(handles), _stream_ptr(stream), ct.byref(out))
    if st != 0:
        msgs = [(_L.lbm_last_error(h) or b"").decode() for h in handles]
        raise LBMError(st, "; ".join(m for m in msgs if m))
    return out


def lbm_batch_step(b, nsteps=1) -> None:
    _bcheck(b, _L.lbm_batch_step(b, int(nsteps)))


def lbm_batch_destroy(b) -> None:
    _L.lbm_batch_destroy(b)


def lbm_batch_set_tile(b, shape) -> None:
    _bcheck(b, _L.lbm_batch_set_tile(b, TILE_SHAPES.index(shape) if isinstance(shape, str) else int(shape)))


def lbm_batch_get_tile(b) -> int:
    s = ct.c_int32(0)
    _bcheck(b, _L.lbm_batch_get_tile(b, ct.byref(s)))
    return s.value


def lbm_batch_autotune(b, trial_steps=5):
    """(chosen shape, per-shape microseconds per batched step-kernel launch)."""
    s = ct.c_int32(0)
    us = (ct.c_double * len(TILE_SHAPES))()
    _bcheck(b, _L.lbm_batch_autotune(b, int(trial_steps), ct.byref(s), us))
    return s.value, list(us)


# ---- convenience object over one handle -----------------------------------------

class Lattice:
    """One handle with the calls above as methods (shapes remembered)."""

    def __init__(self, cfg: LBMConfig):
        self.cfg = cfg
        self.shape = (cfg.nz, cfg.ny, cfg.nx)
        self.h = lbm_create(cfg)
        self._nbt = 0
        self._n_walls = 0
        self._nb = 0

    @classmethod
    def from_case(cls, case, storage="f32", bb_mode="bouzidi", stream=None, max_bodies=None,
                  nan_guard_every=0, init=True, path=None):
        nw = case.n_walls
        cfg = config(case.nx, case.ny, case.nz, case.tau0, case.smag_c, case.rho0, case.body_force,
                     storage=storage, bb_mode=bb_mode,
                     max_bodies=case.n_bodies if max_bodies is None else max_bodies,
                     max_walls=nw, nan_guard_every=nan_guard_every, stream=stream)
        lat = cls(cfg)
        if path is not None:
            lat.set_step_path(path)
        if case.wall_id is not None:
            lat.set_walls(case.wall_id, case.wall_vel, case.wall_ref)
        lat.set_bodies(*case.bodies_at(0))
        if init:
            lat.init_fields(case.rho_init, case.u_init)
        return lat

    def close(self):
        if self.h:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        lbm_set_stream(self.h, stream)

    def set_walls(self, wall_id, wall_vel, wall_ref=None):
        lbm_set_walls(self.h, wall_id, wall_vel, wall_ref)
        self._n_walls = 0 if wall_vel is None else len(np.asarray(wall_vel).reshape(-1, 3))

    def set_bodies(self, X, V, Omega, R):
        lbm_set_bodies(self.h, X, V, Omega, R)
        self._nb_next = len(np.asarray(R).reshape(-1))

    def set_bodies_device(self, n, d_table):
        lbm_set_bodies_device(self.h, n, d_table)

    def init_fields(self, rho=None, u=None):
        lbm_init_fields(self.h, rho, u)

    def step(self, nsteps=1):
        lbm_step(self.h, nsteps)

    def step_noalloc(self, nsteps=1):
        lbm_step_noalloc(self.h, nsteps)

    def get_forces(self):
        return lbm_get_forces(self.h)

    def get_forces_device(self, d_out):
        lbm_get_forces_device(self.h, d_out)

    def get_populations(self):
        return lbm_get_populations(self.h, self.shape)

    def set_populations(self, f):
        lbm_set_populations(self.h, f)

    def get_macro(self):
        return lbm_get_macro(self.h, self.shape)

    def get_owner(self):
        return lbm_get_owner(self.h, self.shape)

    def get_state(self):
        return lbm_get_state(self.h)

    def set_state(self, s):
        lbm_set_state(self.h, s)

    def info(self):
        return lbm_get_info(self.h)

    def count_fluid(self):
        return lbm_count_fluid(self.h)

    def profile(self, every):
        lbm_profile(self.h, every)

    def profile_read(self):
        return lbm_profile_read(self.h)

    def profile_read_parts(self):
        return lbm_profile_read_parts(self.h)

    def set_step_path(self, path):
        lbm_set_step_path(self.h, path)

    @property
    def step_path(self):
        return lbm_get_step_path(self.h)

    def set_zieb(self, z_s, area, volume, v_piston):
        lbm_set_zieb(self.h, z_s, area, volume, v_piston)

    def zieb_state(self):
        return lbm_get_zieb(self.h)

    def set_body_force(self, F):
        lbm_set_body_force(self.h, F)

    def drag_gradient(self, nsteps, ckpt):
        return lbm_drag_gradient(self.h, nsteps, ckpt, self.info()["n_bodies"])

    def set_tile(self, shape):
        lbm_set_tile(self.h, shape)

    @property
    def tile(self):
        return lbm_get_tile(self.h)

    def autotune(self, trial_steps=10, cache_path=None):
        return lbm_autotune_tile(self.h, trial_steps, cache_path)


class Batch:
    """Independent lattices stepped together (one graph replay per step)."""

    def __init__(self, lattices, stream=None):
        self.members = list(lattices)
        self.b = lbm_batch_create([m.h for m in self.members], stream)

    def step(self, nsteps=1):
        lbm_batch_step(self.b, nsteps)

    def set_tile(self, shape):
        lbm_batch_set_tile(self.b, shape)

    @property
    def tile(self):
        return lbm_batch_get_tile(self.b)

    def autotune(self, trial_steps=5):
        return lbm_batch_autotune(self.b, trial_steps)

    def close(self):
        if self.b:
            lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SphereDrag:
    """J = sum_b F_b,x after `nsteps` steps from a fixed start state, as a
    torch function of the body force F (3,) and the sphere velocities
    V (n_bodies, 3); its backward pass is the library's reverse-mode kernels
    (lbm_drag_gradient).  Positions, angular velocities and radii stay
    those given; every evaluation restarts from `start_state` (a checkpoint
    from Lattice.get_state)."""

    def __init__(self, lattice, start_state, X, Omega, R, nsteps, ckpt):
        import torch

        self.lat, self.state = lattice, start_state
        self.X, self.Omega, self.R = np.asarray(X), np.asarray(Omega), np.asarray(R)
        self.nsteps, self.ckpt = int(nsteps), int(ckpt)
        outer = self

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, F, V):
                outer.lat.set_state(outer.state)
                outer.lat.set_body_force(F.detach().cpu().double().numpy())
                outer.lat.set_bodies(outer.X, V.detach().cpu().double().numpy(), outer.Omega, outer.R)
                J, dF, dV = outer.lat.drag_gradient(outer.nsteps, outer.ckpt)
                ctx.save_for_backward(torch.as_tensor(dF, dtype=F.dtype, device=F.device),
                                      torch.as_tensor(dV, dtype=V.dtype, device=V.device))
                return torch.tensor(J, dtype=F.dtype, device=F.device)

            @staticmethod
            def backward(ctx, gJ):
                dF, dV = ctx.saved_tensors
                return gJ * dF, gJ * dV

        self._fn = _Fn

    def __call__(self, F, V):
        return self._fn.apply(F, V)
