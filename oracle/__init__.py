"""FP64 CPU oracle of the D3Q19 moving-boundary LBM step -- test infrastructure.

Only the test suite, the benchmark's CPU-baseline leg and the smoke check may
import this package.  It wraps ``lbm_oracle.c`` (plain C, double precision,
optional OpenMP over z-slabs) through ctypes and keeps the run state in numpy
arrays.  It shares no code with the HIP library.

Step semantics (one call of :meth:`Oracle.step`):
  state P_{n-1} (post-collision, all nodes), owner maps O_{n-1} and O_n,
  bodies B_{n-1} and B_n  ->  pull streaming with Bouzidi bounce-back and the
  moving-boundary term (Sec. 2.3), momentum-exchange force/torque per body
  (Sec. 2.3), moments (eqs. dens, momentum), equilibrium (eq.
  Equilibre_Maxwell_Boltzmann), Smagorinsky tau* (Sec. 2.2), BGK collision
  with a Guo body-force source (eq. Collision_step)  ->  P_n.
Bodies set before step n are the geometry and velocities of step n; the
geometry at initialisation is both O_0 and the geometry of step 1 unless the
bodies are set again before stepping.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ct.CDLL(_LIB)
        L.orc_tables.argtypes = [_ip, _dp, _ip]
        L.orc_equilibrium.argtypes = [ct.c_double] * 4 + [_dp]
        L.orc_relaxation_time.argtypes = [ct.c_double] * 4
        L.orc_relaxation_time.restype = ct.c_double
        L.orc_owner_map.argtypes = [_ip, ct.c_void_p, ct.c_int, ct.c_int, _dp, _dp, _ip]
        body4 = [_dp, _dp, _dp, _dp]
        walls = [ct.c_int, _dp, _dp]
        L.orc_stream.argtypes = ([_ip, _dp, ct.c_int, _dp, _ip, _ip, ct.c_int] + body4 +
                                 [ct.c_int] + body4 + walls + [ct.c_int, _dp, _dp, _dp])
        L.orc_zieb_inflow.argtypes = [_ip, _dp, _ip, _dp, ct.c_int, _dp]
        L.orc_zieb_density.argtypes = [ct.c_double] * 6
        L.orc_zieb_density.restype = ct.c_double
        L.orc_zieb.argtypes = [_ip, ct.c_int, ct.c_double, _ip, _dp, _dp]
        L.orc_collide.argtypes = [_ip, _dp, _ip, ct.c_int] + body4 + walls + [_dp, _dp]
        L.orc_init.argtypes = ([_ip, ct.c_double, _ip, ct.c_int] + body4 + walls +
                               [ct.c_void_p, ct.c_void_p, _dp])
        L.orc_macro.argtypes = [_ip, _dp, _ip, ct.c_int] + body4 + walls + [_dp, _dp, _dp]
        L.orc_set_threads.argtypes = [ct.c_int]
        L.orc_set_threads.restype = ct.c_int
        _lib = L
    return _lib


def tables():
    """(c[19,3] int, w[19], opp[19]) as the oracle holds them."""
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    lib().orc_tables(c, w, opp)
    return c, w, opp


def equilibrium(rho, u):
    out = np.zeros(19)
    lib().orc_equilibrium(float(rho), float(u[0]), float(u[1]), float(u[2]), out)
    return out


def relaxation_time(tau0, C, rho, Q):
    return lib().orc_relaxation_time(float(tau0), float(C), float(rho), float(Q))


def set_threads(n: int) -> int:
    return lib().orc_set_threads(int(n))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """Stateful FP64 run mirroring the library's create/set/init/step/get calls."""

    def __init__(self, nx, ny, nz, tau0, smag_c, rho0=1.0, body_force=(0.0, 0.0, 0.0),
                 halfway=False):
        self.dims = np.array([nx, ny, nz, 0], np.int32)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.N = nx * ny * nz
        self.prm = np.array([tau0, smag_c, rho0, *body_force], np.float64)
        self.rho0 = rho0
        self.halfway = int(bool(halfway))
        self.wall = None
        self.n_walls = 0
        self.Uw = np.zeros((1, 3))
        self.Ref = np.zeros((1, 3))
        self._bodies = self._pack_bodies(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0))
        self._bodies_prev = self._bodies
        self.own = None
        self.own_prev = None
        self.P = None
        self.F = np.zeros((0, 3))
        self.T = np.zeros((0, 3))
        self.steps_done = 0
        self.zieb = None
        self.own = self._owner(self._bodies)

    @classmethod
    def from_case(cls, case, halfway=False, init=True):
        o = cls(case.nx, case.ny, case.nz, case.tau0, case.smag_c, case.rho0,
                case.body_force, halfway=halfway)
        if case.wall_id is not None:
            o.set_walls(case.wall_id, case.wall_vel, case.wall_ref)
        o.set_bodies(*case.bodies_at(0))
        if init:
            o.init_fields(case.rho_init, case.u_init)
        return o

    # -- inputs ---------------------------------------------------------
    @staticmethod
    def _pack_bodies(X, V, W, R):
        n = len(R)
        pad = lambda a: _f64(a, (n, 3)) if n else np.zeros((1, 3))
        return dict(n=n, X=pad(X), V=pad(V), W=pad(W), R=_f64(R) if n else np.zeros(1))

    def set_walls(self, wall_id, wall_vel, wall_ref=None):
        wall_vel = _f64(wall_vel, (-1, 3))
        self.n_walls = len(wall_vel)
        self.wall = np.ascontiguousarray(np.asarray(wall_id, np.uint8).reshape(-1))
        self.Uw = wall_vel if self.n_walls else np.zeros((1, 3))
        self.Ref = (_f64(wall_ref, (-1, 3)) if wall_ref is not None
                    else np.zeros((max(self.n_walls, 1), 3)))
        self.own = self._owner(self._bodies)

    def set_bodies(self, X, V, W, R):
        self._bodies = self._pack_bodies(X, V, W, R)
        self.own = self._owner(self._bodies)

    def _owner(self, B):
        own = np.zeros(self.N, np.int32)
        wall_ptr = self.wall.ctypes.data if self.wall is not None else None
        rc = lib().orc_owner_map(self.dims, wall_ptr, self.n_walls, B["n"], B["X"].reshape(-1),
                                 B["R"], own)
        if rc != 0:
            raise ValueError("wall id exceeds the number of walls")
        return own

    def _bargs(self, B):
        return [B["n"], B["X"].reshape(-1), B["V"].reshape(-1), B["W"].reshape(-1), B["R"]]

    def _wargs(self):
        return [self.n_walls, self.Uw.reshape(-1), self.Ref.reshape(-1)]

    def set_zieb(self, z_s, area, volume, v_piston):
        """Virtual-cylinder inflow (Sec. 2.6) at the plane z = z_s; the layer
        z_s - 1 stands for the removed domain.  The cylinder density starts
        at the plane's mean density of the initial state."""
        self.zieb = dict(z=int(z_s), area=float(area), volume=float(volume), vp=float(v_piston),
                         rho=None, H=0.0)

    def zieb_inflow(self):
        """(v_f, mean density) of the current state at the ZIEB plane."""
        out = np.zeros(2)
        lib().orc_zieb_inflow(self.dims, self.prm, self._state_own(), self.P, self.zieb["z"], out)
        return float(out[0]), float(out[1])

    def init_fields(self, rho=None, u=None):
        self.P = np.zeros(19 * self.N)
        r = _f64(rho).reshape(-1) if rho is not None else None
        v = _f64(u).reshape(-1) if u is not None else None
        lib().orc_init(self.dims, self.rho0, self.own, *self._bargs(self._bodies), *self._wargs(),
                       r.ctypes.data if r is not None else None,
                       v.ctypes.data if v is not None else None, self.P)
        self.own_prev = self.own.copy()
        self._bodies_prev = self._bodies
        nbt = self._bodies["n"] + self.n_walls
        self.F = np.zeros((nbt, 3))
        self.T = np.zeros((nbt, 3))

    # -- stepping -------------------------------------------------------
    def stream(self):
        """Streaming + boundary stage only: (f [19,N] at fluid nodes, F, T).
        With a ZIEB plane, its update of the cylinder density and of the
        plane's populations is part of this stage."""
        nbt = self._bodies["n"] + self.n_walls
        f = np.full(19 * self.N, np.nan)
        F = np.zeros(max(nbt, 1) * 3)
        T = np.zeros(max(nbt, 1) * 3)
        zz = self.zieb["z"] if self.zieb else -1
        if self.zieb:
            z = self.zieb
            vf, rbar = self.zieb_inflow()
            if z["rho"] is None:
                z["rho"] = rbar
            z["rho_next"] = lib().orc_zieb_density(z["rho"], z["vp"], vf, z["area"], z["volume"], z["H"])
            z["vf"] = vf
        lib().orc_stream(self.dims, self.prm, self.halfway, self.P, self.own_prev, self.own,
                         *self._bargs(self._bodies_prev), *self._bargs(self._bodies),
                         *self._wargs(), zz, f, F, T)
        if self.zieb:
            lib().orc_zieb(self.dims, zz, self.zieb["rho_next"], self.own, self.P, f)
        return f, F[:3 * nbt].reshape(nbt, 3), T[:3 * nbt].reshape(nbt, 3)

    def step(self, nsteps=1):
        if self.P is None:
            raise RuntimeError("init_fields first")
        for _ in range(nsteps):
            f, F, T = self.stream()
            Pn = np.zeros(19 * self.N)
            lib().orc_collide(self.dims, self.prm, self.own, *self._bargs(self._bodies),
                              *self._wargs(), f, Pn)
            self.P = Pn
            self.F, self.T = F, T
            if self.zieb:
                self.zieb["rho"] = self.zieb["rho_next"]
                self.zieb["H"] += self.zieb["vp"]
            self.own_prev = self.own.copy()
            self._bodies_prev = self._bodies
            self.steps_done += 1

    # -- outputs --------------------------------------------------------
    def populations(self):
        return self.P.reshape(19, self.nz, self.ny, self.nx)

    def macro(self):
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        lib().orc_macro(self.dims, self.prm, self._state_own(), *self._bargs(self._bodies_prev),
                        *self._wargs(), self.P, rho, u)
        return rho.reshape(self.nz, self.ny, self.nx), u.reshape(3, self.nz, self.ny, self.nx)

    def _state_own(self):
        # geometry of the current state: that of the last step (or of init)
        return self.own_prev if self.own_prev is not None else self.own

    def fluid_mask(self):
        return (self._state_own() < 0).reshape(self.nz, self.ny, self.nx)

    def owner(self):
        return self._state_own().reshape(self.nz, self.ny, self.nx)

    def forces(self):
        return self.F.copy(), self.T.copy()
