"""Seeded synthetic inputs for the D3Q19 moving-boundary LBM step.

This module builds the *inputs* of a run -- box sizes, relaxation and
Smagorinsky parameters, the body-force density, static wall voxels with
their prescribed velocities, sphere tables (centre, velocity, angular
velocity, radius) and initial density/velocity fields.  It holds none of the
method's arithmetic (no equilibria, no rasterisation of spheres onto the
lattice, no streaming): both the FP64 oracle and the HIP library receive the
same arrays from here and nothing else.

Conventions
-----------
* Lattice units throughout (the paper's Sec. 2.2 non-dimensionalisation:
  spacing and time step equal one).
* Node (x, y, z) has linear index ``x + nx*(y + ny*z)``; numpy fields have
  shape ``(nz, ny, nx)``.  Every axis is index-periodic; non-periodic
  boundaries are realised as solid wall voxels.
* ``wall_id`` is uint8, 0 = not a wall, 1..W = wall object; ``wall_vel`` and
  ``wall_ref`` are (W, 3) float64 (velocity, torque reference point).
* Sphere tables are float64: ``X, V, Omega`` (n, 3), ``R`` (n,).
* Velocity fields are component-major: ``u[c, z, y, x]``.

Workloads follow the paper's piston-valve setting (Sec. 3: a piston pushing a
particle-laden fluid through a restriction, particle diameters of a few lattice
cells, uniform polydisperse radii) at the sizes of the benchmark configurations
described in the design notes.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

__all__ = [
    "Case", "rsa_pack", "min_tie_gap", "case_box32", "case_duct", "case_piston_duct", "case_adjoint",
    "case_box", "drift_positions", "case_sweep_instances",
]


@dataclass
class Case:
    """Everything a run needs, as plain arrays (no derived method state)."""
    name: str
    nx: int
    ny: int
    nz: int
    tau0: float
    smag_c: float
    rho0: float = 1.0
    body_force: tuple = (0.0, 0.0, 0.0)
    wall_id: Optional[np.ndarray] = None      # uint8 (nz, ny, nx)
    wall_vel: Optional[np.ndarray] = None     # (W, 3)
    wall_ref: Optional[np.ndarray] = None     # (W, 3)
    X: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    V: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    Omega: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    R: np.ndarray = field(default_factory=lambda: np.zeros((0,)))
    rho_init: Optional[np.ndarray] = None     # (nz, ny, nx) or None -> rho0
    u_init: Optional[np.ndarray] = None       # (3, nz, ny, nx) or None -> 0
    steps: int = 100
    drift: bool = False                       # bodies advance X += V each step

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_walls(self) -> int:
        return 0 if self.wall_vel is None else int(len(self.wall_vel))

    @property
    def n_bodies(self) -> int:
        return int(len(self.R))

    def bodies_at(self, n: int):
        """Body kinematics supplied for step ``n`` (1-based); step 0 = initial."""
        if not self.drift or n == 0:
            return self.X, self.V, self.Omega, self.R
        return drift_positions(self, n), self.V, self.Omega, self.R


def _box(case_or_dims):
    if isinstance(case_or_dims, Case):
        return np.array([case_or_dims.nx, case_or_dims.ny, case_or_dims.nz], float)
    return np.asarray(case_or_dims, float)


def drift_positions(case: Case, n: int) -> np.ndarray:
    """Centres after ``n`` steps of free drift, wrapped into the periodic box."""
    box = _box(case)
    P = np.mod(case.X + n * case.V, box)
    # a tiny negative coordinate wraps to box - tiny, which can round to box
    return np.where(P >= box, 0.0, P)


def min_tie_gap(X: np.ndarray, R: np.ndarray, box) -> float:
    """Smallest | |p - X|^2 - R^2 | over integer nodes p near every sphere.

    Inputs with a value below 1e-6 put a node (numerically) on a sphere
    surface; generators redraw such spheres so that the solid/fluid decision
    of every node is far from a tie in FP64.
    """
    box = np.asarray(box, float)
    best = np.inf
    for c, r in zip(np.asarray(X, float), np.asarray(R, float)):
        rng = [np.arange(np.floor(c[a] - r) - 1, np.ceil(c[a] + r) + 2) for a in range(3)]
        gx, gy, gz = np.meshgrid(*rng, indexing="ij")
        d = np.stack([gx - c[0], gy - c[1], gz - c[2]], -1)
        d -= box * np.round(d / box)
        best = min(best, float(np.min(np.abs((d * d).sum(-1) - r * r))))
    return best


def rsa_pack(rng: np.random.Generator, radii: np.ndarray, lo, hi, gap: float,
             box, periodic=(True, True, True), max_tries: int = 200000):
    """Random sequential addition of non-overlapping spheres.

    Radii are placed largest first.  A centre is drawn uniformly in
    ``[0, box)`` on periodic axes and in ``[lo + r, hi - r]`` on the others,
    and accepted when its surface gap to every
    placed sphere (minimum image on periodic axes) is at least ``gap`` and no
    lattice node lies within 1e-6 (in squared distance) of its surface.
    Returns the centres in the original order of ``radii``.
    """
    radii = np.asarray(radii, float)
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    box = np.asarray(box, float)
    per = np.asarray(periodic, bool)
    order = np.argsort(-radii, kind="stable")
    centres = np.zeros((len(radii), 3))
    placed_c = np.zeros((0, 3))
    placed_r = np.zeros((0,))
    tries = 0
    for idx in order:
        r = radii[idx]
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("rsa_pack: packing too dense for the region")
            c = lo + r + rng.random(3) * np.maximum(hi - lo - 2 * r, 0.0)
            c = np.where(per, rng.random(3) * box, c)
            if len(placed_r):
                d = placed_c - c
                d[:, per] -= box[per] * np.round(d[:, per] / box[per])
                if np.any(np.sqrt((d * d).sum(1)) < placed_r + r + gap):
                    continue
            if min_tie_gap(c[None], np.array([r]), box) < 1e-6:
                continue
            break
        centres[idx] = c
        placed_c = np.vstack([placed_c, c])
        placed_r = np.append(placed_r, r)
    return centres


def case_box32(seed: int = 0) -> Case:
    """Small parity case: 32^3 periodic box, 8 fixed spheres of radius 4.

    BGK+Smagorinsky with C = 0.1, tau0 = 0.6, body force 1e-6 along x,
    density 1 and initial velocity N(0, 0.01^2) per component at every node
    (the library keeps only fluid nodes), spheres at rest with centres drawn
    by RSA with a surface gap of 2 cells.  100 steps.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 32
    R = np.full(8, 4.0)
    X = rsa_pack(rng, R, (0, 0, 0), (n, n, n), gap=2.0, box=(n, n, n))
    u = rng.normal(0.0, 0.01, size=(3, n, n, n))
    return Case(name="box_32cube_8spheres", nx=n, ny=n, nz=n, tau0=0.6, smag_c=0.1,
                body_force=(1e-6, 0.0, 0.0), X=X, V=np.zeros((8, 3)),
                Omega=np.zeros((8, 3)), R=R, u_init=u, steps=100)


def case_duct(nx=128, ny=128, nz=512, n_spheres=4000, r_min=2.0, r_max=6.0,
              piston_u=0.02, orifice_z=384, orifice_thick=4, orifice_r_in=40.0,
              orifice_gap=6.0, pack_z=(20.0, 358.0), tau0=0.55, smag_c=0.17,
              v_sigma=0.005, w_sigma=0.001, seed=1, steps=1000, drift=True,
              name=None) -> Case:
    """Piston duct with an annular orifice plate and polydisperse spheres.

    Walls (static, id 1): the layers x in {0, nx-1} and y in {0, ny-1}.
    Piston (id 2): the layer z = 0 inside the duct, moving at +piston_u along
    z; the z axis is index-periodic, so the piston pushes on its z = 1 face
    and withdraws on its z = nz-1 face.  Orifice plate (id 3, static): the
    layers orifice_z .. orifice_z+thick-1, solid except the annulus
    r_in <= r < r_in + gap about the duct axis.  Spheres: radii uniform in
    [r_min, r_max], RSA with a 1-cell surface gap inside the duct interior
    and z in ``pack_z``; velocities N(0, v_sigma^2), angular velocities
    N(0, w_sigma^2) per component.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    wall = np.zeros((nz, ny, nx), np.uint8)
    wall[:, :, 0] = wall[:, :, nx - 1] = 1
    wall[:, 0, :] = wall[:, ny - 1, :] = 1
    wall[0, 1:ny - 1, 1:nx - 1] = 2
    cy, cx = (ny - 1) / 2.0, (nx - 1) / 2.0
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((xx - cx) ** 2 + (yy - cy) ** 2)
    plate = ~((r >= orifice_r_in) & (r < orifice_r_in + orifice_gap))
    for z in range(orifice_z, orifice_z + orifice_thick):
        layer = wall[z]
        sel = plate & (layer == 0)
        layer[sel] = 3
    wall_vel = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, piston_u], [0.0, 0.0, 0.0]])
    wall_ref = np.array([[cx, cy, nz / 2.0], [cx, cy, 0.0], [cx, cy, orifice_z + orifice_thick / 2.0]])
    R = r_min + (r_max - r_min) * rng.random(n_spheres)
    lo = (1.0 + 1.0, 1.0 + 1.0, pack_z[0])
    hi = (nx - 1.0 - 1.0, ny - 1.0 - 1.0, pack_z[1])
    X = rsa_pack(rng, R, lo, hi, gap=1.0, box=(nx, ny, nz), periodic=(False, False, False))
    V = rng.normal(0.0, v_sigma, size=(n_spheres, 3))
    W = rng.normal(0.0, w_sigma, size=(n_spheres, 3))
    return Case(name=name or f"duct_{nx}x{ny}x{nz}_{n_spheres}spheres", nx=nx, ny=ny, nz=nz,
                tau0=tau0, smag_c=smag_c, wall_id=wall, wall_vel=wall_vel,
                wall_ref=wall_ref, X=X, V=V, Omega=W, R=R, steps=steps, drift=drift)


def case_piston_duct(seed: int = 1, drift: bool = True) -> Case:
    """The full piston-duct slurry: 128x128x512, 4000 spheres, solid fraction 0.25."""
    return case_duct(seed=seed, drift=drift)


def case_box(n=(32, 32, 32), n_spheres=8, radius=(4.0, 4.0), tau0=0.6, smag_c=0.1,
             body_force=(1e-6, 0.0, 0.0), u_sigma=0.01, v_sigma=0.0, w_sigma=0.0,
             gap=2.0, seed=0, drift=False, steps=100, name=None) -> Case:
    """A periodic box with RSA spheres (generalises the small parity case)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = n
    R = radius[0] + (radius[1] - radius[0]) * rng.random(n_spheres)
    if n_spheres:
        X = rsa_pack(rng, R, (0, 0, 0), (nx, ny, nz), gap=gap, box=(nx, ny, nz))
    else:
        X = np.zeros((0, 3))
    V = rng.normal(0.0, v_sigma, size=(n_spheres, 3)) if v_sigma else np.zeros((n_spheres, 3))
    W = rng.normal(0.0, w_sigma, size=(n_spheres, 3)) if w_sigma else np.zeros((n_spheres, 3))
    u = rng.normal(0.0, u_sigma, size=(3, nz, ny, nx)) if u_sigma else None
    return Case(name=name or f"box_{nx}x{ny}x{nz}_{n_spheres}spheres", nx=nx, ny=ny, nz=nz,
                tau0=tau0, smag_c=smag_c, body_force=tuple(body_force), X=X, V=V,
                Omega=W, R=R, u_init=u, steps=steps, drift=drift)


SWEEP_SIZES = [(64, 64, 64), (96, 96, 96), (128, 128, 128), (96, 96, 192), (160, 128, 128)]


def case_sweep_instances(n_instances: int = 48, seed: int = 3, steps: int = 500):
    """Independent periodic boxes of a parameter sweep.

    Per instance (seed + index): size drawn from SWEEP_SIZES, tau0 in
    [0.52, 0.8], C in [0.1, 0.2], body force magnitude in [1e-7, 1e-5] along
    x, packing fraction in [0, 0.35] of spheres with radius uniform in
    [2, 5]; the sphere count is min(1500, round(phi * V / E[V_sphere])) with
    E[V_sphere] = (4/3) pi E[R^3], E[R^3] = (5^4 - 2^4) / (4 * 3).  Spheres
    are placed by random sequential addition without a surface gap (they may
    touch, never overlap): with a one-cell gap the densest instances (phi
    near 0.35) cannot be packed that way.
    """
    out = []
    ev = 4.0 / 3.0 * np.pi * (5.0 ** 4 - 2.0 ** 4) / (4.0 * 3.0)
    for k in range(n_instances):
        rng = np.random.Generator(np.random.PCG64(seed + k))
        nx, ny, nz = SWEEP_SIZES[int(rng.integers(len(SWEEP_SIZES)))]
        tau0 = float(rng.uniform(0.52, 0.8))
        cs = float(rng.uniform(0.1, 0.2))
        fmag = float(rng.uniform(1e-7, 1e-5))
        phi = float(rng.uniform(0.0, 0.35))
        nsph = int(min(1500, round(phi * nx * ny * nz / ev)))
        R = 2.0 + 3.0 * rng.random(nsph)
        X = (rsa_pack(rng, R, (0, 0, 0), (nx, ny, nz), gap=0.0, box=(nx, ny, nz), max_tries=400000)
             if nsph else np.zeros((0, 3)))
        out.append(Case(name=f"sweep{k}_{nx}x{ny}x{nz}_{nsph}spheres", nx=nx, ny=ny, nz=nz,
                        tau0=tau0, smag_c=cs, body_force=(fmag, 0.0, 0.0), X=X,
                        V=np.zeros((nsph, 3)), Omega=np.zeros((nsph, 3)), R=R, steps=steps))
    return out


def case_adjoint(seed: int = 4, steps: int = 200) -> Case:
    """Drag-gradient workload: 96x96x192 periodic box, 300 spheres of radius
    4 (RSA, 2-cell surface gap), body force 5e-6 along x, fluid at rest,
    tau0 = 0.6, C = 0.1; sphere velocities N(0, 0.005^2) per component, held
    in place (the gradient is taken with respect to the body force and the
    300 x 3 velocities)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = 96, 96, 192
    R = np.full(300, 4.0)
    X = rsa_pack(rng, R, (0, 0, 0), (nx, ny, nz), gap=2.0, box=(nx, ny, nz))
    V = rng.normal(0.0, 0.005, size=(300, 3))
    return Case(name="adjoint_96x96x192_300spheres", nx=nx, ny=ny, nz=nz, tau0=0.6, smag_c=0.1,
                body_force=(5e-6, 0.0, 0.0), X=X, V=V, Omega=np.zeros((300, 3)), R=R, steps=steps)


def with_steps(case: Case, steps: int) -> Case:
    return replace(case, steps=steps)
