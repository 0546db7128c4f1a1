"""The largest lattice the library takes: 1024 x 1024 x 1023 nodes (1.07e9,
just under the 2^30 node limit of lbm_create, up to which the byte offset of
a population within its direction's array fits in 32 bits).  One sphere moves
at the far end of the index range, a body force acts everywhere, the fluid
starts at rest.  After two steps:

* the 24^3 block at the end of the index range that holds the sphere equals,
  in density and velocity at every node of its interior (3 nodes in from its
  faces, beyond what two steps can carry across them), the FP64 oracle on a
  periodic 24^3 box with the same sphere; the sphere's force and torque equal
  the oracle's (the box holds the sphere and all that two steps reach);
* nodes far from the sphere, the first and the last of the index range among
  them, equal the oracle's nodes far from its sphere.

FP32 and FP16 storage: about 200 and 120 GB of device memory, 34 GB of host
memory for the read-back.  Bars: FP32 1e-6 on density and velocity, 1e-4 on
force and torque (norm-relative).  FP16 (eps = 2^-11): 3 eps on force and
8 eps on torque, and 0.01 eps on density and velocity far from the sphere, as
in test_gpu_storage; in the sphere's block each of the two steps rounds every
stored deviation g_i by at most eps |g_i|, and the density and momentum are
sums of them, so there the bar is 2 eps max_node sum_i |g_i| (from the
oracle's populations, 0.057 here) on top of FP32's 1e-6: next to a sphere
moving at 0.02 the largest sum_i |g_i| is about thirty times that of the 32^3
case after its 100 steps (0.0018).
"""
import numpy as np
import pytest

import lbm_workloads as W

pytestmark = pytest.mark.gpu

NX, NY, NZ = 1024, 1024, 1023
P = 24                                   # the block, and the oracle's box
X0, Y0, Z0 = NX - P, NY - P, NZ - P      # the block's origin in the lattice
XC = np.array([[11.25, 11.75, 12.375]])  # sphere centre in the block: binary fractions,
R = np.array([5.2])                      # so that both sides see the same offsets
V = np.array([[0.02, -0.01, 0.015]])
OM = np.array([[0.001, -0.002, 0.0015]])
TAU0, SMAG_C, FORCE = 0.6, 0.1, (1e-5, -2e-6, 3e-6)
EPS16 = 2.0 ** -11
BARS = {"f32": (1e-6, 1e-6, 1e-4, 1e-4), "f16": (0.01 * EPS16, 0.01 * EPS16, 3 * EPS16, 8 * EPS16)}


def _case(name, n, origin):
    nx, ny, nz = n
    return W.Case(name=name, nx=nx, ny=ny, nz=nz, tau0=TAU0, smag_c=SMAG_C, body_force=FORCE,
                  X=XC + np.asarray(origin, float), V=V.copy(), Omega=OM.copy(), R=R.copy(), drift=False)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_largest_lattice(storage, torch_stream):
    import oracle
    from paper_1703_05158_amd import LBMError, Lattice

    o = oracle.Oracle.from_case(_case("max_size_block", (P, P, P), (0, 0, 0)))
    o.step(2)
    ro, uo = o.macro()
    Fo, To = o.forces()
    _, w, _ = oracle.tables()
    s = slice(3, P - 3)
    g_sum = np.abs(o.populations() - w[:, None, None, None] * o.rho0).sum(axis=0)[s, s, s].max()

    big = _case("max_size", (NX, NY, NZ), (X0, Y0, Z0))
    assert big.n_nodes < 2 ** 30
    try:
        lat = Lattice.from_case(big, storage=storage, stream=torch_stream)
    except LBMError as e:
        pytest.skip(f"the lattice does not fit in this device's memory: {e}")
    try:
        lat.step(2)
        Fg, Tg = lat.get_forces()
        rho, u = lat.get_macro()
    finally:
        lat.close()
    b_rho, b_u, b_f, b_t = BARS[storage]
    blk_bar = 1e-6 + (2 * EPS16 * g_sum if storage == "f16" else 0.0)

    # the block that holds the sphere, interior nodes
    blk_rho = rho[Z0:, Y0:, X0:][s, s, s]
    blk_u = u[:, Z0:, Y0:, X0:][:, s, s, s]
    dr = float(np.max(np.abs(blk_rho - ro[s, s, s])))
    du = float(np.max(np.abs(blk_u - uo[:, s, s, s])))

    # nodes far from the sphere: the first and last of the index range, the
    # block's far corner, and a seeded sample; against the oracle's far corner
    rng = np.random.Generator(np.random.PCG64(30))
    N = big.n_nodes
    idx = np.concatenate([[0, 1, NX - 1, NX * NY, N - NX, N - 2, N - 1], rng.integers(0, N, 20000)])
    z, r = np.divmod(idx, NX * NY)
    y, x = np.divmod(r, NX)
    d = np.stack([x, y, z], 1) - (XC[0] + [X0, Y0, Z0])
    d -= np.array([NX, NY, NZ]) * np.round(d / np.array([NX, NY, NZ]))
    far = np.linalg.norm(d, axis=1) > R[0] + 4.0
    assert far[[0, 1, 6]].all()  # the first node and the last
    z, y, x = z[far], y[far], x[far]
    fr = float(np.max(np.abs(rho[z, y, x] - ro[0, 0, 0])))
    fu = float(np.max(np.abs(u[:, z, y, x] - uo[:, 0, 0, 0][:, None])))
    del rho, u

    fe = float(np.linalg.norm(Fg[0] - Fo[0]) / np.linalg.norm(Fo[0]))
    te = float(np.linalg.norm(Tg[0] - To[0]) / np.linalg.norm(To[0]))
    print(f"{storage}: block rho {dr:.2e} u {du:.2e} (bar {blk_bar:.2e}); "
          f"far rho {fr:.2e} u {fu:.2e} ({far.sum()} nodes); "
          f"F {fe:.2e} T {te:.2e}")
    assert dr <= blk_bar and du <= blk_bar
    assert fr <= b_rho and fu <= b_u
    assert fe <= b_f and te <= b_t
