"""The inflow plane fed by a virtual cylinder (Sec. 2.6) on the GPU, against
the FP64 oracle: a duct closed at its far end, with spheres, compressed by
the virtual piston through the plane z = 1.  Same bars as the step itself
(populations 1e-5 relative, forces 1e-4 norm-relative); the cylinder state
to 1e-6; checkpoints carry the cylinder state.
"""
import numpy as np
import pytest

import lbm_workloads as W
from ._pair import force_rel_err, pop_rel_err

pytestmark = pytest.mark.gpu


def _case():
    nx, ny, nz = 24, 20, 48
    w = np.zeros((nz, ny, nx), np.uint8)
    w[:, :, 0] = w[:, :, nx - 1] = 1
    w[:, 0, :] = w[:, ny - 1, :] = 1
    w[0] = 1            # stands for the removed domain below the plane z = 1
    w[nz - 1] = 1       # closed far end
    rng = np.random.Generator(np.random.PCG64(31))
    R = np.array([3.0, 2.5, 3.5])
    X = W.rsa_pack(rng, R, (2, 2, 6), (nx - 2, ny - 2, nz - 4), gap=1.0, box=(nx, ny, nz),
                   periodic=(False, False, False))
    u = rng.normal(0.0, 0.005, size=(3, nz, ny, nx))
    case = W.Case(name="zieb_duct", nx=nx, ny=ny, nz=nz, tau0=0.7, smag_c=0.1, wall_id=w,
                  wall_vel=np.zeros((1, 3)), wall_ref=np.zeros((1, 3)), X=X, V=np.zeros((3, 3)),
                  Omega=np.zeros((3, 3)), R=R, u_init=u)
    fluid_plane = float((w[1] == 0).sum())
    volume = 2.0 * float((w == 0).sum())
    return case, (1, fluid_plane, volume, 0.01)


def _pair(torch_stream, storage="f32"):
    import oracle
    from paper_1703_05158_amd import Lattice
    case, zp = _case()
    o = oracle.Oracle.from_case(case, init=False)
    o.set_zieb(*zp)
    o.init_fields(case.rho_init, case.u_init)
    lat = Lattice.from_case(case, storage=storage, stream=torch_stream, init=False)
    lat.set_zieb(*zp)
    lat.init_fields(case.rho_init, case.u_init)
    return o, lat, case, zp


def test_zieb_parity(torch_stream):
    o, lat, case, _ = _pair(torch_stream)
    for n in range(60):
        o.step(1)
        lat.step(1)
    pe = pop_rel_err(o, lat)
    fe, te = force_rel_err(o, lat)
    rho, H, vf = lat.zieb_state()
    print(f"pop {pe:.2e} F {fe:.2e} T {te:.2e} rho {rho:.8f} (oracle {o.zieb['rho']:.8f}) vf {vf:.3e}")
    assert pe <= 1e-5 and fe <= 1e-4 and te <= 1e-4
    assert rho == pytest.approx(o.zieb["rho"], rel=1e-6)
    assert H == pytest.approx(o.zieb["H"], rel=1e-12)
    assert vf == pytest.approx(o.zieb["vf"], abs=1e-7)
    assert rho > 1.0           # the piston has compressed the cylinder
    lat.close()


def test_zieb_checkpoint_resume(torch_stream):
    from paper_1703_05158_amd import Lattice
    _, lat, case, zp = _pair(torch_stream)
    lat.step(20)
    state = lat.get_state()
    lat.step(15)
    P_ref, z_ref = lat.get_populations(), lat.zieb_state()
    lat2 = Lattice.from_case(case, stream=torch_stream, init=False)
    lat2.set_zieb(*zp)
    lat2.set_state(state)
    lat2.step(15)
    assert np.array_equal(lat2.get_populations(), P_ref)
    assert lat2.zieb_state() == z_ref
    lat.close()
    lat2.close()


def test_zieb_rejects_bad_planes(torch_stream):
    from paper_1703_05158_amd import Batch, LBMError, Lattice
    case, (z, a, v, vp) = _case()
    lat = Lattice.from_case(case, stream=torch_stream, init=False)
    with pytest.raises(LBMError):
        lat.set_zieb(5, a, v, vp)       # the layer below z = 5 is not all wall
    with pytest.raises(LBMError):
        lat.set_zieb(z, -1.0, v, vp)
    lat.set_zieb(z, a, v, vp)
    lat.init_fields()
    with pytest.raises(LBMError):
        lat.set_zieb(z, a, v, vp)       # after lbm_init_fields
    with pytest.raises(LBMError):
        Batch([lat])
    lat.close()


def test_zieb_with_spheres_crossing_the_plane(torch_stream):
    """Drifting spheres next to the plane cover and uncover plane nodes: the
    plane mean, the density update and the redistribution then run over a
    changing set of fluid nodes, on both sides."""
    import dataclasses

    import oracle
    from paper_1703_05158_amd import Lattice
    case, zp = _case()
    X = np.array([[8.0, 7.0, 4.6], [16.0, 12.5, 5.2], [12.0, 9.0, 14.0]])
    V = np.array([[0.02, 0.01, -0.03], [-0.01, 0.02, -0.035], [0.0, 0.0, 0.01]])
    case = dataclasses.replace(case, X=X, V=V, R=np.array([3.0, 2.5, 3.5]), drift=True)
    o = oracle.Oracle.from_case(case, init=False)
    o.set_zieb(*zp)
    o.init_fields(case.rho_init, case.u_init)
    lat = Lattice.from_case(case, stream=torch_stream, init=False)
    lat.set_zieb(*zp)
    lat.init_fields(case.rho_init, case.u_init)
    covered = []
    for n in range(1, 61):
        Xn, Vn, On, Rn = case.bodies_at(n)
        o.set_bodies(Xn, Vn, On, Rn)
        lat.set_bodies(Xn, Vn, On, Rn)
        o.step(1)
        lat.step(1)
        covered.append(int((o.owner()[1] >= 0).sum()))
    np.testing.assert_array_equal(lat.get_owner(), o.owner())
    pe = pop_rel_err(o, lat)
    fe, te = force_rel_err(o, lat)
    rho, H, vf = lat.zieb_state()
    print(f"pop {pe:.2e} F {fe:.2e} T {te:.2e} rho {rho:.8f} ({o.zieb['rho']:.8f}); plane solid nodes {covered[0]}..{max(covered)}")
    assert max(covered) > min(covered)   # the plane's solid set changed
    assert pe <= 1e-5 and fe <= 1e-4 and te <= 1e-4
    assert rho == pytest.approx(o.zieb["rho"], rel=1e-6)
    lat.close()


def test_zieb_plane_wider_than_the_reduction_grid(torch_stream):
    """A plane of 520 x 520 nodes: more than the plane reduction's largest
    grid covers at one node per thread (1024 workgroups of 256), so its
    workgroups loop over the plane; the cylinder state and the populations
    against the oracle."""
    import oracle
    from paper_1703_05158_amd import Lattice
    nx, ny, nz = 520, 520, 5
    assert nx * ny > 1024 * 256
    w = np.zeros((nz, ny, nx), np.uint8)
    w[0] = 1            # the removed domain below the plane z = 1
    w[nz - 1] = 1       # closed far end
    w[:, 0, :] = 1
    rng = np.random.Generator(np.random.PCG64(41))
    case = W.Case(name="zieb_wide", nx=nx, ny=ny, nz=nz, tau0=0.8, smag_c=0.1, wall_id=w,
                  wall_vel=np.zeros((1, 3)), wall_ref=np.zeros((1, 3)),
                  X=np.array([[100.5, 200.2, 2.4]]), V=np.zeros((1, 3)), Omega=np.zeros((1, 3)), R=np.array([1.4]),
                  u_init=rng.normal(0.0, 0.005, size=(3, nz, ny, nx)))
    zp = (1, float((w[1] == 0).sum()), 2.0 * float((w == 0).sum()), 0.01)
    o = oracle.Oracle.from_case(case, init=False)
    o.set_zieb(*zp)
    o.init_fields(case.rho_init, case.u_init)
    lat = Lattice.from_case(case, stream=torch_stream, init=False)
    lat.set_zieb(*zp)
    lat.init_fields(case.rho_init, case.u_init)
    for n in range(2):
        o.step(1)
        lat.step(1)
    rho, H, vf = lat.zieb_state()
    pe = pop_rel_err(o, lat)
    print(f"pop {pe:.2e} rho {rho:.10f} (oracle {o.zieb['rho']:.10f}) vf {vf:.3e} ({o.zieb['vf']:.3e})")
    assert pe <= 1e-5
    assert rho == pytest.approx(o.zieb["rho"], rel=1e-6)
    assert vf == pytest.approx(o.zieb["vf"], abs=1e-7)
    lat.close()


@pytest.mark.parametrize("storage,pop_bar,rho_bar", [("f16", 5e-3, 1e-4), ("bf16", 4e-2, 1e-3)])
def test_zieb_reduced_precision(torch_stream, storage, pop_bar, rho_bar):
    """The inflow plane with 16-bit population storage, 30 steps.  Each
    store rounds a deviation to half a unit in its last place (2^-12 and
    2^-9 of it, up to 3e-4 and 3e-3 of the smallest weight), growing about
    like the square root of the step count: bars of 5e-3 and 4e-2 on the
    populations in units of each direction's weight.  The cylinder density
    comes from the mean over the plane's nodes, where the roundings average
    out: 1e-4 and 1e-3 relative."""
    from ._pair import pop_weight_err
    o, lat, case, _ = _pair(torch_stream, storage=storage)
    for n in range(30):
        o.step(1)
        lat.step(1)
    pe = pop_weight_err(o, lat)
    rho, H, vf = lat.zieb_state()
    print(f"{storage}: pop/w {pe:.2e} rho {rho:.8f} (oracle {o.zieb['rho']:.8f})")
    assert pe <= pop_bar
    assert rho == pytest.approx(o.zieb["rho"], rel=rho_bar)
    assert H == pytest.approx(o.zieb["H"], rel=1e-12)
    lat.close()


def test_zieb_on_the_full_duct(torch_stream):
    """The inflow-plane workload the bench times, at its full size: the
    128x128x512 duct with 4000 drifting spheres, the piston layer held still
    and the plane z = 1 fed by a virtual cylinder of the duct's cross-section
    moving at the piston's speed; 3 steps with the sphere table set before
    each, against the FP64 oracle at the step's bars and the cylinder state
    to 1e-6."""
    import dataclasses

    import oracle
    from paper_1703_05158_amd import Lattice
    from ._pair import advance
    oracle.set_threads(16)
    base = W.case_piston_duct(drift=True)
    v_piston = float(base.wall_vel[1][2])
    wv = base.wall_vel.copy()
    wv[1] = 0.0
    case = dataclasses.replace(base, wall_vel=wv)
    area = float((case.wall_id[1] == 0).sum())
    zp = (1, area, area * case.nz / 2, v_piston)
    o = oracle.Oracle.from_case(case, init=False)
    o.set_zieb(*zp)
    o.init_fields(case.rho_init, case.u_init)
    lat = Lattice.from_case(case, stream=torch_stream, init=False)
    lat.set_zieb(*zp)
    lat.init_fields(case.rho_init, case.u_init)
    advance(o, lat, case, 0, 3)
    pe = pop_rel_err(o, lat)
    fe, te = force_rel_err(o, lat)
    rho, H, vf = lat.zieb_state()
    print(f"pop {pe:.2e} F {fe:.2e} T {te:.2e} rho {rho:.10f} (oracle {o.zieb['rho']:.10f}) vf {vf:.3e}")
    assert pe <= 1e-5 and fe <= 1e-4 and te <= 1e-4
    assert rho == pytest.approx(o.zieb["rho"], rel=1e-6)
    assert H == pytest.approx(o.zieb["H"], rel=1e-12)
    assert vf == pytest.approx(o.zieb["vf"], abs=1e-7)
    lat.close()
