"""Edge cases of the geometry on the GPU, against the FP64 oracle (same bars
as the step: populations 1e-5 relative, forces and torques 1e-4
norm-relative; owner maps bit for bit).

* spheres large enough that their candidate links do not fit one list, so
  the link pass takes them in rounds of box nodes;
* overlapping spheres, a sphere overlapping a wall and spheres across the
  periodic boundary (precedence: walls, then the lower sphere index);
* a box a few nodes wide;
* no solids at all;
* random small lattices with walls and drifting, overlapping spheres;
* the full id range with spheres that cover one node or none;
* a sphere at the radius limit, next to its own periodic image.
"""
import numpy as np
import pytest

import lbm_workloads as W
from ._pair import advance, force_rel_err, make_pair, pop_rel_err

pytestmark = pytest.mark.gpu


def _check(o, lat, pop_bar=1e-5, force_bar=1e-4):
    np.testing.assert_array_equal(lat.get_owner(), o.owner())
    pe = pop_rel_err(o, lat)
    fe, te = force_rel_err(o, lat)
    print(f"pop {pe:.2e}  F {fe:.2e}  T {te:.2e}")
    assert pe <= pop_bar and fe <= force_bar and te <= force_bar


def test_large_spheres_take_rounds(torch_stream):
    rng = np.random.Generator(np.random.PCG64(21))
    R = np.array([7.8, 9.5, 11.0])
    X = np.array([[12.3, 14.1, 13.7], [36.6, 33.2, 15.4], [22.5, 30.8, 38.9]])
    case = W.Case(name="large_spheres", nx=48, ny=48, nz=52, tau0=0.65, smag_c=0.12,
                  body_force=(2e-6, 0.0, 0.0), X=X, V=rng.normal(0.0, 0.02, (3, 3)),
                  Omega=rng.normal(0.0, 0.002, (3, 3)), R=R, u_init=rng.normal(0.0, 0.01, (3, 52, 48, 48)),
                  drift=True)
    o, lat = make_pair(case, stream=torch_stream)
    advance(o, lat, case, 0, 20)
    _check(o, lat)
    lat.close()


def test_overlaps_walls_and_periodic_images(torch_stream):
    nx, ny, nz = 34, 30, 40
    w = np.zeros((nz, ny, nx), np.uint8)
    w[:, :, 0] = 1                  # wall 1: the plane x = 0 (moving along y)
    w[20:23, 10:20, 14:18] = 2      # wall 2: a block, static
    rng = np.random.Generator(np.random.PCG64(8))
    X = np.array([[2.2, 15.3, 10.4],    # overlaps wall 1
                  [8.1, 14.7, 11.2],    # overlaps sphere 0
                  [16.2, 15.1, 21.6],   # overlaps the block
                  [30.6, 0.7, 38.9],    # across three periodic boundaries
                  [20.4, 27.9, 4.1]])
    R = np.array([4.0, 4.5, 3.5, 3.2, 2.6])
    case = W.Case(name="overlaps", nx=nx, ny=ny, nz=nz, tau0=0.7, smag_c=0.1, body_force=(1e-6, 0.0, 0.0),
                  wall_id=w, wall_vel=np.array([[0.0, 0.01, 0.0], [0.0, 0.0, 0.0]]),
                  wall_ref=np.array([[0.0, 15.0, 20.0], [16.0, 15.0, 21.5]]),
                  X=X, V=rng.normal(0.0, 0.03, (5, 3)), Omega=rng.normal(0.0, 0.003, (5, 3)), R=R,
                  u_init=rng.normal(0.0, 0.01, (3, nz, ny, nx)), drift=True)
    o, lat = make_pair(case, stream=torch_stream)
    np.testing.assert_array_equal(lat.get_owner(), o.owner())
    advance(o, lat, case, 0, 25)
    _check(o, lat)
    lat.close()


def test_box_a_few_nodes_wide(torch_stream):
    rng = np.random.Generator(np.random.PCG64(5))
    case = W.Case(name="tiny", nx=8, ny=9, nz=7, tau0=0.8, smag_c=0.1, body_force=(1e-6, 0.0, 0.0),
                  X=np.array([[3.6, 4.2, 0.4]]), V=np.array([[0.05, -0.04, 0.03]]),
                  Omega=np.array([[0.0, 0.01, 0.0]]), R=np.array([2.3]),
                  u_init=rng.normal(0.0, 0.01, (3, 7, 9, 8)), drift=True)
    o, lat = make_pair(case, stream=torch_stream)
    advance(o, lat, case, 0, 30)
    _check(o, lat)
    lat.close()


def test_no_solids(torch_stream):
    case = W.case_box(n=(20, 12, 18), n_spheres=0, tau0=0.58, smag_c=0.18, body_force=(3e-6, -1e-6, 0.0),
                      u_sigma=0.02, seed=11)
    o, lat = make_pair(case, stream=torch_stream)
    advance(o, lat, case, 0, 40)
    _check(o, lat)
    F, T = lat.get_forces()
    assert F.shape == (0, 3) and T.shape == (0, 3)
    lat.close()


def test_surface_ties_decided_like_the_oracle(torch_stream):
    """Centres on a 0.1 grid and radii on a 0.5 grid put many nodes exactly,
    or within an ulp, on a sphere surface.  The owner test is an FP64
    product-sum without fused multiply-add on both sides, so the owner maps
    agree node for node: fresh, and after drift steps that vacate and stamp
    (velocities on a 0.1 grid as well)."""
    import oracle
    from paper_1703_05158_amd import Lattice
    rng = np.random.Generator(np.random.PCG64(17))
    nx, ny, nz = 40, 36, 44
    n = 60
    X = np.round(rng.uniform(0, 1, (n, 3)) * [nx, ny, nz], 1) % [nx, ny, nz]
    R = rng.integers(4, 10, n) * 0.5
    V = rng.integers(-3, 4, (n, 3)) * 0.1
    case = W.Case(name="ties", nx=nx, ny=ny, nz=nz, tau0=0.7, smag_c=0.1, X=X, V=V,
                  Omega=np.zeros((n, 3)), R=R, drift=True)
    # the first centre gives an exact tie at node (6, 9, 4) with R = 3
    case.X[0] = [8.4, 7.2, 4.6 - 0.6]
    case.R[0] = 3.0
    o = oracle.Oracle.from_case(case)
    lat = Lattice.from_case(case, stream=torch_stream)
    np.testing.assert_array_equal(lat.get_owner(), o.owner())
    assert o.owner()[4, 9, 6] == 0
    for step in range(1, 6):
        Xs, Vs, Os, Rs = case.bodies_at(step)
        o.set_bodies(Xs, Vs, Os, Rs)
        lat.set_bodies(Xs, Vs, Os, Rs)
        o.step(1)
        lat.step(1)
        np.testing.assert_array_equal(lat.get_owner(), o.owner())
    lat.close()


def _random_case(seed, v_step=0.05):
    """Random small lattice; sphere velocity components are v_step times an
    integer in [-2, 2]."""
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    nx, ny, nz = (int(v) for v in rng.integers(18, 34, 3))
    w = np.zeros((nz, ny, nx), np.uint8)
    n_walls = 3
    for k in range(1, n_walls + 1):
        a = [int(rng.integers(0, d)) for d in (nz, ny, nx)]
        e = [int(rng.integers(1, 5)), int(rng.integers(2, ny)), int(rng.integers(2, nx))]
        w[a[0]:a[0] + e[0], a[1]:a[1] + e[1], a[2]:a[2] + e[2]] = k
    nb = int(rng.integers(4, 12))
    X = np.round(rng.uniform(0, 1, (nb, 3)) * [nx, ny, nz], 1) % [nx, ny, nz]
    R = rng.integers(4, 11, nb) * 0.5
    return W.Case(name=f"random_{seed}", nx=nx, ny=ny, nz=nz, tau0=float(rng.uniform(0.55, 0.9)),
                  smag_c=float(rng.uniform(0.0, 0.2)), body_force=tuple(rng.normal(0, 2e-6, 3)),
                  wall_id=w, wall_vel=rng.normal(0, 0.01, (n_walls, 3)), wall_ref=rng.uniform(0, 20, (n_walls, 3)),
                  X=X, V=rng.integers(-2, 3, (nb, 3)) * v_step, Omega=rng.normal(0, 0.005, (nb, 3)), R=R,
                  u_init=rng.normal(0.0, 0.01, (3, nz, ny, nx)), drift=True)


@pytest.mark.parametrize("seed,storage,pop_bar,force_bar", [(1, "f16", 5e-3, 2e-2), (3, "bf16", 4e-2, 1e-1)])
def test_random_geometry_reduced_precision(torch_stream, seed, storage, pop_bar, force_bar):
    """The random lattices with 16-bit population storage.  Each store
    rounds a deviation g = f - w rho0 to half a unit in its last place,
    2^-12 |g| (FP16) or 2^-9 |g| (BF16); with |g| up to about 0.04 next to
    the fastest spheres that is 3e-4 and 3e-3 of the smallest weight (1/36),
    and over 15 steps it grows like a random walk by about 4.  The bars, on
    the population error in units of each direction's weight (a relative
    error per population is ill-conditioned where a population comes near
    zero beside a fast sphere), are 5e-3 and 4e-2; on the norm-relative
    forces 2e-2 and 1e-1.  The owner maps stay bit for bit."""
    from ._pair import pop_weight_err
    case = _random_case(seed)
    o, lat = make_pair(case, storage=storage, stream=torch_stream)
    advance(o, lat, case, 0, 15)
    np.testing.assert_array_equal(lat.get_owner(), o.owner())
    pe = pop_weight_err(o, lat)
    fe, te = force_rel_err(o, lat)
    print(f"pop/w {pe:.2e}  F {fe:.2e}  T {te:.2e}")
    assert pe <= pop_bar and fe <= force_bar and te <= force_bar
    lat.close()


@pytest.mark.parametrize("seed,halfway", [(1, False), (2, True), (3, False)])
def test_random_geometry_parity(torch_stream, seed, halfway):
    """Random small lattices: a few wall slabs and blocks (static and moving),
    spheres on a 0.1 grid (near-ties), overlaps allowed, drift with rotation;
    the same bars as the step.  Sphere speeds stay at most 0.1 per component
    (lattice Mach number well below 1, the method's regime): at speeds near
    0.35 some populations next to a sphere fall to about 1e-3 of their weight,
    and a relative bar on them would measure FP32 rounding of the larger
    populations they are made from."""
    case = _random_case(seed)
    o, lat = make_pair(case, halfway=halfway, stream=torch_stream)
    np.testing.assert_array_equal(lat.get_owner(), o.owner())
    advance(o, lat, case, 0, 15)
    _check(o, lat)
    lat.close()


@pytest.mark.parametrize("seed,halfway", [(1, False), (4, True)])
def test_random_geometry_fast_spheres(torch_stream, seed, halfway):
    """The random lattices with sphere speeds up to 0.2 per component (0.35
    in norm), FP32.  Next to such a sphere some populations fall to about
    1e-3 of their weight or change sign, so a relative error per population
    is ill-conditioned there; the error is measured in units of each
    direction's weight instead.  Bar: every step rounds each population in
    FP32 (unit roundoff 2^-24 = 6e-8 of values up to a few weights) and the
    link values combine at most three of them with coefficients of at most 6
    (3/q for q >= 1/2), so one step adds at most a few 1e-7 of a weight;
    over 15 steps 1e-5 leaves a margin of a few times.  Forces and torques
    keep the step's 1e-4 norm-relative bar.  (Seed 3 at these speeds
    diverges in the FP64 oracle itself, so it is not a parity case.)"""
    from ._pair import pop_weight_err
    case = _random_case(seed, v_step=0.1)
    assert np.max(np.abs(case.V)) == pytest.approx(0.2)
    o, lat = make_pair(case, halfway=halfway, stream=torch_stream)
    advance(o, lat, case, 0, 15)
    np.testing.assert_array_equal(lat.get_owner(), o.owner())
    pe = pop_weight_err(o, lat)
    fe, te = force_rel_err(o, lat)
    print(f"pop/w {pe:.2e}  F {fe:.2e}  T {te:.2e}")
    assert pe <= 1e-5 and fe <= 1e-4 and te <= 1e-4
    lat.close()


def test_id_range_full_with_tiny_spheres(torch_stream):
    """As many bodies as the owner codes can name (3 walls and 32763 spheres:
    the last sphere id is the largest the library accepts), most of them so
    small that they cover one node or none, overlapping, drifting; the
    owner map, populations and every body's force against the oracle."""
    rng = np.random.Generator(np.random.PCG64(77))
    nx, ny, nz = 64, 64, 48
    w = np.zeros((nz, ny, nx), np.uint8)
    w[:, :, 0] = 1
    w[10:12, 20:40, 20:44] = 2
    w[30, :, :] = 3
    nb = 32763
    X = rng.uniform(0, 1, (nb, 3)) * [nx, ny, nz]
    case = W.Case(name="tiny_many", nx=nx, ny=ny, nz=nz, tau0=0.7, smag_c=0.12, body_force=(1e-6, 0.0, 0.0),
                  wall_id=w, wall_vel=np.array([[0.0, 0.01, 0.0], [0.0, 0.0, 0.0], [0.005, 0.0, 0.0]]),
                  wall_ref=np.array([[0.0, 32.0, 24.0], [32.0, 30.0, 10.5], [32.0, 32.0, 30.0]]),
                  X=X, V=rng.normal(0.0, 0.02, (nb, 3)), Omega=rng.normal(0.0, 0.01, (nb, 3)),
                  R=rng.uniform(0.3, 1.3, nb), u_init=rng.normal(0.0, 0.01, (3, nz, ny, nx)), drift=True)
    o, lat = make_pair(case, stream=torch_stream, max_bodies=nb)
    own = o.owner()
    covering = np.unique(own[own >= 3])
    assert own.max() > 32700 and len(covering) < nb   # ids near the top; some spheres cover no node
    advance(o, lat, case, 0, 4)
    _check(o, lat)
    lat.close()


def test_sphere_at_the_radius_limit(torch_stream):
    """A sphere just below the largest radius the library accepts (half the
    smallest box side minus one): its box nearly spans the periodic lattice
    and it nearly touches its own periodic image, with a small sphere in the
    gap; drifting and spinning, both link modes."""
    rng = np.random.Generator(np.random.PCG64(31))
    nx, ny, nz = 24, 26, 28
    for halfway in (False, True):
        case = W.Case(name="radius_limit", nx=nx, ny=ny, nz=nz, tau0=0.65, smag_c=0.1, body_force=(1e-6, 0.0, 0.0),
                      X=np.array([[11.3, 12.6, 13.9], [23.4, 12.2, 13.1]]), V=np.array([[0.02, -0.01, 0.01], [0.0, 0.01, 0.0]]),
                      Omega=np.array([[0.002, 0.001, -0.003], [0.0, 0.0, 0.01]]), R=np.array([10.95, 0.9]),
                      u_init=rng.normal(0.0, 0.01, (3, nz, ny, nx)), drift=True)
        o, lat = make_pair(case, halfway=halfway, stream=torch_stream)
        np.testing.assert_array_equal(lat.get_owner(), o.owner())
        advance(o, lat, case, 0, 12)
        _check(o, lat)
        lat.close()


def test_long_axis_geometry(torch_stream):
    """Spheres straddling and drifting across the periodic ends of an
    8192-node axis, and one far from the origin: the re-rasterisation takes offsets from each
    sphere's box origin, so its FP32 bounds hold at any coordinate size.
    Owner maps bit for bit, populations and forces at the FP32 bars."""
    rng = np.random.Generator(np.random.PCG64(21))
    nx, ny, nz = 20, 18, 8192
    X = np.array([[9.3, 8.7, 8190.6], [10.1, 9.4, 1.2], [6.2, 5.5, 4096.35], [13.7, 11.1, 8185.45],
                  [9.0, 9.0, 8191.5]])
    R = np.array([4.3, 3.7, 5.1, 2.9, 3.0])
    V = np.array([[0.02, -0.01, 0.1], [-0.01, 0.02, -0.1], [0.01, 0.01, 0.05], [0.0, -0.02, 0.1],
                  [0.01, 0.0, -0.1]])
    case = W.Case(name="long_axis", nx=nx, ny=ny, nz=nz, tau0=0.7, smag_c=0.1, body_force=(0.0, 0.0, 1e-6),
                  X=X, V=V, Omega=rng.normal(0.0, 0.005, (len(R), 3)), R=R,
                  u_init=rng.normal(0.0, 0.005, (3, nz, ny, nx)), drift=True)
    o, lat = make_pair(case, stream=torch_stream)
    advance(o, lat, case, 0, 12)
    np.testing.assert_array_equal(lat.get_owner(), o.owner())
    pe = pop_rel_err(o, lat)
    fe, te = force_rel_err(o, lat)
    print(f"pop {pe:.2e}  F {fe:.2e}  T {te:.2e}")
    assert pe <= 1e-5 and fe <= 1e-4 and te <= 1e-4
    lat.close()
