"""Oracle pins for the step: invariants, brute force on tiny inputs, symmetry.

What pins what:
* fixed point / uniform acceleration -- equilibrium, Guo source, half-force
  velocity shift (closed forms of a spatially uniform state);
* exact mass and momentum balances -- streaming, link completeness, the
  sign and normalisation of the momentum-exchange force (Sec. 2.3);
* quiescent body -- interpolation weights of both Bouzidi branches sum to one
  and the force/torque assembly cancels around closed bodies;
* single moving voxel -- sign and size of the moving-boundary term
  (eq. moving_boundary_velocity) against the hand-derived F = -2 rho0 U;
* brute-force links -- link enumeration, q found by bisection, pull
  indexing, torque arm, solid velocity (tiny boxes);
* Bouzidi continuity at q = 1/2 (the two branches of Sec. 2.3 meet);
* owner map against an all-pairs check; refill of uncovered nodes;
* integer shift and 90-degree rotation covariance (table consistency).
"""
import numpy as np
import pytest

import lbm_workloads as W


def _oracle(orc, n, tau0=0.7, C=0.0, F=(0, 0, 0), halfway=False):
    return orc.Oracle(n[0], n[1], n[2], tau0, C, 1.0, F, halfway=halfway)


def _rand_state(o, rng, amp=0.05):
    c, w, _ = _tables(o)
    P = w[:, None] * (1.0 + amp * rng.standard_normal((19, o.N)))
    o.P = np.ascontiguousarray(P.reshape(-1))


def _tables(o):
    import oracle
    return oracle.tables()


def test_fixed_point_uniform_state(orc):
    o = _oracle(orc, (6, 5, 4), tau0=0.63, C=0.17)
    u0 = np.array([0.03, -0.02, 0.01])
    o.init_fields(np.full((4, 5, 6), 1.0), np.broadcast_to(u0[:, None, None, None], (3, 4, 5, 6)))
    P0 = o.P.copy()
    o.step(5)
    np.testing.assert_allclose(o.P, P0, rtol=0, atol=2e-16)


def test_uniform_acceleration_guo(orc):
    """Guo forcing adds exactly F of momentum per node per step; rho stays."""
    F = np.array([2e-5, -1e-5, 3e-6])
    o = _oracle(orc, (5, 4, 3), tau0=0.8, C=0.2, F=F)
    u0 = np.array([0.01, 0.02, -0.015])
    o.init_fields(None, np.broadcast_to(u0[:, None, None, None], (3, 3, 4, 5)))
    c, _, _ = orc.tables()
    for n in range(1, 8):
        o.step(1)
        P = o.populations().reshape(19, -1)
        j = c.T.astype(float) @ P
        rho = P.sum(0)
        np.testing.assert_allclose(rho, 1.0, rtol=0, atol=1e-14)
        np.testing.assert_allclose(j, (u0 + n * F)[:, None] * np.ones((1, o.N)), rtol=0, atol=1e-15)
        # velocity used by the collision of step n: u0 + (n - 1/2) F
        rho_m, u_m = o.macro()
        np.testing.assert_allclose(u_m.reshape(3, -1), (u0 + (n - 0.5) * F)[:, None] * np.ones((1, o.N)),
                                   rtol=0, atol=1e-15)


def _fluid_momentum(o, c):
    P = o.populations().reshape(19, -1)
    m = o.fluid_mask().reshape(-1)
    return c.T.astype(float) @ P[:, m].sum(1), m.sum()


@pytest.mark.parametrize("halfway", [False, True])
def test_momentum_balance_exact(orc, halfway):
    """M_n - M_{n-1} = N_fluid F - sum_b F_b for fixed geometry (moving surfaces)."""
    case = W.case_box(n=(14, 12, 16), n_spheres=3, radius=(2.2, 3.1), tau0=0.66, smag_c=0.15,
                      body_force=(3e-5, -2e-5, 1e-5), u_sigma=0.02, v_sigma=0.01, w_sigma=0.003, seed=5)
    wall = np.zeros(case.shape, np.uint8)
    wall[:, 0, :] = 1
    wall[:, 6, 2:5] = 2
    case.wall_id, case.wall_vel, case.wall_ref = wall, np.array([[0.01, 0, 0.005], [0, 0.0, -0.01]]), None
    o = orc.Oracle.from_case(case, halfway=halfway)
    c, _, _ = orc.tables()
    F = np.array(case.body_force)
    M0, nf = _fluid_momentum(o, c)
    for _ in range(4):
        o.step(1)
        M1, _ = _fluid_momentum(o, c)
        Fb, _ = o.forces()
        np.testing.assert_allclose(M1 - M0, nf * F - Fb.sum(0), rtol=0, atol=1e-11)
        M0 = M1


def test_mass_exact_halfway_moving_surfaces(orc):
    """Halfway bounce-back with rigidly moving spheres and walls conserves mass."""
    case = W.case_box(n=(12, 12, 12), n_spheres=2, radius=(2.5, 3.0), tau0=0.7, smag_c=0.1,
                      u_sigma=0.02, v_sigma=0.01, w_sigma=0.004, seed=2)
    o = orc.Oracle.from_case(case, halfway=True)
    m = o.fluid_mask()
    M0 = o.populations()[:, m].sum()
    o.step(6)
    assert o.populations()[:, m].sum() == pytest.approx(M0, rel=1e-14)


def test_mass_exact_piston_treadmill_halfway(orc):
    """Small duct: static walls, moving piston pushing on one face and
    withdrawing on the periodic other face, halfway links: exact mass."""
    case = W.case_duct(nx=12, ny=12, nz=24, n_spheres=0, orifice_z=16, orifice_thick=2,
                       orifice_r_in=2.0, orifice_gap=2.0, pack_z=(4, 12), seed=3, steps=5)
    o = orc.Oracle.from_case(case, halfway=True)
    m = o.fluid_mask()
    M0 = o.populations()[:, m].sum()
    o.step(5)
    assert o.populations()[:, m].sum() == pytest.approx(M0, rel=1e-14)


def test_quiescent_body_feels_nothing(orc):
    """Fluid and bodies at rest: every Bouzidi branch returns w_k rho0, F = T = 0."""
    case = W.case_box(n=(20, 18, 22), n_spheres=5, radius=(2.0, 4.5), u_sigma=0.0,
                      body_force=(0, 0, 0), gap=2.0, seed=7)
    o = orc.Oracle.from_case(case)
    o.step(2)
    F, T = o.forces()
    assert np.abs(F).max() < 1e-13 and np.abs(T).max() < 1e-13
    _, w, _ = orc.tables()
    m = o.fluid_mask()
    np.testing.assert_allclose(o.populations()[:, m], np.broadcast_to(w[:, None], (19, m.sum())),
                               rtol=0, atol=1e-15)


def test_single_moving_voxel_force(orc):
    """One wall voxel moving at U in fluid at rest, one step.

    Each of the 18 neighbours x = s - c_k reflects f_i = w_k (1 + 6 c_i.U),
    so the momentum exchanged is sum_k (2 w_k - 6 w_k c_k.U) c_k = -2 rho0 U
    (sum_k w_k c_k c_k = I/3).  Torque about ref: (s - ref) x F.
    """
    n = (7, 6, 5)
    s = np.array([3, 2, 2])
    U = np.array([0.02, -0.01, 0.005])
    ref = s + np.array([1.0, 2.0, 3.0])
    o = _oracle(orc, n, tau0=0.9)
    wall = np.zeros((n[2], n[1], n[0]), np.uint8)
    wall[s[2], s[1], s[0]] = 1
    o.set_walls(wall, U[None], ref[None])
    o.init_fields()
    f, F, T = o.stream()
    np.testing.assert_allclose(F[0], -2.0 * U, rtol=1e-13, atol=1e-17)
    np.testing.assert_allclose(T[0], np.cross(s - ref, -2.0 * U), rtol=1e-12, atol=1e-17)
    c, w, opp = orc.tables()
    f = f.reshape(19, n[2], n[1], n[0])
    for k in range(1, 19):
        x = s - c[k]
        i = opp[k]
        assert f[i, x[2], x[1], x[0]] == pytest.approx(w[k] * (1 + 6 * c[i] @ U), rel=1e-14)


def _brute_owner(n, wall, X, R, nwalls):
    nx, ny, nz = n
    own = np.full((nz, ny, nx), -1, np.int64)
    box = np.array([nx, ny, nz], float)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    p = np.stack([x, y, z], -1).astype(float)
    for b in range(len(R)):
        d = p - X[b]
        d -= box * np.round(d / box)
        inside = (d * d).sum(-1) <= R[b] ** 2
        own[(own < 0) & inside] = nwalls + b
    if wall is not None:
        own[wall > 0] = wall[wall > 0].astype(np.int64) - 1
    return own


def test_owner_map_all_pairs(orc):
    rng = np.random.default_rng(11)
    n = (9, 8, 10)
    X = rng.random((6, 3)) * np.array(n)
    R = 1.2 + 2.0 * rng.random(6)   # overlapping on purpose
    wall = np.zeros((n[2], n[1], n[0]), np.uint8)
    wall[:, 0, :] = 1
    wall[3, :, 4] = 2
    o = _oracle(orc, n)
    o.set_walls(wall, np.zeros((2, 3)))
    o.set_bodies(X, np.zeros((6, 3)), np.zeros((6, 3)), R)
    np.testing.assert_array_equal(o.own.reshape(n[2], n[1], n[0]), _brute_owner(n, wall, X, R, 2))


def _brute_stream(P, own, n, X, V, Om, R, nwalls, Uw, halfway=False):
    """Independent enumeration of links with q by bisection (tiny boxes only)."""
    import oracle
    c, w, opp = oracle.tables()
    nx, ny, nz = n
    box = np.array(n, float)
    P = P.reshape(19, nz, ny, nx)
    own = own.reshape(nz, ny, nx)
    f = np.full((19, nz, ny, nx), np.nan)
    nb = len(R)
    F = np.zeros((nb + nwalls, 3))
    T = np.zeros((nb + nwalls, 3))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if own[z, y, x] >= 0:
                    continue
                xv = np.array([x, y, z])
                f[0, z, y, x] = P[0, z, y, x]
                for i in range(1, 19):
                    src = (xv - c[i]) % np.array(n)
                    o = own[src[2], src[1], src[0]]
                    if o < 0:
                        f[i, z, y, x] = P[i, src[2], src[1], src[0]]
                        continue
                    k = opp[i]          # link direction x -> solid
                    ck = c[k].astype(float)
                    if o < nwalls:
                        q = 0.5
                        uw = Uw[o]
                        arm = None
                    else:
                        b = o - nwalls
                        d = xv - X[b]
                        d -= box * np.round(d / box)
                        g = lambda s: ((d + s * ck) ** 2).sum() - R[b] ** 2
                        lo, hi = 0.0, 1.0
                        assert g(lo) > 0 and g(hi) <= 0
                        for _ in range(200):
                            mid = 0.5 * (lo + hi)
                            if g(mid) > 0:
                                lo = mid
                            else:
                                hi = mid
                        q = 0.5 if halfway else hi
                        arm = d + q * ck
                        uw = V[b] + np.cross(Om[b], arm)
                    cu = c[i] @ uw
                    fk = P[k, z, y, x]
                    if q < 0.5:
                        back = (xv - c[k]) % np.array(n)
                        if own[back[2], back[1], back[0]] < 0:
                            val = 2 * q * fk + (1 - 2 * q) * P[k, back[2], back[1], back[0]] + 6 * w[k] * cu
                        else:
                            val = fk + 6 * w[k] * cu
                    else:
                        val = fk / (2 * q) + (2 * q - 1) / (2 * q) * P[i, z, y, x] + 3 / q * w[k] * cu
                    f[i, z, y, x] = val
                    slot = (o - nwalls) if o >= nwalls else nb + o
                    mom = (fk + val) * ck
                    F[slot] += mom
                    if arm is not None:
                        T[slot] += np.cross(arm, mom)
    return f, F, T


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_stream_brute_force_sphere(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = (7, 8, 6)
    nb = 2
    R = np.array([1.7, 1.35])
    while True:
        X = rng.random((nb, 3)) * np.array(n)
        if W.min_tie_gap(X, R, n) > 1e-3:
            break
    V = rng.normal(0, 0.02, (nb, 3))
    Om = rng.normal(0, 0.01, (nb, 3))
    o = _oracle(orc, n)
    wall = np.zeros((n[2], n[1], n[0]), np.uint8)
    wall[0, 0, :] = 1
    Uw = np.array([[0.01, 0.0, -0.02]])
    o.set_walls(wall, Uw)
    o.set_bodies(X, V, Om, R)
    o.init_fields()
    _rand_state(o, rng)
    f, F, T = o.stream()
    fb, Fb, Tb = _brute_stream(o.P, o.own, n, X, V, Om, R, 1, Uw)
    m = o.fluid_mask()
    np.testing.assert_allclose(f.reshape(19, *m.shape)[:, m], fb[:, m], rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(F, Fb, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(T[:nb], Tb[:nb], rtol=1e-12, atol=1e-15)


def _link_q(xv, ck, Xb, R, box):
    """Fraction of the link xv -> xv + ck inside the fluid, by bisection."""
    d = xv - Xb
    d -= box * np.round(d / box)
    g = lambda s: ((d + s * ck) ** 2).sum() - R ** 2
    lo, hi = 0.0, 1.0
    assert g(lo) > 0 and g(hi) <= 0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            lo = mid
        else:
            hi = mid
    return hi


@pytest.mark.parametrize("seed", [0, 1])
def test_bouzidi_reads_a_linear_field_at_the_characteristic_foot(orc, seed):
    """Interpolated bounce-back (Sec. 2.3) follows the particle that reaches
    the fluid node x along k' = opposite(k) after one step: it travels one
    link length with a specular reflection at the wall, a fraction q of the
    link x -> x + c_k away.  For q < 1/2 it left x - (1 - 2q) c_k moving
    along k; the rule interpolates the k population linearly between x - c_k
    and x, so when that population is a linear function G of the position on
    the link's line, the value received is G at that foot point.  For
    q >= 1/2 the particle reflected from x ends the step at x + (2q - 1) c_k
    and the rule interpolates linearly, at x, between it and the k' particle
    leaving x towards x - c_k; with the two values taken from one linear G
    on the line (G at x + (2q - 1) c_k for the reflected one, G at x - c_k for
    the other), the value received is G(x).  A swapped weight, a wrong
    second population or a misplaced interpolation point in either branch
    moves the point at which G is read.  Each link gets its own random G;
    the sphere is at rest, so the moving-boundary term is zero; q by
    bisection; links that would share a population are left out."""
    import oracle
    c, w, opp = oracle.tables()
    rng = np.random.default_rng(40 + seed)
    n = (18, 17, 19)
    box = np.array(n, float)
    X = np.array([[8.6 + 0.3 * seed, 8.2, 9.3 - 0.2 * seed]])
    R = np.array([4.4 + 0.3 * seed])
    o = _oracle(orc, n)
    o.set_bodies(X, np.zeros((1, 3)), np.zeros((1, 3)), R)
    o.init_fields()
    own = o.own.reshape(n[2], n[1], n[0])
    P = np.broadcast_to(w[:, None, None, None], (19, n[2], n[1], n[0])).copy()
    set_by = {}
    links = []
    for z, y, x in zip(*np.nonzero(own < 0)):
        xv = np.array([x, y, z])
        for k in range(1, 19):
            p = (xv + c[k]) % n
            if own[p[2], p[1], p[0]] < 0:
                continue
            q = _link_q(xv.astype(float), c[k].astype(float), X[0], R[0], box)
            back = (xv - c[k]) % n
            behind = own[back[2], back[1], back[0]] < 0
            a, b = w[k] * (1 + 0.1 * rng.standard_normal()), 0.05 * w[k] * rng.standard_normal()
            if q < 0.5 and behind:
                # G(s) = a + b s, s measured from x along c_k
                entries = {(k, z, y, x): a, (k, back[2], back[1], back[0]): a - b}
                expect = a - b * (1 - 2 * q)
            elif q >= 0.5:
                entries = {(k, z, y, x): a + b * (2 * q - 1), (opp[k], z, y, x): a - b}
                expect = a
            else:
                continue
            if any(e in set_by for e in entries):
                continue
            for e, v in entries.items():
                set_by[e] = (z, y, x, k)
                P[e] = v
            links.append((opp[k], z, y, x, expect, q))
    # every population a link reads must be one this test set for that link
    for i, z, y, x, _, _ in links:
        k = opp[i]
        for e in ((k, z, y, x), (i, z, y, x)):
            assert set_by.get(e, (z, y, x, k)) == (z, y, x, k)
    o.P = np.ascontiguousarray(P.reshape(-1))
    f, _, _ = o.stream()
    f = f.reshape(19, n[2], n[1], n[0])
    qs = np.array([l[5] for l in links])
    assert (qs < 0.5).sum() > 100 and (qs >= 0.5).sum() > 100
    got = np.array([f[i, z, y, x] for i, z, y, x, _, _ in links])
    want = np.array([l[4] for l in links])
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=0)


def test_bouzidi_continuous_at_half(orc):
    """Shifting a sphere so one link's q crosses 1/2 changes f only by O(shift)."""
    rng = np.random.default_rng(3)
    n = (12, 9, 9)
    R = np.array([2.3])
    V = np.array([[0.01, 0.02, -0.01]])
    Om = np.zeros((1, 3))
    outs = []
    for eps in (-1e-9, 1e-9):
        X = np.array([[3 + 0.5 + R[0] + eps, 4.0, 4.0]])
        o = _oracle(orc, n)
        o.set_bodies(X, V, Om, R)
        o.init_fields()
        _rand_state(o, np.random.default_rng(3))
        f, F, T = o.stream()
        outs.append((f.reshape(19, -1)[:, o.fluid_mask().reshape(-1)], F))
    assert W.min_tie_gap(np.array([[3 + 0.5 + R[0], 4.0, 4.0]]), R, n) > 1e-3
    np.testing.assert_allclose(outs[0][0], outs[1][0], rtol=0, atol=1e-8)
    np.testing.assert_allclose(outs[0][1], outs[1][1], rtol=0, atol=1e-8)


def test_uncovered_node_gets_previous_solid_equilibrium(orc):
    n = (12, 10, 10)
    R = np.array([2.6])
    X0 = np.array([[5.3, 4.6, 5.1]])
    V0 = np.array([[0.03, -0.01, 0.02]])
    Om0 = np.array([[0.0, 0.01, 0.02]])
    o = _oracle(orc, n)
    o.set_bodies(X0, V0, Om0, R)
    o.init_fields()
    o.step(1)
    X1 = X0 + np.array([[0.8, 0.0, 0.0]])
    o.set_bodies(X1, 2 * V0, -Om0, R)
    own0 = o.own_prev.reshape(n[2], n[1], n[0])
    own1 = o.own.reshape(n[2], n[1], n[0])
    unc = np.argwhere((own0 >= 0) & (own1 < 0))
    assert len(unc) > 0
    f, _, _ = o.stream()
    f = f.reshape(19, n[2], n[1], n[0])
    _, w, _ = orc.tables()
    for z, y, x in unc:
        d = np.array([x, y, z]) - X0[0]
        us = V0[0] + np.cross(Om0[0], d)
        assert f[0, z, y, x] == pytest.approx(w[0] * (1 - 1.5 * us @ us), rel=1e-14)


def _run(orc, case, steps, halfway=False):
    o = orc.Oracle.from_case(case, halfway=halfway)
    o.step(steps)
    return o


def test_integer_shift_covariance(orc):
    case = W.case_box(n=(10, 12, 9), n_spheres=2, radius=(2.0, 2.8), tau0=0.65, smag_c=0.14,
                      body_force=(1e-5, 2e-5, 0), u_sigma=0.02, v_sigma=0.01, w_sigma=0.005, seed=9)
    a = _run(orc, case, 3)
    sh = np.array([3, -2, 4])
    case2 = W.Case(**{**case.__dict__})
    case2.X = np.mod(case.X + sh, [10, 12, 9])
    case2.u_init = np.roll(case.u_init, shift=(sh[2], sh[1], sh[0]), axis=(1, 2, 3))
    b = _run(orc, case2, 3)
    Pa = np.roll(a.populations(), shift=(sh[2], sh[1], sh[0]), axis=(1, 2, 3))
    np.testing.assert_allclose(b.populations(), Pa, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(b.forces()[0], a.forces()[0], rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(b.forces()[1], a.forces()[1], rtol=1e-9, atol=1e-14)


def test_rotation_covariance(orc):
    """Rotate everything by +90 degrees about z: (x, y) -> (-y, x)."""
    n = 10
    case = W.case_box(n=(n, n, 8), n_spheres=2, radius=(2.0, 2.6), tau0=0.7, smag_c=0.12,
                      body_force=(1e-5, -3e-5, 2e-5), u_sigma=0.02, v_sigma=0.01, w_sigma=0.005, seed=4)
    a = _run(orc, case, 3)
    c, _, _ = orc.tables()
    rot = lambda v: np.stack([-v[..., 1], v[..., 0], v[..., 2]], -1)
    perm = [int(np.nonzero((c == rot(c[i])).all(1))[0][0]) for i in range(19)]
    case2 = W.Case(**{**case.__dict__})
    case2.X = np.mod(rot(case.X), n)
    case2.V, case2.Omega = rot(case.V), rot(case.Omega)
    case2.body_force = tuple(rot(np.array(case.body_force)))

    def rot_field(fld):   # fld[..., z, y, x] -> value at (x', y') = (-y, x)
        out = np.empty_like(fld)
        for y in range(n):
            for x in range(n):
                out[..., (x) % n, (-y) % n] = fld[..., y, x]
        return out
    u = case.u_init
    case2.u_init = np.stack([-rot_field(u[1]), rot_field(u[0]), rot_field(u[2])])
    b = _run(orc, case2, 3)
    Pa = a.populations()
    Pr = np.empty_like(Pa)
    for i in range(19):
        Pr[perm[i]] = rot_field(Pa[i])
    np.testing.assert_allclose(b.populations(), Pr, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(b.forces()[0], rot(a.forces()[0]), rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(b.forces()[1], rot(a.forces()[1]), rtol=1e-9, atol=1e-14)
