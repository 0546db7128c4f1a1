"""Pins of the oracle's Zoom-in with Effective Boundaries inflow (Sec. 2.6).

The removed domain is a cylinder of volume V0 and piston area A whose fluid,
of uniform density rho, is pushed through the plane z = 1 by a piston moving
at v_p; the layer z = 0 stands for the removed domain.  Checked here:

  * the density update of eq. (ZIEBdesity8), iterated with a constant
    interface velocity, converges to the exact solution of eq. (mass_conv),
    rho(t) = rho0 (1 - A v_p t / V0)^(-(v_p - v_f) / v_p), as the step shrinks;
  * a fluid at rest with the piston at rest is a fixed point;
  * after every step the plane holds the equilibrium at the cylinder's new
    density and the plane's velocity (eq. ZIEBdesity9 then the equilibrium
    redistribution), with exactly that density;
  * the mass balance behind eq. (mass_conv): in a duct closed at its far end,
    the mass of the cylinder, rho (V0 - A H_p), plus the mass in the simulated
    domain stays constant while the piston pushes, up to the explicit time
    integration of eq. (ZIEBdesity8); the cylinder's density rises.
"""
import numpy as np
import pytest


def _closed_duct(nx=12, ny=12, nz=40):
    w = np.zeros((nz, ny, nx), np.uint8)
    w[:, :, 0] = w[:, :, nx - 1] = 1
    w[:, 0, :] = w[:, ny - 1, :] = 1
    w[0] = 1           # stands for the removed domain below the plane z = 1
    w[nz - 1] = 1      # closed far end
    return w


def _oracle(orc, vp, v0_over_domain, tau0=0.8, C=0.0, u=None):
    w = _closed_duct()
    nz, ny, nx = w.shape
    o = orc.Oracle(nx, ny, nz, tau0, C)
    o.set_walls(w, np.zeros((1, 3)))
    o.init_fields(None, u)
    fluid = w == 0
    area = float(fluid[1].sum())
    vdom = float(fluid.sum())
    o.set_zieb(1, area, v0_over_domain * vdom, vp)
    return o, fluid, area, vdom


@pytest.mark.parametrize("vf", [0.004, 0.0, 0.013])
def test_density_update_integrates_the_mass_balance(orc, vf):
    A, V0, vp, T = 100.0, 1000.0, 0.01, 500.0   # the piston sweeps half the cylinder
    exact = (1.0 - A * vp * T / V0) ** (-(vp - vf) / vp)
    errs = []
    for k in (1, 4):                            # time step 1/k, scaled to lattice time
        rho, H = 1.0, 0.0
        for _ in range(int(T * k)):
            rho = orc.lib().orc_zieb_density(rho, vp / k, vf / k, A, V0, H)
            H += vp / k
        errs.append(abs(rho - exact))
    assert errs[0] < 2e-3 * exact                # within the explicit integration error
    assert errs[1] < 0.3 * errs[0]               # first order: shrinks with the step


def test_rest_is_a_fixed_point(orc):
    o, *_ = _oracle(orc, 0.0, 4.0)
    P0 = o.populations().copy()
    o.step(6)
    assert np.max(np.abs(o.populations() - P0)) < 1e-14
    assert o.zieb["rho"] == pytest.approx(1.0, abs=1e-15)


def test_plane_is_equilibrium_at_cylinder_density(orc):
    rng = np.random.Generator(np.random.PCG64(5))
    u0 = rng.normal(0.0, 0.01, size=(3, 40, 12, 12))
    o, fluid, *_ = _oracle(orc, 0.01, 2.0, C=0.1, u=u0)
    for _ in range(8):
        o.step(1)
        rho_c = o.zieb["rho"]
        P = o.populations()
        rho, u = o.macro()
        plane = np.argwhere(fluid[1])
        for y, x in plane[::7]:
            feq = orc.equilibrium(rho_c, u[:, 1, y, x])
            assert np.max(np.abs(P[:, 1, y, x] - feq)) < 1e-14
            assert rho[1, y, x] == pytest.approx(rho_c, abs=1e-14)


@pytest.mark.parametrize("v0_over_domain", [4.0, 1.0])
def test_cylinder_and_domain_mass_balance(orc, v0_over_domain):
    vp = 0.002
    o, fluid, area, vdom = _oracle(orc, vp, v0_over_domain)
    V0 = v0_over_domain * vdom
    m0 = V0 + vdom            # both at density 1
    rho_prev = 1.0
    for n in range(1, 401):
        o.step(1)
        assert o.zieb["rho"] > rho_prev    # the piston compresses the cylinder
        rho_prev = o.zieb["rho"]
    rho, _ = o.macro()
    H = o.zieb["H"]
    assert H == pytest.approx(400 * vp)
    mass = o.zieb["rho"] * (V0 - area * H) + rho[fluid].sum()
    injected = o.zieb["rho"] * area * H   # mass the piston displaced, to first order
    assert abs(mass - m0) < 0.02 * injected
