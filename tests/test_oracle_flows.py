"""Oracle pins against closed-form flows (steady states of the FP64 oracle).

* Couette between walls moving at +-U with halfway bounce-back: the linear
  profile is an exact steady solution of BGK for any tau (C = 0).
* Couette with the Smagorinsky closure: uniform shear rate g = 2U/H, so the
  Hou et al. closure of Sec. 2.2 gives nu_t = C^2 g exactly and a wall stress
  rho0 (c_s^2 (tau0 - 1/2) + C^2 g) g.  The literal reading of the printed
  tau_t formula with Pi = sqrt(2 Pi:Pi) would give sqrt(2) C^2 g instead; the
  test separates the two readings by several percent.
* Body-force Poiseuille flow with halfway walls at tau = 1/2 + sqrt(3)/4 (the
  BGK case of the two-relaxation-time result Lambda = 3/16): the parabola
  F/(2 nu) (y - y1)(y2 - y) with walls midway between nodes is exact; the
  walls carry exactly N_fluid F at steady state.
* Hasimoto (1959) drag on a simple-cubic periodic array of spheres:
  F = 6 pi rho nu a U K with 1/K = 1 - 1.7601 c^(1/3) + c - 1.5593 c^2
  (1.7601 c^(1/3) = 2.8373 a/L, Hasimoto's periodic Stokeslet constant),
  U the superficial velocity.
* Stokes torque on a sphere rotating in fluid at rest: T = -8 pi rho nu a^3 Omega.
"""
import numpy as np
import pytest


def _channel(orc, ny, tau0, C, F=(0, 0, 0), Ubot=(0, 0, 0), Utop=(0, 0, 0), steps=1000):
    o = orc.Oracle(1, ny, 1, tau0, C, 1.0, F)
    wall = np.zeros((1, ny, 1), np.uint8)
    wall[0, 0, 0] = 1
    wall[0, ny - 1, 0] = 2
    o.set_walls(wall, np.array([Ubot, Utop], float))
    o.init_fields()
    o.step(steps)
    return o


H = 8
Y = np.arange(1, H + 1)


@pytest.mark.parametrize("tau0", [0.55, 0.8, 1.3])
def test_couette_linear_exact(orc, tau0):
    U = 0.01
    nu = (tau0 - 0.5) / 3
    steps = int(40 * H * H / (np.pi ** 2 * nu)) + 200
    o = _channel(orc, H + 2, tau0, 0.0, Ubot=(-U, 0, 0), Utop=(U, 0, 0), steps=steps)
    _, u = o.macro()
    np.testing.assert_allclose(u[0, 0, 1:H + 1, 0], -U + 2 * U * (Y - 0.5) / H, rtol=0, atol=1e-13)
    np.testing.assert_allclose(u[1:, 0, 1:H + 1, 0], 0, atol=1e-13)


@pytest.mark.slow
@pytest.mark.parametrize("tau0,C,steps", [(0.51, 0.4, 60000), (0.55, 0.3, 25000)])
def test_couette_smagorinsky_wall_stress(orc, tau0, C, steps):
    U = 0.01
    g = 2 * U / H
    o = _channel(orc, H + 2, tau0, C, Ubot=(-U, 0, 0), Utop=(U, 0, 0), steps=steps)
    F, _ = o.forces()
    nu_hou = (tau0 - 0.5) / 3 + C * C * g
    nu_lit = (tau0 - 0.5) / 3 + np.sqrt(2) * C * C * g
    assert F[1, 0] == pytest.approx(-nu_hou * g, rel=1e-6)      # top wall dragged back
    assert F[0, 0] == pytest.approx(+nu_hou * g, rel=1e-6)
    assert (nu_lit - nu_hou) / nu_hou > 1e-3                     # readings far apart vs rel=1e-6
    _, u = o.macro()
    np.testing.assert_allclose(u[0, 0, 1:H + 1, 0], -U + 2 * U * (Y - 0.5) / H, rtol=0, atol=1e-9)


def test_poiseuille_exact_at_magic_tau(orc):
    tau = 0.5 + np.sqrt(3) / 4
    nu = (tau - 0.5) / 3
    Fx = 1e-6
    o = _channel(orc, H + 2, tau, 0.0, F=(Fx, 0, 0), steps=6000)
    _, u = o.macro()
    exact = Fx / (2 * nu) * (Y - 0.5) * (H + 0.5 - Y)
    np.testing.assert_allclose(u[0, 0, 1:H + 1, 0], exact, rtol=1e-9, atol=0)
    F, _ = o.forces()
    np.testing.assert_allclose(F.sum(0), [Fx * H, 0, 0], rtol=1e-9, atol=1e-15)


@pytest.mark.slow
def test_hasimoto_drag(orc):
    L, a, tau, Fx = 24, 4.0, 0.8, 1e-6
    nu = (tau - 0.5) / 3
    o = orc.Oracle(L, L, L, tau, 0.0, 1.0, (Fx, 0, 0))
    o.set_bodies(np.array([[L / 2 + 0.13, L / 2 - 0.21, L / 2 + 0.07]]), np.zeros((1, 3)),
                 np.zeros((1, 3)), np.array([a]))
    o.init_fields()
    o.step(5000)
    F, _ = o.forces()
    _, u = o.macro()
    m = o.fluid_mask()
    assert F[0, 0] == pytest.approx(Fx * m.sum(), rel=0.015)          # near steady state
    U = u[0][m].sum() / L ** 3
    c = 4 / 3 * np.pi * a ** 3 / L ** 3
    K_th = 1 / (1 - 1.7601 * c ** (1 / 3) + c - 1.5593 * c * c)
    K = F[0, 0] / (6 * np.pi * nu * a * U)
    assert K == pytest.approx(K_th, rel=0.04)
    assert abs(F[0, 1]) < 1e-3 * F[0, 0] and abs(F[0, 2]) < 1e-3 * F[0, 0]


def test_rotating_sphere_torque(orc):
    L, a, tau, Om = 24, 4.0, 0.8, 1e-3
    nu = (tau - 0.5) / 3
    o = orc.Oracle(L, L, L, tau, 0.0, 1.0, (0, 0, 0))
    o.set_bodies(np.array([[L / 2 + 0.13, L / 2 - 0.21, L / 2 + 0.07]]), np.zeros((1, 3)),
                 np.array([[0, 0, Om]]), np.array([a]))
    o.init_fields()
    o.step(1000)
    F, T = o.forces()
    T_th = -8 * np.pi * nu * a ** 3 * Om
    assert T[0, 2] == pytest.approx(T_th, rel=0.05)
    assert abs(T[0, 0]) < 2e-3 * abs(T_th) and abs(T[0, 1]) < 2e-3 * abs(T_th)
