"""Reduced-precision population storage against the FP64 oracle.

The 16-bit paths store the deviations g = f - w_i rho0 as FP16 or BF16
(round to nearest even) and keep the collision in FP32 and the force and
torque sums in FP64.  Every step rounds each stored deviation with a
relative error of at most the unit roundoff eps of the format (2^-11 for
FP16, 2^-8 for BF16), so the errors against the oracle scale with eps; the
bars below are stated as multiples of eps and hold for both formats:

    populations   max |P - P_ref| / |P_ref|                 <= 0.05 eps
    density       max |rho - rho_ref|                       <= 0.01 eps
    velocity      max |u - u_ref|                           <= 0.01 eps
    force         max_b |F_b - F_ref,b| / max_b |F_ref,b|   <= 3 eps
    torque        same norm                                 <= 8 eps

(32^3 parity case, 100 steps; FP16 errors are about a fifth of these bars,
BF16 errors about a sixth.)  The statement for the 128x128x512 piston duct
after 1000 steps compares against the stored oracle run in
tests/golden/duct_reference.npz.
"""
import os

import numpy as np
import pytest

import lbm_workloads as W
from ._pair import advance, force_rel_err, make_pair, pop_rel_err

pytestmark = pytest.mark.gpu

EPS = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "duct_reference.npz")


def _macro_err(o, lat):
    m = o.fluid_mask()
    ro, uo = o.macro()
    rg, ug = lat.get_macro()
    return float(np.max(np.abs(rg[m] - ro[m]))), float(np.max(np.linalg.norm(ug[:, m] - uo[:, m], axis=0)))


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_box32_reduced_precision_error(storage, torch_stream):
    case = W.case_box()
    o, lat = make_pair(case, storage=storage, stream=torch_stream)
    advance(o, lat, case, 0, case.steps)
    eps = EPS[storage]
    pe = pop_rel_err(o, lat)
    dr, du = _macro_err(o, lat)
    fe, te = force_rel_err(o, lat)
    print(f"{storage}: pop {pe:.2e} rho {dr:.2e} u {du:.2e} F {fe:.2e} T {te:.2e}")
    assert pe <= 0.05 * eps
    assert dr <= 0.01 * eps
    assert du <= 0.01 * eps
    assert fe <= 3 * eps
    assert te <= 8 * eps
    lat.close()


def test_reduced_precision_is_not_fp32(torch_stream):
    """The 16-bit paths really round: their state differs from FP32's."""
    case = W.case_box(n=(24, 20, 28), n_spheres=3, radius=(3.0, 3.0), seed=4)
    from paper_1703_05158_amd import Lattice
    P = {}
    for st in ("f32", "f16", "bf16"):
        lat = Lattice.from_case(case, storage=st, stream=torch_stream)
        lat.step(5)
        P[st] = lat.get_populations()
        assert lat.info()["storage_bytes"] == (4 if st == "f32" else 2)
        lat.close()
    d16 = np.max(np.abs(P["f16"] - P["f32"]))
    db = np.max(np.abs(P["bf16"] - P["f32"]))
    assert 0 < d16 < db


@pytest.mark.skipif(not os.path.exists(REF), reason="duct_reference.npz not generated")
def test_duct_precision_statement(torch_stream):
    """Density, velocity and force error of each storage format after 100 and
    1000 steps of the piston duct, against the stored FP64 oracle run."""
    import torch
    from paper_1703_05158_amd import Lattice
    ref = np.load(REF)
    marks = [int(s) for s in ref["steps"]]
    case = W.case_piston_duct(drift=True)
    nb = case.n_bodies
    tabs = torch.empty((marks[-1], nb, 10), dtype=torch.float64, device="cuda")
    for n in range(1, marks[-1] + 1):
        X, V, Om, R = case.bodies_at(n)
        tabs[n - 1] = torch.from_numpy(np.concatenate([X, V, Om, R[:, None]], 1))
    bars = {"f32": (1e-4, 1e-4, 1e-3), "f16": (1e-2, 1e-2, 3e-2), "bf16": (5e-2, 5e-2, 1e-1)}
    for st in ("f32", "f16", "bf16"):
        lat = Lattice.from_case(case, storage=st, stream=torch_stream)
        for n in range(1, marks[-1] + 1):
            lat.set_bodies_device(nb, tabs[n - 1])
            lat.step(1)
            if n in marks:
                idx = ref[f"idx_{n}"]
                rho, u = lat.get_macro()
                assert np.all(lat.get_owner().ravel()[idx] < 0)
                dr = np.max(np.abs(rho.ravel()[idx] - ref[f"rho_{n}"]))
                ur = ref[f"u_{n}"]
                umax = np.max(np.linalg.norm(ur, axis=0))
                du = np.max(np.linalg.norm(u.reshape(3, -1)[:, idx] - ur, axis=0)) / umax
                F, T = lat.get_forces()
                Fr = ref[f"F_{n}"]
                fe = np.max(np.linalg.norm(F - Fr, axis=1)) / np.max(np.linalg.norm(Fr, axis=1))
                print(f"{st} step {n}: rho {dr:.2e}  u/umax {du:.2e}  F {fe:.2e}")
                br, bu, bf = bars[st]
                assert dr <= br and du <= bu and fe <= bf
        lat.close()
