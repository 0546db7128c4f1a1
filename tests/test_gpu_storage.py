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


def _bf16_nearest_even(x32):
    """FP32 values rounded to BF16 by the definition of round to nearest,
    ties to even: of the two BF16 neighbours (the value with its low 16 bits
    cut, and the next one away from zero) the nearer, on a tie the one whose
    last kept bit is 0.  Distances in FP64, where they are exact."""
    u = x32.view(np.uint32).astype(np.uint64)
    lo = (u >> 16) << 16
    hi = lo + (1 << 16)
    as_f = lambda b: b.astype(np.uint32).view(np.float32).astype(np.float64)
    x, xl, xh = x32.astype(np.float64), as_f(lo), as_f(hi)
    dl, dh = np.abs(x - xl), np.abs(xh - x)
    odd = ((lo >> 16) & 1) == 1
    return np.where((dh < dl) | ((dh == dl) & odd), xh, xl)


def _rounding_cases(rng, n):
    """n FP32 deviations per direction with 2^-30 <= |g| <= 2^-8 (so that
    g + w rho0 and its difference with w rho0 are exact in FP64 for every
    weight), mixing random values with the cases rounding decides on:
    BF16 ties and near-ties, FP16 ties and near-ties in the normal range,
    and FP16 subnormal ties (odd multiples of 2^-25)."""
    k = n // 8
    sign = lambda m: np.where(rng.random(m) < 0.5, -1.0, 1.0)
    mag = lambda m: rng.uniform(1.0, 2.0, m) * 2.0 ** rng.integers(-30, -8, m)
    parts = [(sign(2 * k) * mag(2 * k)).astype(np.float32)]
    base = (sign(k) * mag(k)).astype(np.float32).view(np.uint32)
    for low in (0x8000, 0x7FFF, 0x8001):  # BF16: tie, just below, just above
        parts.append(((base & np.uint32(0xFFFF0000)) | np.uint32(low)).view(np.float32))
    b16 = (sign(k) * rng.uniform(1.0, 2.0, k) * 2.0 ** rng.integers(-14, -8, k)).astype(np.float32).view(np.uint32)
    for low in (0x1000, 0x0FFF):  # FP16 (13 bits dropped in its normal range): tie, just below
        parts.append(((b16 & np.uint32(0xFFFFE000)) | np.uint32(low)).view(np.float32))
    odd = 2 * rng.integers(0, 256, n - 7 * k) + 1  # FP16 subnormal ties
    parts.append((sign(n - 7 * k) * odd * 2.0 ** -25).astype(np.float32))
    g = np.concatenate(parts)
    rng.shuffle(g)
    return g


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_storage_rounds_to_nearest_even(storage, torch_stream):
    """R19: a stored deviation is the FP32 deviation rounded to nearest, ties
    to even (FP16 with subnormals, by numpy's IEEE conversion; BF16 by the
    definition above; FP32 unchanged).  Populations set through the C ABI
    and read back give the stored values exactly: with rho0 = 1 and the
    deviations of _rounding_cases, f = g + w, g = f - w and f' = h + w are all
    exact in FP64, on the host and in the library."""
    from paper_1703_05158_amd import Lattice
    case = W.case_box(n=(16, 16, 16), n_spheres=0, seed=2)
    lat = Lattice.from_case(case, storage=storage, stream=torch_stream)
    import oracle
    c, wt, _ = oracle.tables()
    w = np.asarray(wt, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(19))
    N = 16 ** 3
    g = np.stack([_rounding_cases(rng, N) for _ in range(19)]).reshape(19, 16, 16, 16)
    f = g.astype(np.float64) + w[:, None, None, None]
    assert np.array_equal(f - w[:, None, None, None], g.astype(np.float64))
    lat.set_populations(f)
    h = lat.get_populations() - w[:, None, None, None]
    if storage == "f32":
        want = g.astype(np.float64)
    elif storage == "f16":
        want = g.astype(np.float16).astype(np.float64)
    else:
        want = _bf16_nearest_even(g.reshape(-1)).reshape(g.shape)
    bad = np.flatnonzero(h.reshape(-1) != want.reshape(-1))
    assert bad.size == 0, f"{bad.size} values differ, first: g={g.reshape(-1)[bad[0]]!r} stored={h.reshape(-1)[bad[0]]!r} want={want.reshape(-1)[bad[0]]!r}"
    lat.close()
