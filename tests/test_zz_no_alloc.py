"""lbm_step_noalloc (force sums in the library's static device array, no
allocation) against lbm_step on the same seeded cases, through the C ABI.

Both run the fused kernel with the same per-link fixed-point terms, so the
populations and the forces must agree bit for bit.  Two calls of the new
entry point in a row share the static array: a larger case first (several
steps per call, so both halves of the array are used), then a smaller one
(fewer spheres, a smaller lattice), then the larger handle again.
"""
import numpy as np
import pytest

import lbm_workloads as W

pytestmark = pytest.mark.gpu


def _pair(case, stream):
    from paper_1703_05158_amd import Lattice
    ref = Lattice.from_case(case, stream=stream)
    new = Lattice.from_case(case, stream=stream)
    return ref, new


def _advance(ref, new, case, n0, calls, per_call):
    """`calls` calls of `per_call` steps each, new bodies before every call."""
    n = n0
    for _ in range(calls):
        n += 1
        if case.drift:
            ref.set_bodies(*case.bodies_at(n))
            new.set_bodies(*case.bodies_at(n))
        ref.step(per_call)
        new.step_noalloc(per_call)
    return n


def _same(ref, new):
    np.testing.assert_array_equal(new.get_populations(), ref.get_populations())
    np.testing.assert_array_equal(new.get_owner(), ref.get_owner())
    Fr, Tr = ref.get_forces()
    Fn, Tn = new.get_forces()
    np.testing.assert_array_equal(Fn, Fr)
    np.testing.assert_array_equal(Tn, Tr)
    assert np.all(np.isfinite(Fn)) and np.abs(Fn).sum() > 0


def test_noalloc_step_matches_step_on_two_calls(torch_stream):
    big = W.case_duct(nx=48, ny=40, nz=96, n_spheres=40, orifice_z=70, orifice_r_in=12, orifice_gap=4,
                      pack_z=(6, 60), seed=31, drift=True)
    small = W.case_box(n=(24, 20, 28), n_spheres=3, radius=(2.0, 3.5), v_sigma=0.01, seed=4, drift=True)
    ref_b, new_b = _pair(big, torch_stream)
    nb = _advance(ref_b, new_b, big, 0, 2, 5)       # first call: 5 steps, bodies moved before each call
    _same(ref_b, new_b)
    ref_s, new_s = _pair(small, torch_stream)
    _advance(ref_s, new_s, small, 0, 2, 3)          # second call: a smaller input
    _same(ref_s, new_s)
    _advance(ref_b, new_b, big, nb, 1, 4)           # the larger handle again after the smaller one
    _same(ref_b, new_b)
    for lat in (ref_b, new_b, ref_s, new_s):
        lat.close()


def test_noalloc_step_mixes_with_step(torch_stream):
    """Plain steps whose forces are still pending, then the new entry point,
    then plain steps again: the same as plain steps throughout."""
    case = W.case_box(n=(32, 28, 36), n_spheres=5, radius=(2.0, 4.0), v_sigma=0.01, seed=6, drift=True)
    ref, new = _pair(case, torch_stream)
    for n in range(1, 7):
        for lat in (ref, new):
            lat.set_bodies(*case.bodies_at(n))
        ref.step(1)
        (new.step_noalloc if n in (3, 4) else new.step)(1)
    _same(ref, new)
    ref.close()
    new.close()


def test_noalloc_step_rejects_too_many_bodies(torch_stream):
    from paper_1703_05158_amd import LBMError, Lattice
    rng = np.random.Generator(np.random.PCG64(2))
    nb = 11000  # 6 (11000 + 64 n_walls) > 65536 sums
    case = W.Case(name="many", nx=64, ny=64, nz=64, tau0=0.7, smag_c=0.1, X=rng.uniform(0, 1, (nb, 3)) * 64,
                  V=np.zeros((nb, 3)), Omega=np.zeros((nb, 3)), R=np.full(nb, 0.6))
    lat = Lattice.from_case(case, stream=torch_stream, max_bodies=nb)
    with pytest.raises(LBMError) as ei:
        lat.step_noalloc(1)
    assert "static scratch" in str(ei.value)
    lat.step(1)  # the handle itself still steps
    lat.close()
