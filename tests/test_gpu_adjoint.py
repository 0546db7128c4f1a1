"""The library's reverse-mode kernels (lbm_drag_gradient) against the FP64
reference of oracle/adjoint.py.

J = sum_b F_b,x after n steps from a fixed state, with fixed spheres; the
gradient with respect to the body force and the sphere velocities.  The GPU
runs FP32 forward and reverse steps, so the bar is relative to the size of
each gradient: 1e-3 in norm (the FP32 parity bar of the step is 1e-5 on
populations, and the gradient accumulates n steps of it).
"""
import dataclasses

import numpy as np
import pytest

import lbm_workloads as W

pytestmark = pytest.mark.gpu


def _case(n=(24, 24, 24), n_spheres=3, seed=12):
    case = W.case_box(n=n, n_spheres=n_spheres, radius=(3.0, 3.0), tau0=0.6, smag_c=0.1,
                      body_force=(5e-6, 0.0, 0.0), u_sigma=0.0, gap=2.0, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    return dataclasses.replace(case, V=rng.normal(0.0, 0.01, size=(n_spheres, 3)))


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.mark.parametrize("halfway", [False, True])
def test_gradient_matches_fp64_reference(torch_stream, halfway):
    import oracle
    from oracle.adjoint import DragProblem
    from paper_1703_05158_amd import Lattice
    case = _case()
    steps = 30
    o = oracle.Oracle.from_case(case, halfway=halfway)
    Jr, gFr, gVr = DragProblem(o).gradient(o.populations(), case.body_force, case.V, steps)
    lat = Lattice.from_case(case, bb_mode="halfway" if halfway else "bouzidi", stream=torch_stream)
    J, gF, gV = lat.drag_gradient(steps, 7)
    print(f"J {J:.9e} ({Jr:.9e})  dF {gF} ({gFr})  dV err {_rel(gV, gVr):.2e}")
    assert J == pytest.approx(Jr, rel=1e-5)
    assert _rel(gF, gFr) < 1e-3
    assert _rel(gV, gVr) < 1e-3
    lat.close()


def test_checkpoint_interval_and_final_state(torch_stream):
    from paper_1703_05158_amd import Lattice
    case = _case(n=(32, 24, 20), n_spheres=2, seed=5)
    steps = 24
    ref = Lattice.from_case(case, stream=torch_stream)
    ref.step(steps)
    P_ref = ref.get_populations()
    F_ref = ref.get_forces()
    out = []
    for ckpt in (1, 5, 24, 100):
        lat = Lattice.from_case(case, stream=torch_stream)
        out.append(lat.drag_gradient(steps, ckpt))
        assert np.array_equal(lat.get_populations(), P_ref)
        F, T = lat.get_forces()
        assert np.array_equal(F, F_ref[0]) and np.array_equal(T, F_ref[1])
        assert lat.info()["steps_done"] == steps
        lat.close()
    J0, gF0, gV0 = out[0]
    for J, gF, gV in out[1:]:
        assert J == J0
        assert _rel(gF, gF0) < 1e-5 and _rel(gV, gV0) < 1e-5
    ref.close()


def test_torch_function_and_directional_difference(torch_stream):
    import torch
    from paper_1703_05158_amd import Lattice, SphereDrag
    case = _case()
    lat = Lattice.from_case(case, stream=torch_stream)
    start = lat.get_state()
    fn = SphereDrag(lat, start, case.X, case.Omega, case.R, nsteps=20, ckpt=5)
    F = torch.tensor(case.body_force, dtype=torch.float64, requires_grad=True)
    V = torch.tensor(case.V, dtype=torch.float64, requires_grad=True)
    J = fn(F, V)
    gF, gV = torch.autograd.grad(J, (F, V))
    J2, gF2, gV2 = Lattice.from_case(case, stream=torch_stream).drag_gradient(20, 5)
    assert float(J.detach()) == pytest.approx(J2, rel=1e-12)
    assert np.allclose(gF.numpy(), gF2, rtol=1e-5) and np.allclose(gV.numpy(), gV2, rtol=1e-5, atol=1e-9)
    # J is linear in V: a directional difference on the GPU matches dJ/dV . d
    rng = np.random.Generator(np.random.PCG64(4))
    d = torch.tensor(rng.normal(size=case.V.shape))
    h = 1e-3
    with torch.no_grad():
        Jp = float(fn(F, V + h * d))
        Jm = float(fn(F, V - h * d))
    fd = (Jp - Jm) / (2 * h)
    assert fd == pytest.approx(float((gV * d).sum()), rel=1e-3)
    lat.close()


def test_drag_gradient_rejects_unsupported(torch_stream):
    from paper_1703_05158_amd import LBMError, Lattice
    case = _case(n=(16, 16, 16), n_spheres=1, seed=2)
    lat = Lattice.from_case(case, storage="f16", stream=torch_stream)
    with pytest.raises(LBMError):
        lat.drag_gradient(4, 2)
    lat.close()
    duct = W.case_duct(nx=24, ny=24, nz=48, n_spheres=3, orifice_z=30, orifice_r_in=5, orifice_gap=2,
                       pack_z=(4, 24), seed=3, drift=False)
    lat = Lattice.from_case(duct, stream=torch_stream)
    with pytest.raises(LBMError):
        lat.drag_gradient(4, 2)   # walls
    lat.close()


def test_drag_gradient_out_of_memory_leaves_the_handle_usable(torch_stream):
    """A gradient whose checkpoints cannot fit in device memory (300 states
    of a 256^3 box, 1.27 GB each, about 385 GB) is refused with LBM_ERR_OOM,
    its buffers are freed, and the handle steps on as before: the state and
    forces of two steps after the refusal equal those of a handle that never
    asked (and profiling is left as it was)."""
    from paper_1703_05158_amd import LBMError, Lattice
    case = _case(n=(256, 256, 256), n_spheres=4, seed=5)
    lat = Lattice.from_case(case, stream=torch_stream)
    ref = Lattice.from_case(case, stream=torch_stream)
    lat.profile(1)
    with pytest.raises(LBMError) as e:
        lat.drag_gradient(300, 1)
    assert e.value.status == 2  # LBM_ERR_OOM
    lat.step(2)
    ref.step(2)
    _, steps = lat.profile_read_parts()
    assert steps == 2
    F, T = lat.get_forces()
    Fr, Tr = ref.get_forces()
    assert np.array_equal(F, Fr) and np.array_equal(T, Tr) and np.isfinite(F).all()
    rho, u = lat.get_macro()
    rr, ur = ref.get_macro()
    assert np.array_equal(rho, rr) and np.array_equal(u, ur)
    lat.close()
    ref.close()


def test_gradient_on_a_32cube_subset_of_the_adjoint_workload(torch_stream):
    """The 96x96x192 drag-gradient workload cut to a 32^3 subset (about its
    sphere density: 5 spheres of radius 4; body force 5e-6 along x, tau0
    0.6, C 0.1): the GPU gradient against the FP64 reverse-mode reference,
    and dJ/dV against central differences with h = 1e-4 of J run forward
    on the GPU (J is linear in V, so the difference is exact up to the FP32
    rounding of J)."""
    import oracle
    from oracle.adjoint import DragProblem
    from paper_1703_05158_amd import Lattice
    base = W.case_box(n=(32, 32, 32), n_spheres=5, radius=(4.0, 4.0), tau0=0.6, smag_c=0.1,
                      body_force=(5e-6, 0.0, 0.0), u_sigma=0.0, gap=2.0, seed=21)
    rng = np.random.Generator(np.random.PCG64(121))
    case = dataclasses.replace(base, V=rng.normal(0.0, 0.01, size=(5, 3)))
    steps, ckpt = 40, 10
    o = oracle.Oracle.from_case(case)
    Jr, gFr, gVr = DragProblem(o).gradient(o.populations(), case.body_force, case.V, steps)
    lat = Lattice.from_case(case, stream=torch_stream)
    J, gF, gV = lat.drag_gradient(steps, ckpt)
    lat.close()
    print(f"J {J:.9e} ({Jr:.9e})  dF err {_rel(gF, gFr):.2e}  dV err {_rel(gV, gVr):.2e}")
    assert J == pytest.approx(Jr, rel=1e-5)
    assert _rel(gF, gFr) < 1e-3 and _rel(gV, gVr) < 1e-3

    def J_of(V):
        l = Lattice.from_case(dataclasses.replace(case, V=V), stream=torch_stream)
        l.step(steps)
        F, _ = l.get_forces()
        l.close()
        return float(F[:case.n_bodies, 0].sum())
    h = 1e-4
    for b, a in ((0, 0), (2, 1), (4, 2)):
        Vp, Vm = case.V.copy(), case.V.copy()
        Vp[b, a] += h
        Vm[b, a] -= h
        fd = (J_of(Vp) - J_of(Vm)) / (2 * h)
        print(f"dJ/dV[{b},{a}] {gV[b, a]:.6e} fd {fd:.6e}")
        assert gV[b, a] == pytest.approx(fd, rel=2e-3, abs=2e-3 * np.max(np.abs(gV)))


def test_adjoint_workload_at_full_size(torch_stream):
    """The drag-gradient workload at its full size (96x96x192, 300 spheres
    of radius 4, body force 5e-6 along x, 200 steps) in the bench's launch
    configuration (a checkpoint every 20 steps), checked by what holds at
    any size: J equals, bit for bit, the summed x-force after a plain
    forward run of 200 steps, whose final state the gradient leaves behind;
    a checkpoint every 50 steps gives the same J and gradients to 1e-5; and
    central differences of J run forward on the GPU agree with the gradient
    along its own direction (h = 1e-4 on the unit vector of dJ/dV), in
    dJ/dF_x (h = 5e-8, 1% of the force) and in the three largest components
    of dJ/dV (h = 1e-4), to 1e-3 (the FP32 gradient's bar against the FP64
    reference; measured 3e-5 to 1e-4)."""
    from paper_1703_05158_amd import Lattice
    case = W.case_adjoint()
    steps, ckpt = 200, 20
    nb = case.n_bodies

    def J_of(V=None, F=None):
        c = case
        if V is not None:
            c = dataclasses.replace(c, V=V)
        if F is not None:
            c = dataclasses.replace(c, body_force=F)
        lat = Lattice.from_case(c, stream=torch_stream)
        lat.step(steps)
        Fo, To = lat.get_forces()
        P = lat.get_populations() if V is None and F is None else None
        lat.close()
        return float(Fo[:nb, 0].sum()), (Fo, To, P)

    J_fwd, (F_ref, T_ref, P_ref) = J_of()
    lat = Lattice.from_case(case, stream=torch_stream)
    J, gF, gV = lat.drag_gradient(steps, ckpt)
    assert lat.info()["steps_done"] == steps
    assert np.array_equal(lat.get_populations(), P_ref)
    F1, T1 = lat.get_forces()
    assert np.array_equal(F1, F_ref) and np.array_equal(T1, T_ref)
    lat.close()
    del P_ref
    print(f"J {J:.12e} forward {J_fwd:.12e}  dJ/dF {gF}  |dJ/dV| {np.linalg.norm(gV):.6e}")
    assert J == J_fwd

    lat = Lattice.from_case(case, stream=torch_stream)
    J50, gF50, gV50 = lat.drag_gradient(steps, 50)
    lat.close()
    assert J50 == J
    assert _rel(gF50, gF) < 1e-5 and _rel(gV50, gV) < 1e-5

    h = 1e-4
    d = gV / np.linalg.norm(gV)
    fd = (J_of(V=case.V + h * d)[0] - J_of(V=case.V - h * d)[0]) / (2 * h)
    print(f"along dJ/dV: {np.linalg.norm(gV):.6e} fd {fd:.6e}")
    assert fd == pytest.approx(np.linalg.norm(gV), rel=1e-3)

    hF = 5e-8
    Fp, Fm = np.array(case.body_force, float), np.array(case.body_force, float)
    Fp[0] += hF
    Fm[0] -= hF
    fd = (J_of(F=tuple(Fp))[0] - J_of(F=tuple(Fm))[0]) / (2 * hF)
    print(f"dJ/dF_x {gF[0]:.6e} fd {fd:.6e}")
    assert gF[0] == pytest.approx(fd, rel=1e-3)

    for k in np.argsort(-np.abs(gV).ravel())[:3]:
        b, a = divmod(int(k), 3)
        Vp, Vm = case.V.copy(), case.V.copy()
        Vp[b, a] += h
        Vm[b, a] -= h
        fd = (J_of(V=Vp)[0] - J_of(V=Vm)[0]) / (2 * h)
        print(f"dJ/dV[{b},{a}] {gV[b, a]:.6e} fd {fd:.6e}")
        assert gV[b, a] == pytest.approx(fd, rel=1e-3)
