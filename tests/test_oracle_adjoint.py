"""Pins of the FP64 reference for the drag gradient (oracle/adjoint.py).

The restated step must reproduce the C oracle's step (populations at fluid
nodes and sphere forces), and its reverse-mode gradient of
J = sum_b F_b,x (after n steps from a fixed state) with respect to the body
force and the sphere velocities must match central differences of the C
oracle itself.  J is linear in V (V enters only the moving-boundary term,
and the spheres do not move) up to the non-linear collision, so central
differences are accurate to a few parts in 1e7.
"""
import dataclasses

import numpy as np
import pytest

import lbm_workloads as W


def _case(halfway_seed=3):
    case = W.case_box(n=(16, 16, 16), n_spheres=2, radius=(3.0, 3.0), tau0=0.6, smag_c=0.1,
                      body_force=(5e-6, 0.0, 0.0), u_sigma=0.0, gap=2.0, seed=halfway_seed)
    rng = np.random.Generator(np.random.PCG64(9))
    return dataclasses.replace(case, V=rng.normal(0.0, 0.01, size=(2, 3)))


def _J(orc, case, P0, F, V, steps, halfway):
    o = orc.Oracle.from_case(dataclasses.replace(case, body_force=tuple(F), V=V), halfway=halfway)
    o.P = P0.reshape(-1).copy()
    o.step(steps)
    return o.forces()[0][:case.n_bodies, 0].sum()


@pytest.mark.parametrize("halfway", [False, True])
def test_restated_step_matches_oracle(orc, halfway):
    import torch
    from oracle.adjoint import DragProblem
    case = _case()
    o = orc.Oracle.from_case(case, halfway=halfway)
    dp = DragProblem(o)
    P = torch.tensor(o.populations().reshape(19, -1))
    for _ in range(5):
        P, Fb = dp.step(P, case.body_force, case.V)
    o.step(5)
    fl = dp.fluid.numpy()
    assert np.max(np.abs(P.numpy()[:, fl] - o.populations().reshape(19, -1)[:, fl])) < 1e-12
    assert np.max(np.abs(Fb.numpy() - o.forces()[0][:case.n_bodies])) < 1e-10


@pytest.mark.parametrize("halfway", [False, True])
def test_gradient_matches_central_differences(orc, halfway):
    from oracle.adjoint import DragProblem
    case = _case()
    steps = 20
    o = orc.Oracle.from_case(case, halfway=halfway)
    P0 = o.populations().copy()
    J, gF, gV = DragProblem(o).gradient(P0, case.body_force, case.V, steps)
    assert J == pytest.approx(_J(orc, case, P0, case.body_force, case.V, steps, halfway), rel=1e-12)
    F0 = np.array(case.body_force)
    for a, h in ((0, 1e-6), (1, 1e-6)):
        e = np.zeros(3)
        e[a] = h
        fd = (_J(orc, case, P0, F0 + e, case.V, steps, halfway) - _J(orc, case, P0, F0 - e, case.V, steps, halfway)) / (2 * h)
        assert gF[a] == pytest.approx(fd, rel=1e-5, abs=1e-6 * abs(gF[0]))
    for b, a in ((0, 0), (1, 2), (0, 1)):
        h = 1e-4
        Vp, Vm = case.V.copy(), case.V.copy()
        Vp[b, a] += h
        Vm[b, a] -= h
        fd = (_J(orc, case, P0, F0, Vp, steps, halfway) - _J(orc, case, P0, F0, Vm, steps, halfway)) / (2 * h)
        assert gV[b, a] == pytest.approx(fd, rel=1e-5, abs=1e-5 * np.max(np.abs(gV)))
