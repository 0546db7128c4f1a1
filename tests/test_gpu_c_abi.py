"""The library called from plain C (tests/c_abi_driver.c, built by
__graft_entry__.build() into _build/): the C caller's forces and torques
after 20 steps equal, bit for bit, those of the same run through the Python
binding, and a rejected call returns its documented status."""
import os
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "_build", "c_abi_driver")


def test_c_caller_matches_python_binding():
    assert os.path.exists(EXE), "the C caller is not built; run __graft_entry__.build()"
    out = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.split("\n")
    head = lines[0].split()
    assert head[2] == "steps" and int(head[3]) == 20 and int(head[5]) == 2
    rows = np.array([[float(v) for v in ln.split()[2:]] for ln in lines if ln.startswith("body")])
    assert "rejected 1" in out.stdout  # LBM_ERR_ARG for nsteps < 0

    from paper_1703_05158_amd import Lattice, config
    lat = Lattice(config(32, 32, 32, tau0=0.6, smag_c=0.1, body_force=(1e-5, 0.0, 0.0), max_bodies=2))
    lat.set_bodies(np.array([[10.3, 11.7, 12.2], [22.6, 20.1, 19.4]]),
                   np.array([[0.01, 0.0, -0.005], [0.0, 0.002, 0.0]]),
                   np.array([[0.0, 0.0, 0.001], [0.0, 0.0, 0.0]]), np.array([4.2, 3.6]))
    lat.init_fields()
    lat.step(20)
    F, T = lat.get_forces()
    lat.close()
    np.testing.assert_array_equal(rows[:, :3], F)
    np.testing.assert_array_equal(rows[:, 3:], T)
    assert np.all(np.abs(F[:, 0]) > 0)
