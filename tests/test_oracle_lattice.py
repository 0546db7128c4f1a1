"""Oracle pins: lattice tables, equilibrium moments, Smagorinsky closure.

Each test checks the FP64 oracle against something fixed outside it: the
paper's printed Table 1 and weights, textbook isotropy of the D3Q19 lattice,
exact moment identities of the discrete equilibrium, and the defining relation
of the Hou et al. Smagorinsky closure (Sec. 2.2).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    rows = []
    for line in open(os.path.join(GOLDEN, "d3q19_table1.txt")):
        line = line.split("#")[0].strip()
        if line:
            i, cx, cy, cz, w = line.split()
            rows.append((int(i), int(cx), int(cy), int(cz), float(Fraction(w))))
    return rows


def test_table1_matches_paper(orc):
    c, w, opp = orc.tables()
    rows = _table1()
    assert len(rows) == 19
    for i, cx, cy, cz, wi in rows:
        assert tuple(c[i]) == (cx, cy, cz), f"direction {i}"
        assert w[i] == pytest.approx(wi, rel=0, abs=1e-16)


def test_opposite_map_is_i_plus_9(orc):
    c, w, opp = orc.tables()
    assert opp[0] == 0
    for i in range(1, 10):
        assert opp[i] == i + 9 and opp[i + 9] == i
    for i in range(19):
        assert tuple(c[opp[i]]) == tuple(-c[i])


def test_isotropy_moments(orc):
    """Textbook D3Q19 lattice moments up to fourth order."""
    c, w, _ = orc.tables()
    c = c.astype(float)
    d = np.eye(3)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), d / 3, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ig->abg", w, c, c, c), 0, atol=1e-16)
    iso4 = (np.einsum("ab,gd->abgd", d, d) + np.einsum("ag,bd->abgd", d, d)
            + np.einsum("ad,bg->abgd", d, d)) / 9
    np.testing.assert_allclose(np.einsum("i,ia,ib,ig,id->abgd", w, c, c, c, c), iso4, atol=1e-16)
    # sound speed: c_s^2 = sum_i w_i c_ix^2 = 1/3
    assert np.sum(w * c[:, 0] ** 2) == pytest.approx(1 / 3, abs=1e-16)


def test_zieb_unknown_set_is_the_plus_z_directions(orc):
    """Sec. 2.6 lists 7, 9, 12, 15, 17 as the unknowns at a plane normal to z."""
    c, _, _ = orc.tables()
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "zieb_unknowns.txt"))
            if ln.strip() and not ln.startswith("#")]
    fix = {r[0]: [int(t) for t in r[1:]] for r in rows}
    paper = sorted(fix["unknown"])
    assert fix["normal"] == [12]
    assert sorted(np.nonzero(c[:, 2] == 1)[0].tolist()) == paper
    assert tuple(c[12]) == (0, 0, 1)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(orc, seed):
    """sum f = rho, sum f c = rho u, sum f c c = rho/3 I + rho u u (exact for D3Q19)."""
    rng = np.random.default_rng(seed)
    rho = 0.8 + 0.4 * rng.random()
    u = rng.normal(0, 0.05, 3)
    c, _, _ = orc.tables()
    c = c.astype(float)
    f = orc.equilibrium(rho, u)
    assert f.sum() == pytest.approx(rho, rel=1e-14)
    np.testing.assert_allclose(f @ c, rho * u, atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", f, c, c),
                               rho / 3 * np.eye(3) + rho * np.outer(u, u), atol=1e-15)


def test_equilibrium_at_rest_is_weights(orc):
    _, w, _ = orc.tables()
    np.testing.assert_array_equal(orc.equilibrium(1.0, (0, 0, 0)), w)


@pytest.mark.parametrize("tau0,C,rho,Q", [(0.6, 0.1, 1.0, 1e-6), (0.55, 0.17, 1.02, 3e-5),
                                          (0.5001, 0.4, 0.97, 2e-4), (0.8, 0.2, 1.0, 1e-9)])
def test_smagorinsky_closure(orc, tau0, C, rho, Q):
    """tau* solves the Hou et al. closure of Sec. 2.2.

    eddy viscosity nu_t = c_s^2 (tau* - tau0) must equal (C dx)^2 |S| with
    |S| = sqrt(2 S:S) and S = Pi / (2 rho c_s^2 tau*), i.e.
    |S| = sqrt(2 Q) / (2 rho c_s^2 tau*), Q = Pi:Pi.
    """
    ts = orc.relaxation_time(tau0, C, rho, Q)
    cs2 = 1 / 3
    S = np.sqrt(2 * Q) / (2 * rho * cs2 * ts)
    assert cs2 * (ts - tau0) == pytest.approx(C * C * S, rel=1e-12)
    assert ts > tau0


def test_smagorinsky_limits(orc):
    assert orc.relaxation_time(0.6, 0.0, 1.0, 1e-3) == 0.6
    assert orc.relaxation_time(0.6, 0.3, 1.0, 0.0) == 0.6
