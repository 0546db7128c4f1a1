"""Run the HIP library and the FP64 oracle side by side on the same inputs."""
import numpy as np

import lbm_workloads as W


def make_pair(case, storage="f32", halfway=False, stream=None, max_bodies=None):
    import oracle
    from paper_1703_05158_amd import Lattice
    o = oracle.Oracle.from_case(case, halfway=halfway)
    lat = Lattice.from_case(case, storage=storage, bb_mode="halfway" if halfway else "bouzidi",
                            stream=stream, max_bodies=max_bodies)
    return o, lat


def advance(o, lat, case, start, steps):
    """Steps start+1 .. start+steps, re-setting the bodies before each step
    when the case drifts (both sides get the same FP64 arrays)."""
    for n in range(start + 1, start + steps + 1):
        if case.drift:
            X, V, Om, R = case.bodies_at(n)
            o.set_bodies(X, V, Om, R)
            lat.set_bodies(X, V, Om, R)
        o.step(1)
        lat.step(1)


def pop_rel_err(o, lat):
    """max over fluid nodes and directions of |P_gpu - P_ref| / |P_ref|."""
    m = o.fluid_mask()
    Po = o.populations()[:, m]
    Pg = lat.get_populations()[:, m]
    return float(np.max(np.abs(Pg - Po) / np.abs(Po)))


def pop_weight_err(o, lat):
    """max over fluid nodes and directions of |P_gpu - P_ref| / (w_i rho0):
    the error on the scale of each direction's population.  For 16-bit
    storage, whose rounding is a fraction of the deviation from w_i rho0, this
    stays meaningful where a population itself comes near zero."""
    import oracle
    _, w, _ = oracle.tables()
    m = o.fluid_mask()
    Po = o.populations()[:, m]
    Pg = lat.get_populations()[:, m]
    return float(np.max(np.abs(Pg - Po) / (w[:, None] * o.rho0)))


def force_rel_err(o, lat):
    """max_b |F_gpu,b - F_ref,b| / max_b |F_ref,b|, same for torques (spheres
    and walls together, in the library's order)."""
    Fg, Tg = lat.get_forces()
    Fo, To = o.forces()
    assert Fg.shape == Fo.shape
    if len(Fo) == 0:
        return 0.0, 0.0
    fe = np.max(np.linalg.norm(Fg - Fo, axis=1)) / max(np.max(np.linalg.norm(Fo, axis=1)), 1e-300)
    te = np.max(np.linalg.norm(Tg - To, axis=1)) / max(np.max(np.linalg.norm(To, axis=1)), 1e-300)
    return float(fe), float(te)
