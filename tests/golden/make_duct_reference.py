"""Write duct_reference.npz: the FP64 oracle on the 128x128x512 piston duct
with 4000 drifting spheres (the generator in lbm_workloads), the reference
for the reduced-precision error statement.

At each step in STEPS it stores, for SAMPLES fluid nodes drawn with a fixed
seed, the linear node index, the density and the velocity, and the force and
torque on every body (spheres, then walls).  Only the oracle computes the
stored values.

    python tests/golden/make_duct_reference.py [--threads N] [--steps 100,1000]

The oracle needs about 3 GB of memory and, on 8 cores, roughly half an hour
for 1000 steps.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import lbm_workloads as W  # noqa: E402
import oracle  # noqa: E402

SAMPLES = 20000


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--steps", default="100,1000")
    ap.add_argument("--out", default=os.path.join(HERE, "duct_reference.npz"))
    args = ap.parse_args()
    marks = sorted(int(s) for s in args.steps.split(","))
    oracle.set_threads(args.threads)
    case = W.case_piston_duct(drift=True)
    o = oracle.Oracle.from_case(case)
    rng = np.random.Generator(np.random.PCG64(11))
    out = {"steps": np.array(marks), "samples": np.array(SAMPLES)}
    t0 = time.perf_counter()
    for n in range(1, marks[-1] + 1):
        o.set_bodies(*case.bodies_at(n))
        o.step(1)
        if n in marks:
            fluid = np.flatnonzero(o.fluid_mask().ravel())
            idx = np.sort(rng.choice(fluid, size=SAMPLES, replace=False))
            rho, u = o.macro()
            F, T = o.forces()
            out[f"idx_{n}"] = idx.astype(np.int64)
            out[f"rho_{n}"] = rho.ravel()[idx]
            out[f"u_{n}"] = u.reshape(3, -1)[:, idx]
            out[f"F_{n}"] = F
            out[f"T_{n}"] = T
            print(f"step {n}: {time.perf_counter() - t0:.0f} s", flush=True)
    np.savez_compressed(args.out, **out)
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
