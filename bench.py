#!/usr/bin/env python3
"""Throughput of the fused D3Q19 moving-boundary LBM step on one MI355X.

Workload: the piston duct -- 128x128x512 nodes, static side walls, a piston
layer moving at 0.02 along z, an annular orifice plate, 4000 polydisperse
spheres (R in [2, 6], solid fraction 0.25 in the packed chamber) drifting
with their own velocities and spinning, Smagorinsky C = 0.17, tau0 = 0.55,
FP32 storage.  Every step the sphere kinematics of that step are handed to
the library (device table, as a GPU-resident DEM would), the library
re-rasterises the spheres and runs the fused step, and the per-body force and
torque are copied into a device history buffer (the DEM consumes them every
step).  Inputs are resident in HBM before the timed region starts.

Prints one JSON line: MLUPS (all nodes) over the timed steps; the roofline
of the dominant kernel (the fused step kernel: boundary links, streaming,
collision) from HIP events on its stream and its algorithmic bytes per
launch (`frac`), and of the whole step (`frac_step`: the same bytes over the
wall-clock time per step), with the time of every part of the step from HIP
events in the same timed run; and the FP64 CPU oracle timed on a bounded
sample of the same workload on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
METRIC = "MLUPS and % of HBM roofline; mixed-precision vs FP32 at stated error"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fused_piston_duct_traffic.json")
# the step kernel's source and the headers it is compiled with
KERNEL_SRC = [os.path.join(ROOT, "paper_1703_05158_amd", "csrc", f)
              for f in ("lbm_fused.hip", "lbm_collide.h", "lbm_linkmath.h", "lbm_device.h", "lbm_internal.h")]
TRAFFIC_WORKLOAD = "piston_duct_128x128x512_4000spheres_drift"
REFERENCE = os.path.join(ROOT, "tests", "golden", "duct_reference.npz")


def kernel_sha():
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _counters(d):
    """Counter value of every dispatch of every kernel, {kernel: {dispatch:
    value}}, from a rocprofv3 --pmc CSV output directory."""
    import csv
    import glob
    f = glob.glob(os.path.join(d, "**", "run_counter_collection.csv"), recursive=True)
    if len(f) != 1:
        raise SystemExit(f"expected one run_counter_collection.csv under {d}, found {len(f)}")
    per = {}
    for r in csv.DictReader(open(f[0])):
        per.setdefault(r["Kernel_Name"], {}).setdefault(r["Dispatch_Id"], 0.0)
        per[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return per


def _copy_kib(d):
    """The counter of the largest copy dispatch (the 1 GiB copy)."""
    return max(v for k, per in _counters(d).items() if "copyBuffer" in k for v in per.values())


def record_traffic(d):
    """Write the step kernel's HBM bytes per launch from rocprofv3 counter
    runs under d: pc_fetch and pc_write (FETCH_SIZE and WRITE_SIZE of the
    --calibrate-copy run), pb_fetch_<s> and pb_write_<s> (the same counters
    of --steps 4 --warmup 2 --cpu-steps 0 --no-mixed --no-sweep --no-adjoint
    --storage <s>, for s in f32 and f16).  The bench's tile autotuner runs
    every tile shape of the step kernel on the workload, so each shape gets
    its own figure.  Each counter (KiB per dispatch, the mean over that
    kernel's dispatches) is scaled by what it reads for a copy of 1 GiB read
    and 1 GiB written."""
    import re
    gib = 1 << 30
    copy_f = _copy_kib(os.path.join(d, "pc_fetch"))
    copy_w = _copy_kib(os.path.join(d, "pc_write"))
    fs, ws = gib / 1024 / copy_f, gib / 1024 / copy_w
    cmd = ("rocprofv3 --pmc {c} --output-format csv -d <out> -o run -- python3 <repo>/bench.py --steps 4 "
           "--warmup 2 --cpu-steps 0 --no-mixed --no-sweep --no-adjoint --storage {s}")
    out = {}
    for st, sv in (("f32", 0), ("f16", 1)):
        per = []
        for c in ("fetch", "write"):
            m = {}
            for k, v in _counters(os.path.join(d, f"pb_{c}_{st}")).items():
                g = re.search(rf"k_fused<{sv}, (\d+), (\d+), (\d+)>", k)
                if g:
                    m["x".join(g.groups())] = sum(v.values()) / len(v)
            per.append(m)
        tiles = sorted(set(per[0]) & set(per[1]))
        if not tiles:
            raise SystemExit(f"no k_fused<{sv},...> kernel in both pb_fetch_{st} and pb_write_{st}")
        out[st] = {"kernel_sha": kernel_sha(), "workload": TRAFFIC_WORKLOAD,
                   "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
                   "commands": [cmd.format(c="FETCH_SIZE", s=st), cmd.format(c="WRITE_SIZE", s=st)],
                   "tiles": {t: {"kernel": f"k_fused<{sv},{t.replace('x', ',')}>",
                                 "fetch_kib_per_dispatch": round(per[0][t], 1),
                                 "write_kib_per_dispatch": round(per[1][t], 1),
                                 "bytes_per_launch": round(per[0][t] * 1024 * fs + per[1][t] * 1024 * ws)}
                             for t in tiles}}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def measured_traffic(storage, tile):
    """HBM bytes per launch of the step kernel with this tile shape
    ("64x2x2", ...) from committed rocprofv3 counters, only if they were
    taken on the current kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    rec = d.get(storage)
    if not rec or rec.get("kernel_sha") != kernel_sha():
        return None
    return rec.get("tiles", {}).get(tile, {}).get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(case, sample_steps, threads, box32_steps=100):
    """The FP64 oracle on the host's cores over a bounded sample of the same
    workload, then one step of it on a single thread, and the 32^3 parity box
    (8 spheres) for `box32_steps` steps beside the GPU's figure for it."""
    import lbm_workloads as W
    import oracle
    used = oracle.set_threads(threads)
    o = oracle.Oracle.from_case(case)
    t0 = time.perf_counter()
    for n in range(1, sample_steps + 1):
        o.set_bodies(*case.bodies_at(n))
        o.step(1)
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    o.set_bodies(*case.bodies_at(sample_steps + 1))
    t1 = time.perf_counter()
    o.step(1)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    box = W.case_box32()
    ob = oracle.Oracle.from_case(box)
    t2 = time.perf_counter()
    ob.step(box32_steps)
    dt2 = time.perf_counter() - t2
    return {"value": round(case.n_nodes * sample_steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": used, "kind": "oracle",
            "sample": f"{sample_steps} drift steps of the same 128x128x512 duct (FP64 C oracle, "
                      f"OpenMP over z), {dt:.1f} s",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": round(case.n_nodes / dt1 / 1e6, 3), "unit": "MLUPS",
                              "sample": f"1 drift step on 1 thread, {dt1:.1f} s"},
            "box32": {"value": round(box.n_nodes * box32_steps / dt2 / 1e6, 2), "unit": "MLUPS",
                      "sample": f"{box32_steps} steps of the 32^3 box with 8 spheres, {dt2:.2f} s"}}


def box32_run(steps=100):
    """The 32^3 parity box (8 spheres, 100 steps) on the GPU, for the record:
    32 k nodes are far too few to load the GPU (the oracle's figure for the
    same box is in the CPU baseline)."""
    import torch

    import lbm_workloads as W
    from paper_1703_05158_amd import Lattice

    case = W.case_box32()
    lat = Lattice.from_case(case, stream=torch.cuda.current_stream().cuda_stream)
    lat.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat.close()
    return {"workload": "box_32cube_8spheres", "steps": steps,
            "gpu_mlups": round(case.n_nodes * steps / dt / 1e6, 1)}


def copy_bandwidth():
    """Device-to-device copy of 1 GiB (read + write), GB/s: the practical
    bandwidth reference beside the HBM peak."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return 2 * (1 << 30) / sec / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--static", action="store_true", help="bodies fixed (no per-step re-rasterisation)")
    ap.add_argument("--path", default="fused", choices=["fused", "split"],
                    help="step path of the timed lattice: the fused kernel, or the boundary-link pass "
                         "followed by the pull-collide kernel (same populations bit for bit)")
    ap.add_argument("--no-mixed", dest="mixed", action="store_false",
                    help="skip the FP16/BF16 runs and their error against the stored FP64 run")
    ap.add_argument("--no-sweep", dest="sweep", action="store_false",
                    help="skip the batched 48-instance parameter sweep")
    ap.add_argument("--sweep-steps", type=int, default=500)
    ap.add_argument("--no-zieb", dest="zieb", action="store_false",
                    help="skip the run with the inflow plane")
    ap.add_argument("--no-adjoint", dest="adjoint", action="store_false",
                    help="skip the drag-gradient run")
    ap.add_argument("--cpu-steps", type=int, default=15, help="oracle sample steps (0: skip)")
    ap.add_argument("--cpu-threads", type=int, default=int(os.environ.get("OMP_NUM_THREADS", "16")))
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter scale reference)")
    ap.add_argument("--record-traffic", metavar="DIR",
                    help="write the step kernel's HBM bytes per launch from rocprofv3 counter runs under DIR")
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(args.record_traffic)
        return
    if args.calibrate_copy:
        import torch
        torch.cuda.set_device(0)
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": a.numel() * 4, "bytes_written": a.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); the multi-GPU "
              "sharding of this step is a design note, not a built path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lbm_workloads as W

    torch.cuda.set_device(0)
    case = W.case_piston_duct(drift=not args.static)
    K, Wm = args.steps, args.warmup
    main_run = timed_run(case, args.storage, K, Wm, args.path)
    copy_gbs = copy_bandwidth()
    main_run["roofline"]["copy_gbs"] = round(copy_gbs, 1)
    main_run["roofline"]["frac_of_copy"] = round(main_run["roofline"]["achieved"] / copy_gbs, 4)
    N = case.n_nodes
    out = {
        "metric": METRIC, "value": main_run["value"], "unit": "MLUPS", "n_gpus": 1,
        "steps": K, "warmup": Wm, "ms_per_step": main_run["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {"workload": "piston_duct_128x128x512_4000spheres" + ("_static" if args.static else "_drift"),
                   "nodes": N, "fluid_nodes": main_run["fluid_nodes"], "spheres": case.n_bodies,
                   "walls": case.n_walls, "tau0": case.tau0, "smag_c": case.smag_c, "storage": args.storage,
                   "path": args.path,
                   "per_step": "set_bodies_device + step + get_forces_device" if case.drift
                   else "step + get_forces_device"},
        "mflups": main_run["mflups"],
        "ms_per_step_median5": main_run["ms_per_step_median5"],
        "ms_per_step_host_forces": main_run["ms_per_step_host_forces"],
        "ms_per_step_host_io": main_run["ms_per_step_host_io"],
        "roofline": main_run["roofline"],
    }
    if args.mixed and args.storage == "f32" and not args.static:
        # the same workload with 16-bit deviation storage: throughput, speedup
        # over the FP32 step, and the error against the stored FP64 run
        mixed = {}
        for st in ("f16", "bf16"):
            r = timed_run(case, st, K, Wm)
            mixed[st] = {"value": r["value"], "unit": "MLUPS", "ms_per_step": r["ms_per_step"],
                         "speedup_vs_f32": round(r["value"] / main_run["value"], 3),
                         "kernel_ms": r["roofline"]["kernel_ms"], "roofline_frac": r["roofline"]["frac"],
                         "roofline_frac_step": r["roofline"]["frac_step"]}
        errs = precision_errors(case)
        if errs:
            for st, e in errs.items():
                mixed.setdefault(st, {})["error_vs_fp64"] = e
        out["mixed_precision"] = mixed
    if args.sweep and args.storage == "f32" and not args.static:
        out["batched_sweep"] = sweep_run(args.sweep_steps)
    if args.zieb and args.storage == "f32" and not args.static:
        out["zieb"] = zieb_run(main_run["ms_per_step"])
    if args.adjoint and args.storage == "f32" and not args.static:
        out["adjoint"] = adjoint_run()
    if args.cpu_steps > 0 and not args.static:
        out["box32"] = box32_run()
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_steps, args.cpu_threads)
        out["cpu_baseline"]["gpu_over_oracle"] = round(out["value"] / out["cpu_baseline"]["value"], 1)
    print(json.dumps(out), flush=True)


def zieb_run(plain_ms, steps=100, warmup=10):
    """The duct with the paper's inflow plane (Sec. 2.6) in place of the
    piston: the piston layer z = 0 held still, the plane z = 1 fed by a
    virtual cylinder of the duct's cross-section moving at the piston's
    speed, the spheres drifting as in the main run.  Per step as the main
    run: the bodies' device table, the step, the forces into a device
    history."""
    import dataclasses

    import numpy as np
    import torch

    import lbm_workloads as W
    from paper_1703_05158_amd import Lattice

    base = W.case_piston_duct(drift=True)
    v_piston = float(base.wall_vel[1][2])
    wv = base.wall_vel.copy()
    wv[1] = 0.0
    case = dataclasses.replace(base, wall_vel=wv)
    area = float((case.wall_id[1] == 0).sum())
    volume = area * case.nz / 2
    stream = torch.cuda.current_stream()
    lat = Lattice.from_case(case, stream=stream.cuda_stream, init=False)
    lat.set_zieb(1, area, volume, v_piston)
    lat.init_fields(case.rho_init, case.u_init)
    nb, nbt = case.n_bodies, case.n_bodies + case.n_walls
    tabs = torch.empty((warmup + steps, nb, 10), dtype=torch.float64, device="cuda")
    for n in range(1, warmup + steps + 1):
        X, V, Om, R = case.bodies_at(n)
        tabs[n - 1] = torch.from_numpy(np.concatenate([X, V, Om, R[:, None]], 1))
    hist = torch.zeros((steps, nbt, 6), dtype=torch.float64, device="cuda")
    for n in range(warmup):
        lat.set_bodies_device(nb, tabs[n])
        lat.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(steps):
        lat.set_bodies_device(nb, tabs[warmup + n])
        lat.step(1)
        lat.get_forces_device(hist[n])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rho, H, vf = lat.zieb_state()
    lat.close()
    assert torch.isfinite(hist).all().item()
    ms = dt / steps * 1e3
    return {"workload": "piston_duct_128x128x512_4000spheres_drift_inflow_plane", "plane_z": 1,
            "area": area, "volume": volume, "v_piston": v_piston, "steps": steps,
            "ms_per_step": round(ms, 4), "value": round(case.n_nodes / ms / 1e3, 1), "unit": "MLUPS",
            "over_piston_duct": round(ms / plain_ms, 3), "rho_cylinder": rho, "piston_travel": H}


def adjoint_run(steps=200, ckpt=20):
    """Gradient of the summed sphere drag on the 96x96x192 box with 300
    fixed spheres: the plain forward run of `steps` steps, then the gradient
    (forward with a checkpoint every `ckpt` steps, reverse with recompute)
    from the same start state."""
    import numpy as np
    import torch

    import lbm_workloads as W
    from paper_1703_05158_amd import Lattice

    stream = torch.cuda.current_stream()
    case = W.case_adjoint(steps=steps)
    lat = Lattice.from_case(case, stream=stream.cuda_stream)
    start = lat.get_state()
    lat.step(5)
    lat.set_state(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    lat.set_state(start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, dF, dV = lat.drag_gradient(steps, ckpt)
    t_grad = time.perf_counter() - t0
    lat.close()
    return {"workload": "periodic_96x96x192_300spheres", "steps": steps, "ckpt": ckpt,
            "parameters": 3 + 3 * case.n_bodies, "J": J, "dJdF": [float(v) for v in dF],
            "dJdV_norm": float(np.linalg.norm(dV)), "forward_ms": round(t_fwd * 1e3, 2),
            "gradient_ms": round(t_grad * 1e3, 2), "gradient_over_forward": round(t_grad / t_fwd, 2)}


def sweep_run(steps, warmup=20):
    """The 48-instance parameter sweep (periodic boxes of five sizes, static
    spheres, FP32): tile shapes autotuned per box size, then the instances
    stepped one after another with plain launches, then the same instances
    stepped as one batch (one graph replay per step)."""
    import tempfile

    import torch

    import lbm_workloads as W
    from paper_1703_05158_amd import TILE_SHAPES, Batch, Lattice

    stream = torch.cuda.current_stream()
    cases = W.case_sweep_instances()
    lats = [Lattice.from_case(c, stream=stream.cuda_stream) for c in cases]
    nodes = sum(c.n_nodes for c in cases)
    tiles = {}
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tiles.json")
        for c, lat in zip(cases, lats):
            shape, _ = lat.autotune(trial_steps=5, cache_path=cache)
            tiles[f"{c.nx}x{c.ny}x{c.nz}"] = TILE_SHAPES[shape]
    for lat in lats:
        lat.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in lats:
        lat.step(steps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    batch = Batch(lats, stream=stream)
    bshape, _ = batch.autotune(trial_steps=5)
    tiles["batch"] = TILE_SHAPES[bshape]
    batch.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    batch.close()
    for lat in lats:
        lat.close()
    return {"instances": len(cases), "nodes": nodes, "steps": steps, "tiles": tiles,
            "sequential_mlups": round(nodes * steps / t_seq / 1e6, 1),
            "batched_mlups": round(nodes * steps / t_bat / 1e6, 1),
            "speedup": round(t_seq / t_bat, 3)}


def timed_run(case, storage, K, Wm, path="fused"):
    """Warm up, then time K steps of the case (per step: the bodies' table of
    that step handed over on the device, the step, the forces copied into a
    device history); the step kernel is timed with HIP events on its stream."""
    import numpy as np
    import torch
    from paper_1703_05158_amd import Lattice

    stream = torch.cuda.current_stream()
    lat = Lattice.from_case(case, storage=storage, stream=stream.cuda_stream, path=path)
    nb = case.n_bodies
    nbt = nb + case.n_walls
    # per-step kinematics, resident in HBM before timing (the DEM's output)
    tabs = None
    K2 = min(K, 50)
    nr = max(K // 5, 1)
    nt = Wm + K + 5 * nr + 2 * K2
    if case.drift:
        tabs = torch.empty((nt, nb, 10), dtype=torch.float64, device="cuda")
        for n in range(1, nt + 1):
            X, V, Om, R = case.bodies_at(n)
            tabs[n - 1] = torch.from_numpy(np.concatenate([X, V, Om, R[:, None]], 1))
    hist = torch.zeros((K, nbt, 6), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    for n in range(Wm):
        if tabs is not None:
            lat.set_bodies_device(nb, tabs[n])
        lat.step(1)
    torch.cuda.synchronize()
    n_fluid = lat.count_fluid()
    # the step kernel's tile shape for this box (timed launches that leave
    # the state as it is)
    from paper_1703_05158_amd import TILE_SHAPES
    shape, shape_us = lat.autotune(trial_steps=10)

    # the step kernel's own start and end events on every 10th step of the
    # timed region (each event costs its step a few microseconds)
    lat.profile(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(K):
        if tabs is not None:
            lat.set_bodies_device(nb, tabs[Wm + n])
        lat.step(1)
        lat.get_forces_device(hist[n])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    parts, launches = lat.profile_read_parts()
    kms = parts["step"]
    lat.profile(False)
    n_fluid_end = lat.count_fluid()
    assert torch.isfinite(hist).all().item()
    # five more repetitions of K/5 steps each, for a median
    reps = []
    for r in range(5):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for n in range(nr):
            if tabs is not None:
                lat.set_bodies_device(nb, tabs[Wm + K + r * nr + n])
            lat.step(1)
            lat.get_forces_device(hist[n])
        torch.cuda.synchronize()
        reps.append((time.perf_counter() - t1) / nr)
    # K2 more steps with the forces copied to the host after every step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(K2):
        if tabs is not None:
            lat.set_bodies_device(nb, tabs[Wm + K + 5 * nr + n])
        lat.step(1)
        lat.get_forces()
    dt_host = time.perf_counter() - t0
    # K2 more steps as a host-side DEM would couple: the bodies' host arrays
    # handed over (copied to the device by the library), the step, the
    # forces copied back to the host
    first = Wm + K + 5 * nr + K2 + 1
    host_tabs = [case.bodies_at(n) for n in range(first, first + K2)] if case.drift else []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(K2):
        if host_tabs:
            lat.set_bodies(*host_tabs[n])
        lat.step(1)
        lat.get_forces()
    dt_host_io = time.perf_counter() - t0
    lat.close()

    N = case.n_nodes
    sbytes = 4 if storage == "f32" else 2
    nf = 0.5 * (n_fluid + n_fluid_end)
    # algorithmic bytes of one step (and of one launch of the fused step
    # kernel, which does all of it but the re-rasterisation): every fluid
    # node reads and writes 19 populations; every node's owner code (2 B) is
    # read once
    alg_bytes = 2 * 19 * sbytes * nf + 2 * N
    k_avg_s = kms / launches * 1e-3
    achieved = alg_bytes / k_avg_s / 1e9
    step_s = dt / K
    traffic = measured_traffic(storage, TILE_SHAPES[shape]) if path == "fused" else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "frac_step": round(alg_bytes / step_s / 1e9 / HBM_PEAK_GBS, 4),
            "step_achieved": round(alg_bytes / step_s / 1e9, 1),
            "frac_measured": None if traffic is None else round(traffic / k_avg_s / 1e9 / HBM_PEAK_GBS, 4),
            "kernel_mlups": round(N / k_avg_s / 1e6, 1),
            "kernel": f"{'k_fused' if path == 'fused' else 'k_step'}<{storage},{TILE_SHAPES[shape].replace('x', ',')}>",
            "kernel_ms": round(k_avg_s * 1e3, 4),
            "parts_ms_per_step": {k: round(v / launches, 4) for k, v in parts.items()},
            "tile": TILE_SHAPES[shape], "tile_us": {TILE_SHAPES[i]: round(float(t), 1) for i, t in enumerate(shape_us)},
            "alg_bytes_per_launch": int(alg_bytes)}
    return {"value": round(N * K / dt / 1e6, 1), "ms_per_step": round(dt / K * 1e3, 4),
            "ms_per_step_median5": round(float(np.median(reps)) * 1e3, 4),
            "ms_per_step_host_forces": round(dt_host / K2 * 1e3, 4),
            "ms_per_step_host_io": round(dt_host_io / K2 * 1e3, 4),
            "mflups": round(nf * K / dt / 1e6, 1), "fluid_nodes": int(nf), "roofline": roof}


def precision_errors(case):
    """Density, velocity and force error of each storage format against the
    stored FP64 oracle run of the same drifting duct (tests/golden), at the
    steps it holds."""
    import numpy as np
    import torch
    from paper_1703_05158_amd import Lattice

    if not os.path.exists(REFERENCE):
        return None
    ref = np.load(REFERENCE)
    marks = [int(s) for s in ref["steps"]]
    nb = case.n_bodies
    tabs = torch.empty((marks[-1], nb, 10), dtype=torch.float64, device="cuda")
    for n in range(1, marks[-1] + 1):
        X, V, Om, R = case.bodies_at(n)
        tabs[n - 1] = torch.from_numpy(np.concatenate([X, V, Om, R[:, None]], 1))
    stream = torch.cuda.current_stream()
    res = {}
    for st in ("f32", "f16", "bf16"):
        lat = Lattice.from_case(case, storage=st, stream=stream.cuda_stream)
        e = {}
        for n in range(1, marks[-1] + 1):
            lat.set_bodies_device(nb, tabs[n - 1])
            lat.step(1)
            if n in marks:
                idx = ref[f"idx_{n}"]
                rho, u = lat.get_macro()
                ur = ref[f"u_{n}"]
                umax = float(np.max(np.linalg.norm(ur, axis=0)))
                F, _ = lat.get_forces()
                Fr = ref[f"F_{n}"]
                dr = rho.ravel()[idx] - ref[f"rho_{n}"]
                du = np.linalg.norm(u.reshape(3, -1)[:, idx] - ur, axis=0)
                e[f"step_{n}"] = {
                    "rho_abs": float(np.max(np.abs(dr))),
                    "rho_rms": float(np.sqrt(np.mean(dr * dr))),
                    "u_abs": float(np.max(du)),
                    "u_rms": float(np.sqrt(np.mean(du * du))),
                    "u_max": umax,
                    "force_rel": float(np.max(np.linalg.norm(F - Fr, axis=1)) / np.max(np.linalg.norm(Fr, axis=1))),
                    "sampled_nodes": int(len(idx))}
        res[st] = e
        lat.close()
    return res


if __name__ == "__main__":
    main()
