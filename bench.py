#!/usr/bin/env python3
"""Throughput benchmark of the fused colour-gradient LBM step on one MI355X.

One "step" is one time step of every domain of the workload (the whole hot path: gather with
bounce-back and open boundaries, wetting boundary, curvature/force, MRT collision, recolouring,
store).  Inputs are resident in HBM before timing starts.

Default headline: the batched fingering sweep (320 channels, H in {50,75,100,150,200}, L = 16H,
M x Ca x theta factorial) with 16-bit populations (the C16 format: sign, 4-bit exponent, 11-bit
fraction, per-direction power-of-two scales; it meets the reduced-precision accuracy bar, which
IEEE binary16 misses on the finger length) and FP32 arithmetic, in one launch per step.  The same JSON line reports the plain FP64 single-domain throughput on the 16384 x 512
fingering channel and the ratio of the two, a live roofline of the dominant kernel
(algorithmic bytes / HIP-event time) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per fluid-node update: the node's 9 populations and 3 colour-state values
# read once and written once (storage bytes 8/4/2 for populations, 8/4/4 for colour state).
BYTES_PER_LUP = {"f64": 2 * (9 * 8 + 3 * 8), "f32": 2 * (9 * 4 + 3 * 4), "f16": 2 * (9 * 2 + 3 * 4),
                 "c16": 2 * (9 * 2 + 3 * 4)}
ARITH = {"f64": "f64", "f32": "f32", "f16": "f32", "c16": "f32"}
KERNEL = {"f64": "double", "f32": "float", "f16": "__half", "c16": "lbmcg::C16"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sweep",
                    choices=["sweep", "fingering_large", "fingering", "droplet", "x8", "x9"])
    ap.add_argument("--storage", default=None, choices=["f64", "f32", "f16", "c16"])
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--chunk-rows", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="pick the tile shape of the timed lattice with lbm_autotune first (its trial "
                         "launches are step kernels too: leave it off when profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 2 GiB read + 2 GiB write elementwise kernel, the "
                         "reference for scaling HBM byte counters")
    ap.add_argument("--traffic", default=None,
                    help="profile summary with measured HBM bytes per launch of the step kernel "
                         "(default: profiles/step_kernel_<workload>_<storage>_hbm_bytes.md)")
    return ap.parse_args()


def copy_calibration():
    """Plain elementwise kernel of known traffic: reads 2 GiB and writes 2 GiB (fp32 x * 1)."""
    import torch
    n = 512 * 1024 * 1024
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: 3 launches of {n * 4} bytes read + {n * 4} bytes written",
          flush=True)
    del x, y
    torch.cuda.empty_cache()


def build_workload(name):
    from paper_1707_00198_amd import workloads as W
    if name == "sweep":
        return W.cfg_sweep(), "c16", ("batched fingering sweep: 320 channels, H in {50,75,100,150,200}"
                                      " (64 each), L = 16H, M x Ca x theta factorial, one launch per step")
    if name == "fingering_large":
        return [W.cfg_fingering_large()], "f64", "fingering channel 16384 x 512, M = 50, theta = 30 deg"
    if name == "fingering":
        return [W.cfg_fingering()], "f64", "fingering channel 2000 x 100, M = 10, theta = 60 deg"
    if name == "x8":
        return W.cfg_x8(), "f64", ("wettability sweep of Sec. III D 2: 15 channels 630 x 60, theta 20..160,"
                                   " M = 1, u0 = 0.1, one launch per step")
    if name == "x9":
        return W.cfg_x9(), "f64", ("viscosity-ratio / capillary-number sweep of Sec. III D 4: 44 channels"
                                   " 630 x 60, M 1..1000, Ca 0.36..0.72, one launch per step")
    return [W.cfg_droplet_flat()], "f64", "static droplet on a flat wall, 200 x 100, theta = 60 deg"


def time_lattice(setups, storage, steps, warmup, chunk_rows=0, autotune=False):
    import torch
    from paper_1707_00198_amd.lbm import Lattice
    lat = Lattice(setups, storage=storage)
    if chunk_rows:
        lat.set_tile(chunk_rows)
    if autotune:
        print(f"[bench] autotuned tile: {lat.autotune(steps=10)}", flush=True)
    tile = dict(lat.tile, rule="autotuned" if autotune else ("set" if chunk_rows else "built-in"))
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    mass = lat.mass()  # also raises if a non-finite value appeared
    fluid = sum(s.fluid_nodes for s in setups)
    del lat
    torch.cuda.empty_cache()
    return dict(fluid=fluid, event_ms=ev_ms, wall_s=wall, mlups=fluid * steps / (ev_ms * 1e-3) / 1e6,
                ms_per_step=ev_ms / steps, mass=mass, tile=tile)


def measured_traffic(path, workload, storage):
    """HBM bytes per launch from a committed counter summary (FETCH_SIZE + WRITE_SIZE, scaled by
    a copy kernel), or None if there is none or the kernel source has changed since."""
    import hashlib
    import re
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    t = json.loads(m.group(1))
    src = os.path.join(ROOT, "paper_1707_00198_amd", "csrc", "lbm_kernels.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if t.get("kernel_source_sha256") != h or t.get("workload") != workload or t.get("storage") != storage:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(seconds):
    """The FP64 oracle, as it is, on one H = 50 channel of the sweep (800 x 52 lattice),
    as many steps as fit in about `seconds`."""
    import oracle
    from paper_1707_00198_amd import workloads as W
    s = W.fingering_channel(nx=800, h=50, x_interface=100.0, M=10.0, theta_deg=60.0, ca=0.1,
                            nu_r=0.5, sigma=0.05)
    o = oracle.Oracle(s.solid, s.rho_r0, s.rho_b0, **s.oracle_kwargs())
    o.step(5)

    def rate(budget):
        n, t = 0, 0.0
        while t < budget:
            t0 = time.perf_counter()
            o.step(20)
            t += time.perf_counter() - t0
            n += 20
        return n, t

    cores = oracle.threads()
    n, t = rate(seconds)
    # the same oracle on one thread, for a fifth of the time
    oracle.set_threads(1)
    n1, t1 = rate(seconds / 5.0)
    oracle.set_threads(cores)
    return dict(value=s.fluid_nodes * n / t / 1e6, unit="MLUPS", cores=cores, kind="oracle",
                sample=f"one 800 x 50 fingering channel of the sweep, {n} steps in {t:.1f} s, FP64",
                value_one_thread=round(s.fluid_nodes * n1 / t1 / 1e6, 3))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.calibrate_copy:
        copy_calibration()

    setups, storage, desc = build_workload(args.workload)
    if args.storage:
        storage = args.storage
    print(f"[bench] workload {args.workload}: {len(setups)} domains, "
          f"{sum(s.fluid_nodes for s in setups)} fluid nodes, storage {storage}", flush=True)
    head = time_lattice(setups, storage, args.steps, args.warmup, args.chunk_rows, args.autotune)
    print(f"[bench] {args.workload} {storage}: {head['mlups']:.1f} MLUPS, "
          f"{head['ms_per_step']:.4f} ms/step", flush=True)
    del setups

    ref = None
    if not args.no_fp64_reference and not (args.workload == "fingering_large" and storage == "f64"):
        ref_setups, _, _ = build_workload("fingering_large")
        ref_steps = max(20, args.steps // 2)
        ref = time_lattice(ref_setups, "f64", ref_steps, args.warmup)
        print(f"[bench] fingering_large f64: {ref['mlups']:.1f} MLUPS", flush=True)
        del ref_setups

    # Roofline of the dominant (and only per-step) kernel, the fused step kernel.
    bpl = BYTES_PER_LUP[storage]
    lups_per_launch = head["fluid"]
    achieved = bpl * lups_per_launch / (head["ms_per_step"] * 1e-3) / 1e9
    traffic = measured_traffic(args.traffic or os.path.join(
        ROOT, "profiles", f"step_kernel_{args.workload}_{storage}_hbm_bytes.md"), args.workload, storage)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel=f"step_kernel<{KERNEL[storage]}>",
                    bytes_per_lup=bpl, lups_per_launch=lups_per_launch)

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_seconds)

    out = {
        "metric": "MLUPS (fluid-node updates per second) of the fused colour-gradient LBM step",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ARITH[storage],
        "data": "synthetic",
        "config": {"workload": desc, "storage": storage, "domains": len(head["mass"]),
                   "fluid_nodes": head["fluid"], "tile": head["tile"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if ref is not None:
        out["fp64_single_domain"] = {"workload": "fingering channel 16384 x 512 (FP64 storage and arithmetic)",
                                     "mlups": round(ref["mlups"], 1),
                                     "ms_per_step": round(ref["ms_per_step"], 5),
                                     "hbm_frac": round(BYTES_PER_LUP["f64"] * ref["mlups"] * 1e6 / 1e9 / HBM_PEAK_GBS, 4)}
        out["ratio_vs_fp64_single_domain"] = round(head["mlups"] / ref["mlups"], 3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
