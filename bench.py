#!/usr/bin/env python3
"""Throughput benchmark of the fused colour-gradient LBM step on one MI355X.

One "step" is one time step of every domain of the workload (the whole hot path: gather with
bounce-back and open boundaries, wetting boundary, curvature/force, MRT collision, recolouring,
store).  Inputs are resident in HBM before timing starts.

Default headline: the batched fingering sweep (320 channels, H in {50,75,100,150,200}, L = 16H,
M x Ca x theta factorial) with populations stored as IEEE binary16 deviations from the weights
(per-direction power-of-two scales, stochastically rounded stores) and FP32 arithmetic; ``--storage
c16`` selects the 16-bit format with one more fraction bit.  Timed in the form the sweep is
meant to run: the autotuned tile shape, steps replayed as HIP graphs.  The same JSON line
reports the sweep with the built-in shape launched step by step, the plain FP64 single-domain
throughput on the 16384 x 512 fingering channel and the ratio of the two, the accuracy of the
16-bit sweep against FP64 on a sample of its own channels (finger length, contact line) and on
the Table I droplets (contact angle), a live roofline of the dominant kernel (algorithmic bytes
/ HIP-event time) and the CPU oracle timed on a bounded sample.

``--workload wetting_batch`` runs the curved-wall and capillary batch as two contexts (FP32 and
16-bit storage, alternating domains) and reports their combined throughput.
``--baseline-table`` times every named workload on the GPU and the oracle on the host and
prints the table of measured values (markdown and JSON).
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
WORKLOADS = ["sweep", "fingering_large", "fingering", "droplet", "x8", "x9", "wetting_batch"]


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sweep", choices=WORKLOADS)
    ap.add_argument("--storage", default=None, choices=["f64", "f32", "f16", "c16"],
                    help="storage of the timed lattice (wetting_batch: of its 16-bit context)")
    ap.add_argument("--tile", default=None, choices=["builtin", "autotune"],
                    help="tile shape of the timed lattice (default: autotune for the sweep, else "
                         "the built-in rule)")
    ap.add_argument("--graph", type=int, default=-1,
                    help="step launches per HIP graph replay (0: direct launches; default: graphs "
                         "for the sweep, as many launches as the timed steps allow up to 100)")
    ap.add_argument("--chunk-rows", type=int, default=0)
    ap.add_argument("--shape", default=None,
                    help="waves,cols,cols_per_lane of the timed lattice's tile (lbm_set_tile; implies "
                         "--tile builtin for the chunk height unless --chunk-rows is given)")
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--no-builtin-figure", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 2 GiB read + 2 GiB write elementwise kernel, the "
                         "reference for scaling HBM byte counters")
    ap.add_argument("--traffic", default=None,
                    help="profile summary with measured HBM bytes per launch of the step kernel "
                         "(default: profiles/step_kernel_<workload>_<storage>_hbm_bytes.md)")
    ap.add_argument("--baseline-table", action="store_true",
                    help="time every named workload on the GPU and the oracle on the host")
    return ap.parse_args(argv)


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
        return W.cfg_sweep(), "f16", ("batched fingering sweep: 320 channels, H in {50,75,100,150,200}"
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
    if name == "wetting_batch":
        return W.cfg_wetting_batch(), "c16", ("curved-wall and capillary batch: 128 droplets on cylinders in "
                                              "400 x 400 boxes and 64 capillary channels, FP32 and 16-bit "
                                              "contexts (alternating domains)")
    return [W.cfg_droplet_flat()], "f64", "static droplet on a flat wall, 200 x 100, theta = 60 deg"


def graph_launches(requested, steps, default_on):
    if requested == 0 or (requested < 0 and not default_on):
        return 0
    n = requested if requested > 0 else min(100, steps)
    n -= n % 2
    return n if n >= 2 else 0


def time_lattice(setups, storage, steps, warmup, chunk_rows=0, tile="builtin", graph=0, lat=None,
                 shape=None):
    """Build a lattice (or reuse `lat`), set its shape and graph mode, run `warmup` untimed steps,
    then time `steps` steps with HIP events on the lattice's stream."""
    import torch
    from paper_1707_00198_amd.lbm import Lattice
    own = lat is None
    if own:
        lat = Lattice(setups, storage=storage)
    lat.set_graph(0)
    if tile == "autotune":
        t = lat.autotune(steps=10)
        print(f"[bench] autotuned tile: {t}", flush=True)
    else:
        lat.set_tile(chunk_rows, *(shape or ()))
    rule = "autotuned" if tile == "autotune" else ("set" if chunk_rows or shape else "built-in")
    shape = dict(lat.tile, rule=rule)
    lat.set_graph(graph)
    # the warm-up includes at least one replay of every graph the timed steps use
    lat.step(max(warmup, 2 * graph + 1) if graph else warmup)
    torch.cuda.synchronize()
    stream = lat.stream
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
    out = dict(fluid=fluid, event_ms=ev_ms, wall_s=wall, mlups=fluid * steps / (ev_ms * 1e-3) / 1e6,
               ms_per_step=ev_ms / steps, mass=mass, tile=shape, graph_launches=graph)
    if own:
        del lat
        torch.cuda.empty_cache()
    return out


def roofline_of(storage, fluid, ms_per_step, workload=None, traffic_path=None, tile=None):
    """Roofline record of the step launch: algorithmic bytes over the event-timed launch, and the
    counter-measured HBM bytes when a profile of this kernel source, workload, storage and tile
    shape exists.  `tile` is the lattice's tile dict (the two-column kernel when
    cols_per_lane = 2)."""
    bpl = BYTES_PER_LUP[storage]
    achieved = bpl * fluid / (ms_per_step * 1e-3) / 1e9
    traffic = None
    if workload is not None:
        traffic = measured_traffic(traffic_path or os.path.join(
            ROOT, "profiles", f"step_kernel_{workload}_{storage}_hbm_bytes.md"), workload, storage, tile)
    pair = bool(tile) and tile.get("cols_per_lane", 1) == 2
    kernel = f"pair_kernel<{KERNEL[storage]}>" if pair else f"step_kernel<{KERNEL[storage]}>"
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel=kernel, bytes_per_lup=bpl, lups_per_launch=fluid)


TILE_KEYS = ("chunk_rows", "waves", "cols", "cols_per_lane")


def measured_traffic(path, workload, storage, tile=None):
    """HBM bytes per launch from a committed counter summary (FETCH_SIZE + WRITE_SIZE, scaled by
    a copy kernel), or None if there is none, the kernel source has changed since, or the summary
    names a tile shape other than `tile` (when both are given)."""
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
    if tile and t.get("tile") and any(t["tile"].get(k) != tile.get(k, 1 if k == "cols_per_lane" else None)
                                      for k in TILE_KEYS):
        return None
    return t.get("bytes_per_launch")


# ------------------------------------------------------------------ accuracy of the 16-bit sweep
ACC_STEPS = 8000
ACC_THETA_STEPS = 6000


def accuracy_sample():
    """Two channels of each height of the sweep with Ca = 0.2 (the fastest fronts), so that the
    finger is tens to hundreds of nodes long after ACC_STEPS steps; indices into cfg_sweep()."""
    from paper_1707_00198_amd import workloads as W
    setups = W.cfg_sweep()
    pick, count = [], {}
    for d, s in enumerate(setups):
        if s.meta["ca"] == 0.2 and count.get(s.ny, 0) < 2:
            pick.append(d)
            count[s.ny] = count.get(s.ny, 0) + 1
    return [setups[d] for d in pick], pick


def sweep_accuracy(storage):
    """The 16-bit sweep's accuracy against FP64, outside the timed region: finger length and
    contact line of a sample of the sweep's own channels after ACC_STEPS steps, and the static
    contact angle of the Table I droplets (M = 1, five angles) after ACC_THETA_STEPS steps."""
    import torch
    from paper_1707_00198_amd import workloads as W
    from paper_1707_00198_amd.diagnostics import channel_interface
    from paper_1707_00198_amd.lbm import Lattice
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import physics

    chans, idx = accuracy_sample()
    res = {}
    for st in ("f64", storage):
        lat = Lattice(chans, storage=st).step(ACC_STEPS)
        res[st] = [channel_interface(lat, d, s.solid) for d, s in enumerate(chans)]
        del lat
    len_err = max(abs(g["length"] - r["length"]) / abs(r["length"]) for g, r in zip(res[storage], res["f64"]))
    cl_err = max(abs(g["contact_line"] - r["contact_line"]) for g, r in zip(res[storage], res["f64"]))
    travel = min(r["contact_line"] - s.meta["x_interface"] for r, s in zip(res["f64"], chans))

    boxes = [W.droplet_box(theta_deg=t, M=1.0, xc_offset=0.37) for t in (30.0, 60.0, 90.0, 120.0, 150.0)]
    ang = {}
    for st in ("f64", storage):
        lat = Lattice(boxes, storage=st).step(ACC_THETA_STEPS)
        ang[st] = []
        for d, s in enumerate(boxes):
            rr, rb = lat.densities(d)
            tot = np.where(rr + rb > 0, rr + rb, 1.0)
            ang[st].append(physics.flat_contact_angle((rr - rb) / tot, s.solid, 0.5)[0])
        del lat
    torch.cuda.empty_cache()
    th_err = max(abs(a - b) for a, b in zip(ang[storage], ang["f64"]))
    return dict(storage=storage, reference="f64",
                sample=f"{len(chans)} sweep channels (Ca = 0.2, two per height, indices {idx}), "
                       f"{ACC_STEPS} steps; Table I droplets (M = 1, theta 30..150), {ACC_THETA_STEPS} steps",
                finger_length_max_rel_err=round(len_err, 6), contact_line_max_abs_err=round(cl_err, 4),
                contact_line_min_travel=round(travel, 2), theta_max_abs_err_deg=round(th_err, 4),
                meets_gate=bool(len_err <= 0.01 and th_err <= 0.5))


# --------------------------------------------------------------------------- CPU oracle timing
def oracle_rate(setups, seconds, threads=None, chunk=20):
    """Fluid-node updates per second of the FP64 oracle stepping each domain in turn, for about
    `seconds` of wall time (at least one chunk per domain)."""
    import oracle
    cores = oracle.threads()
    if threads:
        oracle.set_threads(threads)
    try:
        orcs = [oracle.Oracle(s.solid, s.rho_r0, s.rho_b0, **s.oracle_kwargs()) for s in setups]
        for o in orcs:
            o.step(1)
        lups, t = 0, 0.0
        while t < seconds or lups == 0:
            for o, s in zip(orcs, setups):
                t0 = time.perf_counter()
                o.step(chunk)
                t += time.perf_counter() - t0
                lups += s.fluid_nodes * chunk
        return lups / t / 1e6, lups, t
    finally:
        oracle.set_threads(cores)


def cpu_baseline(seconds):
    """The FP64 oracle, as it is, on one H = 50 channel of the sweep (800 x 52 lattice),
    as many steps as fit in about `seconds`."""
    import oracle
    from paper_1707_00198_amd import workloads as W
    s = W.fingering_channel(nx=800, h=50, x_interface=100.0, M=10.0, theta_deg=60.0, ca=0.1,
                            nu_r=0.5, sigma=0.05)
    cores = oracle.threads()
    v, lups, t = oracle_rate([s], seconds)
    v1, _, _ = oracle_rate([s], seconds / 5.0, threads=1)
    return dict(value=v, unit="MLUPS", cores=cores, kind="oracle",
                sample=f"one 800 x 50 fingering channel of the sweep, {lups // s.fluid_nodes} steps in "
                       f"{t:.1f} s, FP64",
                value_one_thread=round(v1, 3))


# ------------------------------------------------------------------------- wetting batch
def run_wetting_batch(args, storage16):
    """Two contexts (domains alternate FP32 / 16-bit), each timed on its own; the combined rate
    is all fluid nodes over the summed step times."""
    setups, _, desc = build_workload("wetting_batch")
    parts = {"f32": setups[0::2], storage16: setups[1::2]}
    res = {}
    for st, doms in parts.items():
        r = time_lattice(doms, st, args.steps, args.warmup, args.chunk_rows,
                         args.tile or "builtin", graph_launches(args.graph, args.steps, False))
        r["roofline"] = roofline_of(st, r["fluid"], r["ms_per_step"], tile=r["tile"])
        res[st] = r
        print(f"[bench] wetting_batch {st} context: {len(doms)} domains, {r['fluid']} fluid nodes, "
              f"{r['mlups']:.1f} MLUPS, {r['ms_per_step']:.4f} ms/step", flush=True)
    fluid = sum(r["fluid"] for r in res.values())
    ms = sum(r["ms_per_step"] for r in res.values())
    dom = max(res, key=lambda k: res[k]["ms_per_step"])
    return desc, fluid, ms, res, dom


# ------------------------------------------------------------------------- baseline table
def baseline_table(args):
    """GPU MLUPS of every named workload and oracle MLUPS on the host (1 thread and all threads),
    printed as a markdown table and as JSON."""
    import oracle
    import torch
    from paper_1707_00198_amd import workloads as W
    rows = []
    cores = oracle.threads()

    def gpu(setups, storage, steps, tile="builtin", graph=0):
        r = time_lattice(setups, storage, steps, 20, 0, tile, graph)
        return round(r["mlups"], 1), round(BYTES_PER_LUP[storage] * r["mlups"] * 1e6 / 1e9 / HBM_PEAK_GBS, 4)

    def cpu(setups, seconds, chunk):
        v, _, _ = oracle_rate(setups, seconds, chunk=chunk)
        v1, _, _ = oracle_rate(setups, seconds / 2.0, threads=1, chunk=chunk)
        return round(v1, 2), round(v, 1)

    d = [W.cfg_droplet_flat()]
    rows.append(("cfg 1 droplet 200x100", "f64", *gpu(d, "f64", 5000), *cpu(d, 8.0, 100)))
    f = [W.cfg_fingering()]
    rows.append(("cfg 2 fingering 2000x100", "f64", *gpu(f, "f64", 2000), *cpu(f, 8.0, 20)))
    big = [W.cfg_fingering_large()]
    c1, c16 = cpu(big, 10.0, 2)
    for st in ("f64", "f32", "f16", "c16"):
        rows.append(("cfg 3 fingering 16384x512", st, *gpu(big, st, 500), c1, c16))
    sweep = W.cfg_sweep()
    heights, sample = set(), []
    for s in sweep:
        if s.ny not in heights:
            heights.add(s.ny)
            sample.append(s)
    cs = cpu(sample, 10.0, 4)
    g = graph_launches(-1, 500, True)
    for st in ("c16", "f16"):
        rows.append(("cfg 4 sweep 320 channels (graphs, autotuned)", st, *gpu(sweep, st, 500, "autotune", g), *cs))
    wb = W.cfg_wetting_batch()
    cw = cpu([wb[0], wb[1], wb[128], wb[129]], 10.0, 2)
    for st in ("f32", "c16"):
        part = wb[0::2] if st == "f32" else wb[1::2]
        rows.append((f"cfg 5 wetting batch, {st} context", st, *gpu(part, st, 500), *cw))
    torch.cuda.empty_cache()
    print("| workload | storage | GPU MLUPS | GPU HBM fraction (algorithmic) | oracle MLUPS 1 thread | "
          f"oracle MLUPS {cores} threads |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        print("| " + " | ".join(str(v) for v in r) + " |")
    print(json.dumps(dict(host_threads=cores, rows=rows)), flush=True)


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
    if args.baseline_table:
        baseline_table(args)
        return
    if args.calibrate_copy:
        copy_calibration()

    extra = {}
    if args.workload == "wetting_batch":
        storage = args.storage if args.storage in ("f16", "c16") else "c16"
        desc, fluid, ms, res, dom = run_wetting_batch(args, storage)
        head = dict(fluid=fluid, ms_per_step=ms, mlups=fluid / (ms * 1e-3) / 1e6,
                    tile={k: r["tile"] for k, r in res.items()}, mass=None)
        n_doms = 192
        dtype = "f32"
        roofline = res[dom]["roofline"]
        extra["contexts"] = {k: dict(mlups=round(r["mlups"], 1), ms_per_step=round(r["ms_per_step"], 5),
                                     fluid_nodes=r["fluid"], roofline=r["roofline"]) for k, r in res.items()}
        args.no_fp64_reference = True
        storage_desc = f"f32 + {storage}"
    else:
        setups, storage, desc = build_workload(args.workload)
        if args.storage:
            storage = args.storage
        sweep = args.workload == "sweep"
        shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else None
        tile = args.tile or ("autotune" if sweep and shape is None else "builtin")
        graph = graph_launches(args.graph, args.steps, sweep)
        print(f"[bench] workload {args.workload}: {len(setups)} domains, "
              f"{sum(s.fluid_nodes for s in setups)} fluid nodes, storage {storage}, tile {tile}, "
              f"graph launches {graph}", flush=True)
        from paper_1707_00198_amd.lbm import Lattice
        lat = Lattice(setups, storage=storage)
        head = time_lattice(setups, storage, args.steps, args.warmup, args.chunk_rows, tile, graph, lat=lat,
                            shape=shape)
        print(f"[bench] {args.workload} {storage}: {head['mlups']:.1f} MLUPS, "
              f"{head['ms_per_step']:.4f} ms/step ({head['tile']}, graph launches {graph})", flush=True)
        if not args.no_builtin_figure and (tile != "builtin" or graph):
            b = time_lattice(setups, storage, args.steps, args.warmup, 0, "builtin", 0, lat=lat)
            print(f"[bench] {args.workload} {storage}, built-in shape, direct launches: {b['mlups']:.1f} MLUPS",
                  flush=True)
            extra["builtin_shape_direct_launches"] = dict(mlups=round(b["mlups"], 1),
                                                          ms_per_step=round(b["ms_per_step"], 5),
                                                          tile=b["tile"])
        del lat
        torch.cuda.empty_cache()
        n_doms = len(setups)
        dtype = ARITH[storage]
        roofline = roofline_of(storage, head["fluid"], head["ms_per_step"], args.workload, args.traffic,
                               head["tile"])
        storage_desc = storage
        del setups

    ref = None
    if not args.no_fp64_reference and not (args.workload == "fingering_large" and storage == "f64"):
        ref_setups, _, _ = build_workload("fingering_large")
        ref = time_lattice(ref_setups, "f64", max(20, args.steps // 2), args.warmup)
        print(f"[bench] fingering_large f64: {ref['mlups']:.1f} MLUPS", flush=True)
        del ref_setups

    acc = None
    if args.workload == "sweep" and not args.no_accuracy and storage != "f64":
        acc = sweep_accuracy(storage)
        print(f"[bench] accuracy of the {storage} sweep against FP64: {acc}", flush=True)

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
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": desc, "storage": storage_desc, "domains": n_doms,
                   "fluid_nodes": head["fluid"], "tile": head["tile"],
                   "graph_launches": head.get("graph_launches", 0)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    if acc is not None:
        out["accuracy"] = acc
    if ref is not None:
        out["fp64_single_domain"] = {"workload": "fingering channel 16384 x 512 (FP64 storage and arithmetic)",
                                     "mlups": round(ref["mlups"], 1),
                                     "ms_per_step": round(ref["ms_per_step"], 5),
                                     "hbm_frac": round(BYTES_PER_LUP["f64"] * ref["mlups"] * 1e6 / 1e9 / HBM_PEAK_GBS, 4)}
        out["ratio_vs_fp64_single_domain"] = round(head["mlups"] / ref["mlups"], 3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
