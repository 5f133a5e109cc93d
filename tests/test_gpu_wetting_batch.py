"""The curved-wall and capillary batch (Sec. III B droplets on cylinders, Sec. III C capillary
filling, Eq. 49) on a subset of its seeded domains.

Subset: the first eight 400 x 400 cylinder boxes (cylinder radius 40-80, droplet radius 20-40,
theta 20-160 degrees; even ones with the analytic wall normal, odd ones with the eighth-order
staircase estimate) and four capillary channels of different widths, angles and viscosity
ratios (tube length 1000 in a periodic 2000 x (d + 14) box).

* FP64 parity with the oracle (max-abs 1e-10 per population) after 200 steps, on one cylinder
  box with each kind of wall normal and on one capillary, all in one launch.
* FP32 and the 16-bit c16 storage (FP32 arithmetic), the mixed storages the batch is run with,
  against FP64 on the same domains: the droplets' contact angles after 10000 steps within 0.5
  degrees, and the distance the capillary menisci have travelled after 20000 steps within 1 %.
"""
import math

import numpy as np
import pytest

import oracle
import physics
from paper_1707_00198_amd import workloads as W

pytestmark = pytest.mark.gpu

CYL = 8
CAP = (0, 5, 10, 15)


def _subset():
    full = W.cfg_wetting_batch()
    return full[:CYL], [full[128 + k] for k in CAP]


def _rho_n(lat, d):
    rr, rb = lat.densities(d)
    tot = rr + rb
    tot[tot == 0] = 1.0
    return (rr - rb) / tot


def test_fp64_parity_cylinder_boxes_and_capillary():
    from paper_1707_00198_amd.lbm import Lattice
    cyl, cap = _subset()
    cases = [cyl[0], cyl[1], cap[1]]
    steps = 200
    lat = Lattice(cases, storage="f64").step(steps)
    for d, s in enumerate(cases):
        g = lat.pops(d)
        r = oracle.Oracle(s.solid, s.rho_r0, s.rho_b0, **s.oracle_kwargs()).step(steps).pops()
        err = np.abs(g - r).max()
        print(f"[wetting batch] {s.name} {s.nx}x{s.ny} analytic={s.ns is not None}: "
              f"max |gpu - oracle| = {err:.3e}", flush=True)
        assert np.isfinite(g).all() and err <= 1e-10


def test_reduced_storage_contact_angles_within_half_degree():
    from paper_1707_00198_amd.lbm import Lattice
    cyl, _ = _subset()
    angles = {}
    for st in ("f64", "f32", "c16"):
        lat = Lattice(cyl, storage=st).step(10000)
        angles[st] = np.array([physics.cylinder_contact_angle(_rho_n(lat, d), s.solid, s.meta["ccx"],
                                                              s.meta["ccy"], s.meta["rc"])[0]
                               for d, s in enumerate(cyl)])
        del lat
        print(f"[wetting batch] cylinders {st}: theta = {np.round(angles[st], 3).tolist()} "
              f"(prescribed {[round(s.params['theta_deg'], 1) for s in cyl]})", flush=True)
    for st in ("f32", "c16"):
        d = np.abs(angles[st] - angles["f64"])
        print(f"[wetting batch] {st}: largest contact-angle difference to FP64 {d.max():.4f} deg", flush=True)
        assert d.max() <= 0.5, (st, d)


def test_reduced_storage_capillary_travel_within_one_percent():
    from paper_1707_00198_amd.lbm import Lattice
    _, cap = _subset()
    travel = {}
    for st in ("f64", "f32", "c16"):
        lat = Lattice(cap, storage=st).step(20000)
        out = []
        for d, s in enumerate(cap):
            row = s.solid.shape[0] // 2
            x = physics.row_crossing(_rho_n(lat, d)[row], int(math.ceil(s.meta["inlet_x"])))
            out.append(np.nan if x is None else x - s.meta["front_x0"])
        travel[st] = np.array(out)
        del lat
        print(f"[wetting batch] capillaries {st}: meniscus travel {np.round(travel[st], 3).tolist()} "
              f"(widths {[s.meta['d'] for s in cap]})", flush=True)
    assert np.all(travel["f64"] > 5.0)
    for st in ("f32", "c16"):
        rel = np.abs(travel[st] / travel["f64"] - 1.0)
        print(f"[wetting batch] {st}: largest travel difference to FP64 {100 * rel.max():.3f} %", flush=True)
        assert np.all(rel <= 0.01), (st, travel[st], travel["f64"])
