"""Physics of the GPU path against the paper's printed numbers and closed forms (Secs. III B, C).

* Sec. III B (Tables III, IV): droplets on a cylinder (200 x 200, R = 40 for both), contact
  angles 30..150 degrees, with the eighth-order staircase wall normal and with the analytic
  (curved) one, ten domains in one launch.  After 20000 steps the contact angle from a circle
  fit and the law of cosines is within 3 degrees of the prescribed one up to 120 degrees (the
  paper prints no angles for this case, only Fig. 3; 120 degrees measures 122.6); at
  150 degrees the droplet creeps upward (the paper reports the same), so the angle is only
  bounded.  With the curved normal, |u|max (Table III, Table IV) and E_NPMT (Eq. 47, about
  the initial droplet circle) agree with Table IV within 10 % at every angle (measured: 4 % and
  3 %).  With the staircase normal, |u|max is within a factor 1.5 except at 90 degrees, where
  it grows with time (the droplet slides along the steps) and only the order is checked, and
  E_NPMT within a factor 1.4.
* Sec. III C (Eq. 49): capillary filling of a 21-wide, 201-long tube (400 x 35 periodic box),
  contact angles 10..60 degrees, M = 1 and M = 100, eight domains in one launch.  At M = 1
  Eq. 49 gives a constant speed d sigma cos(theta) / (6 mu L); at M = 100 its integral
  (6/d) [mu_B L x + (mu_R - mu_B) x^2 / 2] = sigma cos(theta) t + C predicts the meniscus.
* Failure handling: a state driven to overflow (sigma = 50) is reported as LBM_ENONFINITE.
"""
import json
import math
import os

import numpy as np
import pytest

import physics
from paper_1707_00198_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def _lattice(setups, storage="f64"):
    from paper_1707_00198_amd.lbm import Lattice
    return Lattice(setups, storage=storage)


def _rho_n(lat, d):
    rr, rb = lat.densities(d)
    tot = rr + rb
    tot[tot == 0] = 1.0
    return (rr - rb) / tot


def test_curved_wall_angles_and_tables_iii_iv():
    from paper_1707_00198_amd.diagnostics import circle_region, e_npmt
    tab = json.load(open(GOLDEN))["table4_cylinder"]
    thetas = tab["theta"]
    setups = [W.cylinder_droplet(theta_deg=float(t), dcx_offset=0.37, name=f"e8_{t}") for t in thetas]
    setups += [W.cylinder_droplet(theta_deg=float(t), dcx_offset=0.37, analytic_normals=True,
                                  name=f"curved_{t}") for t in thetas]
    lat = _lattice(setups).step(20000)
    stats = lat.velocity_stats()
    n = len(thetas)
    failures = []
    for d, s in enumerate(setups):
        k, kind = d % n, ("staircase" if d < n else "curved")
        th = thetas[k]
        angle, _ = physics.cylinder_contact_angle(_rho_n(lat, d), s.solid, s.meta["ccx"],
                                                  s.meta["ccy"], s.meta["rc"])
        region = circle_region(s.solid.shape, s.meta["dcx"], s.meta["dcy"], s.meta["rd"])
        npmt = e_npmt(lat.region_mass(d, region))
        umax = stats[d, 0]
        printed_u = tab[f"umax_1e4_{kind}"][k] * 1e-4
        printed_e = tab[f"npmt_1e2_{kind}"][k] * 1e-2
        print(f"[cylinder] {kind} theta={th}: angle {angle:.2f}, |u|max {umax:.3e} (Table IV "
              f"{printed_u:.2e}), E_NPMT {npmt:.4f} (Table IV {printed_e:.4f})", flush=True)
        ok_angle = abs(angle - th) <= 3.0 if th <= 120 else th <= angle <= th + 15.0
        f = 3.0 if (kind == "staircase" and th == 90) else (1.1 if kind == "curved" else 1.5)
        fe = 1.1 if kind == "curved" else 1.4
        ok_u = printed_u / f < umax < f * printed_u
        ok_e = printed_e / fe < npmt < fe * printed_e
        if not (ok_angle and ok_u and ok_e):
            failures.append((kind, th, angle, umax, npmt))
    assert not failures, failures


def _meniscus(lat, d, row, inlet_x):
    """Position of the red-to-blue rho^N crossing on the tube's centre row, measured from the
    tube inlet."""
    x = physics.row_crossing(_rho_n(lat, d)[row], int(math.ceil(inlet_x)))
    return math.nan if x is None else x - inlet_x


def test_washburn_capillary_filling_eq_49():
    thetas = (10.0, 30.0, 45.0, 60.0)
    setups = [W.capillary(theta_deg=t, M=M) for M in (1.0, 100.0) for t in thetas]
    lat = _lattice(setups)
    row = setups[0].solid.shape[0] // 2
    times, pos = [], []
    for _ in range(10):
        lat.step(20000)
        times.append(lat.steps)
        pos.append([_meniscus(lat, d, row, s.meta["inlet_x"]) for d, s in enumerate(setups)])
    times, pos = np.array(times, float), np.array(pos).T
    for d, s in enumerate(setups):
        p = s.params
        mu_r, mu_b = p["nu_r"], p["nu_b"]
        dd, L = s.meta["d"], s.meta["L"]
        sc = p["sigma"] * math.cos(math.radians(p["theta_deg"]))
        M = mu_r / mu_b
        if M == 1.0:
            speed = np.polyfit(times[1:], pos[d, 1:], 1)[0]
            want = dd * sc / (6.0 * mu_r * L)
            print(f"[washburn] theta={p['theta_deg']} M=1: speed {speed:.4e}, Eq. 49 {want:.4e}",
                  flush=True)
            assert abs(speed / want - 1.0) < 0.08
        else:
            F = lambda x: (6.0 / dd) * (mu_b * L * x + (mu_r - mu_b) * x * x / 2.0)
            a, b = (6.0 / dd) * (mu_r - mu_b) / 2.0, (6.0 / dd) * mu_b * L
            target = F(pos[d, 1]) + sc * (times[-1] - times[1])
            x_pred = (-b + math.sqrt(b * b + 4.0 * a * target)) / (2.0 * a)
            print(f"[washburn] theta={p['theta_deg']} M={M:g}: x(t_end) {pos[d, -1]:.2f}, "
                  f"Eq. 49 {x_pred:.2f}", flush=True)
            assert abs(pos[d, -1] / x_pred - 1.0) < 0.04


def test_overflowing_state_is_reported_as_nonfinite():
    from paper_1707_00198_amd.lbm import LBMError
    s = W.droplet_flat(nx=60, h=30, radius=10.0)
    s.params = dict(s.params, sigma=50.0)
    lat = _lattice([s])
    with pytest.raises(LBMError) as err:
        for _ in range(20):
            lat.step(100)
            lat.mass()
    assert err.value.code == -4
