"""The 16384 x 512 displacement channel (M = 50, theta = 30 degrees, Ca = 0.2) at full size, in
every storage, against the FP64 run (Sec. III D: contact line S(t), finger length L(t)).

Each storage advances the same channel by 30000 steps (the mean front travels about 600 nodes);
every 1000 steps the contact line (rho^N = 0 crossing on the two fluid rows next to the walls),
the tip (crossing on the two centre rows) and the finger length tip - contact line are read on
the device (lbm_diag_crossings).  Measures against FP64:
  - tip velocity, the least-squares slope of the tip over the last 10000 steps, and finger length
    at the end: within 1 % for FP32 and for the 11-bit-fraction 16-bit format (measured 0.001 % /
    0.12 % for FP32 and 0.003 % / 0.001 % for the 16-bit format, whose stores round
    stochastically; with round-to-nearest stores the 16-bit tip had run 0.36 % fast and the
    finger, 42 nodes long, had come out 1.09 % long: a systematic drift that stochastic rounding
    removes);
  - colour masses (FP64 sums) at the end: printed, and within 1e-3 relative (the inlet injects
    red fluid, so the masses are not conserved; the difference to FP64 is the drift);
  - binary16, also with stochastically rounded stores: within 1 % as well (measured 0.004 % tip
    velocity, 0.21 % finger length; with round-to-nearest stores 0.72 % and 2.58 %).
"""
import numpy as np
import pytest

from paper_1707_00198_amd import workloads as W
from paper_1707_00198_amd.diagnostics import channel_interface, rate

pytestmark = pytest.mark.gpu

STEPS = 30000
EVERY = 1000
TIP_WINDOW = 10000


@pytest.fixture(scope="module")
def runs():
    from paper_1707_00198_amd.lbm import Lattice
    import torch
    s = W.cfg_fingering_large()
    out = {}
    for st in ("f64", "f32", "c16", "f16"):
        print(f"[config 3] {st}: {s.nx} x {s.ny}, {STEPS} steps", flush=True)
        lat = Lattice([s], storage=st)
        m0 = lat.mass()[0]
        t, tip, cl, ln = [], [], [], []
        for _ in range(STEPS // EVERY):
            lat.step(EVERY)
            m = channel_interface(lat, 0, s.solid)
            t.append(lat.steps)
            tip.append(np.nan if m["tip"] is None else m["tip"])
            cl.append(np.nan if m["contact_line"] is None else m["contact_line"])
            ln.append(np.nan if m["length"] is None else m["length"])
        m1 = lat.mass()[0]
        del lat
        torch.cuda.empty_cache()
        t, tip, cl, ln = (np.array(v, dtype=np.float64) for v in (t, tip, cl, ln))
        r = dict(t=t, tip=tip, cl=cl, length=ln, mass0=m0, mass=m1,
                 tip_velocity=rate(t, tip, STEPS - TIP_WINDOW))
        print(f"[config 3] {st}: length every {EVERY} steps {np.round(ln, 3).tolist()}", flush=True)
        print(f"[config 3] {st}: contact line {cl[-1]:.3f}, tip {tip[-1]:.3f}, length {ln[-1]:.3f}, "
              f"tip velocity {r['tip_velocity']:.6g}, masses {m1[0]:.9g} / {m1[1]:.9g}", flush=True)
        out[st] = r
    return out


def test_fp64_channel_displaces(runs):
    r = runs["f64"]
    assert np.isfinite(r["tip"]).all() and np.isfinite(r["cl"]).all()
    assert r["cl"][-1] > r["cl"][0] + 100.0       # the contact line advances
    assert r["length"][-1] > 10.0                  # and a finger forms ahead of it
    U = W.cfg_fingering_large().meta["U"]
    assert 0.5 * U < r["tip_velocity"] < 3.0 * U


@pytest.mark.parametrize("storage,bound,len_bound", [("f32", 0.01, 0.01), ("c16", 0.01, 0.01),
                                                     ("f16", 0.01, 0.01)])
def test_reduced_storage_against_fp64(runs, storage, bound, len_bound):
    ref, got = runs["f64"], runs[storage]
    d_len = abs(got["length"][-1] - ref["length"][-1]) / abs(ref["length"][-1])
    d_tip = abs(got["tip_velocity"] - ref["tip_velocity"]) / abs(ref["tip_velocity"])
    d_cl = abs(got["cl"][-1] - ref["cl"][-1])
    d_mass = np.abs(got["mass"] - ref["mass"]) / ref["mass"]
    print(f"[config 3] {storage} vs f64: finger length {100 * d_len:.3f} %, tip velocity "
          f"{100 * d_tip:.3f} %, contact line {d_cl:.3f} nodes, masses {d_mass[0]:.2e} / "
          f"{d_mass[1]:.2e}", flush=True)
    assert np.isfinite(got["length"]).all()
    assert d_len <= len_bound
    assert d_tip <= bound
    assert d_mass.max() < 1e-3
