"""Reduced-precision storage against FP64 storage, on the same seeded setups.

FP32 storage (FP32 arithmetic) and the 16-bit storages (binary16, and the format with an 11-bit
fraction, both with per-direction power-of-two scales, FP32 colour state and arithmetic) must
reproduce the FP64 path's physics:
  - static contact angle (the Table I flat-wall droplets, and droplets on a cylinder with
    staircase and analytic wall normals) within 0.5 degrees;
  - finger length of a displacement channel (tip minus contact line) within 1 %, and the tip
    velocity over the last 2000 steps within 1 % (measured, with the 16-bit stores rounded
    stochastically: at most 0.04 % in every storage; with round-to-nearest stores binary16 had
    been 0.7-1.6 % short and up to 2 % slow);
  - distance travelled by a capillary-filling meniscus (Eq. 49) within 1 % (binary16: 3 %,
    measured 1.0-1.3 %);
  - the spurious-velocity level |u|max of static droplets within 1 % (FP32) or 10 % (16-bit).
Colour-mass drift is printed for the record and only bounded loosely: the FP64 path conserves
it to rounding (tests/test_gpu_parity.py), the reduced paths round every stored population.
"""
import numpy as np
import pytest

from paper_1707_00198_amd import workloads as W
from physics import finger_metrics, flat_contact_angle

pytestmark = pytest.mark.gpu

DROPLETS = [(30.0, 1.0), (60.0, 1.0), (120.0, 10.0), (150.0, 1.0)]  # (theta, M) of Table I
DROPLET_STEPS = 6000
# (M, theta, Ca): cases that grow a finger (tens of lattice units long), so that 1 % is a
# resolvable length
FINGERS = [(1.0, 60.0, 0.2), (5.0, 60.0, 0.2), (1.0, 120.0, 0.1)]
FINGER_STEPS = 12000


def _rho_n(lat, d):
    rr, rb = lat.densities(d)
    s = rr + rb
    s[s == 0] = 1.0
    return (rr - rb) / s


def _run(setups, storage, steps):
    from paper_1707_00198_amd.lbm import Lattice
    lat = Lattice(setups, storage=storage)
    m0 = lat.mass()
    lat.step(steps)
    m1 = lat.mass()
    fields = [_rho_n(lat, d) for d in range(len(setups))]
    del lat
    return fields, m0, m1


@pytest.fixture(scope="module")
def droplet_runs():
    # off the box's mirror axis, so that no Eq. 36 selection is a tie
    setups = [W.droplet_box(theta_deg=th, M=M, xc_offset=0.37) for th, M in DROPLETS]
    out = {}
    for st in ("f64", "f32", "f16", "c16"):
        fields, m0, m1 = _run(setups, st, DROPLET_STEPS)
        angles = [flat_contact_angle(f, s.solid, 0.5)[0] for f, s in zip(fields, setups)]
        drift = np.abs(m1 - m0) / m0
        print(f"[precision] droplets {st}: theta = {np.round(angles, 3).tolist()}, "
              f"max colour-mass drift {drift.max():.2e}", flush=True)
        out[st] = (angles, drift)
    return out


TIP_WINDOW = 2000


@pytest.fixture(scope="module")
def finger_runs():
    from paper_1707_00198_amd.lbm import Lattice
    setups = [W.fingering_channel(nx=800, h=50, x_interface=100.0, M=M, theta_deg=th, ca=ca,
                                  nu_r=0.5, sigma=0.05) for M, th, ca in FINGERS]
    out = {}
    for st in ("f64", "f32", "f16", "c16"):
        lat = Lattice(setups, storage=st).step(FINGER_STEPS - TIP_WINDOW)
        tips = [finger_metrics(_rho_n(lat, d), s.solid)["tip"] for d, s in enumerate(setups)]
        lat.step(TIP_WINDOW)
        metrics = [finger_metrics(_rho_n(lat, d), s.solid) for d, s in enumerate(setups)]
        for m, t0 in zip(metrics, tips):
            m["tip_velocity"] = (m["tip"] - t0) / TIP_WINDOW
        del lat
        print(f"[precision] fingers {st}: length = "
              f"{[round(m['length'], 3) for m in metrics]}, tip velocity = "
              f"{[float('%.5g' % m['tip_velocity']) for m in metrics]}", flush=True)
        out[st] = metrics
    return out


CYLINDER_THETAS = (30.0, 60.0, 90.0, 120.0)
CYLINDER_STEPS = 10000


@pytest.fixture(scope="module")
def cylinder_runs():
    """Droplets on a cylinder (Sec. III B, 200 x 200, R = 40), eighth-order staircase normals and
    analytic ones, off the mirror axis."""
    from physics import cylinder_contact_angle
    setups = [W.cylinder_droplet(theta_deg=t, dcx_offset=0.37, analytic_normals=a, name=f"c{t}{a}")
              for a in (False, True) for t in CYLINDER_THETAS]
    out = {}
    for st in ("f64", "f32", "f16", "c16"):
        fields, _, _ = _run(setups, st, CYLINDER_STEPS)
        out[st] = [cylinder_contact_angle(f, s.solid, s.meta["ccx"], s.meta["ccy"], s.meta["rc"])[0]
                   for f, s in zip(fields, setups)]
        print(f"[precision] cylinders {st}: theta = {np.round(out[st], 3).tolist()}", flush=True)
    return out


@pytest.mark.parametrize("storage", ["f32", "f16", "c16"])
def test_curved_wall_contact_angle_within_half_degree_of_fp64(cylinder_runs, storage):
    d = np.abs(np.array(cylinder_runs[storage]) - np.array(cylinder_runs["f64"]))
    assert d.max() <= 0.5, (storage, d)


def test_spurious_velocity_level_follows_fp64():
    """|u|max (Eq. 46) of static droplets after 20000 steps: five on a cylinder (Tables III-IV,
    analytic normal) and five in the Table I box.  These velocities are 1e-5 to 3e-4, so the
    16-bit rounding of the populations shows: FP32 within 1 % of FP64, binary16 and c16 within
    10 % (measured: 0.2 %, 1.4 % and 6.4 %)."""
    from paper_1707_00198_amd.lbm import Lattice
    thetas = (30.0, 60.0, 90.0, 120.0, 150.0)
    setups = [W.cylinder_droplet(theta_deg=t, dcx_offset=0.37, analytic_normals=True, name=f"c{t}")
              for t in thetas] + [W.droplet_box(theta_deg=t, M=1.0, xc_offset=0.37) for t in thetas]
    umax = {}
    for st in ("f64", "f32", "f16", "c16"):
        lat = Lattice(setups, storage=st).step(20000)
        umax[st] = lat.velocity_stats()[:, 0]
        del lat
    for st, bound in (("f32", 0.01), ("f16", 0.10), ("c16", 0.10)):
        rel = np.abs(umax[st] / umax["f64"] - 1.0)
        print(f"[precision] |u|max {st}: largest deviation from FP64 {100 * rel.max():.2f} %", flush=True)
        assert np.all(rel < bound), (st, umax[st], umax["f64"])


def test_capillary_meniscus_within_one_percent_of_fp64():
    """Capillary filling (Sec. III C, Eq. 49) at theta = 30 and 60 degrees, M = 1 and 100:
    the distance the meniscus has travelled after 60000 steps agrees with FP64 within 1 % for
    FP32 and c16 (measured up to 0.86 %, c16 at M = 100); binary16 is bounded at 3 % (measured
    up to 1.35 %), as for the finger length."""
    from physics import row_crossing
    setups = [W.capillary(theta_deg=t, M=M) for M in (1.0, 100.0) for t in (30.0, 60.0)]
    row = setups[0].solid.shape[0] // 2
    travel = {}
    for st in ("f64", "f32", "f16", "c16"):
        fields, _, _ = _run(setups, st, 60000)
        travel[st] = np.array([row_crossing(f[row], int(np.ceil(s.meta["inlet_x"]))) - s.meta["inlet_x"]
                               for f, s in zip(fields, setups)])
        print(f"[precision] capillaries {st}: meniscus travel {np.round(travel[st], 3).tolist()}",
              flush=True)
    for st, bound in (("f32", 0.01), ("c16", 0.01), ("f16", 0.03)):
        rel = np.abs(travel[st] / travel["f64"] - 1.0)
        print(f"[precision] capillaries {st}: largest deviation from FP64 {100 * rel.max():.2f} %",
              flush=True)
        assert np.all(rel < bound), (st, travel[st], travel["f64"])


@pytest.mark.parametrize("storage", ["f32", "f16", "c16"])
def test_contact_angle_within_half_degree_of_fp64(droplet_runs, storage):
    ref, _ = droplet_runs["f64"]
    got, drift = droplet_runs[storage]
    for (th, M), a64, a in zip(DROPLETS, ref, got):
        assert abs(a - a64) <= 0.5, f"theta={th} M={M}: {storage} {a:.3f} vs f64 {a64:.3f}"
    assert drift.max() < (1e-4 if storage == "f32" else 1e-2)


@pytest.mark.parametrize("storage", ["f32", "c16", "f16"])
def test_finger_length_within_one_percent_of_fp64(finger_runs, storage):
    for (M, th, ca), m64, m in zip(FINGERS, finger_runs["f64"], finger_runs[storage]):
        assert m64["length"] is not None and m["length"] is not None
        rel = abs(m["length"] - m64["length"]) / abs(m64["length"])
        assert rel <= 0.01, (f"M={M} theta={th} Ca={ca}: {storage} length {m['length']:.3f} vs "
                             f"f64 {m64['length']:.3f} ({100 * rel:.2f} %)")


@pytest.mark.parametrize("storage,bound", [("f32", 0.01), ("c16", 0.01), ("f16", 0.01)])
def test_tip_velocity_against_fp64(finger_runs, storage, bound):
    for (M, th, ca), m64, m in zip(FINGERS, finger_runs["f64"], finger_runs[storage]):
        rel = abs(m["tip_velocity"] - m64["tip_velocity"]) / abs(m64["tip_velocity"])
        print(f"[precision] {storage} tip velocity M={M} theta={th} Ca={ca}: "
              f"{m['tip_velocity']:.5g} vs f64 {m64['tip_velocity']:.5g} ({100 * rel:.2f} %)",
              flush=True)
        assert rel <= bound


def test_binary16_finger_length_error_is_reported(finger_runs):
    """binary16 storage: the finger-length deviation from FP64 is recorded (and held to 1 % by
    test_finger_length_within_one_percent_of_fp64)."""
    for (M, th, ca), m64, m in zip(FINGERS, finger_runs["f64"], finger_runs["f16"]):
        rel = abs(m["length"] - m64["length"]) / abs(m64["length"])
        print(f"[precision] f16 finger M={M} theta={th} Ca={ca}: {100 * rel:.2f} %", flush=True)
        assert rel <= 0.01


def test_c16_initial_state_round_trip():
    """Host encoding and device decoding of the 16-bit format agree with the FP64 state to the
    format's rounding: |error| <= 2^-12 |f - w rho0| per population in the normal range, plus
    half a subnormal step (at most 2^-18 / 2^9) below it."""
    from paper_1707_00198_amd.lbm import Lattice
    s = W.droplet_flat(nx=120, h=40, radius=15.0)
    rng = np.random.default_rng(1707)
    fluid = s.solid == 0
    s.rho_r0 = np.where(fluid, s.rho_r0 * rng.uniform(0.9, 1.1, s.rho_r0.shape), 0.0)
    s.rho_b0 = np.where(fluid, s.rho_b0 * rng.uniform(0.9, 1.1, s.rho_b0.shape), 0.0)
    ref = Lattice([s], storage="f64").pops(0)
    got = Lattice([s], storage="c16").pops(0)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
    rho0 = s.params["rho0"]
    tot_ref, tot_got = ref.sum(axis=0), got.sum(axis=0)
    dev = np.abs(tot_ref - w * rho0 * fluid)
    err = np.abs(tot_got - tot_ref)
    assert np.all(err <= dev * 2.0 ** -12 * (1 + 1e-6) + 2.0 ** -27)
    assert err[:, fluid].max() > 0  # the format does round
