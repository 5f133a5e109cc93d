"""The paper's own displacement sweeps (Sec. III D), batched, on the 630 x 60 channel of Fig. 6.

* Sec. III D 2 (Fig. 8, Eqs. 50-51): M = 1, Ca = 0.5, contact angle 20..160 degrees, 15
  channels in one launch.  The steady contact-line speed dS/dt and finger growth dL/dt are
  compared with the printed linear fits, read with S and L exchanged (the printed Eq. 50 would
  put the contact line ahead of the mean injection speed 2 u0 / 3 for theta > 108 degrees,
  which the red volume balance forbids; exchanged, both fits agree with the oracle's runs).
* Sec. III D 4 (Fig. 9): theta = 90 degrees, Ca in {0.36, 0.48, 0.60, 0.72}, M from 1 to 1000,
  44 channels in one launch.  For M > 20 the contact line moves at 2 u0 / 3 and the finger
  length stops growing; below, dS/dt rises with M and falls with Ca.
Both sweeps run in FP64 and in the 16-bit c16 storage of the headline, to the same bounds (the
X9 batch reaches M = 1000, tau_B = 0.5015, over 50000 steps).
"""
import numpy as np
import pytest

import oracle
from paper_1707_00198_amd import workloads as W
from paper_1707_00198_amd.diagnostics import rate, track_channels

pytestmark = pytest.mark.gpu


def _lattice(setups, storage="f64"):
    from paper_1707_00198_amd.lbm import Lattice
    return Lattice(setups, storage=storage)


@pytest.mark.parametrize("case", ["x8_theta20", "x9_M1000_ca0.72"])
def test_parity_fp64_paper_channels(case):
    """FP64 parity with the oracle at the sweeps' extremes: the fast inlet of Sec. III D 2
    (u0 = 0.1) and the most viscous-contrast channel of Sec. III D 4 (nu_B = 0.0005)."""
    s = W.cfg_x8((20,))[0] if case.startswith("x8") else W.cfg_x9((0.72,), (1000,))[0]
    steps = 300
    g = _lattice([s]).step(steps).pops(0)
    r = oracle.Oracle(s.solid, s.rho_r0, s.rho_b0, **s.oracle_kwargs()).step(steps).pops()
    err = np.abs(g - r).max()
    print(f"[parity] {s.name}: max |gpu - oracle| = {err:.3e}", flush=True)
    assert np.isfinite(g).all() and err <= 1e-10


@pytest.mark.parametrize("storage", ["f64", "c16"])
def test_x8_wettability_speeds_follow_eqs_50_51(storage):
    setups = W.cfg_x8()
    lat = _lattice(setups, storage)
    t, S, L = track_channels(lat, range(len(setups)), 4500, 250)
    x0 = np.array([s.meta["x_interface"] - 0.5 for s in setups])
    ds = np.array([rate(t, S[d], 2000) for d in range(len(setups))])
    dl = np.array([rate(t, L[d], 2000) for d in range(len(setups))])
    thetas = np.array([s.params["theta_deg"] for s in setups])
    fit_l = 5.278e-2 + 1.280e-4 * thetas  # printed Eq. 50, read as dL/dt
    fit_s = 3.095e-2 - 1.212e-4 * thetas  # printed Eq. 51, read as dS/dt
    for k, th in enumerate(thetas):
        print(f"[x8 {storage}] theta={th:5.1f}: dS/dt {ds[k]:.5f} (fit {fit_s[k]:.5f}), "
              f"dL/dt {dl[k]:.5f} (fit {fit_l[k]:.5f}), S(4500) {S[k, -1] - x0[k]:.1f}", flush=True)
    U = setups[0].meta["U"]
    assert np.all(ds < U)  # the contact line cannot outrun the injected volume
    assert np.all(np.abs(dl / fit_l - 1) < 0.10)
    assert np.all(np.abs(ds / fit_s - 1) < 0.10)
    slope_s = np.polyfit(thetas, ds, 1)[0]
    slope_l = np.polyfit(thetas, dl, 1)[0]
    print(f"[x8 {storage}] slopes: dS/dt {slope_s:.3e} (fit -1.212e-4), dL/dt {slope_l:.3e} (fit 1.280e-4)")
    assert -1.212e-4 * 1.25 < slope_s < -1.212e-4 / 1.25
    assert 1.280e-4 / 1.25 < slope_l < 1.280e-4 * 1.25


@pytest.mark.parametrize("storage", ["f64", "c16"])
def test_x9_viscosity_ratio_and_capillary_number(storage):
    cas = (0.72, 0.60, 0.48, 0.36)
    Ms = (1, 2, 3, 5, 10, 20, 50, 100, 200, 500, 1000)
    setups = W.cfg_x9(cas, Ms)
    lat = _lattice(setups, storage)
    t, S, L = track_channels(lat, range(len(setups)), 50000, 2500)
    ds = np.array([rate(t, S[d], 20000) for d in range(len(setups))]).reshape(len(cas), len(Ms))
    dl = np.array([rate(t, L[d], 20000) for d in range(len(setups))]).reshape(len(cas), len(Ms))
    u0 = 0.01
    for i, ca in enumerate(cas):
        print(f"[x9 {storage}] Ca={ca}: dS/dt " + " ".join(f"{v:.5f}" for v in ds[i]), flush=True)
        print(f"[x9 {storage}] Ca={ca}: dL/dt " + " ".join(f"{v:+.5f}" for v in dl[i]), flush=True)
    assert np.isfinite(ds).all() and np.isfinite(dl).all()
    high = np.array(Ms) > 20
    assert np.all(np.abs(ds[:, high] / (2 * u0 / 3) - 1) < 0.03)
    assert np.all(np.abs(dl[:, high]) < 0.03 * u0)
    low = ~high
    assert np.all(np.diff(ds[:, low], axis=1) > -1e-5)       # rises with M
    assert np.all(np.diff(ds[:, low], axis=0) > -1e-5)       # falls with Ca (cas descending)
