"""Parity at the full benchmark sizes, in the launch configuration bench.py times.

The oracle cannot step the full domains in test time, so the GPU state after k steps is read
back and the oracle advances sampled parts of it by one step from exactly that state; the
GPU's own step k+1 must agree.

* 16384 x 512 fingering channel, FP64: full-height windows 48 columns wide at the inlet, at the
  interface, in the middle and at the outlet.  The oracle treats a window's cut edges as
  periodic (or as an open end), which changes results only within the step's dependency radius
  (5 columns) of a cut; columns at least 8 away from every cut are compared, element by element,
  to 1e-10.
* The 320-channel sweep in both 16-bit storages (binary16, the benchmark's, and the format with
  an 11-bit fraction): 30 steps as graph replays of the built-in shape (which the autotuner
  keeps on this batch), then four whole channels (one of each height but one) are stepped by
  the oracle from the decoded state.  The GPU computes in FP32 and rounds the stored
  deviations to 16 bits, so each population must agree within one unit of the format's
  stochastic rounding of its deviation from w rho0 (2^-10 for binary16, 2^-11 for the other)
  plus 2e-6 (FP32 arithmetic on O(1) values).
"""
import numpy as np
import pytest

import oracle
from paper_1707_00198_amd import workloads as W

pytestmark = pytest.mark.gpu

WEIGHTS = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
MARGIN = 8


def _window_oracle(s, pops, x0, x1, open_x):
    """Oracle on columns [x0, x1) of setup s, holding the given (2, 9, ny, nx) state."""
    kw = s.oracle_kwargs()
    kw["open_x"] = open_x
    if not open_x:
        kw.pop("inlet_ux", None)
    sub = lambda a: np.ascontiguousarray(a[:, x0:x1])
    if kw.get("ns") is not None:
        kw["ns"] = sub(kw["ns"])
    o = oracle.Oracle(sub(s.solid), sub(s.rho_r0), sub(s.rho_b0), **kw)
    o.set_pops(np.ascontiguousarray(pops[:, :, :, x0:x1]))
    return o


def test_fullsize_fp64_channel_sampled_windows():
    from paper_1707_00198_amd.lbm import Lattice
    s = W.cfg_fingering_large()
    nx = s.solid.shape[1]
    lat = Lattice([s], storage="f64")
    lat.step(20)
    before = lat.pops(0)
    lat.step(1)
    after = lat.pops(0)
    del lat
    # (x0, x1, open_x, compared columns relative to x0)
    windows = [(0, 48, True, (0, 48 - MARGIN)),                     # real inlet
               (1000, 1048, False, (MARGIN, 48 - MARGIN)),          # interface
               (8000, 8048, False, (MARGIN, 48 - MARGIN)),          # bulk
               (nx - 48, nx, True, (MARGIN, 48))]                   # real outlet
    for x0, x1, open_x, (c0, c1) in windows:
        o = _window_oracle(s, before, x0, x1, open_x).step(1)
        ref = o.pops()[:, :, :, c0:c1]
        got = after[:, :, :, x0 + c0:x0 + c1]
        err = np.abs(got - ref).max()
        print(f"[fullsize] 16384x512 window [{x0}, {x1}): max |gpu - oracle| = {err:.3e}", flush=True)
        assert np.isfinite(got).all()
        assert err <= 1e-10


@pytest.mark.parametrize("storage,rel", [("f16", 2.0 ** -10), ("c16", 2.0 ** -11)])
def test_fullsize_sweep_sampled_channels(storage, rel):
    from paper_1707_00198_amd.lbm import Lattice
    setups = W.cfg_sweep()
    lat = Lattice(setups, storage=storage)
    # the built-in launch configuration: 64-row chunks of 56-column strips, 4 wavefronts
    assert lat.tile == dict(chunk_rows=64, waves=4, cols=1, items=30592, cols_per_lane=1)
    lat.set_graph(10)
    lat.step(30)
    lat.set_graph(0)
    heights = {}
    for d, s in enumerate(setups):
        heights.setdefault(s.solid.shape[0], d)
    sample = sorted(heights.values())[:4]
    before = {d: lat.pops(d) for d in sample}
    lat.step(1)
    after = {d: lat.pops(d) for d in sample}
    del lat
    for d in sample:
        s = setups[d]
        o = oracle.Oracle(s.solid, s.rho_r0, s.rho_b0, **s.oracle_kwargs())
        o.set_pops(before[d])
        ref = o.step(1).pops()
        fluid = s.solid == 0
        dev = np.abs(ref.sum(axis=0) - WEIGHTS[:, None, None] * s.params["rho0"] * fluid)
        tol = dev * rel + 2e-6  # one unit of the stochastically rounded 16-bit store
        err = np.abs(after[d] - ref)
        worst = (err / tol[None]).max()
        print(f"[fullsize] {storage} sweep channel {d} ({s.solid.shape[1]} x {s.solid.shape[0]}): "
              f"max |gpu - oracle| = {err.max():.3e}, max error / tolerance = {worst:.3f}", flush=True)
        assert np.isfinite(after[d]).all()
        assert worst <= 1.0
