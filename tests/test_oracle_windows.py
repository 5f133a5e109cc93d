"""The windowed one-step check used at full size (test_gpu_fullsize.py), validated on the CPU:
oracle windows cut from a full oracle state and stepped once reproduce the full oracle's next
step on the columns the check compares (at least 8 columns from every cut, with the real inlet
and outlet kept), so the method itself adds no error."""
import numpy as np

import oracle
from paper_1707_00198_amd import workloads as W
from test_gpu_fullsize import MARGIN, _window_oracle


def test_windows_reproduce_the_full_step():
    s = W.fingering_channel(nx=240, h=30, x_interface=60.0, M=10.0, theta_deg=60.0, ca=0.2,
                            nu_r=0.5, sigma=0.05)
    full = oracle.Oracle(s.solid, s.rho_r0, s.rho_b0, **s.oracle_kwargs()).step(120)
    before = full.pops()
    ref = full.step(1).pops()
    nx = s.solid.shape[1]
    for x0, x1, open_x, (c0, c1) in [(0, 40, True, (0, 40 - MARGIN)),
                                      (45, 85, False, (MARGIN, 40 - MARGIN)),
                                      (nx - 40, nx, True, (MARGIN, 40))]:
        got = _window_oracle(s, before, x0, x1, open_x).step(1).pops()[:, :, :, c0:c1]
        assert np.abs(got - ref[:, :, :, x0 + c0:x0 + c1]).max() <= 1e-14, (x0, x1)
