"""The headline workload over a long run: the 320-channel sweep in both 16-bit storages for 5000
steps (Sec. III D displacement channels, one launch per step).

Every channel stays finite, and its colour masses follow the FP64 path: the red-mass growth
(the injected red, Zou-He inlet of Sec. III D) and the total mass of each of the first 40
channels agree with an FP64 run of the same channels: within 1 % (red growth) and 1e-3 (total
mass); measured with stochastically rounded stores: 1.3e-4 and 1.2e-5 (binary16), 2.2e-4 and
4.5e-6 (c16; 1.2e-3 and 1.8e-4 with round-to-nearest stores).  The red mass
grows by 1.00-1.11 times the nominal inflow sum(u_in) t, and the total mass rises by up to 10 %:
the inlet density rises above rho0 with the pressure drop of the high-viscosity-ratio channels,
and the convective outlet pins no density level.  Both paths show the same.
"""
import numpy as np
import pytest

from paper_1707_00198_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 5000
N_REF = 40


def _masses(setups, storage):
    from paper_1707_00198_amd.lbm import Lattice
    lat = Lattice(setups, storage=storage)
    m0 = lat.mass()
    lat.step(STEPS)
    m1 = lat.mass()  # raises LBMError if a non-finite value appeared
    del lat
    return m0, m1


_F64 = {}


def _reference(sw):
    if "m" not in _F64:
        _F64["m"] = _masses(sw[:N_REF], "f64")
    return _F64["m"]


@pytest.mark.parametrize("storage", ["f16", "c16"])
def test_sweep_long_run_follows_fp64(storage):
    sw = W.cfg_sweep()
    m0, m1 = _masses(sw, storage)
    r0, r1 = _reference(sw)
    grow = m1[:N_REF, 0] - m0[:N_REF, 0]
    grow64 = r1[:, 0] - r0[:, 0]
    tot = m1[:N_REF].sum(1)
    tot64 = r1.sum(1)
    e_grow = np.abs(grow / grow64 - 1.0).max()
    e_tot = np.abs(tot / tot64 - 1.0).max()
    flux = np.array([float(np.sum(s.inlet_ux)) for s in sw])
    ratio = (m1[:, 0] - m0[:, 0]) / (flux * STEPS)
    print(f"[longrun] {storage} vs f64 over {N_REF} channels: red growth {e_grow:.2e}, total {e_tot:.2e}; "
          f"red growth / inflow {ratio.min():.4f} .. {ratio.max():.4f}", flush=True)
    assert np.all(np.isfinite(m1))
    assert 0.99 < ratio.min() and ratio.max() < 1.15
    assert e_grow < 0.01 and e_tot < 1e-3
