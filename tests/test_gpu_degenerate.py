"""Degenerate domains inside a batch, in every storage type.

* An all-solid domain has no fluid node: it reads back as zeros, its mass is (0, 0), and it
  does not disturb the domains launched with it.
* A pure phase with no solid (periodic box of red at rho0) has rho^N = 1 everywhere, so the
  colour gradient, the normals, the curvature and the force are exactly zero (Eqs. 28, 22, 13,
  10): the populations stay exactly at w_alpha rho0 in every storage, and the blue set is
  exactly zero.
* A pure blue box between walls stays pure: the red fraction c = rho_R / rho is exactly 0, so
  no red population appears (Eq. 14).  In FP64 the box also stays exactly at rest (the virtual
  rho^N of Eq. 29 is exactly -1); in FP32 arithmetic the wall stage's 1-ulp reciprocal can leave
  a gradient of order 1e-8, so there the populations are only checked to 1e-6.
* A two-phase droplet in the same launch matches the oracle (FP64).
"""
import numpy as np
import pytest

import oracle
from paper_1707_00198_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 200
WTS = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _setups():
    base = W.free_droplet(n=40, radius=8.0)
    solid = np.ones((12, 40), np.uint8)
    z = np.zeros(solid.shape)
    all_solid = W.Setup("all_solid", solid, z, z, dict(base.params))
    red = W.Setup("pure_red", np.zeros((20, 70), np.uint8), np.ones((20, 70)), np.zeros((20, 70)),
                  dict(base.params))
    ws = np.zeros((30, 60), np.uint8)
    ws[0, :] = ws[-1, :] = 1
    blue = W.Setup("pure_blue", ws, np.zeros(ws.shape), np.where(ws == 0, 1.0, 0.0),
                   dict(base.params, theta_deg=40.0))
    drop = W.droplet_flat(nx=90, h=40, radius=14.0, theta_deg=60.0, xc=37.2, name="drop")
    return [all_solid, red, blue, drop]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "c16"])
def test_degenerate_domains_in_a_batch(storage):
    from paper_1707_00198_amd.lbm import Lattice
    setups = _setups()
    lat = Lattice(setups, storage=storage).step(STEPS)
    mass = lat.mass()
    # all solid
    assert not np.any(lat.pops(0)) and np.array_equal(mass[0], [0.0, 0.0])
    # pure red, no solid: exactly at rest
    p = lat.pops(1)
    assert np.array_equal(p[0], np.broadcast_to(WTS[:, None, None], p[0].shape))
    assert not np.any(p[1])
    # pure blue between walls: no red appears
    p = lat.pops(2)
    fluid = setups[2].solid == 0
    assert not np.any(p[0])
    want = np.where(fluid, WTS[:, None, None], 0.0)
    if storage == "f64":
        assert np.array_equal(p[1], want)
    else:
        assert np.abs(p[1] - want).max() < 1e-6
    if storage == "f64":
        s = setups[3]
        ref = oracle.Oracle(s.solid, s.rho_r0, s.rho_b0, **s.oracle_kwargs()).step(STEPS).pops()
        assert np.abs(lat.pops(3) - ref).max() < 1e-10
