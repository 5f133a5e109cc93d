"""A domain at the top of a context filled to its limit.

The step kernel addresses the nine population planes with 32-bit byte offsets, so a context
holds fewer than 2^31 bytes of populations (lbm_create refuses more).  Here a pure-fluid box
fills the planes to over 97 % of that limit and a small two-phase droplet on a wall sits after
it, at the highest offsets.  The droplet's populations after 50 steps are identical, bit for
bit, to those of the same droplet run alone, and in FP64 they match the oracle to 1e-10.
"""
import numpy as np
import pytest

import oracle
from paper_1707_00198_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 50


@pytest.mark.parametrize("storage,fill,bytes_per", [("f64", (1776, 16384), 8), ("c16", (7250, 16384), 2)])
def test_domain_at_the_top_of_a_full_context(storage, fill, bytes_per):
    from paper_1707_00198_amd.lbm import Lattice
    small = W.droplet_flat(nx=120, h=50, radius=18.0, theta_deg=60.0, xc=57.37, name="drop")
    ny, nx = fill
    filler = W.Setup("filler", np.zeros((ny, nx), np.uint8), np.ones((ny, nx)), np.zeros((ny, nx)),
                     dict(small.params))
    nodes = ny * nx + small.solid.size
    share = 9 * bytes_per * nodes / 2.0 ** 31
    print(f"[max] {storage}: {nodes} nodes, population planes at {100 * share:.1f} % of 2^31 bytes",
          flush=True)
    assert 0.97 < share < 1.0
    lat = Lattice([filler, small], storage=storage).step(STEPS)
    got = lat.pops(1)
    lat.mass()  # raises LBMError if any domain, the filler included, went non-finite
    del lat, filler
    alone = Lattice([small], storage=storage).step(STEPS).pops(0)
    assert np.array_equal(got, alone)
    if storage == "f64":
        ref = oracle.Oracle(small.solid, small.rho_r0, small.rho_b0, **small.oracle_kwargs()).step(STEPS).pops()
        assert np.abs(got - ref).max() <= 1e-10
