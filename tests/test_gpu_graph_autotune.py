"""Step graphs and the tile-shape autotuner (include/lbmcg.h: lbm_set_graph, lbm_autotune).

* A graph replays a fixed run of step launches captured once per starting buffer parity; every
  replay is checked bit for bit against direct launches of the same steps, with the program's
  own eager work (mass sums, field reads) and synchronisations between replays, for FP64 and
  C16 storage, across odd remainders, the initial (node-local) state and a restored state.
* The autotuner runs real trial steps and restores the state from a saved copy: afterwards the
  populations and the step count are exactly as before, the shape it reports is one it offers,
  and later steps equal those of an untuned context (results do not depend on the tile shape).
"""
import dataclasses

import numpy as np
import pytest

from paper_1707_00198_amd import workloads as W

pytestmark = pytest.mark.gpu


def _setups():
    a = W.droplet_flat(nx=130, h=60, radius=20.0, theta_deg=50.0, xc=61.3, name="a")
    b = W.cylinder_droplet(n=120, rc=25.0, rd=24.0, theta_deg=120.0, ccx=60.0, ccy=40.0, name="b")
    c = W.fingering_channel(nx=400, h=40, x_interface=80.0, M=10.0, theta_deg=60.0, ca=0.1, name="c")
    d = dataclasses.replace(W.droplet_flat(nx=100, h=50, radius=15.0, theta_deg=120.0, name="d"),
                            wetting=W.WET_SCHEME_B)
    return [a, b, c, d]


def _lat(storage):
    from paper_1707_00198_amd.lbm import Lattice
    return Lattice(_setups(), storage=storage)


def _pops(lat):
    return [lat.pops(i) for i in range(4)]


def _same(p, q):
    return all(np.array_equal(x, y) for x, y in zip(p, q))


@pytest.mark.parametrize("storage", ["f64", "c16"])
def test_graph_replays_match_direct_launches(storage):
    g, ref = _lat(storage).set_graph(8), _lat(storage)
    for n in (1, 7, 8, 16, 3, 24, 2):
        g.step(n)
        ref.step(n)
        mg, mr = g.mass(), ref.mass()  # eager work and a synchronisation between replays
        assert g.steps == ref.steps
        assert np.array_equal(mg, mr), n
        assert _same(_pops(g), _pops(ref)), n
    # restore a state saved on the other parity: replays then start from the other graph
    snap = ref.save_state()
    ref.step(1)
    g.step(1)
    g.load_state(snap)
    ref.load_state(snap)
    g.set_graph(4)
    for n in (4, 9, 12):
        g.step(n)
        ref.step(n)
        g.synchronize()
        assert _same(_pops(g), _pops(ref)), ("after load", n)


def test_graph_of_a_new_context_starts_with_a_direct_step():
    g, ref = _lat("f32").set_graph(2), _lat("f32")
    g.step(2)  # the initial state is node-local: one direct step, then one direct step
    ref.step(2)
    assert g.steps == 2 and _same(_pops(g), _pops(ref))
    g.step(40)
    ref.step(40)
    assert _same(_pops(g), _pops(ref))


def test_set_graph_rejects_odd_and_oversized_counts():
    from paper_1707_00198_amd.lbm import LBMError
    lat = _lat("f32")
    for bad in (3, -2, 1, 2048):
        with pytest.raises(LBMError):
            lat.set_graph(bad)
    lat.set_graph(0).step(5)


@pytest.mark.parametrize("storage", ["f64", "c16"])
def test_autotune_keeps_the_state_and_picks_an_offered_shape(storage):
    lat, ref = _lat(storage), _lat(storage)
    lat.step(50)
    ref.step(50)
    before = _pops(lat)
    info = lat.autotune(steps=3)
    assert lat.steps == 50
    assert _same(_pops(lat), before)
    assert info["chunk_rows"] in (8, 12, 16, 24, 32, 48, 64)
    assert (info["waves"], info["cols"]) in ((4, 1), (8, 1), (4, 2))
    assert info["ms_per_step"] > 0.0
    assert {k: lat.tile[k] for k in ("chunk_rows", "waves", "cols")} == \
        {k: info[k] for k in ("chunk_rows", "waves", "cols")}
    assert lat.tile["items"] > 0
    lat.set_graph(6)  # the tuned shape under replays too
    lat.step(37)
    ref.step(37)
    assert _same(_pops(lat), _pops(ref))
    assert np.array_equal(lat.mass(), ref.mass())
