"""JSON descriptions of the named workloads (python -m paper_1707_00198_amd.workloads <name>)."""
import contextlib
import io
import json

from paper_1707_00198_amd import workloads as W


def _printed(name):
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        W.main([name])
    return json.loads(buf.getvalue())


def test_sweep_description_matches_the_benchmark_batch():
    d = _printed("sweep")
    assert d["seed"] == W.SEED and d["domains"] == 320 and d["fluid_nodes"] == 82_560_000
    heights = sorted({x["ny"] - 2 for x in d["domain_list"]})
    assert heights == [50, 75, 100, 150, 200]
    assert all(x["open_x"] and x["nx"] == 16 * (x["ny"] - 2) for x in d["domain_list"])


def test_every_named_workload_is_described():
    for name in ("droplet", "fingering", "x8"):
        d = _printed(name)
        assert d["domains"] == len(d["domain_list"]) >= 1
        assert all(set(W.PHYS_KEYS) <= set(x["params"]) for x in d["domain_list"])
