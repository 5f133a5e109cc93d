"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every entry point
include/lbmcg.h declares, sizes buffers and rejects invalid parameters before device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1707_00198_amd import lbm, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmcg.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("lbm_create", "lbm_step", "lbm_read_fields", "lbm_mass", "lbm_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = lbm.load_library()
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(declared_functions()) == set(lbm.PROTOTYPES)


def _desc(s):
    keep = []
    d = lbm.DomainDesc()
    solid = np.ascontiguousarray(s.solid, np.uint8)
    rr = np.ascontiguousarray(s.rho_r0)
    rb = np.ascontiguousarray(s.rho_b0)
    keep += [solid, rr, rb]
    d.nx, d.ny, d.open_x = s.nx, s.ny, int(s.open_x)
    d.wetting = s.wetting
    d.solid = solid.ctypes.data_as(C.POINTER(C.c_uint8))
    d.rho_r0 = rr.ctypes.data_as(C.POINTER(C.c_double))
    d.rho_b0 = rb.ctypes.data_as(C.POINTER(C.c_double))
    if s.open_x:
        iu = np.ascontiguousarray(s.inlet_ux)
        keep.append(iu)
        d.inlet_ux = iu.ctypes.data_as(C.POINTER(C.c_double))
    for k, v in s.params.items():
        setattr(d, k, float(v))
    return d, keep


def query(s, storage=0):
    L = lbm.load_library()
    d, keep = _desc(s)
    st, sc = C.c_size_t(), C.c_size_t()
    rc = L.lbm_query_bytes(C.byref(d), 1, storage, C.byref(st), C.byref(sc))
    return rc, st.value, sc.value, L.lbm_last_error().decode()


def test_query_sizes_scale_with_storage():
    s = W.cfg_droplet_flat()
    sizes = [query(s, k)[1] for k in range(3)]
    assert sizes[0] > sizes[1] > sizes[2]
    nodes = s.nx * s.ny
    # two buffers of 9 populations + 3 colour values (+ alignment)
    assert 2 * nodes * 12 * 8 <= sizes[0] < 2 * nodes * 12 * 8 * 1.2


@pytest.mark.parametrize("change,msg", [
    (dict(nu_r=0.0), "viscosity"), (dict(nu_b=-1.0), "viscosity"), (dict(theta_deg=181.0), "theta"),
    (dict(beta=1.5), "beta"), (dict(s_q=2.0), "relaxation"), (dict(eps=0.0), "eps"),
])
def test_invalid_parameters_are_rejected(change, msg):
    s = W.cfg_droplet_flat()
    s.params = dict(s.params, **change)
    rc, *_, err = query(s)
    assert rc == -1 and msg in err


def test_invalid_geometry_is_rejected():
    s = W.cfg_droplet_flat()
    s.rho_r0 = s.rho_r0.copy()
    s.rho_r0[5, 5] = np.nan
    rc, *_, err = query(s)
    assert rc == -1 and "density" in err
    s = W.fingering_channel(nx=40, h=8)
    s.inlet_ux = s.inlet_ux * 1000  # peak 3.0, beyond the lattice speed limit
    rc, *_, err = query(s)
    assert rc == -1 and "inlet" in err
    assert query(s, storage=7)[0] == -1


def test_wetting_flags_validated():
    s = W.cfg_droplet_flat()
    for ok in (W.WET_SCHEME_B, W.WET_SURFACE_ENERGY, W.WET_SCHEME_B | W.WET_SURFACE_ENERGY):
        s.wetting = ok
        assert query(s)[0] == 0
    s.wetting = 4
    rc, *_, err = query(s)
    assert rc == -1 and "wetting" in err


def test_graph_and_autotune_reject_null_arguments():
    L = lbm.load_library()
    assert L.lbm_set_graph(None, 8) == -1 and "null context" in L.lbm_last_error().decode()
    shape = (C.c_int * 4)()
    assert L.lbm_get_tile(None, shape) == -1 and "null" in L.lbm_last_error().decode()
    out = (C.c_double * 4)()
    assert L.lbm_autotune(None, 5, None, out) == -1 and "null" in L.lbm_last_error().decode()


def test_empty_batch_is_rejected():
    L = lbm.load_library()
    st, sc = C.c_size_t(), C.c_size_t()
    assert L.lbm_query_bytes(None, 0, 0, C.byref(st), C.byref(sc)) == -1
    assert "at least one domain" in L.lbm_last_error().decode()


def test_context_beyond_the_buffer_limit_is_rejected_before_device_work():
    """The step kernel addresses the 9 population planes as one buffer below 2^31 bytes: an
    FP64 batch of more than 2^31 / 72 nodes is refused by lbm_create with a clear message, before
    any device buffer is touched (NULL buffers here), while FP32 storage of the same batch fits."""
    ny, nx = 5002, 6000  # 30.0 M nodes: 9 x 8 B x 30 M > 2^31, 9 x 4 B x 30 M < 2^31
    solid = np.zeros((ny, nx), np.uint8)
    solid[0, :] = solid[-1, :] = 1
    rr = np.where(solid == 0, 1.0, 0.0)
    rb = np.zeros_like(rr)
    s = W.Setup("huge", solid, rr, rb, W._phys())
    L = lbm.load_library()
    d, keep = _desc(s)
    h = C.c_void_p()
    rc = L.lbm_create(C.byref(d), 1, 0, None, 0, None, 0, None, C.byref(h))
    assert rc == -1 and "context's limit" in L.lbm_last_error().decode()
    rc = L.lbm_create(C.byref(d), 1, 1, None, 0, None, 0, None, C.byref(h))
    assert rc == -1 and "NULL" in L.lbm_last_error().decode()


def test_lattice_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        lbm.Lattice([W.cfg_droplet_flat()])


def classify(s):
    L = lbm.load_library()
    d, keep = _desc(s)
    if s.ns is not None:
        ns = np.ascontiguousarray(s.ns, dtype=np.float64)
        keep.append(ns)
        d.ns = ns.ctypes.data_as(C.POINTER(C.c_double))
    cls = np.empty((s.ny, s.nx), np.uint8)
    nrm = np.empty((s.ny, s.nx, 2))
    rc = L.lbm_classify(C.byref(d), cls.ctypes.data_as(C.POINTER(C.c_uint8)),
                        nrm.ctypes.data_as(C.POINTER(C.c_double)))
    assert rc == 0, L.lbm_last_error()
    return cls, nrm


def _classify_cases():
    import test_gpu_parity as T
    out = list(T.ragged_cases())
    out += [W.cylinder_droplet(n=96, rc=20.0, rd=18.0, theta_deg=120.0, ccx=48.0, ccy=30.0),
            W.cylinder_droplet(n=64, rc=12.0, rd=10.0, analytic_normals=True, ccx=32.0, ccy=20.0),
            W.capillary(nx=120, ny=30, plate_x0=30, plate_x1=90, thick=5, blue_x0=40, blue_x1=100),
            W.fingering_channel(nx=80, h=12), W.droplet_box(nx=40, ny=30, radius=10.0)]
    return out


@pytest.mark.parametrize("idx", range(13))
def test_library_classification_matches_oracle(idx):
    """Node classes and wall normals (Eqs. 32-33 or analytic) computed by the library's host
    runtime equal the oracle's, bit for bit."""
    import oracle
    s = _classify_cases()[idx]
    cls, nrm = classify(s)
    o = oracle.Oracle(s.solid, s.rho_r0, s.rho_b0, **s.oracle_kwargs())
    assert np.array_equal(cls, o.classes())
    assert np.array_equal(nrm, o.wall_normals())


def test_c_example_is_built_and_reports_a_missing_device():
    """The plain-C driver of the interface (csrc/c_api_example.c) is built with the library; it
    rejects a bad storage name before touching HIP, and without a usable device it says so and
    exits with status 2 instead of crashing."""
    import subprocess
    exe = os.path.join(ROOT, "paper_1707_00198_amd", "lbm_c_example")
    assert os.path.exists(exe), "built by __graft_entry__.build()"
    r = subprocess.run([exe, "f128"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage" in r.stderr
    import torch
    if torch.cuda.is_available():
        return
    r = subprocess.run([exe, "f64", "1"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "no HIP device" in r.stderr
