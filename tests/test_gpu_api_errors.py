"""Error behaviour of the C-ABI on a live context (include/lbmcg.h): every call returns its
documented status, leaves the state untouched, and the context stays usable afterwards."""
import ctypes as C

import numpy as np
import pytest

from paper_1707_00198_amd import workloads as W

pytestmark = pytest.mark.gpu

EINVAL, ENOMEM, ESTATE = -1, -2, -5


def _lat():
    from paper_1707_00198_amd.lbm import Lattice
    s = W.droplet_flat(nx=90, h=40, radius=14.0, theta_deg=60.0, xc=37.2, name="drop")
    return Lattice([s]).step(20)


def _lib():
    from paper_1707_00198_amd.lbm import load_library
    return load_library()


def test_diagnostics_need_an_attached_buffer():
    lat = _lat()
    L = _lib()
    out = np.zeros(4)
    dp = out.ctypes.data_as(C.POINTER(C.c_double))
    assert L.lbm_diag_velocity(lat._h, 0, dp) == ESTATE
    n = C.c_int(-1)
    buf = (C.c_int32 * 8)()
    assert L.lbm_diag_contact_line(lat._h, 0, buf, 8, C.byref(n)) == ESTATE
    assert "diagnostics buffer" in L.lbm_last_error().decode()
    # still usable: attach through the binding and query
    assert lat.velocity_stats().shape == (1, 2)


def test_contact_line_capacity_too_small_reports_the_count():
    lat = _lat()
    full = lat.contact_line(0)
    assert len(full) > 2
    L = _lib()
    n = C.c_int(-1)
    buf = (C.c_int32 * 2)(-7, -7)
    assert L.lbm_diag_contact_line(lat._h, 0, buf, 2, C.byref(n)) == ENOMEM
    assert n.value == len(full)
    assert list(buf) == [-7, -7]  # untouched
    assert L.lbm_diag_contact_line(lat._h, 5, buf, 2, C.byref(n)) == EINVAL


def test_bad_arguments_leave_the_state_untouched():
    lat = _lat()
    before = lat.pops(0)
    L = _lib()
    out = np.zeros(10)
    dp = out.ctypes.data_as(C.POINTER(C.c_double))
    assert L.lbm_read_fields(lat._h, 0, 1, dp, 10) == ENOMEM        # output too small
    assert L.lbm_read_fields(lat._h, 3, 1, dp, 10) == EINVAL        # no such domain
    assert L.lbm_read_fields(lat._h, 0, 64, dp, 10) == EINVAL       # unknown field bit
    assert L.lbm_set_tile(lat._h, 6, 0, 0, 0) == EINVAL                 # chunk not a multiple of 4
    assert L.lbm_set_tile(lat._h, 0, 3, 0, 0) == EINVAL                 # waves
    assert L.lbm_set_tile(lat._h, 0, 8, 2, 0) == EINVAL                 # 8 x 2 not provided
    assert np.array_equal(lat.pops(0), before)
    ref = _lat().step(30).pops(0)
    assert np.array_equal(lat.step(30).pops(0), ref)
