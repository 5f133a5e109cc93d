"""Plain FP64 CPU oracle of the colour-gradient LBM step with the improved wetting boundary
(arXiv:1707.00198, Sec. II).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline
leg of the benchmark.  The GPU library never imports, links or calls anything here, and this
package imports nothing from the GPU library.

The arithmetic lives in ``lbm_oracle.c`` (plain C, FP64, one pass per stage); this module is
argument marshalling only.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

DEFAULTS = dict(
    nu_r=1.0 / 6.0, nu_b=1.0 / 6.0, sigma=0.01, beta=0.7, theta_deg=90.0,
    s_e=1.64, s_eps=1.54, s_q=1.9, rho0=1.0, eps=1e-10, outlet_u=0.0,
    body_fx=0.0, body_fy=0.0,
)

FIELDS = ("rhoR", "rhoB", "rhoN", "gx", "gy", "nx", "ny", "kappa", "Fx", "Fy", "ux", "uy")


class OrcParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("open_x", C.c_int32), ("scheme", C.c_int32),
        ("nu_r", C.c_double), ("nu_b", C.c_double), ("sigma", C.c_double),
        ("beta", C.c_double), ("theta_deg", C.c_double), ("s_e", C.c_double),
        ("s_eps", C.c_double), ("s_q", C.c_double), ("rho0", C.c_double),
        ("eps", C.c_double), ("outlet_u", C.c_double), ("body_fx", C.c_double),
        ("body_fy", C.c_double), ("surface_energy", C.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitize_check(out: str = None) -> str:
    """Compile ``sanitize_check.c`` (the oracle driven over every entry point and the test
    geometries) with gcc's address and undefined-behaviour sanitizers into an executable."""
    out = out or os.path.join(_HERE, "sanitize_check")
    subprocess.check_call(["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall",
                           "-Wno-unknown-pragmas",
                           "-I", _HERE, "-o", out, os.path.join(_HERE, "sanitize_check.c"), "-lm"])
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        u8p = C.POINTER(C.c_uint8)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcParams), u8p, dp, dp, dp, dp]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_get_pops.argtypes = [C.c_void_p, dp]
        L.orc_set_pops.argtypes = [C.c_void_p, dp]
        L.orc_fields.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_fields.restype = C.c_int
        L.orc_classes.argtypes = [C.c_void_p, u8p]
        L.orc_wall_normals.argtypes = [C.c_void_p, dp]
        L.orc_mass.argtypes = [C.c_void_p, dp]
        L.orc_step_count.argtypes = [C.c_void_p]
        L.orc_step_count.restype = C.c_longlong
        L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_guo.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc_collide.argtypes = [C.POINTER(OrcParams), dp, C.c_double, C.c_double,
                                  C.c_double, dp]
        L.orc_collide.restype = C.c_int
        L.orc_recolor.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_double, dp, dp]
        L.orc_wet_correct.argtypes = [C.c_double] * 6 + [dp]
        L.orc_grad48.argtypes = [dp, u8p, dp]
        L.orc_e8_table.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int), dp]
        L.orc_e8_normal.argtypes = [u8p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, dp]
        L.orc_matrices.argtypes = [dp, dp]
        L.orc_lattice.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int), dp]
        L.orc_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def make_params(nx, ny, open_x=False, scheme=0, surface_energy=False, **kw) -> OrcParams:
    """``scheme`` 0 / 1: scheme (a) / (b) of Sec. III A 2; ``surface_energy``: rho^N = cos(theta)
    on outermost solid nodes without the gradient correction (Sec. III A 1)."""
    d = dict(DEFAULTS)
    unknown = set(kw) - set(d)
    if unknown:
        raise TypeError(f"unknown oracle parameters {sorted(unknown)}")
    d.update(kw)
    return OrcParams(nx=nx, ny=ny, open_x=int(bool(open_x)), scheme=scheme,
                     surface_energy=int(bool(surface_energy)), **d)


class Oracle:
    """One lattice: ``solid`` (ny, nx) uint8, initial ``rho_r0``/``rho_b0`` (ny, nx),
    optional analytic wall normals ``ns`` (ny, nx, 2) pointing into the solid and
    ``inlet_ux`` (ny,) for an open x axis."""

    def __init__(self, solid, rho_r0, rho_b0, *, open_x=False, ns=None, inlet_ux=None,
                 scheme=0, surface_energy=False, **params):
        L = lib()
        self.solid = np.ascontiguousarray(solid, dtype=np.uint8)
        self.ny, self.nx = self.solid.shape
        self.params = make_params(self.nx, self.ny, open_x, scheme, surface_energy, **params)
        rr = np.ascontiguousarray(rho_r0, dtype=np.float64)
        rb = np.ascontiguousarray(rho_b0, dtype=np.float64)
        nsa = None if ns is None else np.ascontiguousarray(ns, dtype=np.float64)
        iu = np.zeros(self.ny) if inlet_ux is None else np.ascontiguousarray(inlet_ux, dtype=np.float64)
        assert rr.shape == rb.shape == self.solid.shape
        self._h = L.orc_create(C.byref(self.params), _u8(self.solid),
                               None if nsa is None else _dp(nsa), _dp(iu), _dp(rr), _dp(rb))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        # held by the object: module globals may already be gone when it is collected at exit
        self._destroy = L.orc_destroy

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    def step(self, n=1):
        lib().orc_step(self._h, int(n))
        return self

    @property
    def steps(self):
        return int(lib().orc_step_count(self._h))

    def pops(self):
        """(2, 9, ny, nx) per-colour populations, colour 0 red."""
        out = np.empty((2, 9, self.ny, self.nx))
        lib().orc_get_pops(self._h, _dp(out))
        return out

    def set_pops(self, pops):
        a = np.ascontiguousarray(pops, dtype=np.float64)
        assert a.shape == (2, 9, self.ny, self.nx)
        lib().orc_set_pops(self._h, _dp(a))

    def field(self, name):
        out = np.empty((self.ny, self.nx))
        if lib().orc_fields(self._h, FIELDS.index(name), _dp(out)):
            raise ValueError(name)
        return out

    def classes(self):
        out = np.empty((self.ny, self.nx), dtype=np.uint8)
        lib().orc_classes(self._h, _u8(out))
        return out

    def wall_normals(self):
        out = np.empty((self.ny, self.nx, 2))
        lib().orc_wall_normals(self._h, _dp(out))
        return out

    def mass(self):
        out = np.empty(2)
        lib().orc_mass(self._h, _dp(out))
        return float(out[0]), float(out[1])


# ------------------------------------------------------------ single-node helpers

def lattice():
    ex = (C.c_int * 9)()
    ey = (C.c_int * 9)()
    w = np.empty(9)
    lib().orc_lattice(ex, ey, _dp(w))
    return np.array(ex[:]), np.array(ey[:]), w


def matrices():
    M = np.empty((9, 9))
    Minv = np.empty((9, 9))
    lib().orc_matrices(_dp(M), _dp(Minv))
    return M, Minv


def feq(rho, ux, uy):
    out = np.empty(9)
    lib().orc_feq(rho, ux, uy, _dp(out))
    return out


def guo(ux, uy, Fx, Fy):
    out = np.empty(9)
    lib().orc_guo(ux, uy, Fx, Fy, _dp(out))
    return out


def collide(f, Fx, Fy, rhoN, **params):
    p = make_params(1, 1, **params)
    fa = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(9)
    if lib().orc_collide(C.byref(p), _dp(fa), Fx, Fy, rhoN, _dp(out)):
        raise RuntimeError("singular M")
    return out


def recolor(fp, rR, rB, nx, ny, beta=0.7):
    fa = np.ascontiguousarray(fp, dtype=np.float64)
    oR = np.empty(9)
    oB = np.empty(9)
    lib().orc_recolor(_dp(fa), rR, rB, nx, ny, beta, _dp(oR), _dp(oB))
    return oR, oB


def wet_correct(ns, g, theta_deg, eps=1e-10):
    out = np.empty(2)
    lib().orc_wet_correct(ns[0], ns[1], theta_deg, eps, g[0], g[1], _dp(out))
    return out


def grad48(phi9, fluid9):
    """Eq. 48 at one node: phi9[a] = phi(x + e_a) (phi9[0] = phi(x)), fluid9[a] truthy where
    that neighbour is fluid."""
    phi = np.ascontiguousarray(phi9, dtype=np.float64)
    fl = np.ascontiguousarray(np.asarray(fluid9, dtype=bool), dtype=np.uint8)
    assert phi.shape == (9,) and fl.shape == (9,)
    out = np.empty(2)
    lib().orc_grad48(_dp(phi), _u8(fl), _dp(out))
    return out


def e8_table():
    cx = (C.c_int * 24)()
    cy = (C.c_int * 24)()
    w = np.empty(24)
    lib().orc_e8_table(cx, cy, _dp(w))
    return np.array(cx[:]), np.array(cy[:]), w


def e8_normal(solid, x, y, open_x=False):
    s = np.ascontiguousarray(solid, dtype=np.uint8)
    out = np.empty(2)
    lib().orc_e8_normal(_u8(s), s.shape[1], s.shape[0], int(open_x), x, y, _dp(out))
    return out


def threads():
    return int(lib().orc_threads())


def set_threads(n):
    lib().orc_set_threads(int(n))
