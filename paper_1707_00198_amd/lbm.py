"""Python binding of liblbmcg (include/lbmcg.h): argument marshalling only.

PyTorch supplies the device memory (state and scratch buffers, field read-back buffers) and the
HIP stream; every step of the method runs in the library's HIP kernels.  There is no CPU
fallback: without the built library (``python -m paper_1707_00198_amd.build``) or without a
GPU, constructing a ``Lattice`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbmcg.so")

STORAGE = {"f64": 0, "f32": 1, "f16": 2, "c16": 3}
FIELD_RHO_R, FIELD_RHO_B, FIELD_POPS, FIELD_UX, FIELD_UY = 1, 2, 4, 8, 16

STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
          -4: "LBM_ENONFINITE", -5: "LBM_ESTATE"}
STATUS_CODE = {v: k for k, v in STATUS.items()}

# Exported symbols and their prototypes, as declared in include/lbmcg.h.
_dp = C.POINTER(C.c_double)


# Wetting variants (LBM_WET_* of include/lbmcg.h).
WET_SCHEME_B = 1
WET_SURFACE_ENERGY = 2


class DomainDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("open_x", C.c_int32), ("wetting", C.c_int32),
        ("solid", C.POINTER(C.c_uint8)), ("ns", _dp), ("inlet_ux", _dp), ("rho_r0", _dp),
        ("rho_b0", _dp),
        ("nu_r", C.c_double), ("nu_b", C.c_double), ("sigma", C.c_double), ("beta", C.c_double),
        ("theta_deg", C.c_double), ("s_e", C.c_double), ("s_eps", C.c_double),
        ("s_q", C.c_double), ("rho0", C.c_double), ("eps", C.c_double),
        ("outlet_u", C.c_double),
    ]


PROTOTYPES = {
    "lbm_query_bytes": (C.c_int, [C.POINTER(DomainDesc), C.c_int, C.c_int,
                                  C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "lbm_create": (C.c_int, [C.POINTER(DomainDesc), C.c_int, C.c_int, C.c_void_p, C.c_size_t,
                             C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_classify": (C.c_int, [C.POINTER(DomainDesc), C.POINTER(C.c_uint8), _dp]),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_read_fields": (C.c_int, [C.c_void_p, C.c_int, C.c_uint32, C.c_void_p, C.c_size_t]),
    "lbm_mass": (C.c_int, [C.c_void_p, _dp]),
    "lbm_steps_taken": (C.c_int64, [C.c_void_p]),
    "lbm_set_tile": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int]),
    "lbm_get_tile": (C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    "lbm_set_graph": (C.c_int, [C.c_void_p, C.c_int]),
    "lbm_autotune": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_double)]),
    "lbm_state_size": (C.c_size_t, [C.c_void_p]),
    "lbm_save_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_load_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_diag_bytes": (C.c_size_t, [C.c_void_p]),
    "lbm_diag_attach": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "lbm_diag_velocity": (C.c_int, [C.c_void_p, C.c_int, _dp]),
    "lbm_diag_region_mass": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, _dp]),
    "lbm_diag_crossings": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.c_int, _dp]),
    "lbm_diag_crossings_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.c_int, _dp]),
    "lbm_diag_contact_line": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.c_int,
                                        C.POINTER(C.c_int)]),
    "lbm_last_error": (C.c_char_p, []),
    "lbm_destroy": (None, [C.c_void_p]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbmcg.so and declare its prototypes (no device work; works without a GPU).

    torch is imported first so that the library binds to the HIP runtime torch has loaded: the
    device buffers and the stream handed to the library come from that runtime instance."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (load order: torch's HIP runtime first)
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with python -m paper_1707_00198_amd.build")
        L = C.CDLL(path)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _check(code):
    if code != 0:
        raise LBMError(code, load_library().lbm_last_error().decode())


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class Lattice:
    """A batch of domains advanced together by the fused HIP step.

    ``setups`` are objects with the attributes of ``workloads.Setup`` (solid, rho_r0, rho_b0,
    params, open_x, inlet_ux, ns, and optionally wetting: WET_* flags).  ``storage`` is 'f64', 'f32', 'f16' or 'c16'.
    """

    def __init__(self, setups: Sequence, storage: str = "f64", device="cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("lbmcg needs a GPU; torch.cuda.is_available() is False")
        L = load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.storage = storage
        self.setups = list(setups)
        self._keep = []
        descs = (DomainDesc * len(self.setups))()
        for d, s in zip(descs, self.setups):
            solid = np.ascontiguousarray(s.solid, dtype=np.uint8)
            rr = np.ascontiguousarray(s.rho_r0, dtype=np.float64)
            rb = np.ascontiguousarray(s.rho_b0, dtype=np.float64)
            self._keep += [solid, rr, rb]
            d.nx, d.ny = solid.shape[1], solid.shape[0]
            d.open_x = int(bool(s.open_x))
            d.wetting = int(getattr(s, "wetting", 0))
            d.solid = _ptr(solid, C.c_uint8)
            d.rho_r0 = _ptr(rr, C.c_double)
            d.rho_b0 = _ptr(rb, C.c_double)
            if s.ns is not None:
                ns = np.ascontiguousarray(s.ns, dtype=np.float64)
                self._keep.append(ns)
                d.ns = _ptr(ns, C.c_double)
            if s.open_x:
                iu = np.ascontiguousarray(s.inlet_ux, dtype=np.float64)
                self._keep.append(iu)
                d.inlet_ux = _ptr(iu, C.c_double)
            p = s.params
            for k in ("nu_r", "nu_b", "sigma", "beta", "theta_deg", "s_e", "s_eps", "s_q",
                      "rho0", "eps", "outlet_u"):
                setattr(d, k, float(p[k]))
        self._descs = descs
        st, sc = C.c_size_t(), C.c_size_t()
        _check(L.lbm_query_bytes(descs, len(descs), STORAGE[storage], C.byref(st), C.byref(sc)))
        with torch.cuda.device(self.device):
            self.state_buf = torch.empty(st.value, dtype=torch.uint8, device=self.device)
            self.scratch_buf = torch.empty(sc.value, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            _check(L.lbm_create(descs, len(descs), STORAGE[storage], self.state_buf.data_ptr(),
                                st.value, self.scratch_buf.data_ptr(), sc.value,
                                C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        # held by the object: module globals may already be gone when it is collected at exit
        self._destroy = L.lbm_destroy
        self.state_bytes, self.scratch_bytes = st.value, sc.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._destroy(h)
            self._h = None

    # ----------------------------------------------------------------- stepping
    def step(self, n: int = 1):
        _check(load_library().lbm_step(self._h, int(n)))
        return self

    @property
    def steps(self) -> int:
        return int(load_library().lbm_steps_taken(self._h))

    def set_tile(self, chunk_rows: int = 0, waves: int = 0, cols: int = 0, cols_per_lane: int = 0):
        _check(load_library().lbm_set_tile(self._h, int(chunk_rows), int(waves), int(cols),
                                           int(cols_per_lane)))

    @property
    def tile(self) -> dict:
        """The step's tile shape in use and its work items (blocks per launch)."""
        out = (C.c_int * 5)()
        _check(load_library().lbm_get_tile(self._h, out))
        return dict(chunk_rows=out[0], waves=out[1], cols=out[2], items=out[3], cols_per_lane=out[4])

    def set_graph(self, launches: int):
        """Replay runs of `launches` steps (even; 0 = off) as one HIP graph launch each."""
        _check(load_library().lbm_set_graph(self._h, int(launches)))
        return self

    def autotune(self, steps: int = 20) -> dict:
        """Time every tile shape on this batch and keep the fastest; the state is saved to a
        temporary device buffer and restored, so the simulation is unchanged."""
        n = int(load_library().lbm_state_size(self._h))
        buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        out = (C.c_double * 5)()
        _check(load_library().lbm_autotune(self._h, int(steps), C.c_void_p(buf.data_ptr()), out))
        del buf
        return dict(chunk_rows=int(out[0]), waves=int(out[1]), cols=int(out[2]), ms_per_step=out[3],
                    cols_per_lane=int(out[4]))

    def synchronize(self):
        self.stream.synchronize()

    # ------------------------------------------------------------------ fields
    def read(self, dom: int, which: int):
        """FP64 device tensor (planes, ny, nx) of the selected quantities."""
        s = self.setups[dom]
        ny, nx = s.solid.shape
        planes = (which & 1) + ((which >> 1) & 1) + 18 * ((which >> 2) & 1) + ((which >> 3) & 1) + ((which >> 4) & 1)
        if which & (FIELD_UX | FIELD_UY):
            self._diag()
        out = self.torch.empty((planes, ny, nx), dtype=self.torch.float64, device=self.device)
        _check(load_library().lbm_read_fields(self._h, dom, which, out.data_ptr(), out.numel()))
        return out

    def pops(self, dom: int = 0) -> np.ndarray:
        """(2, 9, ny, nx) per-colour post-streaming populations (red first), FP64."""
        t = self.read(dom, FIELD_POPS)
        self.synchronize()
        return t.cpu().numpy().reshape(2, 9, *t.shape[1:])

    def densities(self, dom: int = 0):
        t = self.read(dom, FIELD_RHO_R | FIELD_RHO_B)
        self.synchronize()
        a = t.cpu().numpy()
        return a[0], a[1]

    def mass(self) -> np.ndarray:
        out = np.empty(2 * len(self.setups))
        _check(load_library().lbm_mass(self._h, _ptr(out, C.c_double)))
        return out.reshape(-1, 2)

    def velocity(self, dom: int = 0):
        """(u_x, u_y) of Eq. 17 that the next collision uses, FP64, solid nodes 0."""
        t = self.read(dom, FIELD_UX | FIELD_UY)
        self.synchronize()
        a = t.cpu().numpy()
        return a[0], a[1]

    # ------------------------------------------------------------- diagnostics
    def _diag(self):
        if getattr(self, "diag_buf", None) is None:
            L = load_library()
            n = int(L.lbm_diag_bytes(self._h))
            self.diag_buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
            _check(L.lbm_diag_attach(self._h, self.diag_buf.data_ptr(), n))

    def velocity_stats(self, snapshot: bool = False) -> np.ndarray:
        """(n_domains, 2): |u|max (Eq. 46) and the largest velocity-component change since the
        last snapshot (Eq. 45 with a 500-step gap; NaN before the first snapshot)."""
        self._diag()
        out = np.empty(2 * len(self.setups))
        _check(load_library().lbm_diag_velocity(self._h, int(bool(snapshot)), _ptr(out, C.c_double)))
        return out.reshape(-1, 2)

    def region_mass(self, dom: int, region) -> np.ndarray:
        """[rho_R inside, rho_R outside, rho_B inside, rho_B outside] for a (ny, nx) region mask:
        a host array, or a contiguous uint8 tensor already on the device (reused as is)."""
        self._diag()
        ny, nx = self.setups[dom].solid.shape
        if isinstance(region, self.torch.Tensor) and region.is_cuda:
            if region.device != self.device:
                raise ValueError(f"region is on {region.device}, the lattice on {self.device}")
            if region.dtype != self.torch.uint8 or not region.is_contiguous() or region.numel() != nx * ny:
                raise ValueError(f"region must be a contiguous uint8 tensor of {ny} x {nx} elements")
            r = region
        else:
            r = self.torch.as_tensor(np.ascontiguousarray(region, dtype=np.uint8), device=self.device)
            if r.numel() != nx * ny:
                raise ValueError(f"region must have {ny} x {nx} elements")
        out = np.empty(4)
        _check(load_library().lbm_diag_region_mass(self._h, dom, r.data_ptr(), _ptr(out, C.c_double)))
        return out

    def crossings(self, dom: int, rows) -> np.ndarray:
        """First rho^N > 0 -> <= 0 crossing x along each row (NaN where none)."""
        self._diag()
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        out = np.empty(len(rows))
        _check(load_library().lbm_diag_crossings(self._h, dom, _ptr(rows, C.c_int32), len(rows),
                                                 _ptr(out, C.c_double)))
        return out

    def crossings_noalloc(self, dom: int, rows) -> np.ndarray:
        """As crossings(), through the entry point that allocates nothing (static device staging,
        no diagnostics buffer)."""
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        out = np.empty(len(rows))
        _check(load_library().lbm_diag_crossings_noalloc(self._h, dom, _ptr(rows, C.c_int32), len(rows),
                                                         _ptr(out, C.c_double)))
        return out

    def contact_line(self, dom: int) -> np.ndarray:
        """Outermost fluid nodes of domain ``dom`` where |grad rho^N| > eps (the nodes the
        wetting condition acts on), as an (n, 2) array of (x, y), ordered by y then x."""
        self._diag()
        L = load_library()
        n = C.c_int()
        cap = 256
        while True:
            out = np.empty(cap, dtype=np.int32)
            rc = L.lbm_diag_contact_line(self._h, dom, _ptr(out, C.c_int32), cap, C.byref(n))
            if rc == STATUS_CODE["LBM_ENOMEM"] and n.value > cap:
                cap = n.value
                continue
            _check(rc)
            break
        nx = self.setups[dom].solid.shape[1]
        idx = out[:n.value]
        return np.stack([idx % nx, idx // nx], axis=1)

    # -------------------------------------------------------------- checkpoints
    def save_state(self):
        n = int(load_library().lbm_state_size(self._h))
        buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        _check(load_library().lbm_save_state(self._h, buf.data_ptr()))
        return buf

    def load_state(self, buf):
        _check(load_library().lbm_load_state(self._h, buf.data_ptr()))
