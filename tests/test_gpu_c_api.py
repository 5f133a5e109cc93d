"""The C interface driven from plain C99 (paper_1707_00198_amd/csrc/c_api_example.c, built by
build() with gcc against liblbmcg.so and the HIP runtime, no Python or torch in the process):
a static droplet on a flat wall advanced 200 steps gives the same colour masses and red
densities, bit for bit, as the Python binding of the same library on the same set-up, in FP64
and in the 16-bit c16 storage; in FP64 the colour masses are conserved to rounding."""
import os
import subprocess

import numpy as np
import pytest

from paper_1707_00198_amd import workloads as W

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1707_00198_amd",
                   "lbm_c_example")
STEPS = 200
SAMPLES = [(32, 1), (32, 8), (40, 5), (10, 20)]


def _setup():
    """The C program's set-up: 64 x 32, solid rows at y = 0 and 31, red inside radius 10 of
    (32, 1), theta = 60 degrees."""
    ny, nx = 32, 64
    solid = np.zeros((ny, nx), np.uint8)
    solid[0, :] = solid[-1, :] = 1
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    fluid = solid == 0
    red = fluid & ((x - 32.0) ** 2 + (y - 1.0) ** 2 < 100.0)
    rr = np.where(red, 1.0, 0.0)
    rb = np.where(fluid & ~red, 1.0, 0.0)
    p = dict(nu_r=1.0 / 6.0, nu_b=1.0 / 6.0, sigma=0.01, beta=0.7, theta_deg=60.0, s_e=1.64,
             s_eps=1.54, s_q=1.9, rho0=1.0, eps=1e-10, outlet_u=0.0)
    return W.Setup("c_example", solid, rr, rb, p)


def _run_c(storage):
    assert os.path.exists(EXE), "the C example is built by __graft_entry__.build()"
    print(f"[c api] {EXE} {storage} {STEPS}", flush=True)
    r = subprocess.run([EXE, storage, str(STEPS)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = {}
    for line in r.stdout.splitlines():
        f = line.split()
        if f[0] in ("mass_before", "mass_after"):
            out[f[0]] = (float(f[1]), float(f[2]))
        elif f[0] == "rho_r":
            out[(int(f[1]), int(f[2]))] = float(f[3])
        elif f[0] == "storage":
            out["steps"] = int(f[3])
    return out


@pytest.mark.parametrize("storage", ["f64", "c16"])
def test_c_program_matches_the_python_binding(storage):
    from paper_1707_00198_amd.lbm import Lattice
    c = _run_c(storage)
    assert c["steps"] == STEPS
    lat = Lattice([_setup()], storage=storage)
    m0 = lat.mass()[0]
    lat.step(STEPS)
    m1 = lat.mass()[0]
    rr, _ = lat.densities(0)
    print(f"[c api] {storage}: C masses {c['mass_after']}, binding {tuple(m1)}", flush=True)
    assert tuple(m0) == c["mass_before"] and tuple(m1) == c["mass_after"]
    for x, y in SAMPLES:
        assert rr[y, x] == c[(x, y)], (x, y, rr[y, x], c[(x, y)])
    if storage == "f64":
        assert abs(c["mass_after"][0] / c["mass_before"][0] - 1) < 1e-12
        assert abs(c["mass_after"][1] / c["mass_before"][1] - 1) < 1e-12
