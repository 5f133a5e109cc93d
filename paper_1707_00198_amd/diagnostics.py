"""Measures of Sec. III built on the library's on-device diagnostics (include/lbmcg.h,
lbm_diag_*): no field is read back to the host.

* ``run_to_steady``: iterate until E1 (Eq. 45, the largest change of a velocity component over
  500 steps) drops below a threshold, then report |u|max (Eq. 46).
* ``e_npmt``: the non-physical mass transfer measure of Eq. 47 from colour masses inside and
  outside the theoretical interface C.  As printed, Eq. 47 divides the red mass *inside* C and
  the blue mass *outside* C by the totals; for a red droplet that ratio is 1, while the paper's
  tabulated values are O(1e-2).  The fictive transfer the text defines is red mass beyond the
  interface and blue mass inside it, so the superscripts are read as swapped:
  E = sqrt((m_R^out / m_R^all)^2 + (m_B^in / m_B^all)^2).
* ``channel_interface``: contact line, tip and finger length of a displacement channel from the
  rho^N = 0 crossings on the rows next to the walls and on the centre line.
* ``track_channels`` / ``rate``: S(t), L(t) of a batch of channels sampled during a run, and
  their steady slopes (the speeds of Eqs. 50-51 and Fig. 9).
"""
from __future__ import annotations

import math

import numpy as np


def e_npmt(masses) -> float:
    """Eq. 47 (with the reading above) from [rho_R in, rho_R out, rho_B in, rho_B out]."""
    r_in, r_out, b_in, b_out = (float(m) for m in masses)
    r_all, b_all = r_in + r_out, b_in + b_out
    return math.hypot(r_out / r_all if r_all else 0.0, b_in / b_all if b_all else 0.0)


def circle_region(shape, xc: float, yc: float, radius: float) -> np.ndarray:
    """(ny, nx) uint8 mask of the node centres inside a circle (the theoretical interface C)."""
    ny, nx = shape
    y, x = np.mgrid[0:ny, 0:nx]
    return ((x - xc) ** 2 + (y - yc) ** 2 <= radius * radius).astype(np.uint8)


def run_to_steady(lat, every: int = 500, tol: float = 1e-7, max_steps: int = 200000):
    """Advance ``lat`` in windows of ``every`` steps until E1 < tol in every domain (or
    max_steps).  Returns (steps taken, per-domain |u|max, per-domain last E1)."""
    lat.velocity_stats(snapshot=True)
    taken = 0
    e1 = None
    stats = None
    while taken < max_steps:
        lat.step(every)
        taken += every
        stats = lat.velocity_stats(snapshot=True)
        e1 = stats[:, 1]
        if np.all(e1 < tol):
            break
    return taken, stats[:, 0], e1


def channel_interface(lat, dom: int, solid: np.ndarray) -> dict:
    """Contact line (mean crossing on the two fluid rows next to the walls), tip (crossing on
    the centre line, mean of the two centre rows for an even height) and length tip - contact
    line, for domain ``dom`` of ``lat`` whose solid mask is ``solid``; None where a row has no
    crossing."""
    fluid_rows = np.nonzero((solid == 0).any(axis=1))[0]
    y0, y1 = int(fluid_rows[0]), int(fluid_rows[-1])
    h = y1 - y0 + 1
    centre = [y0 + h // 2] if h % 2 else [y0 + h // 2 - 1, y0 + h // 2]
    x = lat.crossings(dom, [y0, y1] + centre)
    nan = lambda v: None if math.isnan(v) else float(v)
    cl = None if math.isnan(x[0]) or math.isnan(x[1]) else 0.5 * (x[0] + x[1])
    tip = nan(np.mean(x[2:])) if not np.isnan(x[2:]).any() else None
    return dict(contact_line=cl, tip=tip, length=None if cl is None or tip is None else tip - cl)


def track_channels(lat, doms, steps: int, every: int):
    """Advance ``lat`` by ``steps`` in windows of ``every`` and record, for each domain in
    ``doms``, the contact line and finger length of ``channel_interface`` after every window.
    Returns (times (k,), contact line (len(doms), k), length (len(doms), k)); NaN where a row
    has no crossing."""
    times, cl, ln = [], [], []
    solids = [lat.setups[d].solid for d in doms]
    for _ in range(steps // every):
        lat.step(every)
        times.append(lat.steps)
        row_cl, row_ln = [], []
        for d, solid in zip(doms, solids):
            m = channel_interface(lat, d, solid)
            row_cl.append(np.nan if m["contact_line"] is None else m["contact_line"])
            row_ln.append(np.nan if m["length"] is None else m["length"])
        cl.append(row_cl)
        ln.append(row_ln)
    return np.array(times, dtype=np.float64), np.array(cl).T, np.array(ln).T


def rate(times, values, t_min: float) -> float:
    """Least-squares slope of ``values`` over the samples with time >= t_min (the steady
    speeds dS/dt and dL/dt of Sec. III D)."""
    sel = (times >= t_min) & np.isfinite(values)
    if sel.sum() < 2:
        return math.nan
    return float(np.polyfit(times[sel], values[sel], 1)[0])
