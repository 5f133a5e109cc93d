"""Measurements on colour fields used by the tests: interface points, circle fits, contact
angles, interface positions.  Test infrastructure; independent of both the oracle's and the
GPU library's arithmetic (they only post-process rho^N fields)."""
from __future__ import annotations

import math

import numpy as np


def interface_points(rhoN, fluid, min_dist_solid=0, solid=None, periodic_x=True):
    """Zero crossings of rhoN between horizontally or vertically adjacent fluid nodes,
    linearly interpolated.  Returns (k, 2) array of (x, y)."""
    ny, nx = rhoN.shape
    pts = []
    ok = fluid.copy()
    if min_dist_solid and solid is not None:
        # distance (Chebyshev) to the nearest solid node
        far = np.ones_like(fluid, dtype=bool)
        s = solid.astype(bool)
        for dy in range(-min_dist_solid, min_dist_solid + 1):
            for dx in range(-min_dist_solid, min_dist_solid + 1):
                far &= ~np.roll(np.roll(s, dy, axis=0), dx, axis=1)
        ok &= far
    # horizontal pairs
    a = rhoN
    b = np.roll(rhoN, -1, axis=1)
    okp = ok & np.roll(ok, -1, axis=1)
    if not periodic_x:
        okp[:, -1] = False
    m = okp & (a * b < 0)
    ys, xs = np.nonzero(m)
    t = a[ys, xs] / (a[ys, xs] - b[ys, xs])
    xi = xs + t
    if periodic_x:
        xi = np.mod(xi, nx)
    pts.append(np.stack([xi, ys.astype(float)], axis=1))
    # vertical pairs (no wrap)
    a = rhoN[:-1]
    b = rhoN[1:]
    okp = ok[:-1] & ok[1:]
    m = okp & (a * b < 0)
    ys, xs = np.nonzero(m)
    t = a[ys, xs] / (a[ys, xs] - b[ys, xs])
    pts.append(np.stack([xs.astype(float), ys + t], axis=1))
    return np.concatenate(pts, axis=0)


def fit_circle(pts):
    """Algebraic least-squares circle: returns (xc, yc, R)."""
    x, y = pts[:, 0], pts[:, 1]
    A = np.stack([x, y, np.ones_like(x)], axis=1)
    rhs = -(x * x + y * y)
    (D, E, F), *_ = np.linalg.lstsq(A, rhs, rcond=None)
    xc, yc = -D / 2.0, -E / 2.0
    R = math.sqrt(xc * xc + yc * yc - F)
    return xc, yc, R


def flat_contact_angle(rhoN, solid, wall_y, min_height=3.0):
    """Contact angle (degrees, in the red phase) of a single red droplet on a flat bottom wall
    at height wall_y: circle fit of the interface points at least min_height above the wall,
    cos(theta) = (wall_y - yc) / R."""
    fluid = solid == 0
    pts = interface_points(rhoN, fluid)
    pts = pts[pts[:, 1] >= wall_y + min_height]
    xc, yc, R = fit_circle(pts)
    c = (wall_y - yc) / R
    return math.degrees(math.acos(max(-1.0, min(1.0, c)))), (xc, yc, R)


def cylinder_contact_angle(rhoN, solid, ccx, ccy, rc, min_dist=3.0):
    """Contact angle of a droplet on a cylinder (centre ccx, ccy, radius rc): circle fit of
    interface points at least min_dist from the cylinder surface; by the law of cosines
    cos(theta) = (Rd^2 + Rc^2 - D^2) / (2 Rd Rc)."""
    fluid = solid == 0
    pts = interface_points(rhoN, fluid)
    r = np.hypot(pts[:, 0] - ccx, pts[:, 1] - ccy)
    pts = pts[r >= rc + min_dist]
    xc, yc, R = fit_circle(pts)
    D = math.hypot(xc - ccx, yc - ccy)
    c = (R * R + rc * rc - D * D) / (2.0 * R * rc)
    return math.degrees(math.acos(max(-1.0, min(1.0, c)))), (xc, yc, R)


def row_crossing(rhoN_row, x_from=0):
    """First x (interpolated) along a row where rhoN changes from positive to non-positive,
    scanning in +x from x_from; None if there is none."""
    r = rhoN_row
    for x in range(x_from, len(r) - 1):
        if r[x] > 0.0 and r[x + 1] <= 0.0:
            return x + r[x] / (r[x] - r[x + 1])
    return None


def finger_metrics(rhoN, solid):
    """Channel displacement metrics: contact-line position (mean of the crossings on the fluid
    rows next to the bottom and top walls), tip position (crossing on the centre line,
    mean of the two centre rows for even heights) and finger length tip - contact line."""
    fluid_rows = np.nonzero((solid == 0).any(axis=1))[0]
    y0, y1 = fluid_rows[0], fluid_rows[-1]
    xb = row_crossing(rhoN[y0])
    xt = row_crossing(rhoN[y1])
    h = y1 - y0 + 1
    if h % 2:
        tip = row_crossing(rhoN[y0 + h // 2])
    else:
        a = row_crossing(rhoN[y0 + h // 2 - 1])
        b = row_crossing(rhoN[y0 + h // 2])
        tip = None if a is None or b is None else 0.5 * (a + b)
    cl = None if xb is None or xt is None else 0.5 * (xb + xt)
    length = None if cl is None or tip is None else tip - cl
    return dict(contact_line=cl, tip=tip, length=length)
