"""Pins of the CPU oracle's building blocks against what the paper and the mathematics fix.

Each check is independent of the oracle's own code: expected values come from textbook
definitions (Lallemand-Luo moment polynomials, BGK + Guo forcing), closed forms (moments of
f^eq and of the Guo source), hand-derived geometry (contact-line normals) or exact
properties (isotropy of the stencils, exactness of Eq. 28 on quadratics, Eq. 37).
"""
import math

import numpy as np
import pytest

import oracle

EX_P = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])  # Sec. II A: e_{1,3} = (+-1,0), e_{2,4} = (0,+-1),
EY_P = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])  # e_{5,6} = (+-1,1), e_{7,8} = (-+1,-1)


def moment_matrix():
    """Lallemand-Luo moments as polynomials of e: rho, e, epsilon, j_x, q_x, j_y, q_y,
    p_xx, p_xy (the order of Eq. 3)."""
    ex, ey = EX_P.astype(float), EY_P.astype(float)
    e2 = ex * ex + ey * ey
    rows = [np.ones(9), -4 + 3 * e2, 4 - 10.5 * e2 + 4.5 * e2 * e2, ex, (-5 + 3 * e2) * ex, ey,
            (-5 + 3 * e2) * ey, ex * ex - ey * ey, ex * ey]
    return np.array(rows)


def textbook_feq(rho, u):
    ex, ey = EX_P.astype(float), EY_P.astype(float)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    eu = ex * u[0] + ey * u[1]
    return rho * w * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (u[0] ** 2 + u[1] ** 2))


def textbook_guo(u, F):
    ex, ey = EX_P.astype(float), EY_P.astype(float)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    eu = ex * u[0] + ey * u[1]
    return w * ((3 * (ex - u[0]) + 9 * eu * ex) * F[0] + (3 * (ey - u[1]) + 9 * eu * ey) * F[1])


def test_lattice_matches_paper_and_is_isotropic():
    ex, ey, w = oracle.lattice()
    assert (ex == EX_P).all() and (ey == EY_P).all()
    assert math.isclose(w.sum(), 1.0, rel_tol=0, abs_tol=1e-15)
    # second and fourth moments of the D2Q9 weights (c_s^2 = 1/3)
    assert np.allclose([(w * ex * ex).sum(), (w * ey * ey).sum(), (w * ex * ey).sum()],
                       [1 / 3, 1 / 3, 0], atol=1e-15)
    assert math.isclose((w * ex ** 4).sum(), 3 * (w * ex ** 2 * ey ** 2).sum(), abs_tol=1e-15)


def test_transform_matrix_is_the_moment_basis():
    M, Minv = oracle.matrices()
    assert np.array_equal(M, moment_matrix())
    G = M @ M.T
    assert np.allclose(G, np.diag(np.diag(G)), atol=0)  # rows orthogonal
    assert np.allclose(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    assert np.allclose(Minv @ M, np.eye(9), atol=1e-14)


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0)), (1.03, (0.05, -0.02)), (0.97, (-0.1, 0.08))])
def test_equilibrium_moments(rho, u):
    f = oracle.feq(rho, *u)
    m = moment_matrix() @ f
    ux, uy = u
    uu = ux * ux + uy * uy
    expect = [rho, -2 * rho + 3 * rho * uu, rho - 3 * rho * uu, rho * ux, -rho * ux,
              rho * uy, -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy]
    assert np.allclose(m, expect, atol=1e-15)
    assert np.allclose(f, textbook_feq(rho, u), atol=1e-16)


@pytest.mark.parametrize("u,F", [((0.0, 0.0), (1e-3, 0.0)), ((0.05, -0.02), (2e-4, -3e-4))])
def test_guo_source_moments(u, F):
    s = oracle.guo(*u, *F)
    m = moment_matrix() @ s
    ux, uy = u
    Fx, Fy = F
    uF = ux * Fx + uy * Fy
    expect = [0, 6 * uF, -6 * uF, Fx, -Fx, Fy, -Fy, 2 * (ux * Fx - uy * Fy), ux * Fy + uy * Fx]
    assert np.allclose(m, expect, atol=1e-17)


def _random_state(rng, amp=0.02):
    rho = 1.0 + rng.uniform(-0.02, 0.02)
    u = rng.uniform(-0.05, 0.05, size=2)
    return textbook_feq(rho, u) * (1 + amp * rng.standard_normal(9))


@pytest.mark.parametrize("seed", range(5))
def test_mrt_reduces_to_bgk_guo_when_all_rates_equal(seed):
    rng = np.random.default_rng(seed)
    f = _random_state(rng)
    F = rng.uniform(-1e-3, 1e-3, size=2)
    nu = rng.uniform(0.05, 0.5)
    tau = 3 * nu + 0.5
    rhoN = rng.uniform(-1, 1)
    out = oracle.collide(f, F[0], F[1], rhoN, nu_r=nu, nu_b=nu, s_e=1 / tau, s_eps=1 / tau,
                         s_q=1 / tau)
    rho = f.sum()
    u = np.array([(f * EX_P).sum() + 0.5 * F[0], (f * EY_P).sum() + 0.5 * F[1]]) / rho
    bgk = f - (f - textbook_feq(rho, u)) / tau + (1 - 0.5 / tau) * textbook_guo(u, F)
    assert np.allclose(out, bgk, atol=2e-15)


@pytest.mark.parametrize("seed", range(5))
def test_mrt_moment_relaxation_rates_and_local_viscosity(seed):
    """Each moment relaxes with its own rate of Eq. 6 and the shear rate follows Eqs. 18, 5;
    mass is conserved and momentum changes by exactly F (for any rate)."""
    rng = np.random.default_rng(100 + seed)
    f = _random_state(rng, amp=0.05)
    F = rng.uniform(-1e-3, 1e-3, size=2)
    nu_r, nu_b = 0.35, 0.35 / 7.0
    rhoN = rng.uniform(-1, 1)
    se, seps, sq = 1.64, 1.54, 1.9
    out = oracle.collide(f, F[0], F[1], rhoN, nu_r=nu_r, nu_b=nu_b, s_e=se, s_eps=seps, s_q=sq)
    Mm = moment_matrix()
    rho = f.sum()
    u = np.array([(f * EX_P).sum() + 0.5 * F[0], (f * EY_P).sum() + 0.5 * F[1]]) / rho
    m, meq, mF = Mm @ f, Mm @ textbook_feq(rho, u), Mm @ textbook_guo(u, F)
    nu = 1.0 / ((1 + rhoN) / (2 * nu_r) + (1 - rhoN) / (2 * nu_b))
    sv = 1.0 / (3 * nu + 0.5)
    S = np.array([1.0, se, seps, 1.0, sq, 1.0, sq, sv, sv])
    expect = m - S * (m - meq) + (1 - S / 2) * mF
    assert np.allclose(Mm @ out, expect, atol=2e-15)
    assert math.isclose(out.sum(), rho, rel_tol=0, abs_tol=1e-15)
    assert np.allclose([(out * EX_P).sum() - (f * EX_P).sum(),
                        (out * EY_P).sum() - (f * EY_P).sum()], F, atol=1e-16)


def test_viscosity_interpolation_limits():
    """Pure red / pure blue nodes relax shear moments with 1/(3 nu_k + 1/2)."""
    f = textbook_feq(1.0, (0.0, 0.0)) + 1e-3 * np.array([0, 1, -1, 1, -1, 0, 0, 0, 0])
    Mm = moment_matrix()
    for rhoN, nu in ((1.0, 0.3), (-1.0, 0.03)):
        out = oracle.collide(f, 0.0, 0.0, rhoN, nu_r=0.3, nu_b=0.03)
        pxx_in = (Mm @ f)[7]
        pxx_out = (Mm @ out)[7]
        assert math.isclose(pxx_out, (1 - 1 / (3 * nu + 0.5)) * pxx_in, rel_tol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_recolouring_conserves_colour_and_pushes_red_along_n(seed):
    rng = np.random.default_rng(seed)
    fp = _random_state(rng)
    rR = rng.uniform(0.1, 0.9)
    rB = fp.sum() - rR
    ang = rng.uniform(0, 2 * np.pi)
    n = np.array([math.cos(ang), math.sin(ang)])
    beta = 0.7
    oR, oB = oracle.recolor(fp, rR, rB, n[0], n[1], beta)
    assert math.isclose(oR.sum(), rR, abs_tol=1e-15)
    assert math.isclose(oB.sum(), rB, abs_tol=1e-15)
    assert np.allclose(oR + oB, fp, atol=1e-16)
    rho = rR + rB
    # the red share of the first moment moves by beta (rR rB / rho) c_s^2 n along n
    shift = np.array([((oR - rR / rho * fp) * EX_P).sum(), ((oR - rR / rho * fp) * EY_P).sum()])
    assert np.allclose(shift, beta * rR * rB / rho / 3.0 * n, atol=1e-16)


def test_recolouring_keeps_pure_nodes_pure():
    fp = textbook_feq(1.0, (0.02, 0.01))
    oR, oB = oracle.recolor(fp, fp.sum(), 0.0, 0.6, 0.8)
    assert (oB == 0.0).all() and np.array_equal(oR, fp)


@pytest.mark.parametrize("theta", [30.0, 60.0, 120.0, 150.0])
def test_wetting_direction_flat_wall(theta):
    """Flat bottom wall, n_s = (0, -1) into the solid.  A red droplet's right contact line
    has its interface normal (into red) at (-sin t, -cos t); the left one at (sin t, -cos t)."""
    t = math.radians(theta)
    for g_est, expect in (((-1.0, -0.3), (-math.sin(t), -math.cos(t))),
                          ((1.0, -0.3), (math.sin(t), -math.cos(t)))):
        g = np.array(g_est) * 0.37
        out = oracle.wet_correct((0.0, -1.0), g, theta)
        assert np.allclose(out, np.linalg.norm(g) * np.array(expect), atol=1e-15)


def test_wetting_direction_general_wall_and_ties():
    # left wall (solid at x < 0): n_s = (-1, 0); red below the interface -> normal points down
    t = math.radians(60)
    out = oracle.wet_correct((-1.0, 0.0), (-0.2, -1.0), 60.0)
    assert np.allclose(out, np.hypot(0.2, 1.0) * np.array([-math.cos(t), -math.sin(t)]), atol=1e-15)
    # theta = 0 / 180: both candidates coincide with +-n_s
    assert np.allclose(oracle.wet_correct((0.0, -1.0), (0.3, 0.4), 0.0), [0, -0.5], atol=1e-15)
    assert np.allclose(oracle.wet_correct((0.0, -1.0), (0.3, 0.4), 180.0), [0, 0.5], atol=1e-15)
    # tie D1 == D2 (estimate along n_s at theta = 90) picks the counter-clockwise candidate
    assert np.allclose(oracle.wet_correct((0.0, -1.0), (0.0, -2.0), 90.0), [2.0, 0.0], atol=1e-15)
    # below the threshold nothing is rotated
    assert np.array_equal(oracle.wet_correct((0.0, -1.0), (1e-12, 0.0), 60.0), [1e-12, 0.0])


def test_eighth_order_stencil_isotropy():
    cx, cy, w = oracle.e8_table()
    assert len(set(zip(cx.tolist(), cy.tolist()))) == 24
    r2 = cx ** 2 + cy ** 2
    for k, wk in ((1, 4 / 21), (2, 4 / 45), (4, 1 / 60), (5, 2 / 315), (8, 1 / 5040)):
        assert np.allclose(w[r2 == k], wk)
    assert math.isclose((w * cx * cx).sum(), 1.0, abs_tol=1e-15)
    assert math.isclose((w * cx * cy).sum(), 0.0, abs_tol=1e-15)
    assert math.isclose((w * cx ** 4).sum(), 12 / 7, abs_tol=1e-14)
    assert math.isclose((w * cx ** 2 * cy ** 2).sum(), 4 / 7, abs_tol=1e-14)
    assert math.isclose((w * cx ** 6).sum(), 5 * (w * cx ** 2 * cy ** 4).sum(), rel_tol=1e-13)


def test_eighth_order_wall_normals():
    s = np.zeros((12, 12), dtype=np.uint8)
    s[0, :] = 1
    assert np.allclose(oracle.e8_normal(s, 5, 1), [0, -1], atol=1e-15)
    s = np.zeros((12, 12), dtype=np.uint8)
    s[:, 11] = 1
    assert np.allclose(oracle.e8_normal(s, 10, 6), [1, 0], atol=1e-15)
    # 45-degree staircase: solid where x + y <= 10 -> normal along (-1, -1)/sqrt 2
    y, x = np.mgrid[0:24, 0:24]
    s = ((x + y) <= 10).astype(np.uint8)
    assert np.allclose(oracle.e8_normal(s, 6, 5), [-(0.5 ** 0.5), -(0.5 ** 0.5)], atol=1e-12)
    # staircase circle of radius 40 (node-centre test): the normal field has the circle's
    # eight-fold lattice symmetry exactly, and points radially on average
    c = 60
    y, x = np.mgrid[0:121, 0:121]
    s = (((x - c) ** 2 + (y - c) ** 2) <= 40 ** 2).astype(np.uint8)
    devs = []
    for py in range(121):
        for px in range(121):
            if s[py, px] or not s[py - 1:py + 2, px - 1:px + 2].any():
                continue
            n = oracle.e8_normal(s, px, py)
            dx, dy = px - c, py - c
            for (qx, qy), (mx, my) in (((c - dx, py), (-n[0], n[1])), ((px, c - dy), (n[0], -n[1])),
                                       ((c + dy, c + dx), (n[1], n[0]))):
                assert np.allclose(oracle.e8_normal(s, qx, qy), [mx, my], atol=1e-13)
            radial = np.array([-dx, -dy], float) / math.hypot(dx, dy)
            devs.append(math.degrees(math.acos(min(1.0, float(n @ radial)))))
    assert len(devs) > 300 and np.mean(devs) < 10.0
