"""Pins of the oracle's Cartesian methods (Sec. 3.1, Eq. 6-21, A1-A16):
the cell kernels against 2-D quadrature and the exact self-cell value, their
symmetries, exactness of the second-order method for linear densities
against an independent quadrature of the whole domain, the particle and
modified particle kernels, and convergence on the analytic sigma_D2 disk
(Fig. 3: orders about 2, 1 and 1)."""
import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import analytic

T_NAMES = oracle.CART_TABLE_NAMES


def _cell_quad(m, n, dx, dy, k):
    """Kernel k of source offset (m, n) by nested adaptive quadrature of its
    defining integrand (Eq. 13-15, A5-A7), in coordinates relative to the
    destination."""
    X, Y = -m * dx, -n * dy

    def f(y, x):
        r3 = (x * x + y * y) ** 1.5
        u, v = x - X, y - Y
        return [x / r3, x * u / r3, x * v / r3, y / r3, y * v / r3, y * u / r3][k]

    xs = sorted({X - dx / 2, X + dx / 2} | ({0.0} if abs(X) < dx / 2 else set()))
    ys = sorted({Y - dy / 2, Y + dy / 2} | ({0.0} if abs(Y) < dy / 2 else set()))
    tot = 0.0
    for a, b in zip(xs[:-1], xs[1:]):
        for c, d in zip(ys[:-1], ys[1:]):
            tot += integrate.dblquad(f, a, b, c, d, epsabs=1e-14, epsrel=1e-12)[0]
    return tot


@pytest.mark.parametrize("dx,dy", [(0.1, 0.1), (0.1, 0.25)])
def test_kernels_match_quadrature(dx, dy):
    g = oracle.CartGrid(12, 10, dx, dy)
    T = oracle.cart_tables(g)
    # near cells (closed forms) and far cells (Gauss-Legendre), both signs
    for m, n in [(1, 0), (0, 1), (1, 1), (-2, 1), (2, -2), (3, 1), (-5, 4), (11, -9), (7, 0)]:
        for k in range(6):
            ref = _cell_quad(m, n, dx, dy, k)
            got = T[k, m + g.n_x - 1, n + g.n_y - 1]
            scale = abs(T[0, m + g.n_x - 1, n + g.n_y - 1]) + abs(T[3, m + g.n_x - 1, n + g.n_y - 1])
            assert abs(got - ref) <= 1e-10 * scale, (m, n, T_NAMES[k], got, ref)


def test_self_cell():
    # K^{x,x}_00 of a square cell of side h is 2 h asinh(1) (polar integral of
    # cos^2 t over the square); the first-moment self terms vanish
    for h in (0.125, 0.01):
        g = oracle.CartGrid(4, 4, h, h)
        T = oracle.cart_tables(g)
        c = T[:, 3, 3]
        assert abs(c[1] - 2 * h * np.arcsinh(1.0)) < 1e-14 * h
        assert abs(c[4] - 2 * h * np.arcsinh(1.0)) < 1e-14 * h
        for k in (0, 2, 3, 5):
            assert abs(c[k]) < 1e-15
    # a rectangle: K^{x,x}_00 = int cos^2 t R(t) dt, R the distance to the edge
    dx, dy = 0.1, 0.25
    T = oracle.cart_tables(oracle.CartGrid(4, 4, dx, dy))
    tc = np.arctan2(dy, dx)
    kxx = 4 * (integrate.quad(lambda t: np.cos(t) ** 2 * dx / 2 / np.cos(t), 0, tc, epsabs=1e-15)[0]
               + integrate.quad(lambda t: np.cos(t) ** 2 * dy / 2 / np.sin(t), tc, np.pi / 2,
                                epsabs=1e-15)[0])
    kyy = 4 * (integrate.quad(lambda t: np.sin(t) ** 2 * dx / 2 / np.cos(t), 0, tc, epsabs=1e-15)[0]
               + integrate.quad(lambda t: np.sin(t) ** 2 * dy / 2 / np.sin(t), tc, np.pi / 2,
                                epsabs=1e-15)[0])
    assert abs(T[1, 3, 3] - kxx) < 1e-13 and abs(T[4, 3, 3] - kyy) < 1e-13


def test_kernel_symmetries():
    g = oracle.CartGrid(9, 9, 0.2, 0.2)
    T = oracle.cart_tables(g)
    flip_m = T[:, ::-1, :]
    flip_n = T[:, :, ::-1]
    # parity in m (x offset) and n (y offset) of x0, xx, xy, y0, yy, yx
    pm = [-1, 1, -1, 1, 1, -1]
    pn = [1, 1, -1, -1, 1, -1]
    for k in range(6):
        np.testing.assert_allclose(flip_m[k], pm[k] * T[k], atol=1e-15, rtol=0)
        np.testing.assert_allclose(flip_n[k], pn[k] * T[k], atol=1e-15, rtol=0)
    # square cells: the y kernels are the x kernels with the axes exchanged
    np.testing.assert_allclose(T[3], T[0].T, atol=1e-15, rtol=0)
    np.testing.assert_allclose(T[4], T[1].T, atol=1e-15, rtol=0)
    np.testing.assert_allclose(T[5], T[2].T, atol=1e-15, rtol=0)


def _domain_force(g, a, b, c, x, y):
    """Force at (x, y) of the linear density a + b X + c Y on the whole grid
    domain.  The integrand falls like 1/d^2, so the force is the principal
    value about the point: in polar coordinates (d, t) about it, with R(t)
    the distance to the domain edge,
      F = int u(t) [sigma(x, y) ln R(t) + (grad sigma . u(t)) R(t)] dt,
    u = (cos t, sin t) (the ln of the inner radius cancels over the circle).
    One adaptive quadrature in t, split at the corner directions."""
    xa, xb = g.x0 - x, g.x0 + g.n_x * g.dx - x
    ya, yb = g.y0 - y, g.y0 + g.n_y * g.dy - y
    s0 = a + b * x + c * y

    def R(t):
        ct, st = np.cos(t), np.sin(t)
        rx = (xb if ct > 0 else xa) / ct if abs(ct) > 1e-300 else np.inf
        ry = (yb if st > 0 else ya) / st if abs(st) > 1e-300 else np.inf
        return min(rx, ry)

    corners = sorted(np.mod([np.arctan2(ya, xa), np.arctan2(ya, xb), np.arctan2(yb, xa),
                             np.arctan2(yb, xb)], 2 * np.pi))
    cuts = [0.0] + list(corners) + [2 * np.pi]
    out = []
    for comp in (np.cos, np.sin):
        def f(t):
            r = R(t)
            return comp(t) * (s0 * np.log(r) + (b * np.cos(t) + c * np.sin(t)) * r)
        out.append(sum(integrate.quad(f, lo, hi, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
                       for lo, hi in zip(cuts[:-1], cuts[1:]) if hi > lo))
    return out


def test_second_order_exact_for_linear_density():
    # the method is exact when the density is linear over the whole domain:
    # central and one-sided differences return its slopes exactly
    g = oracle.CartGrid(10, 7, 0.1, 0.15, x0=-0.3, y0=0.2)
    X, Y = g.centres()
    a, b, c = 1.3, -0.7, 2.1
    sig = a + b * X + c * Y
    T = oracle.cart_tables(g)
    dest = np.array([0, 13, 34, 48, 69])
    fx, fy = oracle.cart_forward(g, T, sig, dest)
    for q, cell in enumerate(dest):
        i, j = divmod(int(cell), g.n_y)
        rx, ry = _domain_force(g, a, b, c, X[i, j], Y[i, j])
        assert abs(fx[q] - rx) < 1e-12 * (abs(rx) + 1) and abs(fy[q] - ry) < 1e-12 * (abs(ry) + 1), \
            (cell, fx[q], rx, fy[q], ry)


def test_particle_kernels():
    g = oracle.CartGrid(6, 5, 0.1, 0.2)
    Tp = oracle.cart_tables(g, "particle")
    Tq = oracle.cart_tables(g, "particle+")
    T2 = oracle.cart_tables(g)
    c = (g.n_x - 1, g.n_y - 1)
    # point mass sigma dx dy at the source centre, no self force
    m, n = 2, -3
    X, Y = -m * g.dx, -n * g.dy
    w = g.dx * g.dy / (X * X + Y * Y) ** 1.5
    assert abs(Tp[0, m + c[0], n + c[1]] - w * X) < 1e-15
    assert abs(Tp[3, m + c[0], n + c[1]] - w * Y) < 1e-15
    assert np.all(Tp[[1, 2, 4, 5]] == 0) and Tp[0][c] == 0 and Tp[3][c] == 0
    # the modified method adds K^{x,x}_00 and K^{y,y}_00 only (Eq. 21, A16)
    d = Tq - Tp
    assert d[1][c] == T2[1][c] and d[4][c] == T2[4][c]
    d[1][c] = d[4][c] = 0
    assert np.all(d == 0)
    # far from the source the point kernel approaches the cell kernel, the
    # difference falling like (h / d)^2 (the cell's quadrupole)
    near, far = (g.n_x - 1 + 2, g.n_y - 1 - 1), (g.n_x - 1 + 5, g.n_y - 1 - 4)
    e_near = abs(Tp[0][near] - T2[0][near]) / abs(T2[0][near])
    e_far = abs(Tp[0][far] - T2[0][far]) / abs(T2[0][far])
    assert e_far < 0.03 and e_far < 0.5 * e_near, (e_near, e_far)


def _cart_errors(N, method, M=0.5):
    g = oracle.CartGrid.square(N, M)
    X, Y = g.centres()
    R = np.hypot(X, Y)
    sig = analytic.sigma_dn(R, 2, 0.25)
    fx, fy = oracle.cart_forward(g, oracle.cart_tables(g, method), sig)
    fr = (fx * X + fy * Y) / R
    return oracle.error_norms(fr, analytic.force_dn(R, 2, 0.25))


def test_cartesian_convergence_on_sigma_d2():
    # Fig. 3: second order for the 2nd-order method, about first order for
    # both particle methods, the correction lowering the error
    e = {m: np.array([_cart_errors(N, m) for N in (32, 64, 128)])
         for m in ("second", "particle", "particle+")}
    o = {m: np.log2(v[:-1, 0] / v[1:, 0])
         for m, v in e.items()}
    assert np.all(np.abs(o["second"] - 2.0) < 0.3), o
    assert np.all(np.abs(o["particle"] - 1.0) < 0.3), o
    assert np.all(np.abs(o["particle+"] - 1.1) < 0.4), o
    assert np.all(e["particle+"][:, 0] < 0.5 * e["particle"][:, 0])
    assert np.all(e["second"][:, 0] < e["particle+"][:, 0])
