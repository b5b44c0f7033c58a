"""Pins of the oracle's slopes of Eq. 25 (delta^r = d sigma / dr and
delta^phi = d sigma / dphi at the cell centres, taken from the cell values)
for both difference orders, and of the order-4 forward map and transpose.

Checked against: exactness of the five-point difference on quartic
polynomials in u = ln r (the grid is uniform in u) and of the central and
one-sided differences on densities linear in r; the discrete symbols of the
periodic differences on Fourier modes and their fourth- and second-order
approach to the derivative; fourth-order convergence of the radial slope on
a smooth density; brute-force 2-D quadrature of the force integrals over the
piecewise-linear density built from the order-4 slopes; and the dot-product
identity of the order-4 transpose."""
import math

import numpy as np
import pytest

import oracle
import workloads

from test_oracle_forces import _brute_force


def _grid(n_r=24, n_phi=16, r_min=0.1, r_max=10.0):
    return oracle.Grid(n_r, n_phi, r_min, r_max)


def test_radial_five_point_exact_on_quartics_in_u():
    g = _grid()
    u = np.log(g.r_centres)
    c = (0.3, 0.7, -0.2, 0.05, -0.01)
    P = sum(ck * u ** k for k, ck in enumerate(c))
    dP = sum(k * ck * u ** (k - 1) for k, ck in enumerate(c) if k)
    sig = np.repeat(P[:, None], g.n_phi, 1)
    dr4, dp4 = oracle.channels(g, sig, slope_order=4)
    want = (dP / g.r_centres)[2:-2, None]
    assert np.abs(dr4[2:-2] - want).max() < 1e-12 * np.abs(want).max()
    assert np.abs(dp4).max() < 1e-13 * np.abs(sig).max() / g.dphi
    # the order-2 central difference is not exact here (a dropped order
    # would show)
    dr2, _ = oracle.channels(g, sig)
    assert np.abs(dr2[2:-2] - want).max() > 1e-4 * np.abs(want).max()


@pytest.mark.parametrize("order", [2, 4])
def test_radial_ends_exact_on_densities_linear_in_r(order):
    g = _grid()
    sig = np.repeat((2.0 + 3.0 * g.r_centres)[:, None], g.n_phi, 1)
    dr, _ = oracle.channels(g, sig, slope_order=order)
    ends = [0, 1, g.n_r - 2, g.n_r - 1]
    np.testing.assert_allclose(dr[ends], 3.0, rtol=1e-12)
    if order == 2:
        np.testing.assert_allclose(dr, 3.0, rtol=1e-12)
    else:
        # five points of 2 + 3 e^u: exact only to O(du^4)
        du = math.log(g.beta)
        err = np.abs(dr[2:-2] - 3.0).max()
        assert 0 < err < 3.0 * du ** 4


@pytest.mark.parametrize("m", [1, 2, 3])
def test_azimuthal_symbols_on_fourier_modes(m):
    g = _grid(n_r=6, n_phi=32)
    phi = g.phi_centres
    sig = np.repeat(np.cos(m * phi)[None, :], g.n_r, 0)
    d = g.dphi
    _, dp2 = oracle.channels(g, sig, slope_order=2)
    _, dp4 = oracle.channels(g, sig, slope_order=4)
    s2 = math.sin(m * d) / d
    s4 = (8.0 * math.sin(m * d) - math.sin(2 * m * d)) / (6.0 * d)
    mode = np.broadcast_to(np.sin(m * phi)[None, :], g.shape)
    np.testing.assert_allclose(dp2, -s2 * mode, atol=1e-12 * m)
    np.testing.assert_allclose(dp4, -s4 * mode, atol=1e-12 * m)
    # the symbols approach m to second and fourth order in m dphi
    x = m * d
    assert abs(s2 - m) == pytest.approx(m * x * x / 6, rel=0.05)
    assert abs(s4 - m) == pytest.approx(m * x ** 4 / 30, rel=0.05)


def test_radial_five_point_converges_at_fourth_order():
    errs = []
    for n_r in (32, 64, 128):
        g = _grid(n_r=n_r, n_phi=8)
        u = np.log(g.r_centres)
        sig = np.repeat(np.exp(-u * u)[:, None], g.n_phi, 1)
        want = -2.0 * u * np.exp(-u * u) / g.r_centres
        dr, _ = oracle.channels(g, sig, slope_order=4)
        errs.append(np.abs(dr[2:-2, 0] - want[2:-2]).max())
    r = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(r > 3.7), r


def test_slope_order_is_checked():
    g = _grid(n_r=6, n_phi=8)
    sig = workloads.random_field(g.shape, seed_k=3)
    with pytest.raises(ValueError):
        oracle.channels(g, sig, slope_order=3)


@pytest.mark.slow
def test_order4_forward_matches_brute_force_quadrature():
    # 7 rows: rows 2..4 take the five-point difference
    g = oracle.Grid(7, 8, 0.5, 2.0)
    sig = workloads.random_field(g.shape, seed_k=21)
    sk = oracle.selfcell_cover(g.beta, g.dphi)[:3]
    cells = [(1, 2), (3, 6)]
    dest = [i * g.n_phi + j for i, j in cells]
    T = oracle.tables(g, 799, self_k=sk)
    fr, fp = oracle.forward(g, T, sig, dest, slope_order=4)
    bf = np.array([_brute_force(g, T, sig, i, j, slope_order=4) for i, j in cells])
    scale = np.abs(bf).max()
    # what remains is the trapezoid error of Eq. 41-43 (5.1e-7 of the scale
    # at 799 trapezoids, 2.0e-6 at 399: second order, as for order 2)
    assert np.abs(np.stack([fr, fp], 1) - bf).max() < 1e-6 * scale
    # and the order-2 forward differs from it by far more than that
    f2r, f2p = oracle.forward(g, T, sig, dest)
    assert np.abs(np.stack([f2r, f2p], 1) - bf).max() > 1e-4 * scale


def test_order4_adjoint_dot_product():
    g = _grid()
    T = oracle.tables(g, 19)
    sig = workloads.random_field(g.shape, seed_k=23)
    vr = workloads.random_field(g.shape, seed_k=24)
    vp = workloads.random_field(g.shape, seed_k=25)
    fr, fp = oracle.forward(g, T, sig, slope_order=4)
    gs = oracle.adjoint(g, T, vr, vp, slope_order=4)
    lhs = (fr * vr).sum() + (fp * vp).sum()
    rhs = (sig * gs).sum()
    assert abs(lhs - rhs) < 1e-12 * (np.abs(fr * vr).sum() + np.abs(fp * vp).sum())
    # the order-2 transpose does not satisfy it with the order-4 forward map
    g2 = oracle.adjoint(g, T, vr, vp)
    assert abs(lhs - (sig * g2).sum()) > 1e-6 * abs(lhs)
