"""Pins of the analytic sigma_Dn module (Sec. 5.1, Eq. 50-55).

The Chebyshev closed form (Eq. 53) with the coefficient recursions (Eq. 54-55)
is checked against things it does not contain: the integral recursion Eq. 52
done by numerical quadrature, the textbook Maclaurin disk, continuity at the
disk edge and the far field -M/r^2.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import analytic

ALPHA = 0.25


def test_first_member_is_maclaurin():
    # sigma_D1 = sqrt(1 - r^2/alpha^2): F = -pi^2 r / (2 alpha) inside
    r = np.linspace(0.01, 0.99, 17) * ALPHA
    np.testing.assert_allclose(analytic.force_dn(r, 1, ALPHA),
                               -math.pi ** 2 * r / (2 * ALPHA), rtol=1e-14)


def test_second_member_hand_derived():
    # Eq. 52 applied to the Maclaurin force by hand gives, inside,
    # F_2 = (pi^2/2) [(9/8)(r/a)^3 - (3/2)(r/a)]
    r = np.linspace(0.02, 0.98, 13) * ALPHA
    x = r / ALPHA
    want = 0.5 * math.pi ** 2 * (9.0 / 8.0 * x ** 3 - 1.5 * x)
    np.testing.assert_allclose(analytic.force_dn(r, 2, ALPHA), want, rtol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("rfac", [0.2, 0.6, 0.97, 1.0, 1.3, 3.0])
def test_integral_recursion_eq52(n, rfac):
    # F_{n+1}(r; a) = (2n+1)/a^(2n+1) int_0^a ah^(2n) F_n(r; ah) d ah
    r = rfac * ALPHA
    f = lambda ah: ah ** (2 * n) * float(analytic.force_dn(r, n, ah))
    pts = [r] if r < ALPHA else None
    val, _ = integrate.quad(f, 0.0, ALPHA, points=pts, epsabs=0, epsrel=1e-13, limit=200)
    want = (2 * n + 1) / ALPHA ** (2 * n + 1) * val
    got = float(analytic.force_dn(r, n + 1, ALPHA))
    assert abs(got - want) <= 1e-11 * abs(want)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_density_recursion_eq51_consistency(n):
    # the same recursion on the density side: sigma_{n+1} from sigma_n
    for rfac in (0.1, 0.5, 0.9):
        r = rfac * ALPHA
        f = lambda ah: ah ** (2 * n) * float(analytic.sigma_dn(r, n, ah))
        val, _ = integrate.quad(f, r, ALPHA, epsabs=0, epsrel=1e-13)
        want = (2 * n + 1) / ALPHA ** (2 * n + 1) * val
        assert abs(float(analytic.sigma_dn(r, n + 1, ALPHA)) - want) < 1e-12


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_continuous_at_edge(n):
    # the outside branch has a sqrt(r - alpha) term, so the jump over
    # [alpha(1-e), alpha(1+e)] is O(sqrt(e)) when the branches agree at alpha
    e = 1e-12
    lo = analytic.force_dn(ALPHA * (1 - e), n, ALPHA)
    hi = analytic.force_dn(ALPHA * (1 + e), n, ALPHA)
    assert abs(lo - hi) < 20 * math.sqrt(e) * abs(lo)


@pytest.mark.parametrize("n", [1, 2, 5])
def test_far_field(n):
    # F r^2 / M -> -1, the remainder falling like (alpha/r)^2 (quadrupole)
    M = analytic.disk_mass(n, ALPHA)
    dev = []
    for rf in (8.0, 16.0, 32.0):
        r = rf * ALPHA
        dev.append(float(analytic.force_dn(r, n, ALPHA)) * r * r / M + 1)
    assert abs(dev[0]) < 0.01
    for a, b in zip(dev, dev[1:]):
        assert 3.6 < a / b < 4.4


def test_mass_integral():
    for n in (1, 2, 5):
        val, _ = integrate.quad(lambda r: 2 * math.pi * r * float(analytic.sigma_dn(r, n, ALPHA)),
                                0, ALPHA, epsabs=0, epsrel=1e-12)
        assert abs(val - analytic.disk_mass(n, ALPHA)) < 1e-10


def test_spot_value_by_local_polar_integral():
    # F_2 at an interior point from a direct principal-value integral of the
    # true density in polar coordinates about the point:
    # F_x = int_0^{2pi} cos t int_0^{R(t)} (sigma(x + rho e_t) - sigma(x))/rho drho dt
    #       + sigma(x) int cos t ln R(t) dt,  R(t) = distance to the disk edge.
    n, x0 = 2, 0.3 * ALPHA
    sig = lambda rr: float(analytic.sigma_dn(rr, n, ALPHA))

    def Rt(t):
        c = math.cos(t)
        return -x0 * c + math.sqrt(x0 * x0 * c * c - x0 * x0 + ALPHA * ALPHA)

    def inner(t):
        c, s = math.cos(t), math.sin(t)
        f = lambda rho: (sig(math.hypot(x0 + rho * c, rho * s)) - sig(x0)) / rho
        v, _ = integrate.quad(f, 0, Rt(t), epsabs=1e-13, epsrel=1e-12, limit=200)
        return c * (v + sig(x0) * math.log(Rt(t)))

    val, _ = integrate.quad(inner, 0, 2 * math.pi, epsabs=1e-12, epsrel=1e-11, limit=200)
    assert abs(val - float(analytic.force_dn(x0, n, ALPHA))) < 1e-8


def test_kuzmin_closed_form():
    # potential -2 pi / sqrt(1 + r^2) differentiated numerically
    r = np.array([0.1, 1.0, 3.0])
    h = 1e-6
    pot = lambda x: -2 * math.pi / np.sqrt(1 + x * x)
    fd = -(pot(r + h) - pot(r - h)) / (2 * h)
    np.testing.assert_allclose(analytic.kuzmin_force(r), fd, rtol=1e-8)
