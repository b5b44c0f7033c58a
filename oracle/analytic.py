"""Closed-form forces of the finite thin disks sigma_Dn (Sec. 5.1).

TEST INFRASTRUCTURE ONLY (part of the oracle; see ``oracle/__init__.py``).

sigma_Dn(r; alpha) = (1 - r^2/alpha^2)^(n - 1/2) inside r < alpha, 0 outside
(Eq. 50, sigma_0 = 1, G = 1).  Its mid-plane radial force has the Chebyshev
form of Eq. 53, with coefficients from the recursions Eq. 54-55 started at
a^1_1 = 1, b^1_0 = -1.  Readings taken:
  * Eq. 54's third sum prints a^2_{2k+3}; it is read as a^n_{2k+3}
    (the derivation of App. B, Eq. B20, has a^n);
  * coefficients outside their index range are zero;
  * Eq. 53 gives the force of sigma_Dn itself (n = 1 is the Maclaurin disk).
The module is pinned in the tests against the integral recursion Eq. 52, the
Maclaurin disk, continuity at r = alpha and the far field -M/r^2.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def coefficients_exact(n: int):
    """(a, b) for sigma_Dn as exact rationals: a[k] = a^n_{2k+1},
    b[k] = b^n_{2k}, k = 0..n-1 (Eq. 54-55, a^1_1 = 1, b^1_0 = -1)."""
    if n < 1:
        raise ValueError("n >= 1")
    a = {1: Fraction(1)}   # keyed by the Chebyshev order
    b = {0: Fraction(-1)}
    for m in range(1, n):          # build (a^{m+1}, b^{m+1}) from (a^m, b^m)
        Z = Fraction(0)
        A = lambda q: a.get(q, Z)
        B = lambda q: b.get(q, Z)
        q4, q2, q8 = Fraction(1, 4), Fraction(1, 2), Fraction(1, 8)

        def Fj(j):
            s = Z
            s -= q4 * sum((A(2 * k + 1) / (2 * k + 2) for k in range(j, m + 1)), Z)
            s += q4 * sum((A(2 * k - 1) / (2 * k + 2) for k in range(j, m + 1)), Z)
            s -= q4 * sum((A(2 * k + 3) / (2 * k + 2) for k in range(j, m - 1)), Z)
            s += q4 * sum((A(2 * k + 5) / (2 * k + 2) for k in range(j, m - 2)), Z)
            s += q2 * sum((B(2 * k) / (2 * k + 2) ** 2 for k in range(j, m)), Z)
            s -= q2 * sum((B(2 * k + 4) / (2 * k + 2) ** 2 for k in range(j, m - 2)), Z)
            return s

        def Gj(j):
            return q8 * (B(2 * j - 2) / j - B(2 * j + 2) / j)

        f = 2 * m + 1
        na = {1: f * (Fj(0) + B(0) * q8 + A(1) * q8)}
        for j in range(1, m + 1):
            na[2 * j + 1] = f * Fj(j)
        nb = {0: f * (A(1) * q8 - A(3) * q8)}
        if m >= 1:
            nb[2] = f * (Gj(1) + B(0) * q8)
        for j in range(2, m + 1):
            nb[2 * j] = f * Gj(j)
        a, b = na, nb
    return (tuple(a.get(2 * k + 1, Fraction(0)) for k in range(n)),
            tuple(b.get(2 * k, Fraction(0)) for k in range(n)))


def coefficients(n: int):
    """The coefficients of :func:`coefficients_exact` rounded to float."""
    a, b = coefficients_exact(n)
    return tuple(float(v) for v in a), tuple(float(v) for v in b)


def _cheb_T(k: int, x):
    """Chebyshev polynomial of the first kind by its three-term recursion."""
    x = np.asarray(x)
    t0, t1 = np.ones_like(x), x
    if k == 0:
        return t0
    for _ in range(k - 1):
        t0, t1 = t1, 2 * x * t1 - t0
    return t1


def sigma_dn(r, n: int, alpha: float):
    """Surface density of Eq. 50 (sigma_0 = 1)."""
    r = np.asarray(r, dtype=np.float64)
    q = np.clip(1.0 - (r / alpha) ** 2, 0.0, None)
    return np.where(r < alpha, q ** (n - 0.5), 0.0)


def force_dn(r, n: int, alpha: float):
    """Radial mid-plane force of sigma_Dn about its own centre (Eq. 53).

    Negative values point towards the disk centre."""
    r0 = np.asarray(r, dtype=np.float64)
    r = np.atleast_1d(r0)
    a, b = coefficients(n)
    rr = np.where(r > 0, r, 1.0)
    x = alpha / rr
    pw = (rr / alpha) ** (2 * n - 1)
    sb = sum(b[k] * _cheb_T(2 * k, x) for k in range(n))
    inside = 0.5 * math.pi ** 2 * pw * sb
    # outside the disk the two sums cancel to O((alpha/r)^(2n+1)) of their
    # size, so that branch is evaluated in extended precision
    xo = np.minimum(x, 1.0).astype(np.longdouble)
    sa = sum(np.longdouble(a[k]) * _cheb_T(2 * k + 1, xo) for k in range(n))
    sbo = sum(np.longdouble(b[k]) * _cheb_T(2 * k, xo) for k in range(n))
    pwl = (rr.astype(np.longdouble) / np.longdouble(alpha)) ** (2 * n - 1)
    outside = (np.longdouble(math.pi) * pwl
               * (sbo * np.arcsin(xo) + sa * np.sqrt(np.clip(1 - xo * xo, 0, None))))
    out = np.where(rr <= alpha, inside, outside.astype(np.float64))
    # far from the disk even 64-bit mantissas run out; those few points are
    # done with 60 significant digits
    far = np.nonzero((r > 0) & (x < 0.15))
    if far[0].size:
        out = np.array(out, dtype=np.float64, copy=True)
        for idx in zip(*far):
            out[idx] = _outside_mp(float(rr[idx]), n, alpha)
    return np.where(r > 0, out, 0.0).reshape(r0.shape)


def _outside_mp(r: float, n: int, alpha: float) -> float:
    import mpmath as mp
    a, b = coefficients_exact(n)
    with mp.workdps(60):
        x = mp.mpf(alpha) / mp.mpf(r)
        T = [mp.mpf(1), x]
        for _ in range(2 * n):
            T.append(2 * x * T[-1] - T[-2])
        q = lambda v: mp.mpf(v.numerator) / v.denominator
        sb = mp.fsum(q(b[k]) * T[2 * k] for k in range(n))
        sa = mp.fsum(q(a[k]) * T[2 * k + 1] for k in range(n))
        v = mp.pi * (mp.mpf(r) / alpha) ** (2 * n - 1) * (sb * mp.asin(x) + sa * mp.sqrt(1 - x * x))
        return float(v)


def disk_mass(n: int, alpha: float) -> float:
    """Total mass of sigma_Dn: 2 pi alpha^2 / (2n + 1)."""
    return 2.0 * math.pi * alpha ** 2 / (2 * n + 1)


def offcentre_forces(r, phi, n: int, alpha: float, xc: float, yc: float):
    """(F_r, F_phi) at polar points (r, phi) of a sigma_Dn disk centred at
    (xc, yc): the disk's radial force along (x - x_c)/|x - x_c|, projected
    on the grid's unit vectors r-hat and phi-hat."""
    r = np.asarray(r, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    x, y = r * np.cos(phi), r * np.sin(phi)
    dx, dy = x - xc, y - yc
    d = np.hypot(dx, dy)
    f = force_dn(d, n, alpha)
    ds = np.where(d > 0, d, 1.0)
    fx, fy = f * dx / ds, f * dy / ds
    fr = fx * np.cos(phi) + fy * np.sin(phi)
    fp = -fx * np.sin(phi) + fy * np.cos(phi)
    return fr, fp


def kuzmin_force(r):
    """Kuzmin disk sigma = (1 + r^2)^(-3/2): F_r = -2 pi r / (1 + r^2)^(3/2)
    (potential -2 pi / sqrt(1 + r^2), textbook closed form)."""
    r = np.asarray(r, dtype=np.float64)
    return -2.0 * math.pi * r / (1.0 + r * r) ** 1.5
