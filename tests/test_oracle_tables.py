"""Pins of the oracle's grid, slopes and kernel tables.

Each check compares the oracle against something it does not contain:
scipy quadrature of the kernel integrals (Eq. 30-32, A22-A24), the trapezoid
error law of Eq. 41-43, the parities the paper states for the self cell, the
invariance of Eq. 33, and a principal-value integral of the self cell.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle


def test_gauss_legendre_matches_numpy():
    for n in (2, 7, 16, 24, 32):
        x, w = oracle.gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        np.testing.assert_allclose(np.sort(x), np.sort(xr), atol=2e-15)
        np.testing.assert_allclose(w[np.argsort(x)], wr[np.argsort(xr)], atol=2e-15)


def test_grid_areas_and_log_spacing():
    g = oracle.Grid(40, 24, 0.1, 10.0)
    assert abs(g.cell_areas().sum() - math.pi * (10.0 ** 2 - 0.1 ** 2)) < 1e-10
    du = np.diff(np.log(g.r_centres))
    np.testing.assert_allclose(du, math.log(g.beta), rtol=1e-13)
    # arithmetic-mean centres (Sec. 3.2.1)
    np.testing.assert_allclose(g.r_centres, 0.5 * (g.r_edges[1:] + g.r_edges[:-1]), rtol=1e-15)
    assert abs(g.beta ** 40 - 100.0) < 1e-11


def test_radial_slope_exact_for_linear_density():
    g = oracle.Grid(16, 8, 0.5, 4.0)
    sig = 2.0 + 3.0 * g.r_centres[:, None] + 0 * g.phi_centres[None, :]
    dr, dp = oracle.channels(g, sig)
    np.testing.assert_allclose(dr, 3.0, rtol=1e-12)
    np.testing.assert_allclose(dp, 0.0, atol=1e-12)


def test_azimuthal_slope_closed_form():
    g = oracle.Grid(4, 32, 0.5, 4.0)
    k = 3
    sig = np.cos(k * g.phi_centres)[None, :] * np.ones((4, 1))
    _, dp = oracle.channels(g, sig)
    want = -(math.sin(k * g.dphi) / g.dphi) * np.sin(k * g.phi_centres)
    np.testing.assert_allclose(dp, np.broadcast_to(want, dp.shape), atol=1e-13)


# --------------------------------------------------------------------------
# kernel tables against scipy quadrature
# --------------------------------------------------------------------------
G32 = oracle.Grid(32, 32, 0.01, 1.0)


def _F(eta, xi):
    return np.sqrt(eta * eta - 2 * eta * np.cos(xi) + 1)


def _reference_entry(g, m, n, ntpz):
    """Trapezoid in xi (Eq. 41-43) of the radial integral done by adaptive
    quadrature, and the exact azimuthal kernels by 2-D adaptive quadrature."""
    b, dp = g.beta, g.dphi
    rho = b ** (-m)
    el = 2 * rho / (1 + b)
    eu = b * el
    xc = -n * dp
    nodes = xc - dp / 2 + np.arange(ntpz + 1) * dp / ntpz
    w = np.full(ntpz + 1, dp / ntpz)
    w[0] *= 0.5
    w[-1] *= 0.5

    def I(f, xi):
        pts = [1.0] if el < 1 < eu else None
        return integrate.quad(lambda e: f(e, xi), el, eu, epsabs=0, epsrel=2e-14,
                              limit=200, points=pts)[0]

    fr = lambda e, xi: e * (1 - e * np.cos(xi)) / _F(e, xi) ** 3
    fr2 = lambda e, xi: e * e * (1 - e * np.cos(xi)) / _F(e, xi) ** 3
    fp = lambda e, xi: e * e * np.sin(xi) / _F(e, xi) ** 3
    Ir = np.array([I(fr, x) for x in nodes])
    Ir2 = np.array([I(fr2, x) for x in nodes])
    Ip = np.array([I(fp, x) for x in nodes])
    r0 = -(w * Ir).sum()
    rr = -(w * (Ir2 - rho * Ir)).sum()
    rp = -(w * (nodes - xc) * Ir).sum()
    pp = (w * (nodes - xc) * Ip).sum()
    opts = dict(epsabs=0, epsrel=2e-13)
    p0 = integrate.dblquad(lambda e, xi: fp(e, xi), xc - dp / 2, xc + dp / 2, el, eu, **opts)[0]
    pr = integrate.dblquad(lambda e, xi: fp(e, xi) * (e - rho), xc - dp / 2, xc + dp / 2, el, eu, **opts)[0]
    return np.array([r0, rr, rp, p0, pr, pp])


@pytest.mark.parametrize("m,n", [(0, 1), (1, 0), (-1, 0), (1, 1), (0, 5), (3, -2),
                                 (-7, 4), (20, 9), (-25, 16), (0, 16), (0, -15)])
def test_entries_match_quadrature(m, n):
    t = oracle.table_entry(G32, m, n, 19)
    e = _reference_entry(G32, m, n, 19)
    # absolute agreement on the scale of the largest table entry (O(1))
    np.testing.assert_allclose(t, e, rtol=0, atol=3e-14)


def test_trapezoid_error_law():
    # SIM kernels approach the exact integrals as N_tpz^-2 (Eq. 41-43)
    def exact_r0(m, n):
        b, dp = G32.beta, G32.dphi
        rho = b ** (-m)
        el = 2 * rho / (1 + b)
        xc = -n * dp
        f = lambda e, xi: -e * (1 - e * np.cos(xi)) / _F(e, xi) ** 3
        return integrate.dblquad(f, xc - dp / 2, xc + dp / 2, el, b * el, epsabs=0, epsrel=1e-13)[0]

    for (m, n) in [(1, 1), (-2, 3), (5, 7)]:
        ex = exact_r0(m, n)
        e19 = oracle.table_entry(G32, m, n, 19)[0] - ex
        e39 = oracle.table_entry(G32, m, n, 39)[0] - ex
        assert 3.8 < e19 / e39 < 4.6, (m, n, e19, e39)


def _exact_reference_entry(g, m, n):
    """The six kernels of Eq. 30-32 (A22-A24) as nested adaptive quadrature
    over the whole source cell: the converged definition the exact table
    mode computes (no trapezoid).  The xi range is split at 0 when the cell
    contains it, the eta range at the singular ring eta = 1."""
    b, dp = g.beta, g.dphi
    rho = b ** (-m)
    el = 2 * rho / (1 + b)
    eu = b * el
    xc = -n * dp
    pts = [1.0] if el < 1 < eu else None
    fr = lambda e, xi: e * (1 - e * np.cos(xi)) / _F(e, xi) ** 3
    fp = lambda e, xi: e * e * np.sin(xi) / _F(e, xi) ** 3
    integrands = [lambda e, xi: -fr(e, xi),
                  lambda e, xi: -fr(e, xi) * (e - rho),
                  lambda e, xi: -fr(e, xi) * (xi - xc),
                  lambda e, xi: fp(e, xi),
                  lambda e, xi: fp(e, xi) * (e - rho),
                  lambda e, xi: fp(e, xi) * (xi - xc)]
    lo, hi = xc - dp / 2, xc + dp / 2
    cuts = [lo, 0.0, hi] if lo < 0 < hi else [lo, hi]
    out = []
    for f in integrands:
        inner = lambda xi: integrate.quad(lambda e: f(e, xi), el, eu, epsabs=0, epsrel=2e-14,
                                          limit=200, points=pts)[0]
        out.append(sum(integrate.quad(inner, a, c, epsabs=1e-16, epsrel=1e-13, limit=200)[0]
                       for a, c in zip(cuts[:-1], cuts[1:])))
    return np.array(out)


@pytest.mark.parametrize("m,n", [(0, 1), (1, 0), (-1, 0), (1, 1), (-2, 3), (5, 7), (0, 16)])
def test_exact_entries_match_2d_quadrature(m, n):
    t = oracle.table_entry(G32, m, n, table_mode="exact")
    e = _exact_reference_entry(G32, m, n)
    np.testing.assert_allclose(t, e, rtol=0, atol=2e-13)


def test_trapezoid_tables_converge_to_exact_tables():
    # the SIM tables approach the exact tables as N_tpz^-2 (Eq. 41-43)
    sk = oracle.selfcell_pv(G32.beta, G32.dphi)
    te = oracle.tables(G32, self_k=sk, table_mode="exact")
    err = {}
    for nt in (19, 39):
        ts = oracle.tables(G32, nt, self_k=sk)
        err[nt] = np.array([np.abs(ts[k] - te[k]).max() / np.abs(te[k]).max() for k in range(6)])
    ratio = err[19][[0, 1, 2, 5]] / err[39][[0, 1, 2, 5]]
    np.testing.assert_allclose(ratio, (39 / 19) ** 2, rtol=0.05)
    # K^{phi,0} and K^{phi,r} are exact in both modes (A30-A31)
    assert err[19][3] == 0.0 and err[19][4] == 0.0


def test_parities_and_self_zeros():
    sk = (-0.01, 0.2, 0.3)
    par = np.array([1, 1, -1, -1, -1, 1])
    for m in (-3, -1, 0, 1, 4):
        for n in (1, 2, 7, 15):
            tp = oracle.table_entry(G32, m, n, 19, sk)
            tm = oracle.table_entry(G32, m, -n, 19, sk)
            np.testing.assert_allclose(tm, par * tp, rtol=1e-12, atol=1e-16)
    t0 = oracle.table_entry(G32, 0, 0, 19, sk)
    assert t0[2] == 0 and t0[3] == 0 and t0[4] == 0
    np.testing.assert_array_equal(t0[[0, 1, 5]], sk)
    # n = 0 column of the odd azimuthal kernels is zero away from the self cell
    for m in (-5, 2):
        t = oracle.table_entry(G32, m, 0, 19)
        assert abs(t[2]) < 1e-15 and t[3] == 0.0 and abs(t[4]) < 1e-15


def test_tables_depend_only_on_beta_and_dphi():
    # Eq. 33: the kernels are functions of (beta, dphi, m, n) alone
    a = oracle.tables(oracle.Grid(12, 16, 0.01, 1.0), 19)
    b = oracle.tables(oracle.Grid(12, 16, 3.0, 300.0), 19)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-16)


def test_azimuthal_kernels_sum_to_zero_over_a_ring():
    T = oracle.tables(oracle.Grid(10, 24, 0.1, 10.0), 19)
    for k in (3, 4):
        np.testing.assert_allclose(T[k].sum(axis=1), 0.0, atol=1e-14)


def _self_cell_pv(beta, dphi):
    """Self-cell K^{r,0}_{00}, K^{r,r}_{00} and K^{phi,phi}_{00} in local
    polar coordinates (rho, t) about the fan centre (1, 0):
      K^{r,0}     = int cos t ln rho_max(t) dt           (principal value)
      K^{r,r}     = int cos t int_0^{rho_max} (|x| - 1)/rho drho dt
      K^{phi,phi} = int sin t int_0^{rho_max} phi(x)/rho drho dt."""
    r_in, r_out = 2 / (1 + beta), 2 * beta / (1 + beta)
    a = dphi / 2

    def rho_max(t):
        c, s = math.cos(t), math.sin(t)
        cands = [-c + math.sqrt(c * c + r_out * r_out - 1)]
        disc = c * c - (1 - r_in * r_in)
        if disc >= 0:
            for root in (-c - math.sqrt(disc), -c + math.sqrt(disc)):
                if root > 0:
                    cands.append(root)
        for sa in (a, -a):
            den = s * math.cos(sa) - c * math.sin(sa)
            if den != 0:
                rr = math.sin(sa) / den
                if rr > 0:
                    cands.append(rr)
        return min(cands)

    # split at the directions of the four corners
    corners = []
    for R in (r_in, r_out):
        for sa in (a, -a):
            corners.append(math.atan2(R * math.sin(sa), R * math.cos(sa) - 1) % (2 * math.pi))
    brk = sorted(set([0.0] + corners + [2 * math.pi]))
    k0 = k1 = k2 = 0.0
    for lo, hi in zip(brk[:-1], brk[1:]):
        tol = dict(epsabs=1e-16, epsrel=1e-14, limit=200)
        k0 += integrate.quad(lambda t: math.cos(t) * math.log(rho_max(t)), lo, hi, **tol)[0]

        def inner(t):
            c, s = math.cos(t), math.sin(t)
            f = lambda p: (math.hypot(1 + p * c, p * s) - 1) / p
            return c * integrate.quad(f, 0, rho_max(t), **tol)[0]
        k1 += integrate.quad(inner, lo, hi, **tol)[0]

        def inner_phi(t):
            c, s = math.cos(t), math.sin(t)
            f = lambda p: math.atan2(p * s, 1 + p * c) / p
            return s * integrate.quad(f, 0, rho_max(t), **tol)[0]
        k2 += integrate.quad(inner_phi, lo, hi, **tol)[0]
    return k0, k1, k2


@pytest.mark.parametrize("shape", [(64, 64, 0.01, 1.0), (37, 128, 0.1, 10.0), (16, 8, 0.5, 2.0)])
def test_oracle_principal_value_matches_local_polar_quadrature(shape):
    g = oracle.Grid(*shape)
    ref = _self_cell_pv(g.beta, g.dphi)
    got = oracle.selfcell_pv(g.beta, g.dphi)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-15)


def test_self_cell_cover_converges_to_principal_value():
    g = oracle.Grid(64, 64, 0.01, 1.0)
    pv0, pv1, pv2 = _self_cell_pv(g.beta, g.dphi)
    errs0, errs1, errs2 = [], [], []
    for per in (10, 20, 40):
        c0, c1, c2, _ = oracle.selfcell_cover(g.beta, g.dphi, per)
        errs0.append(abs(c0 - pv0) / abs(pv0))
        errs1.append(abs(c1 - pv1) / abs(pv1))
        errs2.append(abs(c2 - pv2) / abs(pv2))
    # paper's rule (10 per Delta x, Delta y) is within a few percent, and the
    # cover error shrinks under refinement
    assert errs0[0] < 0.05 and errs1[0] < 1e-3 and errs2[0] < 1e-4
    assert errs0[2] < errs0[1] < errs0[0]
    assert errs1[2] < errs1[0]
    assert errs2[2] < errs2[0]


def test_self_cell_cover_counts_match_paper_rule():
    # 10 N x 5 N Cartesian cells for r_max/r_min = 100 (Sec. 4)
    g = oracle.Grid(64, 64, 0.01, 1.0)
    n = oracle.selfcell_cover(g.beta, g.dphi, 10)[3]
    assert 0.3 * 50 * 64 * 64 < n < 50 * 64 * 64


def _selfcell_golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "selfcell_constants.txt")
    rows = []
    with open(path) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("row", _selfcell_golden(), ids=lambda r: "N%d" % r[0])
def test_self_cell_constants_against_independent_values(row):
    """The principal values to 1e-14 and the paper's cover (Sec. 4) to the
    digits of an independent implementation (tests/golden/selfcell_constants.txt):
    a misaligned cover grid or an open-fan inclusion test moves the cover's
    constants in the fourth digit and fails here."""
    N, pv0, pv1, cv0, cv1 = row
    N = int(N)
    g = oracle.Grid(N, N, 0.01, 1.0)
    k0, k1, _ = oracle.selfcell_pv(g.beta, g.dphi)
    # 1e-14 absolute: 12 significant digits at N = 64, 11 at N = 256 (the
    # constants shrink as the cell; the integrands' terms are of order one)
    assert abs(k0 - pv0) <= 1e-14
    assert abs(k1 - pv1) <= 1e-14
    c0, c1, _, _ = oracle.selfcell_cover(g.beta, g.dphi, 10)
    # the golden digits: half a unit in the last place shown
    assert abs(c0 - cv0) <= 5e-7
    assert abs(c1 - cv1) <= 5e-7
