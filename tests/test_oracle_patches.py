"""Pins of the oracle's patch interaction and origin wedges (Sec. 3.2.1,
Eq. 27-29): a source patch at any row offset acting on a destination patch
equals the single-grid double sums on the union grid when the source's edge
rows hold no mass (the only place where slopes taken inside the patch and on
the union differ), for gaps, adjacency and overlap; the particle methods the
same way; the wedge kernels against independent 2-D quadrature and, summed,
the force of a uniform disk."""
import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads


def _union(g, n_src, s0):
    lo = min(s0, 0)
    hi = max(s0 + n_src, g.n_r)
    u = oracle.Grid(hi - lo, g.n_phi, g.r_min * g.beta ** lo, g.r_min * g.beta ** hi)
    return u, lo


def _source(n_src, n_phi, seed):
    s = workloads.random_field((n_src, n_phi), seed) + 0.5
    s[:2] = 0.0
    s[-2:] = 0.0
    return s


@pytest.mark.parametrize("s0", [-9, -6, -3, 2])
def test_patch_sums_equal_union_grid(s0):
    g = oracle.Grid(7, 16, 0.3, 2.0)
    n_src = 6
    sig = _source(n_src, g.n_phi, 21 + s0)
    u, lo = _union(g, n_src, s0)
    sk = oracle.selfcell_cover(g.beta, g.dphi, 10)[:3]
    su = np.zeros(u.shape)
    su[s0 - lo:s0 - lo + n_src] = sig
    Tu = oracle.tables(u, 19, self_k=sk)
    fr_u, fp_u = oracle.forward(u, Tu, su)
    T = oracle.patch_tables(g, n_src, s0, 19, self_k=sk)
    fr, fp = oracle.patch_forward(g, n_src, s0, T, sig)
    d = slice(-lo, -lo + g.n_r)
    scale = np.abs(fr_u[d]).max()
    np.testing.assert_allclose(fr, fr_u[d], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(fp, fp_u[d], rtol=0, atol=1e-12 * scale)
    # particle and modified particle methods
    for plus in (False, True):
        pr_u, pp_u = oracle.forward_particle(u, su, plus=plus, self_k=sk)
        pr, pp = oracle.patch_particle(g, n_src, s0, sig, plus=plus, self_k=sk)
        np.testing.assert_allclose(pr, pr_u[d], rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(pp, pp_u[d], rtol=0, atol=1e-12 * scale)


def test_sampled_destinations():
    g = oracle.Grid(6, 12, 0.5, 3.0)
    sig = _source(5, 12, 4)
    T = oracle.patch_tables(g, 5, -5, 3)
    full = oracle.patch_forward(g, 5, -5, T, sig)
    idx = np.array([0, 7, 30, 71])
    part = oracle.patch_forward(g, 5, -5, T, sig, dest=idx)
    np.testing.assert_array_equal(part[0], full[0].ravel()[idx])
    np.testing.assert_array_equal(part[1], full[1].ravel()[idx])


def _wedge_quad(g, s0, i, n, k):
    """Wedge kernel k at destination row i, offset n, by 2-D quadrature of
    its defining integrand in (eta, xi)."""
    r_w = g.r_min * g.beta ** s0
    ew = r_w / g.r_centres[i]
    ec = 0.5 * ew
    nrep = n if n <= g.n_phi // 2 else n - g.n_phi
    xc = -nrep * g.dphi

    def f(eta, xi):
        F3 = (eta * eta - 2 * eta * np.cos(xi) + 1.0) ** 1.5
        fr = eta * (1 - eta * np.cos(xi)) / F3
        fp = eta * eta * np.sin(xi) / F3
        return [-fr, -fr * (eta - ec), -fr * (xi - xc), fp, fp * (eta - ec), fp * (xi - xc)][k]

    return integrate.dblquad(f, xc - g.dphi / 2, xc + g.dphi / 2, 0.0, ew,
                             epsabs=1e-17, epsrel=1e-12)[0]


def test_wedge_kernels_match_quadrature():
    g = oracle.Grid(5, 8, 0.05, 1.0)
    for s0 in (-3, -1):
        Tw = oracle.wedge_tables(g, s0)
        for i, n in [(0, 0), (0, 1), (2, 3), (4, 7)]:
            for k in range(6):
                ref = _wedge_quad(g, s0, i, n, k)
                scale = abs(Tw[0, i, 0])
                assert abs(Tw[k, i, n] - ref) < 1e-11 * scale, (s0, i, n, k, Tw[k, i, n], ref)


def test_uniform_wedges_are_a_uniform_disk():
    # unit density in every wedge: the force of a uniform disk of radius r_w
    g = oracle.Grid(6, 16, 0.02, 1.0)
    s0 = -4
    r_w = g.r_min * g.beta ** s0
    Tw = oracle.wedge_tables(g, s0)
    for i in (0, 3, 5):
        ri = g.r_centres[i]
        ref = -integrate.dblquad(
            lambda rb, th: rb * (ri - rb * np.cos(th)) / (rb * rb + ri * ri - 2 * rb * ri * np.cos(th)) ** 1.5,
            0, 2 * np.pi, 0, r_w, epsabs=1e-18, epsrel=1e-12)[0]
        assert abs(Tw[0, i].sum() - ref) < 1e-11 * abs(ref)
        # azimuthal force of an axisymmetric ring of wedges vanishes
        assert abs(Tw[3, i].sum()) < 1e-14 * abs(ref)
    # point-mass wedges: the same mass at r_w / 2, within O((r_w / r)^2)
    Tp = oracle.wedge_tables(g, s0, "particle")
    for i in (0, 5):
        assert abs(Tp[0, i].sum() / Tw[0, i].sum() - 1) < 2 * (r_w / g.r_centres[i]) ** 2


@pytest.mark.parametrize("s0", [-9, -6, -3, 2])
def test_patch_adjoint_dot_product(s0):
    # the transpose of the patch map (no wedges): <v, A sigma> = <A^T v, sigma>
    # for any source density (edge rows included) and cotangents
    g = oracle.Grid(7, 16, 0.3, 2.0)
    n_src = 6
    T = oracle.patch_tables(g, n_src, s0, 19)
    sig = workloads.random_field((n_src, g.n_phi), 31 + s0)
    vr = workloads.random_field(g.shape, 41 + s0)
    vp = workloads.random_field(g.shape, 51 + s0)
    fr, fp = oracle.patch_forward(g, n_src, s0, T, sig)
    gs = oracle.patch_adjoint(g, n_src, s0, T, vr, vp)
    assert gs.shape == (n_src, g.n_phi)
    lhs = (fr * vr).sum() + (fp * vp).sum()
    rhs = (gs * sig).sum()
    assert abs(lhs - rhs) < 1e-12 * (np.abs(fr * vr).sum() + np.abs(fp * vp).sum())


def test_patch_adjoint_equals_union_grid_adjoint():
    # on the union grid the patch is a block of the single-grid map: with
    # cotangents zero outside the destination rows, the union transpose on
    # the source rows equals the patch transpose wherever the source's edge
    # rows do not enter (the slopes inside the patch and on the union differ
    # only there)
    g = oracle.Grid(7, 16, 0.3, 2.0)
    n_src, s0 = 8, -3
    u, lo = _union(g, n_src, s0)
    sk = oracle.selfcell_cover(g.beta, g.dphi, 10)[:3]
    T = oracle.patch_tables(g, n_src, s0, 19, self_k=sk)
    Tu = oracle.tables(u, 19, self_k=sk)
    vr = workloads.random_field(g.shape, 61)
    vp = workloads.random_field(g.shape, 62)
    vr_u, vp_u = np.zeros(u.shape), np.zeros(u.shape)
    vr_u[-lo:-lo + g.n_r], vp_u[-lo:-lo + g.n_r] = vr, vp
    gu = oracle.adjoint(u, Tu, vr_u, vp_u)[s0 - lo:s0 - lo + n_src]
    gp = oracle.patch_adjoint(g, n_src, s0, T, vr, vp)
    # rows 2 .. n_src - 3: every slope stencil that reads them is a central
    # difference in both
    inner = slice(2, n_src - 2)
    assert gp[inner].size == (n_src - 4) * g.n_phi
    scale = np.abs(gu).max()
    np.testing.assert_allclose(gp[inner], gu[inner], rtol=0, atol=1e-12 * scale)
    # the source's last row is an end of the patch but not of the union
    # grid: there the one-sided difference of the patch makes them differ
    assert np.abs(gp[-1] - gu[-1]).max() > 1e-6 * scale


def test_patch_adjoint_sampled_equals_full():
    g = oracle.Grid(6, 12, 0.5, 3.0)
    T = oracle.patch_tables(g, 5, -5, 3)
    vr = workloads.random_field(g.shape, 71)
    vp = workloads.random_field(g.shape, 72)
    full = oracle.patch_adjoint(g, 5, -5, T, vr, vp)
    idx = np.array([0, 7, 30, 59])
    part = oracle.patch_adjoint(g, 5, -5, T, vr, vp, src=idx)
    np.testing.assert_array_equal(part, full.ravel()[idx])


@pytest.mark.parametrize("s0,method", [(-6, "sim"), (-3, "sim"), (0, "sim"), (-2, "particle")])
def test_patch_adjoint_with_wedges_dot_product(s0, method):
    # the transpose with the origin wedges: <v, A (sigma, sigma_w)> =
    # <g_src, sigma> + <g_w, sigma_w>; the wedges couple to the first source
    # row through their radial slope, so a dropped or mis-signed slope term
    # breaks the identity on random inputs
    g = oracle.Grid(7, 16, 0.3, 2.0)
    n_src = 6
    T = oracle.patch_tables(g, n_src, s0, 19)
    Tw = oracle.wedge_tables(g, s0, method)
    sig = workloads.random_field((n_src, g.n_phi), 81 - s0)
    sw = workloads.random_field((g.n_phi,), 82 - s0)
    vr = workloads.random_field(g.shape, 83 - s0)
    vp = workloads.random_field(g.shape, 84 - s0)
    fr, fp = oracle.patch_forward(g, n_src, s0, T, sig, Tw=Tw, sigma_w=sw)
    gs, gw = oracle.patch_adjoint(g, n_src, s0, T, vr, vp, Tw=Tw)
    assert gs.shape == (n_src, g.n_phi) and gw.shape == (g.n_phi,)
    lhs = (fr * vr).sum() + (fp * vp).sum()
    rhs = (gs * sig).sum() + (gw * sw).sum()
    assert abs(lhs - rhs) < 1e-12 * (np.abs(fr * vr).sum() + np.abs(fp * vp).sum())
    # the wedge part alone (zero source patch) and the source part alone
    fr0, fp0 = oracle.patch_forward(g, n_src, s0, T, np.zeros_like(sig), Tw=Tw, sigma_w=sw)
    lw = (fr0 * vr).sum() + (fp0 * vp).sum()
    assert abs(lw - (gw * sw).sum()) < 1e-12 * (np.abs(fr0 * vr).sum() + np.abs(fp0 * vp).sum())
    # the wedges' slope reaches the first source row: it differs from the
    # transpose without wedges there and only there
    g0 = oracle.patch_adjoint(g, n_src, s0, T, vr, vp)
    if method == "sim":
        assert np.abs(gs[0] - g0[0]).max() > 1e-6 * np.abs(g0).max()
    else:
        np.testing.assert_array_equal(gs[0], g0[0])
    np.testing.assert_array_equal(gs[1:], g0[1:])


def test_patch_adjoint_wedge_gradient_by_unit_wedges():
    # g_w[j] = <v, A (0, e_j)>: the forward map of one unit wedge at a time
    g = oracle.Grid(5, 8, 0.2, 1.0)
    n_src, s0 = 4, -2
    T = oracle.patch_tables(g, n_src, s0, 19)
    Tw = oracle.wedge_tables(g, s0)
    vr = workloads.random_field(g.shape, 91)
    vp = workloads.random_field(g.shape, 92)
    _, gw = oracle.patch_adjoint(g, n_src, s0, T, vr, vp, Tw=Tw)
    z = np.zeros((n_src, g.n_phi))
    for j in range(g.n_phi):
        e = np.zeros(g.n_phi)
        e[j] = 1.0
        fr, fp = oracle.patch_forward(g, n_src, s0, T, z, Tw=Tw, sigma_w=e)
        want = (fr * vr).sum() + (fp * vp).sum()
        assert abs(gw[j] - want) < 1e-12 * (np.abs(fr * vr).sum() + np.abs(fp * vp).sum())


def _mirror_field(shape, j0, seed):
    # symmetric about the centre of column j0: s[:, j0 + d] = s[:, j0 - d]
    s = workloads.random_field(shape, seed) + 0.5
    n = shape[-1]
    j = np.arange(n)
    return 0.5 * (s + s[..., (2 * j0 - j) % n])


@pytest.mark.parametrize("c0", [3, -5, 21])
def test_turned_patch_mirror_line(c0):
    # a source (patch and wedges) mirror-symmetric about its column j0, turned
    # by c0 cells, is mirror-symmetric about destination column j0 + c0: F_phi
    # vanishes there and F_r is even about it.  A wrong sign or size of the
    # turn moves the line
    g = oracle.Grid(7, 16, 0.3, 2.0)
    n_src, s0, j0 = 6, -6, 2
    T = oracle.patch_tables(g, n_src, s0, 19)
    Tw = oracle.wedge_tables(g, s0)
    sig = _mirror_field((n_src, g.n_phi), j0, 121)
    sw = _mirror_field((g.n_phi,), j0, 122)
    jm = (j0 + c0) % g.n_phi
    j = np.arange(g.n_phi)
    for fr, fp in (oracle.patch_forward(g, n_src, s0, T, sig, Tw=Tw, sigma_w=sw, col0=c0),
                   oracle.patch_particle(g, n_src, s0, sig, sw, col0=c0)):
        scale = np.abs(fp).max()
        assert scale > 1e-3 * np.abs(fr).max()
        np.testing.assert_allclose(fp[:, jm], 0.0, atol=1e-13 * scale)
        np.testing.assert_allclose(fr, fr[:, (2 * jm - j) % g.n_phi], rtol=1e-13)
        np.testing.assert_allclose(fp, -fp[:, (2 * jm - j) % g.n_phi], atol=1e-13 * scale)
        # and not about the unturned column
        if jm != j0:
            assert np.abs(fp[:, j0]).max() > 1e-3 * scale


@pytest.mark.parametrize("plus", [False, True])
def test_turned_patch_equals_rolled_source(plus):
    # turning the source by c0 cells equals rolling its columns by c0 (the
    # tables' own periodicity), for overlapping patches too, where the turn
    # moves the singular self cell with the source
    g = oracle.Grid(7, 16, 0.3, 2.0)
    for n_src, s0, c0 in ((6, -6, 3), (8, -3, -7)):
        T = oracle.patch_tables(g, n_src, s0, 19)
        Tw = oracle.wedge_tables(g, s0) if s0 + n_src <= 0 else None
        sig = workloads.random_field((n_src, g.n_phi), 131) + 0.5
        sw = workloads.random_field((g.n_phi,), 132) + 0.5 if Tw is not None else None
        roll = lambda a: None if a is None else np.roll(a, c0, axis=-1)
        a = oracle.patch_forward(g, n_src, s0, T, sig, Tw=Tw, sigma_w=sw, col0=c0)
        b = oracle.patch_forward(g, n_src, s0, T, roll(sig), Tw=Tw, sigma_w=roll(sw))
        # (the same terms summed from another starting column)
        np.testing.assert_allclose(a[0], b[0], rtol=1e-14, atol=1e-15 * np.abs(b[0]).max())
        np.testing.assert_allclose(a[1], b[1], rtol=1e-14, atol=1e-15 * np.abs(b[1]).max())
        a = oracle.patch_particle(g, n_src, s0, sig, sw, plus=plus, col0=c0)
        b = oracle.patch_particle(g, n_src, s0, roll(sig), roll(sw), plus=plus)
        np.testing.assert_allclose(a[0], b[0], rtol=1e-13, atol=1e-13 * np.abs(b[0]).max())
        np.testing.assert_allclose(a[1], b[1], rtol=1e-13, atol=1e-13 * np.abs(b[1]).max())


@pytest.mark.parametrize("c0", [5, -9])
def test_turned_patch_adjoint_dot_product(c0):
    g = oracle.Grid(7, 16, 0.3, 2.0)
    n_src, s0 = 6, -6
    T = oracle.patch_tables(g, n_src, s0, 19)
    Tw = oracle.wedge_tables(g, s0)
    sig = workloads.random_field((n_src, g.n_phi), 141)
    sw = workloads.random_field((g.n_phi,), 142)
    vr = workloads.random_field(g.shape, 143)
    vp = workloads.random_field(g.shape, 144)
    fr, fp = oracle.patch_forward(g, n_src, s0, T, sig, Tw=Tw, sigma_w=sw, col0=c0)
    gs, gw = oracle.patch_adjoint(g, n_src, s0, T, vr, vp, Tw=Tw, col0=c0)
    lhs = (fr * vr).sum() + (fp * vp).sum()
    rhs = (gs * sig).sum() + (gw * sw).sum()
    assert abs(lhs - rhs) < 1e-12 * (np.abs(fr * vr).sum() + np.abs(fp * vp).sum())
    # the transpose of a turn is the opposite roll of the unturned transpose
    gs0, gw0 = oracle.patch_adjoint(g, n_src, s0, T, vr, vp, Tw=Tw)
    np.testing.assert_allclose(gs, np.roll(gs0, -c0, axis=1), rtol=1e-12,
                               atol=1e-13 * np.abs(gs0).max())
    np.testing.assert_allclose(gw, np.roll(gw0, -c0), rtol=1e-12, atol=1e-13 * np.abs(gw0).max())
