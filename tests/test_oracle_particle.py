"""Pins of the oracle's particle and modified particle methods (Eq. 34-37,
56-62): an independent Cartesian point-mass sum, the self-cell correction
of the modified method, and first-order convergence on the analytic disk
(Table 1's particle columns)."""
import numpy as np

import oracle
import workloads
from oracle import analytic


def _point_mass_forces(g, sig):
    """Newtonian forces of point masses sigma * (exact cell area) at the cell
    centres, in Cartesian coordinates, projected on r-hat and phi-hat; no
    self force."""
    re = g.r_edges
    area = 0.5 * (re[1:] ** 2 - re[:-1] ** 2) * g.dphi
    M = (sig * area[:, None]).ravel()
    x, y = (a.ravel() for a in g.xy())
    phi = np.repeat(g.phi_centres[None, :], g.n_r, axis=0).ravel()
    fr = np.empty(x.size)
    fp = np.empty(x.size)
    for q in range(x.size):
        dx, dy = x - x[q], y - y[q]
        d3 = np.hypot(dx, dy) ** 3
        d3[q] = np.inf
        fx, fy = np.sum(M * dx / d3), np.sum(M * dy / d3)
        fr[q] = fx * np.cos(phi[q]) + fy * np.sin(phi[q])
        fp[q] = -fx * np.sin(phi[q]) + fy * np.cos(phi[q])
    return fr.reshape(g.shape), fp.reshape(g.shape)


def test_particle_method_is_the_point_mass_sum():
    g = oracle.Grid(6, 8, 0.2, 5.0)
    sig = workloads.random_field(g.shape, 7) + 1.0
    fr, fp = oracle.forward_particle(g, sig)
    er, ep = _point_mass_forces(g, sig)
    scale = np.abs(er).max()
    np.testing.assert_allclose(fr, er, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(fp, ep, rtol=0, atol=1e-13 * scale)


def test_modified_method_adds_the_self_cell_correction():
    g = oracle.Grid(12, 16, 0.1, 10.0)
    sig = workloads.single_disk_blobs(g.r_centres, g.phi_centres)
    sk = oracle.selfcell_cover(g.beta, g.dphi, 10)[:3]
    f0 = oracle.forward_particle(g, sig)
    f1 = oracle.forward_particle(g, sig, plus=True, self_k=sk)
    dr, dp = oracle.channels(g, sig)
    corr_r = sig * sk[0] + g.r_centres[:, None] * dr * sk[1]
    corr_p = dp * sk[2]
    np.testing.assert_allclose(f1[0] - f0[0], corr_r, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(f1[1] - f0[1], corr_p, rtol=1e-12, atol=1e-15)
    # sampled destinations equal the full grid
    idx = np.array([0, 5, 17, 100, 191])
    fs = oracle.forward_particle(g, sig, plus=True, self_k=sk, dest=idx)
    np.testing.assert_allclose(fs[0], f1[0].ravel()[idx], rtol=1e-14)


def _errors(N, plus):
    g = oracle.Grid(N, N, 0.01, 1.0)
    sig = workloads.finite_disk(g.r_centres, g.phi_centres, n=5)
    fr, fp = oracle.forward_particle(g, sig, plus=plus)
    R, P = np.meshgrid(g.r_centres, g.phi_centres, indexing="ij")
    ar, ap = analytic.offcentre_forces(R, P, 5, 0.25, 0.5, 0.1)
    return np.array(oracle.error_norms(fr, ar) + oracle.error_norms(fp, ap))


def test_particle_methods_converge_at_first_order():
    # Table 1: particle and particle+ are first order on sigma_D5; the
    # correction lowers the error
    for plus in (False, True):
        e64, e128 = _errors(64, plus), _errors(128, plus)
        o = np.log2(e64 / e128)
        assert np.all(o > 0.6) and np.all(o < 1.6), (plus, o)
    assert np.all(_errors(64, True) < _errors(64, False))
