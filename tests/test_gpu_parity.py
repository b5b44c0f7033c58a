"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative L2 over every compared cell, per component): 1e-11 for
the FP64 path, 1e-5 for the FP32 path.  Kernel tables: the library's FP64
tables against the oracle's, entry by entry, within 1e-13 of the larger of
the table's largest entry and max |K^{r,0}| (the two sides evaluate the same
integrals by different quadratures -- graded Gauss-Legendre against closed
antiderivatives -- each exact to rounding on that scale).
"""
import functools
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1509_01450_amd as pf  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pf.load()


@functools.lru_cache(maxsize=8)
def _oracle_tables(n_r, n_phi, r_min, r_max, n_tpz=19, per=10):
    g = oracle.Grid(n_r, n_phi, r_min, r_max)
    return g, oracle.tables(g, n_tpz, per)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _run(plan, sigma):
    s = torch.tensor(sigma, dtype=plan.torch_dtype, device="cuda")
    fr, fp = plan.forces(s)
    torch.cuda.synchronize()
    return fr.double().cpu().numpy(), fp.double().cpu().numpy()


@pytest.mark.parametrize("shape", [(16, 32, 0.1, 10.0), (37, 64, 0.01, 1.0), (9, 8, 0.5, 2.0)])
def test_tables_match_oracle(shape):
    n_r, n_phi, a, b = shape
    _say("tables", shape)
    plan = pf.Plan(n_r, n_phi, a, b, dtype="f64", keep_tables=True)
    T = plan.tables()
    g, To = _oracle_tables(*shape)
    # both sides are accurate to rounding on the scale of the kernels'
    # antiderivatives, O(max |K^{r,0}|); K^{r,r}, K^{phi,r} carry an extra
    # (eta - beta^-m) = O(ln beta) factor and so sit below that scale
    base = np.abs(To[0]).max()
    for k in range(6):
        scale = max(np.abs(To[k]).max(), base)
        err = np.abs(T[k] - To[k]).max()
        _say("  table", oracle.TABLE_NAMES[k], "max|diff| / scale = %.3e" % (err / scale))
        assert err <= 1e-13 * scale, (k, err, scale)
    sk = plan.selfcell()
    ok = oracle.selfcell_cover(g.beta, g.dphi, 10)[:3]
    np.testing.assert_allclose(sk, ok, rtol=1e-12)


# (16, 8, 0.5, 2.0): the inner circle's tangent point from the cell centre
# lies on the cell's inner arc, so rho_max(t) of the self cell jumps
@pytest.mark.parametrize("shape", [(16, 32, 0.1, 10.0), (37, 64, 0.01, 1.0), (9, 8, 0.5, 2.0),
                                   (16, 8, 0.5, 2.0)])
def test_exact_modes_tables_match_oracle(shape):
    # converged azimuthal integrals and the exact self cell: two independent
    # quadratures (graded Gauss-Legendre panels against adaptive bisection)
    # of the same definitions
    n_r, n_phi, a, b = shape
    _say("exact-mode tables", shape)
    plan = pf.Plan(n_r, n_phi, a, b, dtype="f64", keep_tables=True, table_mode="exact",
                   self_mode="exact")
    T = plan.tables()
    g = oracle.Grid(*shape)
    To = oracle.tables(g, table_mode="exact", self_mode="exact")
    base = np.abs(To[0]).max()
    for k in range(6):
        scale = max(np.abs(To[k]).max(), base)
        err = np.abs(T[k] - To[k]).max()
        _say("  table", oracle.TABLE_NAMES[k], "max|diff| / scale = %.3e" % (err / scale))
        assert err <= 1e-13 * scale, (k, err, scale)
    # the self constants enter the tables on their O(1) scale; K^{r,0}_{00} is
    # a small difference of logarithms, so compare on that scale
    np.testing.assert_allclose(plan.selfcell(), oracle.selfcell_pv(g.beta, g.dphi), rtol=1e-13,
                               atol=1e-14)
    # the modes change the tables: SIM with the cover differs at O(1e-4)
    sim = pf.Plan(n_r, n_phi, a, b, dtype="f64", keep_tables=True).tables()
    assert np.abs(sim[0] - T[0]).max() > 1e-8 * base


@pytest.mark.parametrize("dt,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_exact_modes_forward_matches_oracle(dt, tol):
    shape = (37, 64, 0.01, 1.0)
    g = oracle.Grid(*shape)
    To = oracle.tables(g, table_mode="exact", self_mode="exact")
    sig = workloads.single_disk_blobs(g.r_centres, g.phi_centres)
    fr_o, fp_o = oracle.forward(g, To, sig)
    plan = pf.Plan(*shape, dtype=dt, table_mode="exact", self_mode="exact")
    fr, fp = _run(plan, sig)
    e1, e2 = _rel_l2(fr, fr_o), _rel_l2(fp, fp_o)
    _say("exact modes %s rel-L2 F_r %.3e F_phi %.3e" % (dt, e1, e2))
    assert e1 <= tol and e2 <= tol


@pytest.mark.parametrize("method", ["particle", "particle+"])
@pytest.mark.parametrize("dt,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_particle_methods_match_oracle(method, dt, tol):
    # the particle methods through the same passes, against the oracle's
    # point-mass double sums in physical coordinates (Eq. 34-37)
    shape = (37, 64, 0.01, 1.0)
    g = oracle.Grid(*shape)
    sig = workloads.single_disk_blobs(g.r_centres, g.phi_centres, 0.01, 1.0)
    fr_o, fp_o = oracle.forward_particle(g, sig, plus=(method == "particle+"))
    plan = pf.Plan(*shape, dtype=dt, method=method)
    fr, fp = _run(plan, sig)
    e1, e2 = _rel_l2(fr, fr_o), _rel_l2(fp, fp_o)
    _say("%s %s rel-L2 F_r %.3e F_phi %.3e" % (method, dt, e1, e2))
    assert e1 <= tol and e2 <= tol


def test_particle_plus_full_size_sampled():
    n_r, n_phi, a, b = C2
    g = oracle.Grid(n_r, n_phi, a, b)
    phi = g.phi_centres
    sig = workloads.spiral_disk(g.r_centres, phi)
    idx = np.random.default_rng(11).choice(n_r * n_phi, 256, replace=False)
    fr_o, fp_o = oracle.forward_particle(g, sig, plus=True, dest=idx)
    plan = pf.Plan(n_r, n_phi, a, b, dtype="f32", method="particle+")
    fr, fp = _run(plan, sig)
    e1 = _rel_l2(fr.ravel()[idx], fr_o)
    e2 = _rel_l2(fp.ravel()[idx], fp_o)
    _say("particle+ C2 f32 sampled rel-L2 F_r %.3e F_phi %.3e" % (e1, e2))
    assert e1 <= 1e-5 and e2 <= 1e-5


@pytest.mark.parametrize("shape", [(4, 8, 0.5, 2.0), (5, 16, 0.1, 10.0), (37, 16, 0.1, 10.0),
                                   (64, 8, 0.01, 1.0), (100, 128, 0.01, 100.0),
                                   (33, 256, 0.2, 5.0)])
def test_edge_sizes_fp64_full_grid(shape):
    _say("edge sizes", shape)
    g, T = _oracle_tables(*shape)
    sig = workloads.random_field(g.shape, seed_k=21) + 2.0
    fr_o, fp_o = oracle.forward(g, T, sig)
    plan = pf.Plan(*shape, dtype="f64")
    fr, fp = _run(plan, sig)
    er, ep = _rel_l2(fr, fr_o), _rel_l2(fp, fp_o)
    _say("  rel-L2 F_r %.3e  F_phi %.3e" % (er, ep))
    assert er <= 1e-11 and ep <= 1e-11


C1 = (128, 128, 0.1, 10.0)


@pytest.fixture(scope="module")
def c1_reference():
    g, T = _oracle_tables(*C1)
    sig = workloads.single_disk_blobs(g.r_centres, g.phi_centres)
    fr, fp = oracle.forward(g, T, sig)
    return g, sig, fr, fp


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_c1_full_grid(c1_reference, dtype, tol):
    g, sig, fr_o, fp_o = c1_reference
    plan = pf.Plan(*C1, dtype=dtype)
    fr, fp = _run(plan, sig)
    er, ep = _rel_l2(fr, fr_o), _rel_l2(fp, fp_o)
    _say("C1 %s rel-L2 F_r %.3e F_phi %.3e max-abs %.3e %.3e"
         % (dtype, er, ep, np.abs(fr - fr_o).max(), np.abs(fp - fp_o).max()))
    assert er <= tol and ep <= tol


C2 = (1024, 2048, 0.01, 100.0)


@pytest.fixture(scope="module")
def c2_reference():
    g, T = _oracle_tables(*C2)
    sig = workloads.spiral_disk(g.r_centres, g.phi_centres)
    rng = np.random.default_rng(5)
    idx = rng.choice(g.n_r * g.n_phi, 2048, replace=False)
    # all boundary rows' cells at a stride, plus random cells
    bnd = np.concatenate([np.arange(0, g.n_phi, 16), (g.n_r - 1) * g.n_phi + np.arange(0, g.n_phi, 16),
                          g.n_phi + np.arange(3, g.n_phi, 64), (g.n_r - 2) * g.n_phi + np.arange(5, g.n_phi, 64)])
    idx = np.unique(np.concatenate([idx, bnd]))
    fr, fp = oracle.forward(g, T, sig, idx)
    return g, sig, idx, fr, fp


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_c2_full_size_sampled(c2_reference, dtype, tol):
    g, sig, idx, fr_o, fp_o = c2_reference
    _say("C2", dtype, "cells", idx.size)
    plan = pf.Plan(*C2, dtype=dtype)
    fr, fp = _run(plan, sig)
    fr, fp = fr.reshape(-1)[idx], fp.reshape(-1)[idx]
    er, ep = _rel_l2(fr, fr_o), _rel_l2(fp, fp_o)
    _say("C2 %s rel-L2 F_r %.3e F_phi %.3e max-abs %.3e %.3e"
         % (dtype, er, ep, np.abs(fr - fr_o).max(), np.abs(fp - fp_o).max()))
    assert er <= tol and ep <= tol


def test_axisymmetric_has_zero_azimuthal_force_fp32():
    plan = pf.Plan(256, 256, 0.01, 100.0, dtype="f32")
    g = oracle.Grid(256, 256, 0.01, 100.0)
    sig = workloads.kuzmin(g.r_centres, g.phi_centres)
    fr, fp = _run(plan, sig)
    # odd-kernel k_phi = 0 spectra are exactly zero, so F_phi is pure
    # rounding noise of the FP32 transforms
    assert np.abs(fp).max() < 1e-5 * np.abs(fr).max()


def test_forces_are_deterministic():
    plan = pf.Plan(200, 256, 0.1, 10.0, dtype="f32")
    g = oracle.Grid(200, 256, 0.1, 10.0)
    s = torch.tensor(workloads.single_disk_blobs(g.r_centres, g.phi_centres), dtype=torch.float32,
                     device="cuda")
    a = plan.forces(s)
    b = plan.forces(s)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
