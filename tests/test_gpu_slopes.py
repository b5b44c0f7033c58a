"""GPU parity of the slope-order-4 path (five-point differences for the
slopes of Eq. 25: the spectra's symbols and the eight-row correction of the
column passes) against the FP64 oracle with the same slopes: forward map
and transpose, full grids from the smallest grid the order allows (n_r = 4,
where the boundary rows of both ends overlap) up to several tiles with a
ragged tail, FP64 at 1e-11 and FP32 at 1e-5 relative L2 per component, and
the C2-size grid on sampled cells.  Also: order 2 and order 4 differ by far
more than the tolerance on these inputs (a build that ignored the option
would fail), and batched calls refuse order-4 plans."""
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


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _t(x, plan):
    return torch.tensor(x, dtype=plan.torch_dtype, device="cuda")


SHAPES = [(4, 8, 0.5, 2.0), (5, 16, 0.1, 10.0), (9, 32, 0.2, 5.0), (37, 64, 0.01, 1.0),
          (100, 128, 0.01, 100.0)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dt,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_forward_order4_matches_oracle(shape, dt, tol):
    _say("order-4 forward", shape, dt)
    g = oracle.Grid(*shape)
    T = oracle.tables(g, 19)
    sig = workloads.random_field(g.shape, seed_k=41) + 2.0
    fr_o, fp_o = oracle.forward(g, T, sig, slope_order=4)
    plan = pf.Plan(*shape, dtype=dt, slope_order=4)
    try:
        fr, fp = plan.forces(_t(sig, plan))
        torch.cuda.synchronize()
        fr, fp = fr.double().cpu().numpy(), fp.double().cpu().numpy()
    finally:
        plan.close()
    e1, e2 = _rel_l2(fr, fr_o), _rel_l2(fp, fp_o)
    f2r, f2p = oracle.forward(g, T, sig)
    d = max(_rel_l2(f2r, fr_o), _rel_l2(f2p, fp_o))
    _say("  rel-L2 F_r %.3e F_phi %.3e (order 2 vs 4: %.2e)" % (e1, e2, d))
    assert e1 <= tol and e2 <= tol
    assert d > 100 * tol


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dt,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_transpose_order4_matches_oracle(shape, dt, tol):
    _say("order-4 transpose", shape, dt)
    g = oracle.Grid(*shape)
    T = oracle.tables(g, 19)
    vr = workloads.random_field(g.shape, 42)
    vp = workloads.random_field(g.shape, 43)
    want = oracle.adjoint(g, T, vr, vp, slope_order=4)
    plan = pf.Plan(*shape, dtype=dt, slope_order=4)
    try:
        got = plan.backward(_t(vr, plan), _t(vp, plan))
        torch.cuda.synchronize()
        got = got.double().cpu().numpy()
    finally:
        plan.close()
    e = _rel_l2(got, want)
    d = _rel_l2(oracle.adjoint(g, T, vr, vp), want)
    _say("  rel-L2 %.3e (order 2 vs 4: %.2e)" % (e, d))
    assert e <= tol
    assert d > 100 * tol


def test_particle_plus_order4_matches_oracle():
    # the modified particle method's self correction takes the same slopes
    shape = (37, 64, 0.01, 1.0)
    g = oracle.Grid(*shape)
    sig = workloads.single_disk_blobs(g.r_centres, g.phi_centres, 0.01, 1.0)
    fr_o, fp_o = oracle.forward_particle(g, sig, plus=True, slope_order=4)
    plan = pf.Plan(*shape, dtype="f64", method="particle+", slope_order=4)
    try:
        fr, fp = plan.forces(_t(sig, plan))
        torch.cuda.synchronize()
        e1 = _rel_l2(fr.cpu().numpy(), fr_o)
        e2 = _rel_l2(fp.cpu().numpy(), fp_o)
    finally:
        plan.close()
    _say("particle+ order 4 rel-L2 F_r %.3e F_phi %.3e" % (e1, e2))
    assert e1 <= 1e-11 and e2 <= 1e-11


def test_order4_c2_size_sampled():
    n_r, n_phi, a, b = 512, 1024, 0.01, 100.0
    g = oracle.Grid(n_r, n_phi, a, b)
    sig = workloads.spiral_disk(g.r_centres, g.phi_centres)
    rng = np.random.default_rng(61)
    idx = np.unique(np.concatenate([
        rng.choice(n_r * n_phi, 192, replace=False),
        np.arange(0, 4) * n_phi + 3, (n_r - 4 + np.arange(4)) * n_phi + 5]))
    T = oracle.tables(g, 19)
    fr_o, fp_o = oracle.forward(g, T, sig, dest=idx, slope_order=4)
    for dt, tol in (("f64", 1e-11), ("f32", 1e-5)):
        plan = pf.Plan(n_r, n_phi, a, b, dtype=dt, slope_order=4)
        try:
            fr, fp = plan.forces(_t(sig, plan))
            torch.cuda.synchronize()
            e1 = _rel_l2(fr.double().cpu().numpy().ravel()[idx], fr_o)
            e2 = _rel_l2(fp.double().cpu().numpy().ravel()[idx], fp_o)
        finally:
            plan.close()
        _say("order 4 512x1024 %s sampled rel-L2 F_r %.3e F_phi %.3e" % (dt, e1, e2))
        assert e1 <= tol and e2 <= tol


def test_batched_refuses_order4():
    p2 = pf.Plan(16, 32, 0.1, 10.0, dtype="f32")
    p4 = pf.Plan(16, 32, 0.1, 10.0, dtype="f32", slope_order=4)
    try:
        s = torch.ones(16, 32, device="cuda")
        with pytest.raises(pf.PFError, match="slope order"):
            pf.forces_batched([p2, p4], [s, s])
    finally:
        p2.close()
        p4.close()


def test_order4_fp32_grid_scale():
    # the five-point path runs under the same FP32 grid scale: 2^110 sigma
    # gives 2^110 times the forces bit for bit (normal outputs), forward and
    # transpose
    shape = (37, 64, 0.01, 1.0)
    g = oracle.Grid(*shape)
    sig = workloads.random_field(g.shape, seed_k=44) + 2.0
    plan = pf.Plan(*shape, dtype="f32", slope_order=4)
    try:
        s = _t(sig, plan)
        f = 2.0 ** 110
        fr1, fp1 = [x.clone() for x in plan.forces(s)]
        fr, fp = plan.forces(s * f)
        a = _t(workloads.random_field(g.shape, 45), plan)
        b = _t(workloads.random_field(g.shape, 46), plan)
        d1 = plan.backward(a, b).clone()
        d = plan.backward(a * f, b * f)
        torch.cuda.synchronize()
        for x, x1 in ((fr, fr1), (fp, fp1), (d, d1)):
            got = x.double().cpu().numpy()
            want = x1.double().cpu().numpy() * f
            assert np.isfinite(got).all()
            assert np.array_equal(got[want != 0], want[want != 0])
    finally:
        plan.close()
