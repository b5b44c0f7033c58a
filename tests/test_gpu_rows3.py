"""GPU parity of grids whose azimuthal count is three or nine times a power
of two (N_phi = 2 Q P: the row transforms split into Q P-point transforms
and a radix-Q step, Q = 3 or 9) against the FP64 oracle: forward map and
transpose, full grids from the smallest such grids (N_phi = 24, 72) up to
several row tiles with a ragged radial count, the largest (N_phi = 6144,
4608) on sampled cells, the particle method, patch plans with wedges and
turns, the FP32 grid scale, and the batched path's size limits.  Bars:
relative L2 1e-11 (FP64) and 1e-5 (FP32) per component."""
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _t(x, plan):
    return torch.tensor(x, dtype=plan.torch_dtype, device="cuda")


SHAPES = [(4, 24, 0.5, 2.0), (9, 48, 0.2, 5.0), (37, 96, 0.01, 1.0), (20, 192, 0.1, 10.0),
          (5, 768, 0.3, 3.0), (4, 72, 0.5, 2.0), (21, 144, 0.05, 3.0), (6, 576, 0.2, 4.0)]
TRANSPOSE_SHAPES = [SHAPES[i] for i in (0, 1, 2, 3, 5, 6)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dt,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_forward_matches_oracle(shape, dt, tol):
    _say("3P forward", shape, dt)
    g = oracle.Grid(*shape)
    T = oracle.tables(g, 19)
    sig = workloads.random_field(g.shape, seed_k=71) + 2.0
    fr_o, fp_o = oracle.forward(g, T, sig)
    plan = pf.Plan(*shape, dtype=dt)
    try:
        fr, fp = plan.forces(_t(sig, plan))
        torch.cuda.synchronize()
        e1 = _rel(fr.double().cpu().numpy(), fr_o)
        e2 = _rel(fp.double().cpu().numpy(), fp_o)
    finally:
        plan.close()
    _say("  rel-L2 F_r %.3e F_phi %.3e" % (e1, e2))
    assert e1 <= tol and e2 <= tol


@pytest.mark.parametrize("shape", TRANSPOSE_SHAPES)
@pytest.mark.parametrize("dt,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_transpose_matches_oracle(shape, dt, tol):
    _say("3P transpose", shape, dt)
    g = oracle.Grid(*shape)
    T = oracle.tables(g, 19)
    vr = workloads.random_field(g.shape, 72)
    vp = workloads.random_field(g.shape, 73)
    want = oracle.adjoint(g, T, vr, vp)
    plan = pf.Plan(*shape, dtype=dt)
    try:
        got = plan.backward(_t(vr, plan), _t(vp, plan))
        torch.cuda.synchronize()
        e = _rel(got.double().cpu().numpy(), want)
    finally:
        plan.close()
    _say("  rel-L2 %.3e" % e)
    assert e <= tol


@pytest.mark.parametrize("n_r,n_phi", [(512, 1536), (24, 6144), (16, 4608)])
def test_large_sampled(n_r, n_phi):
    # the largest P (1024 with Q = 3, 256 with Q = 9) and a C2-like size, on
    # sampled cells incl. the first and last columns
    a, b = 0.01, 100.0
    g = oracle.Grid(n_r, n_phi, a, b)
    sig = workloads.spiral_disk(g.r_centres, g.phi_centres)
    rng = np.random.default_rng(74)
    idx = np.unique(np.concatenate([
        rng.choice(n_r * n_phi, 160, replace=False),
        np.array([0, n_phi - 1, n_phi // 3, (n_r - 1) * n_phi + n_phi // 2])]))
    T = oracle.tables(g, 19)
    fr_o, fp_o = oracle.forward(g, T, sig, dest=idx)
    for dt, tol in (("f64", 1e-11), ("f32", 1e-5)):
        plan = pf.Plan(n_r, n_phi, a, b, dtype=dt)
        try:
            fr, fp = plan.forces(_t(sig, plan))
            torch.cuda.synchronize()
            e1 = _rel(fr.double().cpu().numpy().ravel()[idx], fr_o)
            e2 = _rel(fp.double().cpu().numpy().ravel()[idx], fp_o)
        finally:
            plan.close()
        _say("3P %d x %d %s sampled rel-L2 F_r %.3e F_phi %.3e" % (n_r, n_phi, dt, e1, e2))
        assert e1 <= tol and e2 <= tol


@pytest.mark.parametrize("n_phi", [96, 144])
def test_particle_plus_matches_oracle(n_phi):
    shape = (37, n_phi, 0.01, 1.0)
    g = oracle.Grid(*shape)
    sig = workloads.single_disk_blobs(g.r_centres, g.phi_centres, 0.01, 1.0)
    fr_o, fp_o = oracle.forward_particle(g, sig, plus=True)
    for dt, tol in (("f64", 1e-11), ("f32", 1e-5)):
        plan = pf.Plan(*shape, dtype=dt, method="particle+")
        try:
            fr, fp = plan.forces(_t(sig, plan))
            torch.cuda.synchronize()
            e1 = _rel(fr.double().cpu().numpy(), fr_o)
            e2 = _rel(fp.double().cpu().numpy(), fp_o)
        finally:
            plan.close()
        _say("3P particle+ %s rel-L2 F_r %.3e F_phi %.3e" % (dt, e1, e2))
        assert e1 <= tol and e2 <= tol


@pytest.mark.parametrize("c0,n_phi", [(0, 48), (7, 48), (-11, 72)])
def test_patch_with_wedges_and_turn(c0, n_phi):
    n_src, s0, n_dst = 10, -10, 24
    g = oracle.Grid(n_dst, n_phi, 0.05, 2.0)
    T = oracle.patch_tables(g, n_src, s0, 19)
    Tw = oracle.wedge_tables(g, s0)
    sig = workloads.random_field((n_src, n_phi), 75) + 0.3
    sw = workloads.random_field((n_phi,), 76) + 0.5
    vr = workloads.random_field(g.shape, 77)
    vp = workloads.random_field(g.shape, 78)
    o_r, o_p = oracle.patch_forward(g, n_src, s0, T, sig, Tw, sw, col0=c0)
    ws, ww = oracle.patch_adjoint(g, n_src, s0, T, vr, vp, Tw=Tw, col0=c0)
    for dt, tol in (("f64", 1e-11), ("f32", 1e-5)):
        plan = pf.PatchPlan(n_src, s0, n_dst, n_phi, g.r_min, g.r_max, wedges=True, dtype=dt,
                            src_col0=c0)
        try:
            fr, fp = plan.forces(_t(sig, plan), _t(sw, plan))
            gs, gw = plan.backward(_t(vr, plan), _t(vp, plan))
            torch.cuda.synchronize()
            e = [_rel(fr.double().cpu().numpy(), o_r), _rel(fp.double().cpu().numpy(), o_p),
                 _rel(gs.double().cpu().numpy(), ws), _rel(gw.double().cpu().numpy(), ww)]
        finally:
            plan.close()
        _say("3P patch turn %d %s rel-L2 %s" % (c0, dt, " ".join("%.2e" % x for x in e)))
        assert max(e) <= tol


@pytest.mark.parametrize("n_phi", [96, 144])
def test_fp32_grid_scale(n_phi):
    # 2^110 and 2^-100 sigma: forces scaled bit for bit (normal outputs)
    shape = (37, n_phi, 0.01, 1.0)
    g = oracle.Grid(*shape)
    sig = workloads.random_field(g.shape, seed_k=79) + 2.0
    plan = pf.Plan(*shape, dtype="f32")
    try:
        s = _t(sig, plan)
        base = [x.clone() for x in plan.forces(s)]
        for f in (2.0 ** 110, 2.0 ** -100):
            got = plan.forces(s * f)
            torch.cuda.synchronize()
            for x, x1 in zip(got, base):
                a = x.double().cpu().numpy()
                want = x1.double().cpu().numpy() * f
                assert np.isfinite(a).all()
                assert np.array_equal(a[want != 0], want[want != 0]), f
    finally:
        plan.close()


def test_batched_refuses_other_counts():
    # the batched path takes the split rows too, within its row lengths:
    # n_phi = 48 (M = 24) is below them
    p = pf.Plan(64, 48, 0.1, 10.0, dtype="f32")
    try:
        s = torch.ones(64, 48, device="cuda")
        with pytest.raises(pf.PFError, match="batched path needs"):
            pf.forces_batched([p], [s])
    finally:
        p.close()


@pytest.mark.parametrize("n_phi", [96, 144])
def test_fp32_grid_scale_transpose(n_phi):
    # the transpose's scale words through the split rows: 2^110 and 2^-100
    # cotangents give the gradient times the same power bit for bit
    # (normal outputs)
    shape = (37, n_phi, 0.01, 1.0)
    g = oracle.Grid(*shape)
    plan = pf.Plan(*shape, dtype="f32")
    try:
        a = _t(workloads.random_field(g.shape, 81), plan)
        b = _t(workloads.random_field(g.shape, 82), plan)
        base = plan.backward(a, b).clone()
        for f in (2.0 ** 110, 2.0 ** -100):
            got = plan.backward(a * f, b * f)
            torch.cuda.synchronize()
            x = got.double().cpu().numpy()
            want = base.double().cpu().numpy() * f
            normal = np.abs(want) >= float(np.finfo(np.float32).tiny)
            assert np.isfinite(x).all(), f
            assert np.array_equal(x[normal], want[normal]), f
    finally:
        plan.close()


@pytest.mark.parametrize("n_phi", [96, 144])
def test_slope_order4_and_exact_tables(n_phi):
    # the split rows with five-point slopes, and with the exact table and
    # self-cell modes, against the oracle's sums of the same reading
    shape = (20, n_phi, 0.1, 10.0)
    g = oracle.Grid(*shape)
    sig = workloads.random_field(g.shape, seed_k=83) + 2.0
    T = oracle.tables(g, 19)
    fr_o, fp_o = oracle.forward(g, T, sig, slope_order=4)
    for dt, tol in (("f64", 1e-11), ("f32", 1e-5)):
        plan = pf.Plan(*shape, dtype=dt, slope_order=4)
        try:
            fr, fp = plan.forces(_t(sig, plan))
            torch.cuda.synchronize()
            e1 = _rel(fr.double().cpu().numpy(), fr_o)
            e2 = _rel(fp.double().cpu().numpy(), fp_o)
        finally:
            plan.close()
        _say("split rows, slope order 4, %s: rel-L2 %.2e %.2e" % (dt, e1, e2))
        assert e1 <= tol and e2 <= tol
    Te = oracle.tables(g, table_mode="exact", self_mode="exact")
    fr_o, fp_o = oracle.forward(g, Te, sig)
    plan = pf.Plan(*shape, dtype="f64", table_mode="exact", self_mode="exact")
    try:
        fr, fp = plan.forces(_t(sig, plan))
        torch.cuda.synchronize()
        e1 = _rel(fr.cpu().numpy(), fr_o)
        e2 = _rel(fp.cpu().numpy(), fp_o)
    finally:
        plan.close()
    _say("split rows, exact tables: rel-L2 %.2e %.2e" % (e1, e2))
    assert e1 <= 1e-11 and e2 <= 1e-11
