"""GPU transpose (backward) through the C ABI: dot-product identity, the
oracle's transposed direct sum, central finite differences of the
force-matching loss, and the autograd wrapper."""
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


def _t(a, plan):
    return torch.tensor(a, dtype=plan.torch_dtype, device="cuda")


@pytest.mark.parametrize("shape", [(37, 64, 0.01, 1.0), (128, 128, 0.1, 10.0), (5, 8, 0.5, 2.0)])
def test_dot_product_identity_fp64(shape):
    plan = pf.Plan(*shape, dtype="f64")
    g = oracle.Grid(*shape)
    sig = _t(workloads.random_field(g.shape, 31), plan)
    vr = _t(workloads.random_field(g.shape, 32), plan)
    vp = _t(workloads.random_field(g.shape, 33), plan)
    fr, fp = plan.forces(sig)
    gs = plan.backward(vr, vp)
    lhs = float((fr * vr).sum() + (fp * vp).sum())
    rhs = float((sig * gs).sum())
    scale = float((fr * vr).abs().sum() + (fp * vp).abs().sum())
    _say(shape, "dot-product |lhs - rhs| / scale = %.3e" % (abs(lhs - rhs) / scale))
    assert abs(lhs - rhs) <= 1e-13 * scale


@pytest.mark.parametrize("shape,dtype,tol", [((37, 64, 0.01, 1.0), "f64", 1e-11),
                                             ((128, 128, 0.1, 10.0), "f64", 1e-11),
                                             ((128, 128, 0.1, 10.0), "f32", 1e-5)])
def test_backward_matches_oracle_transpose(shape, dtype, tol):
    g = oracle.Grid(*shape)
    T = oracle.tables(g, 19)
    vr = workloads.random_field(g.shape, 34)
    vp = workloads.random_field(g.shape, 35)
    want = oracle.adjoint(g, T, vr, vp)
    plan = pf.Plan(*shape, dtype=dtype)
    got = plan.backward(_t(vr, plan), _t(vp, plan)).double().cpu().numpy()
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    _say(shape, dtype, "backward rel-L2 %.3e max-abs %.3e" % (err, np.abs(got - want).max()))
    assert err <= tol


C5 = (1024, 2048, 0.01, 100.0)


@pytest.fixture(scope="module")
def c5_oracle():
    g = oracle.Grid(*C5)
    return g, oracle.tables(g, 19)


def _sample_cells(g, k):
    rng = np.random.default_rng(55)
    idx = rng.choice(g.n_r * g.n_phi, k, replace=False)
    edge = np.array([0, 7, g.n_phi + 3, (g.n_r - 2) * g.n_phi + 11, (g.n_r - 1) * g.n_phi + 5])
    return np.unique(np.concatenate([idx, edge]))


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_backward_full_size_sampled(c5_oracle, dtype, tol):
    """The adjoint kernel at 1024 x 2048 against the oracle's transposed
    direct sum, on seeded cotangents, at 32 random cells + boundary rows."""
    g, T = c5_oracle
    vr = workloads.random_field(g.shape, 36)
    vp = workloads.random_field(g.shape, 37)
    idx = _sample_cells(g, 32)
    want = oracle.adjoint(g, T, vr, vp, idx)
    plan = pf.Plan(*C5, dtype=dtype)
    got = plan.backward(_t(vr, plan), _t(vp, plan)).double().cpu().numpy().reshape(-1)[idx]
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    _say("C5", dtype, "backward vs oracle transpose rel-L2 %.3e max-abs %.3e"
         % (err, np.abs(got - want).max()))
    assert err <= tol


def test_force_matching_gradient_central_differences():
    """dL/dsigma of L = sum (F - F*)^2 at 1024 x 2048 in FP64 (F* the forces
    of a hidden density: exponential disk + 16 clumps) from the autograd
    wrapper, against central differences of L on 32 random cells; L is
    quadratic, so central differences are exact up to rounding."""
    plan = pf.Plan(*C5, dtype="f64")
    g = oracle.Grid(*C5)
    with torch.no_grad():
        Tr, Tp = plan.forces(_t(workloads.hidden_density(g.r_centres, g.phi_centres), plan))
    sig0 = workloads.start_density(g.r_centres, g.phi_centres)
    sig = _t(sig0, plan).requires_grad_(True)
    fr, fp = pf.forces(sig, plan)
    loss = ((fr - Tr) ** 2).sum() + ((fp - Tp) ** 2).sum()
    loss.backward()
    grad = sig.grad.cpu().numpy().reshape(-1)
    idx = _sample_cells(g, 32)
    eps = 1e-3
    s0 = _t(sig0, plan)
    fd = []
    with torch.no_grad():
        for p in idx:
            e = torch.zeros(g.n_r * g.n_phi, dtype=torch.float64, device="cuda")
            e[int(p)] = eps
            e = e.view(g.n_r, g.n_phi)
            lp = sum(float(((a - b) ** 2).sum()) for a, b in zip(plan.forces(s0 + e), (Tr, Tp)))
            lm = sum(float(((a - b) ** 2).sum()) for a, b in zip(plan.forces(s0 - e), (Tr, Tp)))
            fd.append((lp - lm) / (2 * eps))
    fd = np.array(fd)
    got = grad[idx]
    err = np.abs(fd - got).max() / np.abs(got).max()
    _say("C5 f64 gradient vs central differences max rel %.3e" % err)
    assert err <= 1e-6


def test_autograd_gradcheck_small():
    # the map is linear, so central differences carry no truncation error
    # whatever the step; a step of 1e-3 keeps their rounding (ulp(F) / step)
    # far below atol also for the Jacobian entries that vanish (with 1e-6 it
    # reached ~1e-9 on some draws of the input)
    plan = pf.Plan(6, 8, 0.5, 2.0, dtype="f64")
    gen = torch.Generator().manual_seed(1509)
    s = torch.randn(6, 8, dtype=torch.float64, generator=gen).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: pf.forces(x, plan), (s,), eps=1e-3, atol=1e-9)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_force_matching_recovers_the_hidden_density(dt):
    """The inverse problem the transpose serves: find sigma with
    A sigma = F* (the forces of a hidden density) by conjugate gradients on
    the normal equations (CGLS: one forward map and one transpose per
    iteration), from exp(-r/3) on a 48 x 64 grid.  In exact arithmetic the
    residual norm falls monotonically; after 60 steps it is below 1e-4 of
    its start in FP64 (1e-3 in FP32, where the recursion's rounding limits
    it; 3.7e-5 and 1.3e-4 measured) and the density error below 1e-2 of its
    start (3.6e-4 and 6.4e-4 measured)."""
    g = oracle.Grid(48, 64, 0.1, 10.0)
    plan = pf.Plan(48, 64, 0.1, 10.0, dtype=dt)
    try:
        hidden = _t(workloads.hidden_density(g.r_centres, g.phi_centres, 0.1, 10.0), plan)
        Tr, Tp = [x.clone() for x in plan.forces(hidden)]
        x = _t(workloads.start_density(g.r_centres, g.phi_centres), plan)
        fr, fp = plan.forces(x)
        rr, rp = Tr - fr, Tp - fp
        s = plan.backward(rr, rp)
        p = s.clone()
        gamma = float((s * s).sum())
        res0 = float(torch.sqrt((rr * rr).sum() + (rp * rp).sum()))
        err0 = float((x - hidden).norm())
        res = [res0]
        for _ in range(60):
            qr, qp = plan.forces(p)
            alpha = gamma / float((qr * qr).sum() + (qp * qp).sum())
            x = x + alpha * p
            rr, rp = rr - alpha * qr, rp - alpha * qp
            s = plan.backward(rr, rp)
            gn = float((s * s).sum())
            p = s + (gn / gamma) * p
            gamma = gn
            res.append(float(torch.sqrt((rr * rr).sum() + (rp * rp).sum())))
        torch.cuda.synchronize()
        err = float((x - hidden).norm())
    finally:
        plan.close()
    res = np.array(res)
    _say("%s CGLS residual %.3e -> %.3e after %d steps; density error %.3e -> %.3e"
         % (dt, res[0], res[-1], len(res) - 1, err0, err))
    f64 = dt == "f64"
    assert res[-1] < (1e-4 if f64 else 1e-3) * res[0]
    # monotone up to the rounding of the recursion
    assert np.all(np.diff(res) <= 1e-9 * res[0] + 1e-3 * res[:-1])
    assert err < 1e-2 * err0
