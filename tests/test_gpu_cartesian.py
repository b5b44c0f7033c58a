"""GPU parity and convergence of the Cartesian methods (Sec. 3.1, Eq. 6-21,
A1-A16): the HIP path through the C ABI against the FP64 oracle's direct
sums, element by element, and Fig. 3's orders on the analytic sigma_D2 disk.

* full-grid parity on ragged and non-power-of-two grids spanning several
  tiles, all three methods, FP64 (relative L2 <= 1e-11) and FP32 (<= 1e-5);
* sampled parity at 512 x 512, 1024 x 1024 and the largest grid,
  2048 x 2048 (every boundary row and column plus random cells), FP64 and
  FP32;
* the sigma_D2 disk (alpha = 0.25, centred in [-M, M]^2 with M = 0.5) for
  N = 64 ... 1024: fitted orders of the L1 error of F_r over the last four
  grids within 0.15 of Fig. 3 (2.0, 1.1, 1.0), and the ordering of the
  errors (second order < particle+ < particle).
"""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import analytic

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


def _gpu_forces(g, sig, dtype, method):
    plan = pf.CartPlan(g.n_x, g.n_y, g.dx, g.dy, dtype=dtype, method=method)
    try:
        s = torch.tensor(sig, dtype=plan.torch_dtype, device="cuda")
        fx, fy = plan.forces(s)
        torch.cuda.synchronize()
        return fx.double().cpu().numpy(), fy.double().cpu().numpy()
    finally:
        plan.close()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _density(g, seed):
    X, Y = g.centres()
    smooth = np.exp(-((X - 0.1) ** 2 + (Y + 0.2) ** 2) / 0.1)
    return smooth + 0.5 * workloads.random_field(g.shape, seed)


SHAPES = [(4, 4), (16, 16), (24, 10), (37, 100), (64, 48), (128, 128)]


@pytest.mark.parametrize("method", ["second", "particle", "particle+"])
@pytest.mark.parametrize("shape", SHAPES)
def test_full_grid_parity(shape, method):
    g = oracle.CartGrid(shape[0], shape[1], 1.0 / shape[0], 1.3 / shape[1], -0.5, -0.6)
    sig = _density(g, 11 + shape[0])
    _say("cartesian parity %s %s" % (shape, method))
    ox, oy = oracle.cart_forward(g, oracle.cart_tables(g, method), sig)
    for dt, tol in (("f64", 1e-11), ("f32", 1e-5)):
        fx, fy = _gpu_forces(g, sig, dt, method)
        rx, ry = _rel(fx, ox), _rel(fy, oy)
        _say("  %s rel-L2 F_x %.2e F_y %.2e" % (dt, rx, ry))
        assert rx < tol and ry < tol, (shape, method, dt, rx, ry)


@pytest.mark.parametrize("N", [512, 1024, 2048])
def test_sampled_parity_large(N):
    g = oracle.CartGrid.square(N, 0.5)
    sig = _density(g, 5)
    rng = workloads.rng(9, N)
    edges = np.concatenate([np.arange(N), (N - 1) * N + np.arange(N), np.arange(N) * N,
                            np.arange(N) * N + N - 1])
    dest = np.unique(np.concatenate([rng.integers(0, N * N, 1500), edges]))
    for method in ("second", "particle+"):
        ox, oy = oracle.cart_forward(g, oracle.cart_tables(g, method), sig, dest)
        for dt, tol in (("f64", 1e-11), ("f32", 1e-5)):
            fx, fy = _gpu_forces(g, sig, dt, method)
            rx, ry = _rel(fx.ravel()[dest], ox), _rel(fy.ravel()[dest], oy)
            _say("%d^2 %s %s sampled (%d cells) rel-L2 F_x %.2e F_y %.2e"
                 % (N, method, dt, dest.size, rx, ry))
            assert rx < tol and ry < tol


def _fig3(method):
    path = os.path.join(os.path.dirname(__file__), "golden", "fig3_cartesian_orders.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            m, o = line.split()
            if m == method:
                return float(o)
    raise KeyError(method)


def test_fig3_orders_sigma_d2():
    Ns = [64, 128, 256, 512, 1024]
    errs = {}
    for method in ("second", "particle+", "particle"):
        e = []
        for N in Ns:
            g = oracle.CartGrid.square(N, 0.5)
            X, Y = g.centres()
            R = np.hypot(X, Y)
            sig = analytic.sigma_dn(R, 2, 0.25)
            fx, fy = _gpu_forces(g, sig, "f64", method)
            fr = (fx * X + fy * Y) / R
            e.append(oracle.error_norms(fr, analytic.force_dn(R, 2, 0.25))[0])
        e = np.array(e)
        errs[method] = e
        x = np.log(np.array(Ns[1:], dtype=float))
        order = -np.polyfit(x, np.log(e[1:]), 1)[0]
        _say("%s L1_r %s  order (last four) %.2f  (Fig. 3: %.1f)"
             % (method, np.array2string(e, precision=3), order, _fig3(method)))
        assert abs(order - _fig3(method)) < 0.15, (method, order)
    assert np.all(errs["second"] < errs["particle+"]) and np.all(errs["particle+"] < errs["particle"])


FLT_MIN = float(np.finfo(np.float32).tiny)


@pytest.mark.parametrize("method", ["second", "particle+"])
@pytest.mark.parametrize("shape", [(37, 100), (128, 128), (512, 512)])
def test_fp32_grid_scale(shape, method):
    # the FP32 grid scale of the Cartesian passes: 2^110 sigma gives 2^110
    # times the forces bit for bit (no overflow), 2^-100 sigma 2^-100 times
    # them wherever that is a normal number (no flush of the small values),
    # and the scaled forces still match the oracle
    g = oracle.CartGrid(shape[0], shape[1], 1.0 / shape[0], 1.3 / shape[1], -0.5, -0.6)
    sig = _density(g, 21 + shape[0])
    plan = pf.CartPlan(g.n_x, g.n_y, g.dx, g.dy, dtype="f32", method=method)
    try:
        s = torch.tensor(sig, dtype=torch.float32, device="cuda")
        base = [x.clone() for x in plan.forces(s)]
        torch.cuda.synchronize()
        for f in (2.0 ** 110, 2.0 ** -100):
            got = plan.forces(s * f)
            torch.cuda.synchronize()
            for x, x1 in zip(got, base):
                a = x.double().cpu().numpy()
                want = x1.double().cpu().numpy() * f
                assert np.isfinite(a).all(), f
                normal = np.abs(want) >= FLT_MIN
                assert np.array_equal(a[normal], want[normal]), f
                assert np.all(np.abs(a[~normal] - want[~normal]) <= 2.0 ** -150), f
    finally:
        plan.close()
    if shape[0] <= 128:
        ox, oy = oracle.cart_forward(g, oracle.cart_tables(g, method), sig)
        fx, fy = [x.double().cpu().numpy() for x in base]
        _say("cartesian fp32 scale %s %s: rel-L2 F_x %.2e F_y %.2e" % (shape, method,
                                                                        _rel(fx, ox), _rel(fy, oy)))
        assert _rel(fx, ox) < 1e-5 and _rel(fy, oy) < 1e-5
