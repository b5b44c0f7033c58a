"""The largest plans (N_r = 4096, N_phi = 8192, L = 8192) and degenerate
inputs, against the oracle.

At the largest size the full oracle is out of reach, but the tables depend
only on the offsets, beta and dphi (Eq. 33): a density that is nonzero in one
cell (i0, j0) only acts on destination row i through the entries of the
offsets i - i0 + {-1, 0, 1} (the source and the cells whose slopes it
enters), so an 8-row oracle grid over the same physical rows (same radii,
same beta and dphi) gives the exact forces on those rows.  Rows further away
are checked against the far-field behaviour of a point source: the force
points at the source and falls like its mass over the distance squared."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1509_01450_amd as pf  # noqa: E402

N_R, N_PHI, R_MIN, R_MAX = 4096, 8192, 0.01, 100.0


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pf.load()


@pytest.mark.parametrize("dt,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_largest_plan_single_cell(dt, tol):
    i0, j0 = 2000, 100
    plan = pf.Plan(N_R, N_PHI, R_MIN, R_MAX, dtype=dt)
    try:
        sig = torch.zeros((N_R, N_PHI), dtype=plan.torch_dtype, device="cuda")
        sig[i0, j0] = 1.0
        fr, fp = plan.forces(sig)
        torch.cuda.synchronize()
        fr = fr.double().cpu().numpy()
        fp = fp.double().cpu().numpy()
        rc, re, dphi = plan.geometry()
    finally:
        plan.close()
    # the 8-row grid over rows i0 - 3 ... i0 + 4 of the large one
    lo = i0 - 3
    g = oracle.Grid(8, N_PHI, re[lo], re[lo + 8])
    assert abs(g.beta / (re[1] / re[0]) - 1) < 1e-13
    s = np.zeros(g.shape)
    s[3, j0] = 1.0
    T = oracle.tables(g, 19)
    ofr, ofp = oracle.forward(g, T, s)
    er = np.linalg.norm(fr[lo:lo + 8] - ofr) / np.linalg.norm(ofr)
    ep = np.linalg.norm(fp[lo:lo + 8] - ofp) / np.linalg.norm(ofp)
    _say("%d x %d %s single cell: near rows rel-L2 F_r %.2e F_phi %.2e" % (N_R, N_PHI, dt, er, ep))
    assert er < tol and ep < tol
    # far rows: the force of a point source of the cell's mass, to O((h/d)^2);
    # in FP32 the transforms' rounding is relative to the largest force of
    # the field, not to the small far values, hence the floor
    floor = 0.0 if dt == "f64" else 1e-6 * max(np.abs(fr).max(), np.abs(fp).max())
    mass = 0.5 * (re[i0 + 1] ** 2 - re[i0] ** 2) * dphi
    x0 = rc[i0] * np.cos((j0 + 0.5) * dphi)
    y0 = rc[i0] * np.sin((j0 + 0.5) * dphi)
    for i in (0, 500, 3500, N_R - 1):
        for j in (0, N_PHI // 3, N_PHI // 2 + 7):
            ph = (j + 0.5) * dphi
            dx, dy = x0 - rc[i] * np.cos(ph), y0 - rc[i] * np.sin(ph)
            d3 = np.hypot(dx, dy) ** 3
            ar = mass * (dx * np.cos(ph) + dy * np.sin(ph)) / d3
            ap = mass * (-dx * np.sin(ph) + dy * np.cos(ph)) / d3
            scale = mass / np.hypot(dx, dy) ** 2
            tol_ij = 1e-3 * scale + floor
            assert abs(fr[i, j] - ar) < tol_ij and abs(fp[i, j] - ap) < tol_ij, \
                (i, j, fr[i, j], ar, fp[i, j], ap)


def test_zero_density_gives_zero_forces():
    for dt in ("f32", "f64"):
        plan = pf.Plan(33, 64, 0.1, 10.0, dtype=dt)
        try:
            fr, fp = plan.forces(torch.zeros((33, 64), dtype=plan.torch_dtype, device="cuda"))
            torch.cuda.synchronize()
            assert float(fr.abs().max()) == 0.0 and float(fp.abs().max()) == 0.0
        finally:
            plan.close()
