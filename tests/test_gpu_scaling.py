"""FP32 scaling per grid: the FP32 path scales each call's grid by a power of
two chosen from max|sigma| (pass A notes it, pass B scales its columns by
2^-e after the first stage of their transforms, pass C multiplies by 2^e and
clears the notes); within |e| <= 32 the scale is one.

At 512 x 1024 the column transforms sum L N_phi = 2^20 values, so a density
of 2^110 would reach 2^130 in them, beyond the FP32 range, without the
scale.  Power-of-two scaling commutes with every rounding of the path, so the
forces of 2^k sigma are 2^k times those of sigma bit for bit for k = +100
and +110 (pass A transforms the density as given, and at these scales none
of its values leaves the normal range); for k = -100 pass A's smallest
spectral components (below 2^-126, i.e. 2^-26 of the largest) reach the
subnormal range, so there the forces agree with 2^k times the unscaled ones
to far below the FP32 tolerance rather than bit for bit.  Every scale
matches the FP64 oracle (times 2^k) to the FP32 tolerance.  The same for the transpose
and for a disk inside a batch."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1509_01450_amd as pf  # noqa: E402

N_R, N_PHI, R_MIN, R_MAX = 512, 1024, 0.01, 100.0
KS = (-100, 100, 110)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pf.load()


@pytest.fixture(scope="module")
def case():
    g = oracle.Grid(N_R, N_PHI, R_MIN, R_MAX)
    sig = workloads.spiral_disk(g.r_centres, g.phi_centres)
    rng = workloads.rng(11, 0)
    dest = np.unique(np.concatenate([rng.integers(0, N_R * N_PHI, 256),
                                     rng.integers(0, N_PHI, 32),
                                     (N_R - 1) * N_PHI + rng.integers(0, N_PHI, 32)]))
    T = oracle.tables(g, 19)
    fr_o, fp_o = oracle.forward(g, T, sig, dest)
    vr = workloads.random_field(g.shape, 51)
    vp = workloads.random_field(g.shape, 52)
    src = np.unique(rng.integers(0, N_R * N_PHI, 128))
    ds_o = oracle.adjoint(g, T, vr, vp, src)
    return sig, dest, fr_o, fp_o, vr, vp, src, ds_o


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


FLT_MIN = float(np.finfo(np.float32).tiny)


def _bitwise_scaled(x, x1, f):
    """x == f x1 wherever f x1 is a normal FP32 number (exactly, in FP64 on
    the host, where f x1 is exact); where it is subnormal the stored value is
    its rounding, within half a subnormal step."""
    x = x.double().cpu().numpy()
    want = x1.double().cpu().numpy() * f
    normal = np.abs(want) >= FLT_MIN
    assert np.array_equal(x[normal], want[normal])
    assert np.all(np.abs(x[~normal] - want[~normal]) <= 2.0 ** -150)
    return int((~normal).sum())


def test_forward_scaled_densities(case):
    sig, dest, fr_o, fp_o = case[:4]
    plan = pf.Plan(N_R, N_PHI, R_MIN, R_MAX, dtype="f32")
    try:
        s = torch.tensor(sig, dtype=torch.float32, device="cuda")
        fr1, fp1 = plan.forces(s)
        torch.cuda.synchronize()
        fr1, fp1 = fr1.clone(), fp1.clone()
        for k in KS:
            f = 2.0 ** k
            fr, fp = plan.forces(s * f)
            torch.cuda.synchronize()
            assert torch.isfinite(fr).all() and torch.isfinite(fp).all(), k
            if k > 0:
                sub = _bitwise_scaled(fr, fr1, f) + _bitwise_scaled(fp, fp1, f)
            else:
                sub = -1
                for x, x1 in ((fr, fr1), (fp, fp1)):
                    want = x1.double().cpu().numpy() * f
                    got = x.double().cpu().numpy()
                    assert np.abs(got - want).max() <= 1e-7 * np.abs(want).max(), k
            a = fr.double().cpu().numpy().reshape(-1)[dest] / f
            b = fp.double().cpu().numpy().reshape(-1)[dest] / f
            e = (_rel(a, fr_o), _rel(b, fp_o))
            _say("sigma * 2^%d: 2^%d x the unscaled forces (%s); vs oracle rel-L2 F_r %.2e "
                 "F_phi %.2e" % (k, k, "bit for bit, %d subnormal outputs rounded" % sub
                                 if sub >= 0 else "to 1e-7 of the largest", e[0], e[1]))
            assert max(e) < 1e-5
    finally:
        plan.close()


def test_transpose_scaled_cotangents(case):
    vr, vp, src, ds_o = case[4:]
    plan = pf.Plan(N_R, N_PHI, R_MIN, R_MAX, dtype="f32")
    try:
        a = torch.tensor(vr, dtype=torch.float32, device="cuda")
        b = torch.tensor(vp, dtype=torch.float32, device="cuda")
        d1 = plan.backward(a, b).clone()
        torch.cuda.synchronize()
        for k in KS:
            f = 2.0 ** k
            d = plan.backward(a * f, b * f)
            torch.cuda.synchronize()
            assert torch.isfinite(d).all(), k
            if k > 0:
                _bitwise_scaled(d, d1, f)
            else:
                want = d1.double().cpu().numpy() * f
                got = d.double().cpu().numpy()
                assert np.abs(got - want).max() <= 1e-7 * np.abs(want).max(), k
            e = _rel(d.double().cpu().numpy().reshape(-1)[src] / f, ds_o)
            _say("cotangents * 2^%d: bit for bit; vs oracle transposed sums rel-L2 %.2e" % (k, e))
            assert e < 1e-5
    finally:
        plan.close()


def test_scaled_disk_in_a_batch():
    sizes = [(256, 512), (N_R, N_PHI), (100, 256)]
    plans, sig = [], []
    for d, (nr, nphi) in enumerate(sizes):
        p = pf.Plan(nr, nphi, R_MIN, R_MAX, dtype="f32")
        rc, _, _ = p.geometry()
        ph = (np.arange(nphi) + 0.5) * (2 * np.pi / nphi)
        plans.append(p)
        # one disk near 2^110, one near 2^-100, one unscaled
        f = (1.0, 2.0 ** 110, 2.0 ** -100)[d]
        sig.append(torch.tensor(workloads.multiarm_disk(rc, ph, d), dtype=torch.float32,
                                device="cuda") * f)
    outs = pf.forces_batched(plans, sig)
    torch.cuda.synchronize()
    for k, (p, s, (fr, fp)) in enumerate(zip(plans, sig, outs)):
        r, q = p.forces(s)
        torch.cuda.synchronize()
        assert torch.isfinite(fr).all() and torch.equal(fr, r) and torch.equal(fp, q), k
    for p in plans:
        p.close()


@pytest.mark.parametrize("cell", [(0, 5), (N_R // 2 + 3, 700), (N_R - 1, N_PHI - 1)])
def test_single_spike_sets_the_scale(case, cell):
    """A density of order one with one cell at 2^110: only the note of the
    wave holding that cell sees 2^110, so the scale is right only if the
    maximum over every note reaches pass B (else the column transforms
    overflow).  FP32 forces agree with the FP64 path on the whole grid."""
    sig = case[0].copy()
    sig[cell] = 2.0 ** 110
    p32 = pf.Plan(N_R, N_PHI, R_MIN, R_MAX, dtype="f32")
    p64 = pf.Plan(N_R, N_PHI, R_MIN, R_MAX, dtype="f64")
    try:
        fr, fp = p32.forces(torch.tensor(sig, dtype=torch.float32, device="cuda"))
        gr, gp = p64.forces(torch.tensor(sig, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert torch.isfinite(fr).all() and torch.isfinite(fp).all(), cell
        e = (_rel(fr.double().cpu().numpy(), gr.cpu().numpy()),
             _rel(fp.double().cpu().numpy(), gp.cpu().numpy()))
        _say("spike 2^110 at %s: FP32 vs FP64 rel-L2 F_r %.2e F_phi %.2e" % (cell, e[0], e[1]))
        assert max(e) < 1e-5
        # the transpose with one cotangent cell at 2^110
        a = np.zeros_like(sig)
        a[cell] = 2.0 ** 110
        b = case[5].copy()
        d32 = p32.backward(torch.tensor(a, dtype=torch.float32, device="cuda"),
                           torch.tensor(b, dtype=torch.float32, device="cuda"))
        d64 = p64.backward(torch.tensor(a, dtype=torch.float64, device="cuda"),
                           torch.tensor(b, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        assert torch.isfinite(d32).all(), cell
        e = _rel(d32.double().cpu().numpy(), d64.cpu().numpy())
        _say("cotangent spike 2^110 at %s: FP32 vs FP64 rel-L2 %.2e" % (cell, e))
        assert e < 1e-5
    finally:
        p32.close()
        p64.close()
