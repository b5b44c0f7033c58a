"""GPU batched path (grouped launches per class of transform length and
tuned launch shape, covering every disk) against the single-disk path -- bit
for bit: the same pass bodies at the same shapes -- and the FP64 oracle."""
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


def _disks(sizes, r_min=0.01, r_max=100.0, dtype="f32"):
    plans, sig = [], []
    for d, (nr, nphi) in enumerate(sizes):
        p = pf.Plan(nr, nphi, r_min, r_max, dtype=dtype)
        rc, _, _ = p.geometry()
        ph = (np.arange(nphi) + 0.5) * (2 * np.pi / nphi)
        plans.append(p)
        sig.append(torch.tensor(workloads.multiarm_disk(rc, ph, d), dtype=p.torch_dtype,
                                device="cuda"))
    return plans, sig


def _rel(a, b):
    return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))


def _check_against_single(plans, sig, outs, tol=1e-6):
    """Worst relative-L2 difference from the single-disk path; each disk must
    also equal it bit for bit."""
    worst = 0.0
    for k, (p, s, (fr, fp)) in enumerate(zip(plans, sig, outs)):
        r, q = p.forces(s)
        torch.cuda.synchronize()
        worst = max(worst, _rel(fr, r), _rel(fp, q))
        assert torch.equal(fr, r) and torch.equal(fp, q), (k, p.shape, _rel(fr, r), _rel(fp, q))
    return worst


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_three_and_nine_split_rows_in_a_batch(dtype):
    # disks with N_phi three or nine times a power of two (split row
    # transforms) batched with power-of-two disks: each equals its own plan
    # bit for bit, the split-row classes included, and the oracle on a
    # small one
    sizes = [(64, 192), (40, 256), (100, 144), (33, 1536), (70, 2304), (64, 128)]
    plans, sig = _disks(sizes, dtype=dtype)
    _say("split-row disks in a batch (%s)" % dtype)
    try:
        outs = pf.forces_batched(plans, sig)
        torch.cuda.synchronize()
        worst = _check_against_single(plans, sig, outs)
        _say("  vs single-disk worst rel-L2 %.3e" % worst)
        g = oracle.Grid(64, 192, 0.01, 100.0)
        T = oracle.tables(g, 19)
        fr_o, fp_o = oracle.forward(g, T, sig[0].double().cpu().numpy())
        fr, fp = outs[0]
        e1 = float(np.linalg.norm(fr.double().cpu().numpy() - fr_o) / np.linalg.norm(fr_o))
        e2 = float(np.linalg.norm(fp.double().cpu().numpy() - fp_o) / np.linalg.norm(fp_o))
        _say("  64 x 192 vs oracle rel-L2 %.3e %.3e" % (e1, e2))
        tol = 1e-11 if dtype == "f64" else 1e-5
        assert e1 <= tol and e2 <= tol
    finally:
        for p in plans:
            p.close()


def test_two_small_disks():
    plans, sig = _disks([(64, 128), (40, 256)])
    _say("two small disks: batched call")
    outs = pf.forces_batched(plans, sig)
    torch.cuda.synchronize()
    worst = _check_against_single(plans, sig, outs)
    _say("two small disks vs single-disk worst rel-L2 %.3e" % worst)
    assert worst <= 1e-6


def test_uneven_batch_matches_single_disk_and_oracle():
    # includes the extremes of the batched size range: n_phi = 128 and 4096,
    # n_r = 37 (L = 128) and 1500 (L = 4096)
    sizes = [(64, 128), (100, 256), (37, 512), (256, 128), (128, 1024), (200, 4096), (1024, 256),
             (1500, 128)]
    plans, sig = _disks(sizes)
    _say("plans built; batched call")
    outs = pf.forces_batched(plans, sig)
    torch.cuda.synchronize()
    worst = _check_against_single(plans, sig, outs)
    _say("uneven batch vs single-disk worst rel-L2 %.3e" % worst)
    assert worst <= 1e-6
    # oracle on two disks, every cell
    for k in (0, 2):
        nr, nphi = sizes[k]
        g = oracle.Grid(nr, nphi, 0.01, 100.0)
        T = oracle.tables(g, 19)
        fr_o, fp_o = oracle.forward(g, T, sig[k].double().cpu().numpy())
        fr = outs[k][0].double().cpu().numpy()
        fp = outs[k][1].double().cpu().numpy()
        er = np.linalg.norm(fr - fr_o) / np.linalg.norm(fr_o)
        ep = np.linalg.norm(fp - fp_o) / np.linalg.norm(fp_o)
        _say("disk %d %s vs oracle rel-L2 F_r %.3e F_phi %.3e" % (k, sizes[k], er, ep))
        assert er <= 1e-5 and ep <= 1e-5


def test_fp64_batch_matches_single_disk_and_oracle():
    # up to n_r = 1500 (L = 4096)
    sizes = [(64, 128), (37, 512), (300, 256), (1024, 128), (1500, 256)]
    plans, sig = _disks(sizes, dtype="f64")
    outs = pf.forces_batched(plans, sig)
    torch.cuda.synchronize()
    worst = _check_against_single(plans, sig, outs)
    _say("FP64 batch vs single-disk worst rel-L2 %.3e" % worst)
    assert worst <= 1e-13
    k = 1
    nr, nphi = sizes[k]
    g = oracle.Grid(nr, nphi, 0.01, 100.0)
    T = oracle.tables(g, 19)
    fr_o, fp_o = oracle.forward(g, T, sig[k].cpu().numpy())
    er = np.linalg.norm(outs[k][0].cpu().numpy() - fr_o) / np.linalg.norm(fr_o)
    ep = np.linalg.norm(outs[k][1].cpu().numpy() - fp_o) / np.linalg.norm(fp_o)
    _say("FP64 disk %d %s vs oracle rel-L2 F_r %.3e F_phi %.3e" % (k, sizes[k], er, ep))
    assert er <= 1e-11 and ep <= 1e-11


def test_replays_with_new_buffers():
    sizes = [(64, 256), (48, 128), (300, 512)]
    plans, sig = _disks(sizes)
    first = pf.forces_batched(plans, sig)
    # power-of-two scalings commute with every rounding of the path (no value
    # comes near the ends of the exponent range), so every call with fresh
    # input and output buffers reproduces the scaled first result bit for bit
    for f in (1.0, 2.0, 4.0, 0.25):
        sig2 = [s * f for s in sig]
        outs = pf.forces_batched(plans, sig2)
        torch.cuda.synchronize()
        for k, ((a, b), (c, d)) in enumerate(zip(outs, first)):
            assert torch.equal(a, c * f) and torch.equal(b, d * f), (f, k)


def test_graph_captured_batch_replays():
    # a repeat call with the buffers of the previous one only enqueues the
    # three launches, so it can be captured; replay several times with eager
    # work in between (the inputs are rescaled in place by powers of two,
    # exact in floating point) and check every replay against the eager
    # single-disk result of the same inputs
    sizes = [(64, 256), (48, 128), (300, 512)]
    plans, sig = _disks(sizes)
    outs = pf.forces_batched(plans, sig)        # uploads the descriptor table
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pf.forces_batched(plans, sig, outs)
    torch.cuda.synchronize()
    for rep, f in enumerate((1.0, 2.0, 0.5, 4.0)):
        for s in sig:
            s.mul_(f)
        g.replay()
        torch.cuda.synchronize()
        replayed = [(a.clone(), b.clone()) for a, b in outs]
        worst = _check_against_single(plans, sig, outs)
        _say("graph replay %d vs single-disk worst rel-L2 %.3e" % (rep, worst))
        assert worst <= 1e-6
        # the same batch called eagerly into fresh buffers: bit for bit the
        # replay's result (the same launches on the same inputs)
        eager = pf.forces_batched(plans, sig)
        torch.cuda.synchronize()
        for k, ((a, b), (c, d)) in enumerate(zip(replayed, eager)):
            assert torch.equal(a, c) and torch.equal(b, d), (rep, k)
        # the next replay writes to the buffers of the most recent call: give
        # the graph's buffers back to the batch before replaying again
        pf.forces_batched(plans, sig, outs)
        torch.cuda.synchronize()
    del g


def test_sixty_four_disk_batch():
    sizes = workloads.batch_sizes(64)
    plans, sig = _disks(sizes)
    outs = pf.forces_batched(plans, sig)
    torch.cuda.synchronize()
    worst = _check_against_single(plans, sig, outs)
    _say("64-disk batch (%d cells) vs single-disk worst rel-L2 %.3e"
         % (sum(a * b for a, b in sizes), worst))
    assert worst <= 1e-6
    # sampled oracle cells on one full-size disk of the batch
    k = int(np.argmax([a * b for a, b in sizes]))
    nr, nphi = sizes[k]
    g = oracle.Grid(nr, nphi, 0.01, 100.0)
    T = oracle.tables(g, 19)
    idx = np.random.default_rng(9).choice(nr * nphi, 512, replace=False)
    fr_o, fp_o = oracle.forward(g, T, sig[k].double().cpu().numpy(), idx)
    fr = outs[k][0].double().cpu().numpy().reshape(-1)[idx]
    fp = outs[k][1].double().cpu().numpy().reshape(-1)[idx]
    er = np.linalg.norm(fr - fr_o) / np.linalg.norm(fr_o)
    ep = np.linalg.norm(fp - fp_o) / np.linalg.norm(fp_o)
    _say("disk %d %s sampled vs oracle rel-L2 F_r %.3e F_phi %.3e" % (k, sizes[k], er, ep))
    assert er <= 1e-5 and ep <= 1e-5


def test_batch_argument_errors():
    p1 = pf.Plan(64, 128, 0.1, 10.0, dtype="f32")
    p2 = pf.Plan(64, 128, 0.1, 10.0, dtype="f64")
    s1 = torch.zeros(64, 128, device="cuda")
    s2 = torch.zeros(64, 128, dtype=torch.float64, device="cuda")
    lib = pf.load()
    with pytest.raises(pf.PFError) as ei:
        pf.pf_forces_batched([p1.handle, p2.handle], [s1.data_ptr(), s2.data_ptr()],
                             [s1.data_ptr(), s2.data_ptr()], [s1.data_ptr(), s2.data_ptr()])
    assert ei.value.code == pf.PF_EINVAL
    with pytest.raises(pf.PFError) as ei:
        pf.forces_batched([p1, p1], [s1, s1])
    assert ei.value.code == pf.PF_EINVAL
    p3 = pf.Plan(8, 64, 0.1, 10.0, dtype="f32")  # below the batched size range
    with pytest.raises(pf.PFError) as ei:
        pf.forces_batched([p3], [torch.zeros(8, 64, device="cuda")])
    assert ei.value.code == pf.PF_EUNSUPPORTED
    p4 = pf.Plan(2100, 128, 0.1, 10.0, dtype="f32")  # L = 8192: beyond the batch range
    with pytest.raises(pf.PFError) as ei:
        pf.forces_batched([p4], [torch.zeros(2100, 128, device="cuda")])
    assert ei.value.code == pf.PF_EUNSUPPORTED


def test_disks_of_one_size_with_different_shapes():
    """Two disks of one size, one at the tuned shapes and one at other valid
    shapes: they fall into different classes, and each still equals its
    single-disk result bit for bit."""
    plans, sig = _disks([(256, 512), (256, 512), (100, 256)])
    base = list(plans[0].schedule())
    # rows: other points per thread; columns (L = 512): 64-thread workgroups
    # of the other radix
    cols = [8, 1] if base[4] == 16 else [16, 2]
    other = [16 if base[0] != 16 else 8, 1, 4, 4] + cols + [base[6], base[7]]
    plans[1].set_schedule(other)
    assert list(plans[1].schedule()) == other
    outs = pf.forces_batched(plans, sig)
    torch.cuda.synchronize()
    worst = _check_against_single(plans, sig, outs)
    _say("mixed-shape batch vs single-disk worst rel-L2 %.3e" % worst)
