"""Every column-pass launch shape against the oracle.

The autotuner keeps one shape per transform size, so the kernel variants it
does not pick -- points per thread E, columns per workgroup G, with the
radial spectrum prefetch in an LDS array of its own (the static-LDS kernels
for G = 1, 2, 4) or without it -- are run here through pf_plan_set_schedule:
forward and transpose, FP32 and FP64, on a grid with L = 2048 (columns of
128 or 256 threads) and on a small grid with L = 64 (columns of fewer than
64 threads), each compared with the FP64 oracle's direct sums (Eq. 27-29,
A19-A21, and their transpose) on sampled cells.  Tolerances as in the other
parity tests: relative L2 1e-5 (FP32), 1e-11 (FP64).  Shapes that do not fit
are refused with PF_EINVAL and leave the plan's shapes as they were.
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

TOL = {"f32": 1e-5, "f64": 1e-11}
GRIDS = {"L2048": (1024, 256, 0.01, 100.0), "L64": (32, 64, 0.1, 10.0)}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pf.load()


@functools.lru_cache(maxsize=4)
def _reference(name):
    """Oracle forward and transpose on sampled cells (all cells of the small
    grid), for a seeded spiral density and seeded cotangents."""
    g = oracle.Grid(*GRIDS[name])
    T = oracle.tables(g, 19)
    sig = workloads.spiral_disk(g.r_centres, g.phi_centres)
    vr = workloads.random_field(g.shape, 61)
    vp = workloads.random_field(g.shape, 62)
    n = g.n_r * g.n_phi
    if n <= 4096:
        idx = np.arange(n)
    else:
        rng = workloads.rng(63, 0)
        edge = np.concatenate([np.arange(0, g.n_phi, 7), (g.n_r - 1) * g.n_phi +
                               np.arange(0, g.n_phi, 9), g.n_phi + np.arange(2, g.n_phi, 31),
                               (g.n_r - 2) * g.n_phi + np.arange(4, g.n_phi, 29)])
        idx = np.unique(np.concatenate([rng.choice(n, 300, replace=False), edge]))
    fr, fp = oracle.forward(g, T, sig, idx)
    ds = oracle.adjoint(g, T, vr, vp, idx)
    return g, sig, vr, vp, idx, fr, fp, ds


def _column_shapes(L):
    """(E, G) candidates of the column passes: E in {8, 16}, 64 to 512
    threads per workgroup (the autotuner's set)."""
    out = []
    for E in (8, 16):
        th = L // E
        for thr in (64, 128, 256, 512):
            if th <= thr:
                out.append((E, thr // th))
    return out


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["L2048", "L64"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_every_column_shape_matches_oracle(name, dtype):
    g, sig, vr, vp, idx, fr_o, fp_o, ds_o = _reference(name)
    plan = pf.Plan(*GRIDS[name], dtype=dtype)
    try:
        base = list(plan.schedule())
        s = torch.tensor(sig, dtype=plan.torch_dtype, device="cuda")
        a = torch.tensor(vr, dtype=plan.torch_dtype, device="cuda")
        b = torch.tensor(vp, dtype=plan.torch_dtype, device="cuda")
        L = 1 << (2 * g.n_r - 1).bit_length()   # zero padding to L >= 2 n_r
        ran, current = [], base
        for E, G in _column_shapes(L):
            shapes = base[:4] + [E, G, E, G]
            try:
                plan.set_schedule(shapes)
            except pf.PFError as exc:
                assert exc.code == pf.PF_EINVAL
                assert list(plan.schedule()) == current
                _say("%s %s (E, G) = (%d, %d): refused (does not fit)" % (name, dtype, E, G))
                continue
            current = shapes
            assert list(plan.schedule()) == shapes
            fr, fp = plan.forces(s)
            ds = plan.backward(a, b)
            torch.cuda.synchronize()
            fr = fr.double().cpu().numpy().reshape(-1)[idx]
            fp = fp.double().cpu().numpy().reshape(-1)[idx]
            ds = ds.double().cpu().numpy().reshape(-1)[idx]
            e = (_rel(fr, fr_o), _rel(fp, fp_o), _rel(ds, ds_o))
            _say("%s %s (E, G) = (%d, %d): rel-L2 F_r %.2e F_phi %.2e dsigma %.2e (%d cells)"
                 % (name, dtype, E, G, e[0], e[1], e[2], idx.size))
            assert max(e) <= TOL[dtype], (E, G, e)
            ran.append((E, G))
        # the static-LDS prefetch kernels of every G the dispatch has
        if name == "L2048" and dtype == "f32":
            assert {(16, 1), (16, 2), (16, 4), (8, 1), (8, 2)} <= set(ran)
        assert ran
    finally:
        plan.close()


def test_bad_shapes_are_refused_and_keep_the_schedule():
    plan = pf.Plan(64, 128, 0.1, 10.0, dtype="f32")
    try:
        base = list(plan.schedule())
        for bad in (base[:4] + [32, 1, 8, 1],          # points per thread not 8 or 16
                    base[:4] + [8, 64, 8, 1],          # more than 512 threads
                    [3, 1] + base[2:],                 # row points per thread
                    base[:4] + [16, 0, 16, 1],         # no columns per workgroup
                    base[:4] + [8, 3, 8, 3],           # columns per workgroup not a power of two
                    base[:4] + [16, 1, 16, 1]):        # L = 128, 8 threads: not a whole wave
            with pytest.raises(pf.PFError) as exc:
                plan.set_schedule(bad)
            assert exc.value.code == pf.PF_EINVAL
            assert list(plan.schedule()) == base
    finally:
        plan.close()


def test_out_tensors_are_checked_before_any_launch():
    plan = pf.Plan(32, 64, 0.1, 10.0, dtype="f32")
    try:
        s = torch.zeros(32, 64, device="cuda")
        good = torch.empty_like(s)
        bad = [torch.empty(32, 32, device="cuda"),                        # too small
               torch.empty(32, 64, dtype=torch.float64, device="cuda"),   # wrong dtype
               torch.empty(64, 32, device="cuda").t(),                     # not contiguous
               torch.empty(32, 64)]                                        # host memory
        for b in bad:
            with pytest.raises(TypeError):
                plan.forces(s, out=(good, b))
            with pytest.raises(TypeError):
                plan.forces(s, out=(b, good))
            with pytest.raises(TypeError):
                plan.backward(s, s, out=b)
            with pytest.raises(TypeError):
                pf.forces_batched([plan], [s], outs=[(good, b)])
        fr, fp = plan.forces(s, out=(good, torch.empty_like(s)))
        torch.cuda.synchronize()
        assert fr.data_ptr() == good.data_ptr()
    finally:
        plan.close()
