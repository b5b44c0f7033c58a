"""pf_forces_batched_noalloc (the batched forward map with its tables in the
library's static device array) against pf_forces_batched, bit for bit, on two
calls in a row, the second with a smaller batch of smaller disks."""
import sys

import numpy as np
import pytest

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


def _disks(sizes, dtype="f32"):
    plans, sig = [], []
    for d, (nr, nphi) in enumerate(sizes):
        p = pf.Plan(nr, nphi, 0.01, 100.0, dtype=dtype)
        rc, _, _ = p.geometry()
        ph = (np.arange(nphi) + 0.5) * (2 * np.pi / nphi)
        plans.append(p)
        sig.append(torch.tensor(workloads.multiarm_disk(rc, ph, d + 7), dtype=p.torch_dtype,
                                device="cuda"))
    return plans, sig


def _call(fn, plans, sig):
    outs = [(torch.full_like(s, float("nan")), torch.full_like(s, float("nan"))) for s in sig]
    fn([p.handle for p in plans], [s.data_ptr() for s in sig],
       [o[0].data_ptr() for o in outs], [o[1].data_ptr() for o in outs],
       torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return outs


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_matches_batched_on_two_calls(dtype):
    big = [(256, 512), (384, 256), (512, 1024), (100, 128), (1024, 256)]
    small = [(64, 128), (40, 256)]
    for name, sizes in (("first call", big), ("second, smaller call", small)):
        plans, sig = _disks(sizes, dtype)
        _say("%s %s: %d disks %s" % (dtype, name, len(sizes), sizes))
        ref = _call(pf.pf_forces_batched, plans, sig)
        got = _call(pf.pf_forces_batched_noalloc, plans, sig)
        for k, ((a, b), (c, d)) in enumerate(zip(got, ref)):
            assert torch.equal(a, c) and torch.equal(b, d), (name, k, sizes[k])
            assert torch.isfinite(a).all() and torch.isfinite(b).all()
        for p in plans:
            p.close()


def test_noalloc_refuses_oversized_batches():
    lib = pf.load()
    assert lib.pf_forces_batched_noalloc(257, None, None, None, None, None) == pf.PF_EINVAL
    assert "256" in pf.pf_last_error()
