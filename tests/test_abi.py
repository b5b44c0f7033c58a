"""The C-ABI library: loads, exports every symbol include/pf.h declares, and
validates arguments on the host (no compute calls; no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1509_01450_amd as pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("pf_plan_create", "pf_kernels_build", "pf_forces", "pf_forces_backward",
              "pf_forces_batched", "pf_plan_destroy", "pf_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pf.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) == set(pf.EXPORTS)


@pytest.mark.parametrize("args", [(3, 64, 0.1, 10.0), (5000, 64, 0.1, 10.0), (16, 36, 0.1, 10.0),
                                  (16, 40, 0.1, 10.0), (16, 12, 0.1, 10.0), (16, 12288, 0.1, 10.0),
                                  (16, 54, 0.1, 10.0), (16, 9216, 0.1, 10.0), (16, 108, 0.1, 10.0),
                                  (16, 4, 0.1, 10.0), (16, 16384, 0.1, 10.0),
                                  (16, 64, 0.0, 10.0), (16, 64, 1.0, 1.0),
                                  (16, 64, float("nan"), 10.0), (16, 64, 0.1, float("inf"))])
def test_plan_create_rejects_bad_grids(args):
    with pytest.raises(pf.PFError) as ei:
        pf.pf_plan_create(*args)
    assert ei.value.code == pf.PF_EINVAL
    assert pf.pf_last_error()


@pytest.mark.parametrize("n_phi", [8, 24, 48, 72, 96, 144, 1536, 4608, 6144, 8192])
def test_plan_create_accepts_azimuthal_counts(n_phi):
    # powers of two, three and nine times powers of two
    h = pf.pf_plan_create(16, n_phi, 0.1, 10.0)
    try:
        rc, re_, dphi = pf.pf_plan_geometry(h, 16)
        assert abs(dphi - 2 * np.pi / n_phi) < 1e-15
    finally:
        pf.pf_plan_destroy(h)


def test_split_row_shapes_are_validated():
    # rows of n_phi = 2 Q P points take 4 or 8 points per thread (Q = 3; 8
    # only in FP32: the plan is unbuilt, so the FP32 default precision
    # applies) or 2 (Q = 9), at most P points; fitting shapes on an unbuilt
    # plan are a state error, the others invalid
    lib = pf.load()
    cols = (16, 1, 16, 1)   # L = 256 at n_r = 100: 16 threads per column -> G = 4 below
    for n_phi, good, bad in ((96, [(4, 4), (8, 8), (4, 64)], [(2, 8), (16, 2), (4, 256)]),
                             (144, [(2, 8), (2, 16)], [(4, 4), (8, 2), (16, 1)])):
        h = pf.pf_plan_create(100, n_phi, 0.1, 10.0)
        try:
            for E, G in good:
                arr = (ctypes.c_int * 8)(E, G, E, G, 16, 4, 16, 4)
                assert lib.pf_plan_set_schedule(h, arr) == pf.PF_ESTATE, (n_phi, E, G)
            for E, G in bad:
                arr = (ctypes.c_int * 8)(E, G, E, G, 16, 4, 16, 4)
                assert lib.pf_plan_set_schedule(h, arr) == pf.PF_EINVAL, (n_phi, E, G)
        finally:
            pf.pf_plan_destroy(h)


def test_plan_geometry_matches_grid_definition():
    h = pf.pf_plan_create(40, 64, 0.01, 100.0)
    try:
        rc, re_, dphi = pf.pf_plan_geometry(h, 40)
    finally:
        pf.pf_plan_destroy(h)
    g = oracle.Grid(40, 64, 0.01, 100.0)
    np.testing.assert_allclose(rc, g.r_centres, rtol=1e-14)
    np.testing.assert_allclose(re_, g.r_edges, rtol=1e-14)
    assert abs(dphi - g.dphi) < 1e-16


def test_unbuilt_plan_and_null_arguments_are_refused():
    lib = pf.load()
    h = pf.pf_plan_create(16, 32, 0.1, 10.0)
    try:
        # not built: refused before any device work
        assert lib.pf_forces(h, 8, 8, 8, None) == pf.PF_ESTATE
        assert lib.pf_forces_backward(h, 8, 8, 8, None) == pf.PF_ESTATE
        assert lib.pf_plan_selfcell(h, None) == pf.PF_EINVAL
        out8 = (ctypes.c_int * 8)()
        assert lib.pf_plan_schedule(h, out8) == pf.PF_ESTATE
        assert lib.pf_plan_schedule(h, None) == pf.PF_EINVAL
        # shapes are checked before the plan's state: zeros do not fit, a
        # fitting shape on an unbuilt plan is a state error
        assert lib.pf_plan_set_schedule(h, out8) == pf.PF_EINVAL
        ok8 = (ctypes.c_int * 8)(8, 2, 8, 2, 8, 1, 8, 1)    # L = 32: 4 threads per column
        assert lib.pf_plan_set_schedule(h, ok8) == pf.PF_EINVAL   # not a whole wave
        ok8 = (ctypes.c_int * 8)(8, 2, 8, 2, 8, 16, 8, 16)  # 64 threads
        assert lib.pf_plan_set_schedule(h, ok8) == pf.PF_ESTATE
        # whole waves but three columns per workgroup: the transpose's column
        # sums combine lanes at distances G, 2G, ... (G a power of two)
        h2 = pf.pf_plan_create(256, 32, 0.1, 10.0)   # L = 512: 64 threads per column at E = 8
        try:
            g3 = (ctypes.c_int * 8)(8, 2, 8, 2, 8, 3, 8, 3)
            assert lib.pf_plan_set_schedule(h2, g3) == pf.PF_EINVAL
            g4 = (ctypes.c_int * 8)(8, 2, 8, 2, 8, 4, 8, 4)
            assert lib.pf_plan_set_schedule(h2, g4) == pf.PF_ESTATE
        finally:
            pf.pf_plan_destroy(h2)
        assert lib.pf_plan_set_schedule(h, None) == pf.PF_EINVAL
        assert lib.pf_plan_set_schedule(None, out8) == pf.PF_EINVAL
        ms3 = (ctypes.c_float * 3)()
        assert lib.pf_forces_timed(h, 0, 8, None, 8, 8, 1, None, ms3) == pf.PF_ESTATE
        # null pointers
        assert lib.pf_forces(h, None, 8, 8, None) == pf.PF_EINVAL
        assert lib.pf_forces(None, 8, 8, 8, None) == pf.PF_EINVAL
        assert lib.pf_forces_batched(0, None, None, None, None, None) == pf.PF_EINVAL
        # the no-allocation form: 1 <= n <= 256, checked before the plans
        arr257 = (ctypes.c_void_p * 257)(*([8] * 257))
        hs257 = (ctypes.c_void_p * 257)(*([h] * 257))
        for n in (0, -1, 257):
            assert lib.pf_forces_batched_noalloc(n, hs257, arr257, arr257, arr257,
                                                 None) == pf.PF_EINVAL
        assert "256" in pf.pf_last_error() or "bad batch" in pf.pf_last_error()
        assert lib.pf_forces_batched_noalloc(1, None, None, None, None, None) == pf.PF_EINVAL
        # within bounds, an unbuilt plan is a state error
        assert lib.pf_forces_batched_noalloc(1, hs257, arr257, arr257, arr257,
                                             None) == pf.PF_ESTATE
        # bad build options are refused before the device is touched
        o = pf.pf_build_opts_default()
        o.n_tpz = 0
        assert lib.pf_kernels_build(h, ctypes.byref(o), None) == pf.PF_EINVAL
        o = pf.pf_build_opts_default()
        o.dtype = 7
        assert lib.pf_kernels_build(h, ctypes.byref(o), None) == pf.PF_EINVAL
        for field, bad in (("table_mode", 2), ("self_mode", 2), ("method", 3), ("method", -1),
                           ("slope_order", 3), ("slope_order", 0)):
            o = pf.pf_build_opts_default()
            setattr(o, field, bad)
            assert lib.pf_kernels_build(h, ctypes.byref(o), None) == pf.PF_EINVAL
        # n_tpz and cover_per are checked only where their mode uses them
        o = pf.pf_build_opts_default()
        o.n_tpz, o.table_mode = 0, pf.PF_TABLE_SIM
        assert lib.pf_kernels_build(h, ctypes.byref(o), None) == pf.PF_EINVAL
        o = pf.pf_build_opts_default()
        o.cover_per, o.self_mode = 0, pf.PF_SELF_CARTESIAN
        assert lib.pf_kernels_build(h, ctypes.byref(o), None) == pf.PF_EINVAL
    finally:
        pf.pf_plan_destroy(h)
    pf.pf_plan_destroy(None)


def _gpu_present():
    import torch
    return torch.cuda.device_count() > 0


@pytest.mark.skipif(_gpu_present(), reason="checks the library's answer when no GPU is present")
def test_no_device_is_reported():
    """Without a GPU the build calls return PF_ENODEV with a message, and the
    per-call entry points, which need a built plan, return PF_ESTATE."""
    lib = pf.load()
    h = pf.pf_plan_create(16, 32, 0.1, 10.0)
    try:
        o = pf.pf_build_opts_default()
        assert lib.pf_kernels_build(h, ctypes.byref(o), None) == pf.PF_ENODEV
        assert "no GPU" in pf.pf_last_error()
        assert lib.pf_forces(h, 8, 8, 8, None) == pf.PF_ESTATE
        assert lib.pf_forces_backward(h, 8, 8, 8, None) == pf.PF_ESTATE
        arr = (ctypes.c_void_p * 1)(8)
        hs = (ctypes.c_void_p * 1)(h)
        assert lib.pf_forces_batched(1, hs, arr, arr, arr, None) == pf.PF_ESTATE
    finally:
        pf.pf_plan_destroy(h)
    c = pf.pf_cart_create(8, 8, 0.1, 0.1)
    try:
        assert lib.pf_cart_build(c, pf.PF_F32, pf.PF_CART_SECOND, None) == pf.PF_ENODEV
        assert "no GPU" in pf.pf_last_error()
        assert lib.pf_cart_forces(c, 8, 8, 8, None) == pf.PF_ESTATE
    finally:
        pf.pf_cart_destroy(c)


def test_default_options():
    o = pf.pf_build_opts_default()
    assert (o.dtype, o.n_tpz, o.cover_per, o.keep_tables) == (pf.PF_F32, 19, 10, 0)
    # the paper's method by default (SIM tables, Cartesian cover of the self cell)
    assert (o.table_mode, o.self_mode) == (pf.PF_TABLE_SIM, pf.PF_SELF_CARTESIAN)
    assert o.method == pf.PF_METHOD_SIM
    assert (pf.PF_METHOD_PARTICLE, pf.PF_METHOD_PARTICLE_PLUS) == (1, 2)
    assert o.slope_order == 2


def test_cartesian_plan_host_checks():
    lib = pf.load()
    for args in [(3, 8, 0.1, 0.1), (8, 2049, 0.1, 0.1), (8, 8, 0.0, 0.1), (8, 8, 0.1, float("inf"))]:
        with pytest.raises(pf.PFError):
            pf.pf_cart_create(*args)
        assert pf.pf_last_error()
    h = pf.pf_cart_create(100, 37, 0.1, 0.2)
    try:
        # padded transform lengths: powers of two of at least twice the grid
        assert pf.pf_cart_geometry(h) == (100, 37, 256, 128)
        ms3 = (ctypes.c_float * 3)()
        assert lib.pf_cart_forces(h, 8, 8, 8, None) == pf.PF_ESTATE
        assert lib.pf_cart_forces_timed(h, 8, 8, 8, 1, None, ms3) == pf.PF_ESTATE
        assert lib.pf_cart_forces(h, None, 8, 8, None) == pf.PF_EINVAL
        assert lib.pf_cart_forces(None, 8, 8, 8, None) == pf.PF_EINVAL
        assert lib.pf_cart_forces_timed(h, 8, 8, 8, 0, None, ms3) == pf.PF_EINVAL
        assert lib.pf_cart_geometry(h, None) == pf.PF_EINVAL
        # bad options are refused before the device is touched
        assert lib.pf_cart_build(h, 7, pf.PF_CART_SECOND, None) == pf.PF_EINVAL
        assert lib.pf_cart_build(h, pf.PF_F32, 3, None) == pf.PF_EINVAL
        assert lib.pf_cart_build(None, pf.PF_F32, 0, None) == pf.PF_EINVAL
    finally:
        pf.pf_cart_destroy(h)
    pf.pf_cart_destroy(None)


def test_patch_plan_host_checks():
    lib = pf.load()
    for args in [(3, -3, 16, 32, 0.1, 1.0, 0), (8, 2, 16, 32, 0.1, 1.0, 1),
                 (8, -70000, 16, 32, 0.1, 1.0, 0), (8, -8, 16, 33, 0.1, 1.0, 0)]:
        with pytest.raises(pf.PFError):
            pf.pf_plan_create_patches(*args)
        assert pf.pf_last_error()
    h = pf.pf_plan_create_patches(10, -10, 16, 32, 0.1, 1.0, 1)
    try:
        rc, re_, dphi = pf.pf_plan_geometry(h, 16)
        assert abs(re_[0] - 0.1) < 1e-15 and abs(re_[-1] - 1.0) < 1e-12
        assert lib.pf_forces(h, 8, 8, 8, None) == pf.PF_ESTATE
        assert lib.pf_forces_patches(h, 8, 8, 8, 8, None) == pf.PF_ESTATE
        assert lib.pf_forces_patches(h, None, 8, 8, 8, None) == pf.PF_EINVAL
        # five-point slopes are not built for patch plans (refused before
        # the device is touched)
        o = pf.pf_build_opts_default()
        o.slope_order = 4
        assert lib.pf_kernels_build(h, ctypes.byref(o), None) == pf.PF_EUNSUPPORTED
        assert "slope order" in pf.pf_last_error()
        # the azimuthal turn: any integer on a patch plan, unbuilt too; the
        # transpose with wedges, unbuilt, is a state error
        for c in (0, 5, -37, 1 << 30):
            assert lib.pf_plan_set_src_col0(h, c) == pf.PF_OK
        assert lib.pf_forces_patches_backward(h, 8, 8, 8, 8, None) == pf.PF_ESTATE
    finally:
        pf.pf_plan_destroy(h)
    g = pf.pf_plan_create(16, 32, 0.1, 1.0)
    try:
        assert lib.pf_plan_set_src_col0(g, 3) == pf.PF_EINVAL
        assert "patch plan" in pf.pf_last_error()
    finally:
        pf.pf_plan_destroy(g)
    assert lib.pf_plan_set_src_col0(None, 3) == pf.PF_EINVAL


def test_dynamic_lds_arrays_are_aligned():
    """Every dynamic LDS array of the kernels is declared 16-byte aligned: a
    kernel that also holds static LDS (the FP32 grid scale's 4-byte slot)
    otherwise gets its dynamic array at byte 4, and every 8- and 16-byte LDS
    access of it is misaligned (a several-fold slower LDS pipe)."""
    import pathlib
    import re
    csrc = pathlib.Path(__file__).resolve().parents[1] / "paper_1509_01450_amd" / "csrc"
    decls = []
    for f in sorted(csrc.glob("*.hip")) + sorted(csrc.glob("*.hpp")):
        for line in f.read_text().splitlines():
            if re.search(r"\bextern\s+__shared__\b", line):
                decls.append((f.name, line.strip()))
    assert decls, "no dynamic LDS declarations found"
    bad = [d for d in decls if "__align__(16)" not in d[1]]
    assert not bad, bad
