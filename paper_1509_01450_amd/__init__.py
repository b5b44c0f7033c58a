"""Python binding of libpf: log-polar thin-disk self-gravity on MI355X.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libpf.so`` behind the C ABI of ``include/pf.h``.  PyTorch is used
for device memory and streams.  The functions ``pf_*`` mirror the C entry
points one to one; :class:`Plan` and :func:`forces` are conveniences on top
(``forces`` is a ``torch.autograd.Function`` whose backward is the library's
transpose kernel).

Method: Wang, Yen & Taam, arXiv:1509.01450 -- second-order forces of an
infinitesimally thin disk on a log-polar grid (Sec. 3.2, Eq. 26-32, A18-A24)
with kernels from the singular integration method (Sec. 4, Eq. 41-46).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpf.so")

PF_OK, PF_EINVAL, PF_ESTATE, PF_ENOMEM, PF_EHIP, PF_ENODEV, PF_EUNSUPPORTED = range(7)
PF_F32, PF_F64 = 0, 1
PF_TABLE_SIM, PF_TABLE_EXACT = 0, 1
PF_SELF_CARTESIAN, PF_SELF_EXACT = 0, 1
PF_METHOD_SIM, PF_METHOD_PARTICLE, PF_METHOD_PARTICLE_PLUS = 0, 1, 2
_METHODS = {"sim": PF_METHOD_SIM, "particle": PF_METHOD_PARTICLE,
            "particle+": PF_METHOD_PARTICLE_PLUS}
_TABLE_MODES = {"sim": PF_TABLE_SIM, "exact": PF_TABLE_EXACT}
_SELF_MODES = {"cartesian": PF_SELF_CARTESIAN, "exact": PF_SELF_EXACT}
_STATUS = {1: "PF_EINVAL", 2: "PF_ESTATE", 3: "PF_ENOMEM", 4: "PF_EHIP", 5: "PF_ENODEV",
           6: "PF_EUNSUPPORTED"}

PF_CART_SECOND, PF_CART_PARTICLE, PF_CART_PARTICLE_PLUS = 0, 1, 2
_CART_METHODS = {"second": PF_CART_SECOND, "particle": PF_CART_PARTICLE,
                 "particle+": PF_CART_PARTICLE_PLUS}

EXPORTS = ("pf_build_opts_default", "pf_plan_create", "pf_kernels_build", "pf_forces",
           "pf_forces_backward", "pf_forces_batched", "pf_forces_batched_noalloc",
           "pf_forces_timed", "pf_plan_geometry",
           "pf_plan_schedule", "pf_plan_set_schedule", "pf_plan_selfcell", "pf_plan_tables",
           "pf_plan_destroy",
           "pf_last_error", "pf_version", "pf_plan_create_patches", "pf_forces_patches",
           "pf_forces_patches_backward", "pf_plan_set_src_col0",
           "pf_cart_create", "pf_cart_build", "pf_cart_forces",
           "pf_cart_forces_timed", "pf_cart_geometry", "pf_cart_destroy")


class PFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_STATUS.get(code, str(code)), msg))
        self.code = code


class pf_build_opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("n_tpz", ctypes.c_int),
                ("cover_per", ctypes.c_int), ("keep_tables", ctypes.c_int),
                ("table_mode", ctypes.c_int), ("self_mode", ctypes.c_int),
                ("method", ctypes.c_int), ("slope_order", ctypes.c_int)]


_lib = None


def build() -> str:
    """Compile libpf.so from csrc/ (hipcc, gfx950)."""
    from . import _build
    return _build.build()


def load():
    """Load libpf.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpf.so is not built (run paper_1509_01450_amd.build()); "
                          "there is no fallback implementation")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.pf_build_opts_default.argtypes = [ctypes.POINTER(pf_build_opts)]
    lib.pf_build_opts_default.restype = None
    lib.pf_plan_create.argtypes = [I, I, D, D]
    lib.pf_plan_create.restype = P
    lib.pf_kernels_build.argtypes = [P, ctypes.POINTER(pf_build_opts), P]
    lib.pf_forces.argtypes = [P, P, P, P, P]
    lib.pf_forces_backward.argtypes = [P, P, P, P, P]
    lib.pf_forces_batched.argtypes = [I, P, P, P, P, P]
    lib.pf_forces_batched_noalloc.argtypes = [I, P, P, P, P, P]
    lib.pf_forces_timed.argtypes = [P, I, P, P, P, P, I, P, P]
    lib.pf_plan_geometry.argtypes = [P, P, P, P]
    lib.pf_plan_selfcell.argtypes = [P, P]
    lib.pf_plan_schedule.argtypes = [P, P]
    lib.pf_plan_set_schedule.argtypes = [P, P]
    lib.pf_plan_tables.argtypes = [P, P]
    for f in ("pf_kernels_build", "pf_forces", "pf_forces_backward", "pf_forces_batched",
              "pf_forces_batched_noalloc",
              "pf_forces_timed",
              "pf_plan_geometry", "pf_plan_selfcell", "pf_plan_schedule", "pf_plan_set_schedule",
              "pf_plan_tables"):
        getattr(lib, f).restype = I
    lib.pf_plan_destroy.argtypes = [P]
    lib.pf_plan_destroy.restype = None
    lib.pf_plan_create_patches.argtypes = [I, I, I, I, D, D, I]
    lib.pf_plan_create_patches.restype = P
    lib.pf_forces_patches.argtypes = [P, P, P, P, P, P]
    lib.pf_forces_patches.restype = I
    lib.pf_forces_patches_backward.argtypes = [P, P, P, P, P, P]
    lib.pf_forces_patches_backward.restype = I
    lib.pf_plan_set_src_col0.argtypes = [P, I]
    lib.pf_plan_set_src_col0.restype = I
    lib.pf_cart_create.argtypes = [I, I, D, D]
    lib.pf_cart_create.restype = P
    lib.pf_cart_build.argtypes = [P, I, I, P]
    lib.pf_cart_forces.argtypes = [P, P, P, P, P]
    lib.pf_cart_forces_timed.argtypes = [P, P, P, P, I, P, P]
    lib.pf_cart_geometry.argtypes = [P, P]
    for f in ("pf_cart_build", "pf_cart_forces", "pf_cart_forces_timed", "pf_cart_geometry"):
        getattr(lib, f).restype = I
    lib.pf_cart_destroy.argtypes = [P]
    lib.pf_cart_destroy.restype = None
    lib.pf_last_error.argtypes = []
    lib.pf_last_error.restype = ctypes.c_char_p
    lib.pf_version.argtypes = []
    lib.pf_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def pf_last_error() -> str:
    return load().pf_last_error().decode()


def _check(rc):
    if rc != PF_OK:
        raise PFError(rc, pf_last_error())


# --------------------------------------------------------------------------
# one-to-one wrappers of the C entry points
# --------------------------------------------------------------------------
def pf_build_opts_default() -> pf_build_opts:
    o = pf_build_opts()
    load().pf_build_opts_default(ctypes.byref(o))
    return o


def pf_plan_create(n_r: int, n_phi: int, r_min: float, r_max: float) -> int:
    h = load().pf_plan_create(int(n_r), int(n_phi), float(r_min), float(r_max))
    if not h:
        raise PFError(PF_EINVAL, pf_last_error())
    return h


def pf_kernels_build(plan: int, opts: pf_build_opts | None = None, stream: int = 0) -> None:
    _check(load().pf_kernels_build(plan, ctypes.byref(opts) if opts is not None else None,
                                   stream or None))


def pf_forces(plan: int, sigma: int, f_r: int, f_phi: int, stream: int = 0) -> None:
    _check(load().pf_forces(plan, sigma, f_r, f_phi, stream or None))


def pf_forces_backward(plan: int, g_fr: int, g_fphi: int, g_sigma: int, stream: int = 0) -> None:
    _check(load().pf_forces_backward(plan, g_fr, g_fphi, g_sigma, stream or None))


def pf_forces_batched(plans, sigma, f_r, f_phi, stream: int = 0) -> None:
    n = len(plans)
    arr = lambda xs: (ctypes.c_void_p * n)(*xs)
    _check(load().pf_forces_batched(n, arr(plans), arr(sigma), arr(f_r), arr(f_phi),
                                    stream or None))


def pf_forces_batched_noalloc(plans, sigma, f_r, f_phi, stream: int = 0) -> None:
    n = len(plans)
    arr = lambda xs: (ctypes.c_void_p * n)(*xs)
    _check(load().pf_forces_batched_noalloc(n, arr(plans), arr(sigma), arr(f_r), arr(f_phi),
                                            stream or None))


def pf_forces_timed(plan: int, backward: bool, in0: int, in1: int, out0: int, out1: int,
                    reps: int = 1, stream: int = 0):
    """Run the forward map (or its transpose), each pass launched `reps`
    times back to back between events; returns the mean duration of one
    launch of each of the three passes in ms."""
    ms = (ctypes.c_float * 3)()
    _check(load().pf_forces_timed(plan, int(bool(backward)), in0, in1 or None, out0,
                                  out1 or None, int(reps), stream or None, ms))
    return [float(v) for v in ms]


def pf_plan_geometry(plan: int, n_r: int):
    rc = np.empty(n_r)
    re = np.empty(n_r + 1)
    dp = np.empty(1)
    _check(load().pf_plan_geometry(plan, rc.ctypes.data, re.ctypes.data, dp.ctypes.data))
    return rc, re, float(dp[0])


def pf_plan_selfcell(plan: int):
    out = np.empty(3)
    _check(load().pf_plan_selfcell(plan, out.ctypes.data))
    return out


def pf_plan_schedule(plan: int):
    """(one-channel row E, G, two-channel row E, G, column E, G, transpose
    column E, G) launch shapes of a built plan."""
    out = np.zeros(8, dtype=np.int32)
    _check(load().pf_plan_schedule(plan, out.ctypes.data))
    return tuple(int(v) for v in out)


def pf_plan_set_schedule(plan: int, shapes) -> None:
    """Set the eight launch-shape numbers (layout of pf_plan_schedule)."""
    a = np.ascontiguousarray(np.asarray(shapes, dtype=np.int32).reshape(8))
    _check(load().pf_plan_set_schedule(plan, a.ctypes.data))


def pf_plan_tables(plan: int, n_r: int, n_phi: int):
    out = np.empty((6, 2 * n_r - 1, n_phi))
    _check(load().pf_plan_tables(plan, out.ctypes.data))
    return out


def pf_plan_destroy(plan: int) -> None:
    load().pf_plan_destroy(plan)


def pf_plan_create_patches(n_src: int, src_row0: int, n_dst: int, n_phi: int, r_min: float,
                           r_max: float, wedges: bool = False) -> int:
    h = load().pf_plan_create_patches(int(n_src), int(src_row0), int(n_dst), int(n_phi),
                                      float(r_min), float(r_max), int(bool(wedges)))
    if not h:
        raise PFError(PF_EINVAL, pf_last_error())
    return h


def pf_forces_patches(plan: int, sigma_src: int, sigma_wedge: int, f_r: int, f_phi: int,
                      stream: int = 0) -> None:
    _check(load().pf_forces_patches(plan, sigma_src, sigma_wedge or None, f_r, f_phi,
                                    stream or None))


def pf_plan_set_src_col0(plan: int, src_col0: int) -> None:
    _check(load().pf_plan_set_src_col0(plan, int(src_col0)))


def pf_forces_patches_backward(plan: int, g_fr: int, g_fphi: int, g_sigma_src: int,
                               g_sigma_wedge: int, stream: int = 0) -> None:
    _check(load().pf_forces_patches_backward(plan, g_fr, g_fphi, g_sigma_src,
                                             g_sigma_wedge or None, stream or None))


def pf_cart_create(n_x: int, n_y: int, dx: float, dy: float) -> int:
    h = load().pf_cart_create(int(n_x), int(n_y), float(dx), float(dy))
    if not h:
        raise PFError(PF_EINVAL, pf_last_error())
    return h


def pf_cart_build(plan: int, dtype: int, method: int, stream: int = 0) -> None:
    _check(load().pf_cart_build(plan, int(dtype), int(method), stream or None))


def pf_cart_forces(plan: int, sigma: int, f_x: int, f_y: int, stream: int = 0) -> None:
    _check(load().pf_cart_forces(plan, sigma, f_x, f_y, stream or None))


def pf_cart_forces_timed(plan: int, sigma: int, f_x: int, f_y: int, reps: int = 1,
                         stream: int = 0):
    ms = (ctypes.c_float * 3)()
    _check(load().pf_cart_forces_timed(plan, sigma, f_x, f_y, int(reps), stream or None, ms))
    return [float(v) for v in ms]


def pf_cart_geometry(plan: int):
    """(N_x, N_y, L_x, L_y)."""
    out = np.zeros(4, dtype=np.int32)
    _check(load().pf_cart_geometry(plan, out.ctypes.data))
    return tuple(int(v) for v in out)


def pf_cart_destroy(plan: int) -> None:
    load().pf_cart_destroy(plan)


# --------------------------------------------------------------------------
# conveniences
# --------------------------------------------------------------------------
def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Plan:
    """A built n_r x n_phi log-polar grid on [r_min, r_max] (owns libpf state)."""

    def __init__(self, n_r, n_phi, r_min, r_max, dtype="f32", n_tpz=19, cover_per=10,
                 keep_tables=False, build=True, table_mode="sim", self_mode="cartesian",
                 method="sim", slope_order=2):
        self.n_r, self.n_phi = int(n_r), int(n_phi)
        self.r_min, self.r_max = float(r_min), float(r_max)
        self.handle = pf_plan_create(n_r, n_phi, r_min, r_max)
        self.dtype = None
        if build:
            self.build(dtype, n_tpz, cover_per, keep_tables, table_mode, self_mode, method,
                       slope_order)

    def build(self, dtype="f32", n_tpz=19, cover_per=10, keep_tables=False, table_mode="sim",
              self_mode="cartesian", method="sim", slope_order=2):
        """method "sim" (second order, SIM kernels), "particle" or "particle+"
        (Eq. 34-37); table_mode "sim" (n_tpz trapezoids, Eq. 41-43) or
        "exact"; self_mode "cartesian" (cover, Eq. 44-46) or "exact";
        slope_order 2 (central differences for the slopes of Eq. 25) or 4
        (five-point differences)."""
        o = pf_build_opts_default()
        o.dtype = PF_F64 if dtype in ("f64", "float64", PF_F64) else PF_F32
        o.n_tpz, o.cover_per, o.keep_tables = int(n_tpz), int(cover_per), int(bool(keep_tables))
        o.table_mode = _TABLE_MODES[table_mode]
        o.self_mode = _SELF_MODES[self_mode]
        o.method = _METHODS[method]
        o.slope_order = int(slope_order)
        pf_kernels_build(self.handle, o, _stream())
        self.dtype = "f64" if o.dtype == PF_F64 else "f32"
        return self

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.dtype == "f64" else torch.float32

    @property
    def shape(self):
        return (self.n_r, self.n_phi)

    def geometry(self):
        return pf_plan_geometry(self.handle, self.n_r)

    def selfcell(self):
        return pf_plan_selfcell(self.handle)

    def tables(self):
        return pf_plan_tables(self.handle, self.n_r, self.n_phi)

    def schedule(self):
        return pf_plan_schedule(self.handle)

    def set_schedule(self, shapes):
        pf_plan_set_schedule(self.handle, shapes)

    def _check_field(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA tensor" % name)
        if t.dtype != self.torch_dtype or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise TypeError("%s must be a contiguous %s tensor of shape %s"
                            % (name, self.torch_dtype, self.shape))

    def forces(self, sigma, out=None):
        import torch
        self._check_field(sigma, "sigma")
        if out is None:
            fr, fp = torch.empty_like(sigma), torch.empty_like(sigma)
        else:
            fr, fp = out
            self._check_field(fr, "out[0]")
            self._check_field(fp, "out[1]")
        pf_forces(self.handle, sigma.data_ptr(), fr.data_ptr(), fp.data_ptr(), _stream())
        return fr, fp

    def backward(self, g_fr, g_fphi, out=None):
        import torch
        self._check_field(g_fr, "g_fr")
        self._check_field(g_fphi, "g_fphi")
        gs = out if out is not None else torch.empty_like(g_fr)
        if out is not None:
            self._check_field(gs, "out")
        pf_forces_backward(self.handle, g_fr.data_ptr(), g_fphi.data_ptr(), gs.data_ptr(),
                           _stream())
        return gs

    def timed(self, a, b=None, backward=False, reps=1):
        """Mean duration (ms) of one launch of each pass of the forward map
        (a = sigma) or its transpose (a, b = g_fr, g_fphi), each pass
        launched `reps` times back to back."""
        import torch
        self._check_field(a, "a")
        if backward:
            self._check_field(b, "b")
            out = torch.empty_like(a)
            return pf_forces_timed(self.handle, True, a.data_ptr(), b.data_ptr(),
                                   out.data_ptr(), 0, reps, _stream())
        fr, fp = torch.empty_like(a), torch.empty_like(a)
        return pf_forces_timed(self.handle, False, a.data_ptr(), 0, fr.data_ptr(),
                               fp.data_ptr(), reps, _stream())

    def close(self):
        if getattr(self, "handle", None):
            pf_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def forces_batched(plans, sigmas, outs=None, noalloc=False):
    """Forward map of many disks (grouped launches covering every disk);
    noalloc: through pf_forces_batched_noalloc (tables in the library's static
    device array, at most 256 disks)."""
    import torch
    if len(plans) != len(sigmas) or (outs is not None and len(outs) != len(plans)):
        raise TypeError("one sigma (and one output pair) per plan")
    for p, s in zip(plans, sigmas):
        p._check_field(s, "sigma")
    if outs is None:
        outs = [(torch.empty_like(s), torch.empty_like(s)) for s in sigmas]
    else:
        for p, o in zip(plans, outs):
            p._check_field(o[0], "outs[k][0]")
            p._check_field(o[1], "outs[k][1]")
    fn = pf_forces_batched_noalloc if noalloc else pf_forces_batched
    fn([p.handle for p in plans], [s.data_ptr() for s in sigmas],
       [o[0].data_ptr() for o in outs], [o[1].data_ptr() for o in outs], _stream())
    return outs


def _make_function():
    import torch

    class _Forces(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sigma, plan):
            ctx.plan = plan
            return plan.forces(sigma.contiguous())

        @staticmethod
        def backward(ctx, g_fr, g_fphi):
            plan = ctx.plan
            z = None
            if g_fr is None:
                g_fr = torch.zeros(plan.shape, dtype=plan.torch_dtype, device=g_fphi.device)
            if g_fphi is None:
                g_fphi = torch.zeros(plan.shape, dtype=plan.torch_dtype, device=g_fr.device)
            return plan.backward(g_fr.contiguous(), g_fphi.contiguous()), z

    class _PatchForces(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sigma_src, sigma_wedge, plan):
            ctx.plan = plan
            w = sigma_wedge.contiguous() if sigma_wedge is not None else None
            return plan.forces(sigma_src.contiguous(), w)

        @staticmethod
        def backward(ctx, g_fr, g_fphi):
            plan = ctx.plan
            if g_fr is None:
                g_fr = torch.zeros(plan.shape, dtype=plan.torch_dtype, device=g_fphi.device)
            if g_fphi is None:
                g_fphi = torch.zeros(plan.shape, dtype=plan.torch_dtype, device=g_fr.device)
            g = plan.backward(g_fr.contiguous(), g_fphi.contiguous())
            if plan.wedges:
                return g[0], g[1], None
            return g, None, None

    return _Forces, _PatchForces


_FN = None


def forces(sigma, plan: Plan):
    """(F_r, F_phi) = A sigma, differentiable in sigma (backward = A^T)."""
    global _FN
    if _FN is None:
        _FN = _make_function()
    return _FN[0].apply(sigma, plan)


def patch_forces(sigma_src, plan, sigma_wedge=None):
    """(F_r, F_phi) on a patch plan's destination from its source patch (and
    wedge densities for plans with wedges), differentiable in both (backward
    = the patch transpose)."""
    global _FN
    if _FN is None:
        _FN = _make_function()
    return _FN[1].apply(sigma_src, sigma_wedge, plan)


class CartPlan:
    """A built N_x x N_y uniform Cartesian grid of cells dx by dy (Sec. 3.1):
    method "second" (Eq. 9-15), "particle" (Eq. 20) or "particle+"
    (Eq. 18-21)."""

    def __init__(self, n_x, n_y, dx, dy, dtype="f32", method="second", build=True):
        self.n_x, self.n_y = int(n_x), int(n_y)
        self.dx, self.dy = float(dx), float(dy)
        self.handle = pf_cart_create(n_x, n_y, dx, dy)
        self.dtype = None
        if build:
            self.build(dtype, method)

    def build(self, dtype="f32", method="second"):
        d = PF_F64 if dtype in ("f64", "float64", PF_F64) else PF_F32
        pf_cart_build(self.handle, d, _CART_METHODS[method], _stream())
        self.dtype = "f64" if d == PF_F64 else "f32"
        return self

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.dtype == "f64" else torch.float32

    @property
    def shape(self):
        return (self.n_x, self.n_y)

    def geometry(self):
        return pf_cart_geometry(self.handle)

    def _check_field(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA tensor" % name)
        if t.dtype != self.torch_dtype or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise TypeError("%s must be a contiguous %s tensor of shape %s"
                            % (name, self.torch_dtype, self.shape))

    def forces(self, sigma, out=None):
        import torch
        self._check_field(sigma, "sigma")
        if out is None:
            fx, fy = torch.empty_like(sigma), torch.empty_like(sigma)
        else:
            fx, fy = out
            self._check_field(fx, "out[0]")
            self._check_field(fy, "out[1]")
        pf_cart_forces(self.handle, sigma.data_ptr(), fx.data_ptr(), fy.data_ptr(), _stream())
        return fx, fy

    def timed(self, sigma, reps=1):
        import torch
        self._check_field(sigma, "sigma")
        fx, fy = torch.empty_like(sigma), torch.empty_like(sigma)
        return pf_cart_forces_timed(self.handle, sigma.data_ptr(), fx.data_ptr(), fy.data_ptr(),
                                    reps, _stream())

    def close(self):
        if getattr(self, "handle", None):
            pf_cart_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PatchPlan(Plan):
    """The force of a source patch (rows src_row0 .. src_row0 + n_src - 1 of
    the log-polar grid of the destination patch [r_min, r_max], n_dst rows)
    on the destination patch, optionally with the origin wedges below the
    source (Sec. 3.2.1, Eq. 27-29); src_col0 turns the source and its
    wedges by that many whole cells in phi (``set_src_col0`` changes it)."""

    def __init__(self, n_src, src_row0, n_dst, n_phi, r_min, r_max, wedges=False, dtype="f32",
                 n_tpz=19, cover_per=10, build=True, table_mode="sim", self_mode="cartesian",
                 method="sim", keep_tables=False, src_col0=0):
        self.n_r, self.n_phi = int(n_dst), int(n_phi)
        self.n_src, self.src_row0 = int(n_src), int(src_row0)
        self.r_min, self.r_max = float(r_min), float(r_max)
        self.wedges = bool(wedges)
        self.handle = pf_plan_create_patches(n_src, src_row0, n_dst, n_phi, r_min, r_max, wedges)
        self.set_src_col0(src_col0)
        self.dtype = None
        if build:
            self.build(dtype, n_tpz, cover_per, keep_tables, table_mode, self_mode, method)

    @property
    def src_shape(self):
        return (self.n_src, self.n_phi)

    def tables(self):
        out = np.empty((6, self.n_src + self.n_r - 1, self.n_phi))
        _check(load().pf_plan_tables(self.handle, out.ctypes.data))
        return out

    def forces(self, sigma_src, sigma_wedge=None, out=None):
        import torch
        if (not isinstance(sigma_src, torch.Tensor) or not sigma_src.is_cuda
                or sigma_src.dtype != self.torch_dtype or tuple(sigma_src.shape) != self.src_shape
                or not sigma_src.is_contiguous()):
            raise TypeError("sigma_src must be a contiguous %s CUDA tensor of shape %s"
                            % (self.torch_dtype, self.src_shape))
        if sigma_wedge is not None and (not isinstance(sigma_wedge, torch.Tensor)
                                        or tuple(sigma_wedge.shape) != (self.n_phi,)
                                        or sigma_wedge.dtype != self.torch_dtype
                                        or not sigma_wedge.is_cuda
                                        or not sigma_wedge.is_contiguous()):
            raise TypeError("sigma_wedge must be a contiguous %s CUDA tensor of shape (%d,)"
                            % (self.torch_dtype, self.n_phi))
        if out is None:
            out = (torch.empty(self.shape, dtype=self.torch_dtype, device=sigma_src.device),
                   torch.empty(self.shape, dtype=self.torch_dtype, device=sigma_src.device))
        fr, fp = out
        self._check_field(fr, "out[0]")   # destination grid: n_dst x n_phi
        self._check_field(fp, "out[1]")
        pf_forces_patches(self.handle, sigma_src.data_ptr(),
                          sigma_wedge.data_ptr() if sigma_wedge is not None else 0,
                          fr.data_ptr(), fp.data_ptr(), _stream())
        return fr, fp

    def set_src_col0(self, src_col0):
        """Turn the source (and wedges) by src_col0 whole cells in phi."""
        pf_plan_set_src_col0(self.handle, src_col0)
        self.src_col0 = int(src_col0)

    def backward(self, g_fr, g_fphi, out=None):
        """Transpose: cotangents on the destination patch [n_dst][n_phi] ->
        gradient on the source patch [n_src][n_phi]; plans with origin
        wedges return (g_src, g_wedge), g_wedge [n_phi] the gradient with
        respect to the wedge densities (out: that pair)."""
        import torch
        self._check_field(g_fr, "g_fr")
        self._check_field(g_fphi, "g_fphi")
        shapes = [self.src_shape] + ([(self.n_phi,)] if self.wedges else [])
        if out is None:
            outs = [torch.empty(sh, dtype=self.torch_dtype, device=g_fr.device) for sh in shapes]
        else:
            outs = list(out) if self.wedges else [out]
        if len(outs) != len(shapes):
            raise TypeError("out must be a pair (g_src, g_wedge) for plans with wedges")
        for o, sh in zip(outs, shapes):
            if (not isinstance(o, torch.Tensor) or not o.is_cuda or o.dtype != self.torch_dtype
                    or tuple(o.shape) != sh or not o.is_contiguous()):
                raise TypeError("out must be a contiguous %s CUDA tensor of shape %s"
                                % (self.torch_dtype, sh))
        pf_forces_patches_backward(self.handle, g_fr.data_ptr(), g_fphi.data_ptr(),
                                   outs[0].data_ptr(),
                                   outs[1].data_ptr() if self.wedges else 0, _stream())
        return tuple(outs) if self.wedges else outs[0]
