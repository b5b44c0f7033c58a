"""FP64 CPU oracle for the log-polar thin-disk self-gravity method.

TEST INFRASTRUCTURE ONLY.  This package is the independent checker of the HIP
library: only the test suite, ``__graft_entry__.smoke()`` and the CPU baseline
leg of ``bench.py`` may import it.  It shares no code with the library and the
library never imports it.

The arithmetic lives in ``pf_oracle.c`` (plain C + OpenMP, FP64); this module
only builds and loads it and marshals numpy arrays.  Each wrapper names the
paper passage that the C function follows (Wang, Yen & Taam,
arXiv:1509.01450).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TABLE_NAMES = ("r0", "rr", "rphi", "phi0", "phir", "phiphi")


def build(force: bool = True) -> str:
    """Compile ``pf_oracle.c`` into ``liboracle.so`` (gcc, -O2, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    d, i, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
    P = ctypes.c_void_p
    lib.or_geometry.argtypes = [i, i, d, d, P, P, P, P]
    lib.or_gauss_legendre.argtypes = [i, P, P]
    lib.or_selfcell_cover.argtypes = [d, d, i, P, P]
    lib.or_selfcell_pv.argtypes = [d, d, P]
    lib.or_table_entry.argtypes = [i, i, d, d, i, i, i, i, P, P]
    lib.or_tables.argtypes = [i, i, d, d, i, i, P, P]
    lib.or_channels.argtypes = [i, i, P, d, P, P, P]
    lib.or_channels_o.argtypes = [i, i, P, d, i, P, P, P]
    lib.or_forward.argtypes = [i, i, d, d, P, P, P, i64, P, P]
    lib.or_forward_o.argtypes = [i, i, d, d, i, P, P, P, i64, P, P]
    lib.or_adjoint.argtypes = [i, i, d, d, P, P, P, P, i64, P]
    lib.or_adjoint_o.argtypes = [i, i, d, d, i, P, P, P, P, i64, P]
    lib.or_forward_particle.argtypes = [i, i, d, d, i, P, P, P, i64, P, P]
    lib.or_forward_particle_o.argtypes = [i, i, d, d, i, i, P, P, P, i64, P, P]
    lib.or_patch_tables.argtypes = [i, i, i, i, d, d, i, i, P, P]
    lib.or_wedge_tables.argtypes = [i, i, d, d, i, i, P]
    lib.or_patch_forward.argtypes = [i, i, i, i, i, d, d, P, P, P, P, P, i64, P, P]
    lib.or_patch_adjoint.argtypes = [i, i, i, i, i, d, d, P, P, P, P, i64, P, P, P]
    lib.or_patch_particle.argtypes = [i, i, i, i, i, d, d, i, P, P, P, P, i64, P, P]
    lib.or_cart_tables.argtypes = [i, i, d, d, i, P]
    lib.or_cart_slopes.argtypes = [i, i, d, d, P, P, P]
    lib.or_cart_forward.argtypes = [i, i, d, d, P, P, P, i64, P, P]
    for f in ("or_geometry", "or_gauss_legendre", "or_selfcell_cover", "or_selfcell_pv",
              "or_table_entry", "or_tables", "or_channels", "or_forward",
              "or_adjoint", "or_forward_particle", "or_channels_o", "or_forward_o",
              "or_adjoint_o", "or_forward_particle_o", "or_patch_tables", "or_wedge_tables",
              "or_patch_forward", "or_patch_adjoint", "or_patch_particle", "or_cart_tables", "or_cart_slopes",
              "or_cart_forward", "or_num_threads"):
        getattr(lib, f).restype = i
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().or_num_threads())


def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes and weights on [-1, 1]."""
    x = np.empty(n)
    w = np.empty(n)
    if _load().or_gauss_legendre(n, _p(x), _p(w)):
        raise ValueError("n out of range")
    return x, w


class Grid:
    """Log-polar grid of Sec. 3.2.1 generalised to N_r x N_phi."""

    def __init__(self, n_r: int, n_phi: int, r_min: float, r_max: float):
        self.n_r, self.n_phi = int(n_r), int(n_phi)
        self.r_min, self.r_max = float(r_min), float(r_max)
        rc = np.empty(self.n_r)
        re = np.empty(self.n_r + 1)
        b = np.empty(1)
        dp = np.empty(1)
        if _load().or_geometry(self.n_r, self.n_phi, self.r_min, self.r_max,
                               _p(rc), _p(re), _p(b), _p(dp)):
            raise ValueError("bad grid")
        self.r_centres, self.r_edges = rc, re
        self.beta, self.dphi = float(b[0]), float(dp[0])
        self.phi_centres = (np.arange(self.n_phi) + 0.5) * self.dphi

    @property
    def shape(self):
        return (self.n_r, self.n_phi)

    def cell_areas(self):
        """Exact polar cell areas (r_out^2 - r_in^2) dphi / 2."""
        re = self.r_edges
        a = 0.5 * (re[1:] ** 2 - re[:-1] ** 2) * self.dphi
        return np.repeat(a[:, None], self.n_phi, axis=1)

    def xy(self):
        r = self.r_centres[:, None]
        p = self.phi_centres[None, :]
        return r * np.cos(p), r * np.sin(p)


def selfcell_cover(beta: float, dphi: float, per: int = 10):
    """Self-cell kernels by the Cartesian cover (Sec. 4, Eq. 44-46).

    Returns (K^{r,0}_{00}, K^{r,r}_{00}, K^{phi,phi}_{00}, n_cells)."""
    out = np.empty(3)
    n = np.zeros(1, dtype=np.int64)
    if _load().or_selfcell_cover(float(beta), float(dphi), int(per), _p(out), _p(n)):
        raise ValueError("bad cover arguments")
    return float(out[0]), float(out[1]), float(out[2]), int(n[0])


def selfcell_pv(beta: float, dphi: float):
    """Self-cell kernels as the exact integrals (principal value for
    K^{r,0}) in local polar coordinates about the cell centre.

    Returns (K^{r,0}_{00}, K^{r,r}_{00}, K^{phi,phi}_{00})."""
    out = np.empty(3)
    if _load().or_selfcell_pv(float(beta), float(dphi), _p(out)):
        raise ValueError("bad self-cell arguments")
    return float(out[0]), float(out[1]), float(out[2])


_TABLE_MODES = {"sim": 0, "exact": 1}


def table_entry(grid: Grid, m: int, n_rep: int, n_tpz: int = 19, self_k=None,
                table_mode: str = "sim"):
    """All six kernels for offset (m, n_rep) (Eq. 30-32, 41-43, A22-A24).

    table_mode "sim": n_tpz trapezoids in the azimuth (Eq. 41-43); "exact":
    the same azimuthal integrals converged.  ``self_k`` supplies the three
    self-cell constants used at (0, 0)."""
    sk = _f64(self_k if self_k is not None else np.zeros(3))
    t = np.empty(6)
    if _load().or_table_entry(grid.n_r, grid.n_phi, grid.r_min, grid.r_max,
                              int(n_tpz), _TABLE_MODES[table_mode], int(m), int(n_rep),
                              _p(sk), _p(t)):
        raise ValueError("bad arguments")
    return t


def tables(grid: Grid, n_tpz: int = 19, cover_per: int = 10, self_k=None,
           table_mode: str = "sim", self_mode: str = "cartesian"):
    """Six kernel tables, shape (6, 2 N_r - 1, N_phi); row m + N_r - 1,
    column n = (j - j') mod N_phi; order r0, rr, rphi, phi0, phir, phiphi.

    table_mode "sim" (the paper's trapezoids, Eq. 41-43) or "exact"
    (converged azimuthal integrals).  The self cell comes from
    :func:`selfcell_cover` (self_mode "cartesian", Sec. 4) or
    :func:`selfcell_pv` (self_mode "exact") unless ``self_k`` is given."""
    if self_k is None:
        if self_mode == "exact":
            self_k = selfcell_pv(grid.beta, grid.dphi)
        elif self_mode == "cartesian":
            self_k = selfcell_cover(grid.beta, grid.dphi, cover_per)[:3]
        else:
            raise ValueError("self_mode must be 'cartesian' or 'exact'")
    sk = _f64(self_k)
    T = np.empty((6, 2 * grid.n_r - 1, grid.n_phi))
    if _load().or_tables(grid.n_r, grid.n_phi, grid.r_min, grid.r_max,
                         int(n_tpz), _TABLE_MODES[table_mode], _p(sk), _p(T)):
        raise ValueError("bad arguments")
    return T


def channels(grid: Grid, sigma, slope_order: int = 2):
    """Radial and azimuthal slopes of Eq. 25 (delta^r = d sigma / dr,
    delta^phi = d sigma / dphi at the cell centres) from the cell values.
    slope_order 2: central differences, one-sided on the first and last rows.
    slope_order 4: five-point central differences (in u = ln r radially)
    where the five points exist, the order-2 ones on the rows next to the
    ends."""
    s = _f64(sigma)
    dr = np.empty_like(s)
    dp = np.empty_like(s)
    if _load().or_channels_o(grid.n_r, grid.n_phi, _p(grid.r_centres),
                             grid.dphi, int(slope_order), _p(s), _p(dr), _p(dp)):
        raise ValueError("bad grid or slope order")
    return dr, dp


def forward(grid: Grid, T, sigma, dest=None, slope_order: int = 2):
    """F_r, F_phi by the plain double sums of Eq. 27-29 and A19-A21, with
    the slopes of :func:`channels` of the given order.

    ``dest``: optional flat destination indices i * N_phi + j; returns the
    forces at those cells (1-D) or on the whole grid (2-D)."""
    s = _f64(sigma)
    T = _f64(T)
    assert s.shape == grid.shape and T.shape == (6, 2 * grid.n_r - 1, grid.n_phi)
    if dest is None:
        fr = np.empty(grid.shape)
        fp = np.empty(grid.shape)
        d, nd = None, 0
    else:
        d = np.ascontiguousarray(dest, dtype=np.int64)
        nd = d.size
        fr = np.empty(nd)
        fp = np.empty(nd)
    rc = _load().or_forward_o(grid.n_r, grid.n_phi, grid.r_min, grid.r_max, int(slope_order),
                              _p(T), _p(s), _p(d), nd, _p(fr), _p(fp))
    if rc:
        raise RuntimeError("or_forward failed (%d)" % rc)
    return fr, fp


def forward_particle(grid: Grid, sigma, plus: bool = False, self_k=None, dest=None,
                     self_mode: str = "cartesian", cover_per: int = 10, slope_order: int = 2):
    """F_r, F_phi of the particle method (plus=False, Eq. 35-36 without the
    correction) or the modified particle method (plus=True, Eq. 34-37): point
    masses sigma r dr dphi at the cell centres, no self force, plus the
    self-cell correction with the constants of :func:`selfcell_cover` (or
    :func:`selfcell_pv` for self_mode "exact") unless ``self_k`` is given.
    ``dest`` as in :func:`forward`."""
    s = _f64(sigma)
    assert s.shape == grid.shape
    if self_k is None:
        self_k = (selfcell_pv(grid.beta, grid.dphi) if self_mode == "exact"
                  else selfcell_cover(grid.beta, grid.dphi, cover_per)[:3])
    sk = _f64(self_k)
    if dest is None:
        fr = np.empty(grid.shape)
        fp = np.empty(grid.shape)
        d, nd = None, 0
    else:
        d = np.ascontiguousarray(dest, dtype=np.int64)
        nd = d.size
        fr = np.empty(nd)
        fp = np.empty(nd)
    rc = _load().or_forward_particle_o(grid.n_r, grid.n_phi, grid.r_min, grid.r_max,
                                       int(bool(plus)), int(slope_order), _p(sk), _p(s), _p(d),
                                       nd, _p(fr), _p(fp))
    if rc:
        raise RuntimeError("or_forward_particle failed (%d)" % rc)
    return fr, fp


def adjoint(grid: Grid, T, v_r, v_phi, src=None, slope_order: int = 2):
    """Transpose of :func:`forward` (same slope order) applied to cotangents
    (v_r, v_phi), as a plain double sum, at flat source indices ``src`` (or
    every cell)."""
    vr, vp, T = _f64(v_r), _f64(v_phi), _f64(T)
    assert vr.shape == grid.shape and vp.shape == grid.shape
    if src is None:
        g = np.empty(grid.shape)
        s, ns = None, 0
    else:
        s = np.ascontiguousarray(src, dtype=np.int64)
        ns = s.size
        g = np.empty(ns)
    rc = _load().or_adjoint_o(grid.n_r, grid.n_phi, grid.r_min, grid.r_max, int(slope_order),
                              _p(T), _p(vr), _p(vp), _p(s), ns, _p(g))
    if rc:
        raise RuntimeError("or_adjoint failed (%d)" % rc)
    return g


def error_norms(num, ana):
    """L1, L2 and L-infinity error norms of Eq. 47-49 over all cells."""
    e = np.abs(np.asarray(num, dtype=np.float64) - np.asarray(ana, dtype=np.float64))
    n = e.size
    return float(e.sum() / n), float(np.sqrt((e * e).sum() / n)), float(e.max())


# ---------------------------------------------------------------------------
# Two patches of one log-polar grid and the origin wedges (Sec. 3.2.1)
# ---------------------------------------------------------------------------
def patch_tables(grid: Grid, n_src: int, s0: int, n_tpz: int = 19, self_k=None,
                 table_mode: str = "sim", self_mode: str = "cartesian", cover_per: int = 10):
    """Tables of the source patch (rows s0 .. s0 + n_src - 1 of the grid of
    the destination patch ``grid``) acting on the destination:
    [6][n_src + n_dst - 1][N_phi], row m' + n_src - 1 for m' = i - i'."""
    if self_k is None:
        self_k = (selfcell_pv(grid.beta, grid.dphi) if self_mode == "exact"
                  else selfcell_cover(grid.beta, grid.dphi, cover_per)[:3])
    sk = _f64(self_k)
    T = np.empty((6, n_src + grid.n_r - 1, grid.n_phi))
    mode = {"sim": 0, "exact": 1}[table_mode]
    if _load().or_patch_tables(int(n_src), int(s0), grid.n_r, grid.n_phi, grid.r_min,
                               grid.r_max, int(n_tpz), mode, _p(sk), _p(T)):
        raise ValueError("bad patch arguments")
    return T


def wedge_tables(grid: Grid, s0: int, method: str = "sim"):
    """Origin-wedge kernels [6][N_dst][N_phi] for wedges of radius
    r_min beta^s0 (method "sim": the integrals; "particle": point masses)."""
    T = np.empty((6, grid.n_r, grid.n_phi))
    m = 0 if method == "sim" else 1
    if _load().or_wedge_tables(grid.n_r, grid.n_phi, grid.r_min, grid.r_max, int(s0), m, _p(T)):
        raise ValueError("bad wedge arguments")
    return T


def _dest(grid, dest):
    if dest is None:
        return None, 0, np.empty(grid.shape), np.empty(grid.shape)
    d = np.ascontiguousarray(dest, dtype=np.int64)
    return d, d.size, np.empty(d.size), np.empty(d.size)


def patch_forward(grid: Grid, n_src: int, s0: int, T, sigma_src, Tw=None, sigma_w=None,
                  dest=None, col0: int = 0):
    """F_r, F_phi on the destination patch from the source patch (and the
    origin wedges when Tw and sigma_w are given), plain double sums; col0
    turns the source (and its wedges) by that many whole cells in phi."""
    s = _f64(sigma_src)
    assert s.shape == (n_src, grid.n_phi)
    T = _f64(T)
    Tw = _f64(Tw) if Tw is not None else None
    sw = _f64(sigma_w) if sigma_w is not None else None
    d, nd, fr, fp = _dest(grid, dest)
    if _load().or_patch_forward(int(n_src), int(s0), int(col0), grid.n_r, grid.n_phi, grid.r_min,
                                grid.r_max, _p(T), _p(s), _p(Tw), _p(sw), _p(d), nd, _p(fr),
                                _p(fp)):
        raise RuntimeError("or_patch_forward failed")
    return fr, fp


def patch_adjoint(grid: Grid, n_src: int, s0: int, T, v_r, v_phi, src=None, Tw=None,
                  col0: int = 0):
    """Transpose of :func:`patch_forward`: cotangents on the destination
    patch -> gradient on the source patch [n_src][n_phi] (or at the flat
    source indices ``src``), plain double sums.  With the wedge tables Tw
    (full source grid only) also the gradient with respect to the wedge
    densities: returns (g_src, g_wedge)."""
    vr, vp, T = _f64(v_r), _f64(v_phi), _f64(T)
    assert vr.shape == grid.shape and vp.shape == grid.shape
    assert Tw is None or src is None
    if src is None:
        s, ns, g = None, 0, np.empty((n_src, grid.n_phi))
    else:
        s = np.ascontiguousarray(src, dtype=np.int64)
        ns, g = s.size, np.empty(s.size)
    Tw = _f64(Tw) if Tw is not None else None
    gw = np.empty(grid.n_phi) if Tw is not None else None
    if _load().or_patch_adjoint(int(n_src), int(s0), int(col0), grid.n_r, grid.n_phi, grid.r_min,
                                grid.r_max, _p(T), _p(vr), _p(vp), _p(s), ns, _p(g), _p(Tw),
                                _p(gw)):
        raise RuntimeError("or_patch_adjoint failed")
    return (g, gw) if Tw is not None else g


def patch_particle(grid: Grid, n_src: int, s0: int, sigma_src, sigma_w=None, plus=False,
                   self_k=None, dest=None, col0: int = 0):
    """Particle (plus=False) or modified particle method between patches,
    point masses in physical coordinates, wedges as point masses."""
    s = _f64(sigma_src)
    if self_k is None:
        self_k = selfcell_cover(grid.beta, grid.dphi, 10)[:3]
    sk = _f64(self_k)
    sw = _f64(sigma_w) if sigma_w is not None else None
    d, nd, fr, fp = _dest(grid, dest)
    if _load().or_patch_particle(int(n_src), int(s0), int(col0), grid.n_r, grid.n_phi, grid.r_min,
                                 grid.r_max, int(bool(plus)), _p(sk), _p(s), _p(sw), _p(d), nd,
                                 _p(fr), _p(fp)):
        raise RuntimeError("or_patch_particle failed")
    return fr, fp


def patch_centres(grid: Grid, n_src: int, s0: int):
    """Centres of the source rows and the wedge centre r_w / 2."""
    k = s0 + np.arange(n_src)
    rc = grid.r_min * grid.beta ** k * 0.5 * (1.0 + grid.beta)
    return rc, 0.5 * grid.r_min * grid.beta ** s0


# ---------------------------------------------------------------------------
# Cartesian coordinates (Sec. 3.1, Eq. 6-21, A1-A16)
# ---------------------------------------------------------------------------
CART_TABLE_NAMES = ("x0", "xx", "xy", "y0", "yy", "yx")
CART_METHODS = {"second": 0, "particle": 1, "particle+": 2}


class CartGrid:
    """Uniform N_x x N_y grid of cells Delta x by Delta y (Sec. 3.1.1); cell
    (i, j) has centre (x0 + (i + 1/2) Delta x, y0 + (j + 1/2) Delta y)."""

    def __init__(self, n_x: int, n_y: int, dx: float, dy: float, x0: float = 0.0,
                 y0: float = 0.0):
        self.n_x, self.n_y = int(n_x), int(n_y)
        self.dx, self.dy = float(dx), float(dy)
        self.x0, self.y0 = float(x0), float(y0)

    @classmethod
    def square(cls, n: int, half_width: float):
        """The paper's domain [-M, M]^2 with N_d = n cells per side."""
        h = 2.0 * half_width / n
        return cls(n, n, h, h, -half_width, -half_width)

    @property
    def shape(self):
        return (self.n_x, self.n_y)

    def centres(self):
        x = self.x0 + (np.arange(self.n_x) + 0.5) * self.dx
        y = self.y0 + (np.arange(self.n_y) + 0.5) * self.dy
        return np.meshgrid(x, y, indexing="ij")


def cart_tables(grid: CartGrid, method: str = "second"):
    """The six Cartesian kernel tables [6][2N_x - 1][2N_y - 1], offsets
    m = i - i', n = j - j' at [k][m + N_x - 1][n + N_y - 1]; kernels in the
    order of ``CART_TABLE_NAMES`` (Eq. 13-15, A5-A13; particle kernels of
    Eq. 20 and A15 with masses sigma Dx Dy, plus the self terms of Eq. 21 and
    A16 for "particle+")."""
    T = np.empty((6, 2 * grid.n_x - 1, 2 * grid.n_y - 1))
    if _load().or_cart_tables(grid.n_x, grid.n_y, grid.dx, grid.dy, CART_METHODS[method], _p(T)):
        raise ValueError("bad Cartesian grid")
    return T


def cart_slopes(grid: CartGrid, sigma):
    """delta^x, delta^y: central differences, one-sided at the edges."""
    s = _f64(sigma)
    gx = np.empty_like(s)
    gy = np.empty_like(s)
    if _load().or_cart_slopes(grid.n_x, grid.n_y, grid.dx, grid.dy, _p(s), _p(gx), _p(gy)):
        raise ValueError("bad Cartesian grid")
    return gx, gy


def cart_forward(grid: CartGrid, T, sigma, dest=None):
    """F^x, F^y by the plain double sums of Eq. 9-12 and A1-A4 with tables
    ``T`` from :func:`cart_tables`; ``dest``: optional flat indices
    i * N_y + j."""
    s = _f64(sigma)
    T = _f64(T)
    assert s.shape == grid.shape and T.shape == (6, 2 * grid.n_x - 1, 2 * grid.n_y - 1)
    if dest is None:
        fx = np.empty(grid.shape)
        fy = np.empty(grid.shape)
        d, nd = None, 0
    else:
        d = np.ascontiguousarray(dest, dtype=np.int64)
        nd = d.size
        fx = np.empty(nd)
        fy = np.empty(nd)
    if _load().or_cart_forward(grid.n_x, grid.n_y, grid.dx, grid.dy, _p(T), _p(s), _p(d), nd,
                               _p(fx), _p(fy)):
        raise RuntimeError("or_cart_forward failed")
    return fx, fy
