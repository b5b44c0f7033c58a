"""Seeded synthetic surface densities for the log-polar self-gravity path.

This module holds no arithmetic of the force method: it only draws seeded
parameters and evaluates density formulas at points that the caller supplies
(the cell centres, taken from whichever side -- library or oracle -- the
caller uses).  The oracle, the tests and the benchmark all draw their inputs
from here, so that both sides of a parity test see the same numbers.

Seeds: ``numpy.random.default_rng(150901450 + k + 1000 * d)`` for workload k
and disk d.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 150901450


def rng(k: int, d: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + k + 1000 * d)


def _rphi(r, phi):
    r = np.asarray(r, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    return np.broadcast_arrays(r[:, None], phi[None, :])


def kuzmin(r, phi):
    """Axisymmetric (1 + r^2)^(-3/2)."""
    R, _ = _rphi(r, phi)
    return (1.0 + R * R) ** -1.5


def blobs(r, phi, n_blobs: int, g: np.random.Generator, r_min: float,
          r_max: float):
    """Sum of Gaussian blobs A exp(-|x - x_k|^2 / (2 w_k^2)) with
    A ~ U[0.1, 1], ln r_k ~ U[ln r_min, ln r_max], phi_k ~ U[0, 2 pi),
    w_k = U[0.05, 0.5] r_k."""
    R, P = _rphi(r, phi)
    X, Y = R * np.cos(P), R * np.sin(P)
    out = np.zeros_like(R)
    for _ in range(n_blobs):
        A = g.uniform(0.1, 1.0)
        rk = math.exp(g.uniform(math.log(r_min), math.log(r_max)))
        pk = g.uniform(0.0, 2 * math.pi)
        wk = g.uniform(0.05, 0.5) * rk
        xk, yk = rk * math.cos(pk), rk * math.sin(pk)
        out += A * np.exp(-((X - xk) ** 2 + (Y - yk) ** 2) / (2 * wk * wk))
    return out


def single_disk_blobs(r, phi, r_min=0.1, r_max=10.0, seed_k=1):
    """128 x 128 workload on [0.1, 10]: Kuzmin profile + 8 seeded blobs."""
    return kuzmin(r, phi) + blobs(r, phi, 8, rng(seed_k), r_min, r_max)


def spiral_disk(r, phi, seed_k=2, amp=0.2, arms=2, scale=3.0):
    """Exponential disk exp(-r/scale) with a logarithmic m-armed spiral of
    relative amplitude ``amp``: pitch p ~ U[10, 30] deg, phase ~ U[0, 2 pi)."""
    g = rng(seed_k)
    p = math.radians(g.uniform(10.0, 30.0))
    ph0 = g.uniform(0.0, 2 * math.pi)
    R, P = _rphi(r, phi)
    return np.exp(-R / scale) * (1.0 + amp * np.cos(arms * (P - np.log(R) / math.tan(p)) + ph0))


def finite_disk(r, phi, n=5, alpha=0.25, xc=0.5, yc=0.1):
    """sigma_Dn(|x - x_c|; alpha) = (1 - d^2/alpha^2)^(n - 1/2) inside."""
    R, P = _rphi(r, phi)
    d = np.hypot(R * np.cos(P) - xc, R * np.sin(P) - yc)
    q = np.clip(1.0 - (d / alpha) ** 2, 0.0, None)
    return np.where(d < alpha, q ** (n - 0.5), 0.0)


def multiarm_disk(r, phi, d: int, seed_k=4):
    """Exponential disk with seeded m = 1..4 logarithmic spirals (disk d):
    R_d ~ U[1, 5], a_m ~ U[0, 0.15], p_m ~ U[10, 30] deg, phase ~ U[0, 2 pi)."""
    g = rng(seed_k, d)
    Rd = g.uniform(1.0, 5.0)
    R, P = _rphi(r, phi)
    pert = np.ones_like(R)
    for m in range(1, 5):
        a = g.uniform(0.0, 0.15)
        p = math.radians(g.uniform(10.0, 30.0))
        ph = g.uniform(0.0, 2 * math.pi)
        pert += a * np.cos(m * (P - np.log(R) / math.tan(p)) + ph)
    return np.exp(-R / Rd) * pert


def batch_sizes(n_disks=64, seed_k=4):
    """Seeded (N_r, N_phi) for each disk of the uneven batch."""
    g = rng(seed_k, 999)
    nr = g.choice([256, 384, 512, 768, 1024], size=n_disks)
    nphi = g.choice([256, 512, 1024, 2048], size=n_disks)
    return [(int(a), int(b)) for a, b in zip(nr, nphi)]


def hidden_density(r, phi, r_min=0.01, r_max=100.0, seed_k=5):
    """Target of the force-matching problem: exp(-r/3) + 16 seeded clumps."""
    R, _ = _rphi(r, phi)
    return np.exp(-R / 3.0) + blobs(r, phi, 16, rng(seed_k), r_min, r_max)


def start_density(r, phi):
    """Starting guess of the force-matching problem: exp(-r/3)."""
    R, _ = _rphi(r, phi)
    return np.exp(-R / 3.0)


def random_field(shape, seed_k=7, d=0):
    """Plain N(0, 1) field (cotangents, perturbations)."""
    return rng(seed_k, d).standard_normal(shape)
