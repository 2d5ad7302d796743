"""Closed-form flow fields and seeded random vectors.

Fields are evaluated at caller-supplied points ``x`` of shape (npnt, dim) and
return (npnt, dim) velocities or (npnt,) pressures.
"""
import math

import numpy as np


def random_vector(n, seed, dtype=np.float64):
    """N(0, 1) entries from numpy's PCG64 generator seeded with ``seed``."""
    return np.random.default_rng(seed).standard_normal(int(n)).astype(dtype)


# -- 2D Taylor-Green ---------------------------------------------------------
def taylor_green_2d(x, t, Re):
    """Taylor-Green vortex on (0, 2 pi)^2 as printed in the paper
    (eq. greentaylor); returns (u, p)."""
    x1, x2 = x[:, 0], x[:, 1]
    fu = math.exp(-2.0 * t / Re)
    fp = math.exp(-4.0 * t / Re)
    u = np.stack([np.cos(x1) * np.sin(x2) * fu, -np.sin(x1) * np.cos(x2) * fu], axis=1)
    p = -0.25 * (np.cos(2 * x1) + np.cos(2 * x2)) * fp
    return u, p


def taylor_green_2d_unit(x, t, nu):
    """u = (sin 2pi x cos 2pi y, -cos 2pi x sin 2pi y) e^{-8 pi^2 nu t} on the
    unit square, p = +1/4 (cos 4pi x + cos 4pi y) e^{-16 pi^2 nu t}
    (u . grad u = -grad p fixes the sign for this orientation)."""
    tp = 2.0 * math.pi
    X, Y = tp * x[:, 0], tp * x[:, 1]
    fu = math.exp(-2.0 * tp * tp * nu * t)
    fp = math.exp(-4.0 * tp * tp * nu * t)
    u = np.stack([np.sin(X) * np.cos(Y) * fu, -np.cos(X) * np.sin(Y) * fu], axis=1)
    p = 0.25 * (np.cos(2 * X) + np.cos(2 * Y)) * fp
    return u, p


# -- 3D Taylor-Green (initial data only) --------------------------------------
def tgv3d_velocity(x):
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    return np.stack([np.sin(X) * np.cos(Y) * np.cos(Z),
                     -np.cos(X) * np.sin(Y) * np.cos(Z),
                     np.zeros_like(X)], axis=1)


def tgv3d_pressure(x):
    """Solution of -lap p = div(u0 . grad u0) for the 3D vortex above."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    return (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0


# -- Kovasznay ------------------------------------------------------------------
def kovasznay(x, Re):
    """Steady Kovasznay flow; returns (u, p) with p = (1 - e^{2 lam x})/2."""
    lam = 0.5 * Re - math.sqrt(0.25 * Re * Re + 4.0 * math.pi * math.pi)
    X, Y = x[:, 0], x[:, 1]
    e = np.exp(lam * X)
    u = np.stack([1.0 - e * np.cos(2 * math.pi * Y),
                  lam / (2 * math.pi) * e * np.sin(2 * math.pi * Y)], axis=1)
    p = 0.5 * (1.0 - np.exp(2.0 * lam * X))
    return u, p


# -- random-phase divergence-free fields -------------------------------------
def random_phase_velocity(x, seed, modes=8, kmax=4.0):
    """Sum of ``modes`` Fourier modes a_m cos(kappa_m . x + phi_m) with integer
    wave vectors 1 <= |kappa| <= kmax, amplitudes N(0, I)/|kappa|^2 projected
    orthogonal to kappa (so each mode is divergence free)."""
    rng = np.random.default_rng(seed)
    dim = x.shape[1]
    r = int(math.floor(kmax))
    grid = np.stack(np.meshgrid(*[np.arange(-r, r + 1)] * dim, indexing="ij"), -1).reshape(-1, dim)
    norms = np.linalg.norm(grid, axis=1)
    cand = grid[(norms >= 1.0) & (norms <= kmax)]
    u = np.zeros((x.shape[0], dim))
    for _ in range(modes):
        kap = cand[rng.integers(len(cand))].astype(np.float64)
        kn = np.linalg.norm(kap)
        a = rng.standard_normal(dim) / kn ** 2
        a -= (a @ kap) / (kn * kn) * kap
        phi = rng.uniform(0.0, 2.0 * math.pi)
        u += np.cos(x @ kap + phi)[:, None] * a[None, :]
    return u


# -- layout helpers -------------------------------------------------------------
def nodal_velocity(values, dim, nodes_per_cell):
    """Pack point values (Nc * nb, dim) given in [cell][node] order into the
    [cell][component][node] velocity layout."""
    v = np.asarray(values, dtype=np.float64).reshape(-1, nodes_per_cell, dim)
    return np.ascontiguousarray(np.transpose(v, (0, 2, 1))).reshape(-1)


def nodal_scalar(values):
    return np.ascontiguousarray(np.asarray(values, dtype=np.float64).reshape(-1))


# -- distorted meshes ---------------------------------------------------------
def sine_vertex_map(amp):
    """Vertex displacement x' = x + amp sin(2 pi x) sin(2 pi y) (same shift in
    y), applied to the vertices of a 2D box; cells stay bilinear.  It vanishes
    on the lines x, y in Z/2, so the boundary of [-0.5, 1] x [-0.5, 1.5] is
    fixed."""
    def f(X):
        d = amp * np.sin(2 * math.pi * X[:, 0]) * np.sin(2 * math.pi * X[:, 1])
        return X + np.stack([d, d], axis=1)
    return f
