"""Pins of the oracle's h/p-multigrid against mathematics and library routines.

* SplitMix64 reproduces the published first outputs from state 0;
* prolongation reproduces a globally multilinear field exactly (the coarse
  spaces are nested in the fine ones);
* the Chebyshev recurrence multiplies the error by the closed-form scaled
  Chebyshev polynomial (numpy's chebval on the eigen-decomposition);
* the Lanczos estimate lies just below the largest eigenvalue from a dense
  eigensolver;
* the V-cycle is a symmetric positive definite operator, the coarse solve
  equals a dense solve, and a one-level hierarchy is the exact inverse;
* flexible CG with the V-cycle reaches the sparse-LU solution.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import BoxMesh, Discretization, TRBDF2
from oracle.multigrid import (Multigrid, chebyshev_smooth, flexible_pcg, lanczos_largest,
                              lanczos_start, splitmix64)


def _disc(dim, n, k):
    mesh = BoxMesh(dim, (n,) * dim, (0.0,) * dim, (1.0,) * dim, (True,) * dim)
    return Discretization(mesh, k, nu=0.01)


def _alpha(disc, dt=0.01, s=1):
    return TRBDF2(disc, dt).alpha(s)


def test_splitmix64_published_outputs():
    assert splitmix64(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    v = lanczos_start(1000, seed=0)
    assert v.min() >= -0.5 and v.max() < 0.5 and abs(v.mean()) < 0.05


@pytest.mark.parametrize("dim,n,k", [(2, 8, 3), (2, 8, 4), (3, 4, 3)])
def test_prolongation_reproduces_multilinear_fields(dim, n, k):
    disc = _disc(dim, n, k)
    mg = Multigrid(disc, _alpha(disc), coarse_cells=8 if dim == 3 else 16)
    assert len(mg.levels) >= 3

    def f(x):
        out = np.ones(len(x))
        for a in range(dim):
            out *= 1.0 + (a + 1) * x[:, a]
        return out

    for i, P in enumerate(mg.P):
        xf = mg.levels[i].disc.node_coords("p")
        xc = mg.levels[i + 1].disc.node_coords("p")
        assert np.allclose(P @ f(xc), f(xf), rtol=0, atol=1e-13)
        # the transpose keeps the integral of a residual: 1^T (P^T r) = (P 1)^T r
        r = np.random.default_rng(i).standard_normal(P.shape[0])
        assert math.isclose((P.T @ r).sum(), r @ (P @ np.ones(P.shape[1])), rel_tol=1e-12)


def test_chebyshev_matches_closed_form_polynomial():
    disc = _disc(2, 4, 3)
    lv = Multigrid(disc, _alpha(disc)).levels[0]
    H = lv.H.toarray()
    d = lv.d
    S = H / np.sqrt(np.outer(d, d))
    lam, Q = np.linalg.eigh(S)
    lo, hi = lam.max() / 15.0, 1.1 * lam.max()
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    e0 = np.random.default_rng(3).standard_normal(len(d))
    for degree in (1, 2, 3, 5):
        x = chebyshev_smooth(lv.H, 1.0 / d, H @ e0, None, degree, lo, hi)
        cdeg = np.zeros(degree + 1)
        cdeg[-1] = 1.0
        R = np.polynomial.chebyshev.chebval((theta - lam) / delta, cdeg) / \
            np.polynomial.chebyshev.chebval(theta / delta, cdeg)
        # error x - e0 = D^{-1/2} Q R(Lambda) Q^T D^{1/2} (0 - e0)
        expect = -(Q @ (R * (Q.T @ (np.sqrt(d) * e0)))) / np.sqrt(d)
        assert np.allclose(x - e0, expect, rtol=0, atol=1e-11 * np.abs(e0).max())


@pytest.mark.parametrize("dim,n,k", [(2, 8, 3), (3, 4, 3)])
def test_lanczos_estimate_bounds(dim, n, k):
    disc = _disc(dim, n, k)
    mg = Multigrid(disc, _alpha(disc), coarse_cells=8 if dim == 3 else 16)
    for lv, lam in zip(mg.levels[:-1], mg.lam):
        S = lv.H.toarray() / np.sqrt(np.outer(lv.d, lv.d))
        lmax = np.linalg.eigvalsh(S).max()
        assert lam <= lmax * (1 + 1e-12) and lam >= 0.9 * lmax, (lam, lmax)
    # direct call: a diagonal matrix is resolved exactly once steps >= size
    H = np.diag(np.arange(1.0, 6.0))
    assert math.isclose(lanczos_largest(H, np.ones(5), 10, lanczos_start(5)), 5.0, rel_tol=1e-12)


@pytest.mark.parametrize("dim,n,k", [(2, 8, 3), (3, 4, 2)])
def test_vcycle_symmetric_positive_definite(dim, n, k):
    disc = _disc(dim, n, k)
    mg = Multigrid(disc, _alpha(disc), degree=3, coarse_cells=8 if dim == 3 else 16)
    N = mg.levels[0].N
    B = np.stack([mg.vcycle(e) for e in np.eye(N)], axis=1)
    assert np.abs(B - B.T).max() <= 1e-11 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0.0
    # coarse solve equals a dense solve
    Hc = mg.levels[-1].H.toarray()
    b = np.random.default_rng(1).standard_normal(Hc.shape[0])
    assert np.allclose(mg.vcycle(b, len(mg.levels) - 1), np.linalg.solve(Hc, b), rtol=1e-12, atol=0)


def test_single_level_is_exact_inverse():
    disc = _disc(2, 3, 2)           # 3x3 cells of Q1: no coarsening possible
    mg = Multigrid(disc, _alpha(disc))
    assert len(mg.levels) == 1
    H = mg.levels[0].H
    b = np.random.default_rng(2).standard_normal(H.shape[0])
    assert np.allclose(H @ mg.vcycle(b), b, rtol=0, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("dim,n,k", [(2, 8, 3), (2, 8, 5), (3, 4, 3)])
def test_mg_pcg_reaches_direct_solution(dim, n, k):
    disc = _disc(dim, n, k)
    a = _alpha(disc)
    mg = Multigrid(disc, a, degree=3, coarse_cells=8 if dim == 3 else 16)
    H = mg.levels[0].H
    b = H @ np.random.default_rng(4).standard_normal(H.shape[0])
    x, its, hist = flexible_pcg(H, b, np.zeros_like(b), mg.vcycle, 1e-10)
    assert hist[-1] <= 1e-10 and its <= 25, (its, hist)
    xd = spla.splu(H.tocsc()).solve(b)
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)
    # Jacobi-preconditioned CG needs many more iterations
    _, its_j, _ = flexible_pcg(H, b, np.zeros_like(b), lambda r: r / mg.levels[0].d, 1e-10, 2000)
    assert its_j > 2 * its
