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

Velocity-component hierarchy (field "u"):
* theta_s nu times its level-0 operator is the stepper's stage-s momentum
  operator on one component with no advecting field (walls included);
* its prolongations reproduce multilinear fields on the velocity nodes;
* the cycle is symmetric positive definite on walled and mixed boxes;
* flexible CG with it reaches the sparse-LU solution in a bounded number of
  iterations on two mesh sizes, and preconditioned GMRES on the full
  momentum operator (advection included) converges fast.
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


def _walled(dim, n, k, periodic):
    mesh = BoxMesh(dim, (n,) * dim, (0.0,) * dim, (1.0,) * dim, periodic)
    return Discretization(mesh, k, nu=0.05)


def _alpha_u(ts, s):
    return ts.m(s) / (ts.theta[s] * ts.disc.nu)


@pytest.mark.parametrize("dim,periodic", [(2, (False, False)), (2, (True, False)), (3, (False, True, False))])
def test_velocity_level0_is_stage_operator_without_advection(dim, periodic):
    disc = _walled(dim, 4, 2, periodic)
    ts = TRBDF2(disc, 0.02, uD=lambda x, t: np.zeros((len(x), dim)))
    for s in (1, 2):
        mg = Multigrid(disc, _alpha_u(ts, s), field="u", coarse_cells=4 if dim == 2 else 8)
        A = ts.momentum_scalar(s, np.zeros(disc.N_u), 0.0).toarray()
        H = ts.theta[s] * disc.nu * mg.levels[0].H.toarray()
        assert np.abs(H - A).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("dim,n,k", [(2, 8, 3), (3, 4, 2)])
def test_velocity_prolongation_reproduces_multilinear_fields(dim, n, k):
    disc = _walled(dim, n, k, (False,) * dim)
    mg = Multigrid(disc, 10.0, field="u", coarse_cells=8 if dim == 3 else 16)
    assert len(mg.levels) >= 3 and mg.levels[0].q == k

    def f(x):
        out = np.ones(len(x))
        for a in range(dim):
            out *= 1.0 + (a + 1) * x[:, a]
        return out

    for i, P in enumerate(mg.P):
        xf = mg.levels[i].disc.node_coords("u")
        xc = mg.levels[i + 1].disc.node_coords("u")
        assert np.allclose(P @ f(xc), f(xf), rtol=0, atol=1e-13)


@pytest.mark.parametrize("periodic", [(False, False), (True, False)])
def test_velocity_vcycle_symmetric_positive_definite(periodic):
    disc = _walled(2, 8, 2, periodic)
    ts = TRBDF2(disc, 0.02)
    mg = Multigrid(disc, _alpha_u(ts, 2), degree=3, field="u")
    N = mg.levels[0].N
    B = np.stack([mg.vcycle(e) for e in np.eye(N)], axis=1)
    assert np.abs(B - B.T).max() <= 1e-11 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0.0


@pytest.mark.parametrize("n", [8, 16])
def test_velocity_mg_pcg_iterations_bounded(n):
    """Diffusion-dominated stage operator (nu dt / h^2 up to 5 on the finer
    mesh): the V-cycle keeps flexible CG at a few iterations on both meshes,
    while Jacobi needs many more."""
    disc = _walled(2, n, 3, (False, False))
    ts = TRBDF2(disc, 0.25)
    a = _alpha_u(ts, 1)
    mg = Multigrid(disc, a, degree=4, field="u")
    H = mg.levels[0].H
    b = H @ np.random.default_rng(5).standard_normal(H.shape[0])
    x, its, hist = flexible_pcg(H, b, np.zeros_like(b), mg.vcycle, 1e-10)
    assert hist[-1] <= 1e-10 and its <= 20, (its, hist)
    xd = spla.splu(H.tocsc()).solve(b)
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
    _, its_j, _ = flexible_pcg(H, b, np.zeros_like(b), lambda r: r / mg.levels[0].d, 1e-10, 4000)
    assert its_j > 3 * its


def test_velocity_mg_preconditions_the_momentum_operator():
    """Right-preconditioned GMRES on the stage operator with a non-zero
    advecting field (Re = 20 on the unit box, walls): P^{-1} = the V-cycle
    of the symmetric part divided by theta nu."""
    disc = _walled(2, 8, 3, (False, False))
    ts = TRBDF2(disc, 0.1, uD=lambda x, t: np.zeros((len(x), 2)))
    xu = disc.node_coords("u")
    w = np.stack([np.sin(np.pi * xu[:, 0]) * np.cos(np.pi * xu[:, 1]),
                  -np.cos(np.pi * xu[:, 0]) * np.sin(np.pi * xu[:, 1])], 1)
    import synthetic
    w = synthetic.nodal_velocity(w, 2, disc.nbu)
    s = 1
    A = ts.momentum_scalar(s, w, 0.0)
    mg = Multigrid(disc, _alpha_u(ts, s), degree=4, field="u")
    tn = ts.theta[s] * disc.nu
    b = np.random.default_rng(6).standard_normal(A.shape[0])
    counts = {}
    for name, pre in (("mg", lambda r: mg.vcycle(r) / tn), ("jacobi", lambda r: r / A.diagonal())):
        Pinv = spla.LinearOperator(A.shape, matvec=pre)
        AP = spla.LinearOperator(A.shape, matvec=lambda v: A @ pre(v))
        its = [0]
        y, info = spla.gmres(AP, b, rtol=1e-10, restart=60, maxiter=20,
                             callback=lambda r: its.__setitem__(0, its[0] + 1), callback_type="pr_norm")
        x = pre(y)
        assert info == 0 and np.linalg.norm(b - A @ x) <= 1e-9 * np.linalg.norm(b), name
        counts[name] = its[0]
    assert counts["mg"] <= 25 and counts["jacobi"] > 3 * counts["mg"], counts
