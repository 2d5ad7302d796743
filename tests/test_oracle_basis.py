"""Pins of the oracle's quadrature, bases and geometry against mathematics.

Each expected value here comes from a closed form or an identity, not from
the oracle itself.
"""
import math

import numpy as np
import pytest

from oracle import BoxMesh, Discretization, gauss_legendre_01, lagrange_values, lagrange_derivatives


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_exactness(n):
    x, w = gauss_legendre_01(n)
    for m in range(2 * n):
        assert abs(np.dot(w, x ** m) - 1.0 / (m + 1)) < 1e-14
    # degree 2n is not integrated exactly
    assert abs(np.dot(w, x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-8


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_lagrange_identities(n):
    z, _ = gauss_legendre_01(n)
    xs = np.linspace(-0.3, 1.4, 37)
    V = lagrange_values(z, xs)
    assert np.allclose(V.sum(axis=1), 1.0, atol=1e-13)          # partition of unity
    assert np.allclose(lagrange_values(z, z), np.eye(n), atol=1e-14)
    D = lagrange_derivatives(z, xs)
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-11)
    # derivative exact on polynomials of degree <= n-1
    rng = np.random.default_rng(n)
    coef = rng.standard_normal(n)
    poly = np.polynomial.Polynomial(coef)
    assert np.allclose(D @ poly(z), poly.deriv()(xs), atol=1e-10)


def _sine_map(X):
    d = 0.05 * np.sin(2 * math.pi * X[:, 0]) * np.sin(2 * math.pi * X[:, 1])
    return X + np.stack([d, d], axis=1)


@pytest.mark.parametrize("mapped", [False, True])
def test_geometry(mapped):
    mesh = BoxMesh(2, (5, 4), (0.0, 0.0), (1.0, 1.0), (False, False),
                   vertex_map=_sine_map if mapped else None)
    disc = Discretization(mesh, 3, nu=1.0)
    vol = sum(disc.cell_measure(c) for c in range(mesh.N))
    assert abs(vol - 1.0) < 1e-13          # the displacement vanishes on the boundary
    for c in range(mesh.N):
        assert np.all(disc.cell(c)["det"] > 0)
        for a in range(2):
            nb = mesh.neighbor(c, a, 1)
            if nb is None:
                continue
            fm = disc.face(c, a, 1)
            fp = disc.face(nb, a, 0)
            assert np.allclose(fm["x"], fp["x"], atol=1e-14)
            assert np.allclose(fm["n"], -fp["n"], atol=1e-14)
            assert np.allclose(fm["dS"], fp["dS"], atol=1e-14)
            assert np.allclose(np.linalg.norm(fm["n"], axis=1), 1.0)


def test_affine_3d_measures():
    mesh = BoxMesh(3, (2, 3, 4), (0.0, 0.0, 0.0), (1.0, 2.0, 3.0), (True, True, True))
    disc = Discretization(mesh, 2, nu=1.0)
    h = np.array([0.5, 2.0 / 3.0, 0.75])
    assert abs(sum(disc.cell_measure(c) for c in range(mesh.N)) - 6.0) < 1e-12
    for a in range(3):
        tang = [b for b in range(3) if b != a]
        assert abs(disc.face_measure(0, a, 1) - h[tang[0]] * h[tang[1]]) < 1e-14


def test_dof_counts_match_paper():
    # Sec. 4 (3D lid-driven cavity): 64 x 64 x 48 Q2-Q1 cells carry
    # 15 925 248 velocity and 1 572 864 pressure unknowns.
    mesh = BoxMesh(3, (64, 64, 48), (0.0, 0.0, 0.0), (1.0, 1.0, 0.75), (False, False, False))
    disc = Discretization(mesh, 2, nu=1.0)
    assert disc.N_u == 15925248
    assert disc.N_p == 1572864
