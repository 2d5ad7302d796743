"""Quadrature and nodal bases on the unit interval (oracle; test infrastructure).

Sec. 3 of the paper uses Q_k for each velocity component and Q_{k-1} for the
pressure but does not name a basis or a quadrature rule ("appropriate
quadrature rules" for the algebraic systems).  Reading used throughout: a
Lagrange basis whose nodes are the n Gauss-Legendre points of [0,1]
(n = k+1 for velocity, n = k for pressure), integrated with the same n-point
Gauss-Legendre rule, so the velocity and pressure mass matrices are diagonal.
"""
import numpy as np


def gauss_legendre_01(n):
    """n-point Gauss-Legendre points and weights mapped from [-1,1] to [0,1].

    numpy's ``leggauss`` is used as the library primitive; it is exact for
    polynomials of degree <= 2n-1.
    """
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """V[q, i] = l_i(x_q) for the Lagrange polynomials l_i on ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                V[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return V


def lagrange_derivatives(nodes, x):
    """D[q, i] = l_i'(x_q), the product rule applied to the Lagrange product."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for j in range(n):
                if j != i and j != m:
                    term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            D[:, i] += term
    return D


def tensor(tables):
    """Tensor product of per-direction tables; direction 0 (x) runs fastest.

    ``tables[a]`` has shape (points_a, functions_a); the result has shape
    (prod points, prod functions) with lexicographic x-fastest ordering on
    both axes.
    """
    out = tables[0]
    for t in tables[1:]:
        out = np.kron(t, out)
    return out


def tensor_points(points_1d_per_dir):
    """Lexicographic (x fastest) tensor grid; returns shape (N, dim)."""
    grids = np.meshgrid(*points_1d_per_dir[::-1], indexing="ij")
    cols = [g.reshape(-1) for g in grids[::-1]]
    return np.stack(cols, axis=1)


def tensor_weights(weights_1d_per_dir):
    w = np.asarray(weights_1d_per_dir[0], dtype=np.float64)
    for wd in weights_1d_per_dir[1:]:
        w = np.kron(np.asarray(wd, dtype=np.float64), w)
    return w
