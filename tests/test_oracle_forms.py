"""Pins of the oracle's assembled DG forms against mathematics.

Expected values are properties that the paper's forms must have (symmetry,
null spaces, conservation, integration-by-parts adjointness), closed-form
spectra and manufactured solutions, or an independently coded upwind
discretisation built here by brute force with a different quadrature.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla
from scipy.special import roots_legendre

from oracle import BoxMesh, Discretization
from synthetic import random_vector


def _periodic(dim, n, k, L=1.0):
    mesh = BoxMesh(dim, (n,) * dim, (0.0,) * dim, (L,) * dim, (True,) * dim)
    return Discretization(mesh, k, nu=1.0)


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (2, 4), (2, 5), (3, 2), (3, 3)])
def test_sip_symmetric_null_space(dim, k):
    n = 3 if dim == 2 else 2
    d = _periodic(dim, n, k)
    for A in (d.sip_p().toarray(), d.sip_u().toarray()):
        scale = np.abs(A).max()
        assert np.abs(A - A.T).max() <= 1e-13 * scale
        assert np.abs(A.sum(axis=1)).max() <= 1e-12 * scale        # A 1 = 0
        ev = np.linalg.eigvalsh(A)
        assert ev[0] > -1e-12 * scale
        assert ev[1] > 1e-6 * scale                                   # one-dimensional null space


@pytest.mark.parametrize("k", [2, 3])
def test_pressure_spectrum_converges(k):
    """Smallest non-zero generalised eigenvalue of (K, M^p) on the periodic
    unit square is 4 pi^2 (fourfold) in the limit."""
    errs = []
    for n in (4, 8, 16):
        d = _periodic(2, n, k)
        K = d.sip_p().toarray()
        Mp = d.mass_p().toarray()
        ev = np.sort(sla.eigh(K, Mp, eigvals_only=True))
        assert abs(ev[0]) < 1e-9
        lam = ev[1:5]
        assert np.ptp(lam) < 1e-8 * lam[0]
        errs.append(abs(lam[0] / (4 * math.pi ** 2) - 1.0))
    # eigenvalue error decays at least like h^(2 k_p) = h^(2k-2)
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0, errs
    assert errs[2] < 2e-2


@pytest.mark.parametrize("k,rate", [(2, 2.0), (3, 3.0)])
def test_pressure_helmholtz_mms(k, rate):
    """(M^p + K) p = M^p f with p = sin 2pi x sin 2pi y, f = (1 + 8 pi^2) p:
    the L2 error converges at order k_p + 1 = k."""
    errs = []
    for n in (4, 8, 16):
        d = _periodic(2, n, k)
        xp = d.node_coords("p")
        pex = lambda x: np.sin(2 * math.pi * x[:, 0]) * np.sin(2 * math.pi * x[:, 1])
        Mp = d.mass_p()
        H = (Mp + d.sip_p()).tocsc()
        rhs = Mp @ ((1.0 + 8 * math.pi ** 2) * pex(xp))
        ph = spla.spsolve(H, rhs)
        e, r = d.l2_error(ph, pex, field="p")
        errs.append(e / r)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] > rate - 0.3, rates


def test_mass_matrices():
    d = _periodic(3, 2, 3, L=2.0)
    M = d.mass_u()
    Mp = d.mass_p()
    for A in (M, Mp):
        Ad = A.toarray()
        assert np.abs(Ad - np.diag(np.diag(Ad))).max() == 0.0
        assert abs(A.diagonal().sum() - 8.0) < 1e-12


def _lagrange_poly(nodes, i):
    """Lagrange polynomial via numpy Polynomial roots (independent of the oracle)."""
    others = np.delete(nodes, i)
    p = np.polynomial.Polynomial.fromroots(others)
    return p / p(nodes[i])


def _upwind_matrix(d, w):
    """Brute-force upwind DG advection matrix for a constant field w on a
    periodic Cartesian 2D mesh, integrated with a 12-point Gauss rule:
    -int u w.grad v + sum_faces int (w.n) u_upwind (v_own - v_other)."""
    mesh = d.mesh
    nodes = d.zu
    n = len(nodes)
    polys = [_lagrange_poly(nodes, i) for i in range(n)]
    dpolys = [p.deriv() for p in polys]
    xg, wg = roots_legendre(12)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    V = np.array([[p(x) for p in polys] for x in xg])          # (12, n)
    D = np.array([[p(x) for p in dpolys] for x in xg])
    V0 = np.array([p(0.0) for p in polys])
    V1 = np.array([p(1.0) for p in polys])
    h = (mesh.hi - mesh.lo) / np.array(mesh.n_cells)
    nb = n * n
    A = np.zeros((d.n_scalar, d.n_scalar))
    # volume: -int u (w . grad v), basis index i = ix + n iy
    Mx = (V * wg[:, None]).T @ V               # int l_j l_i (1D, reference)
    Sx = (D * wg[:, None]).T @ V               # int l_j l_i'
    vol = -(w[0] * h[1] * np.kron(Mx, Sx) + w[1] * h[0] * np.kron(Sx, Mx))
    for c in range(mesh.N):
        A[c * nb:(c + 1) * nb, c * nb:(c + 1) * nb] += vol
        for a in range(2):
            nbr = mesh.neighbor(c, a, 1)
            wn = w[a]                          # w . n for the face normal +e_a
            other = 1 - a
            Mt = (V * wg[:, None]).T @ V * h[other]
            # traces: test/trial on c at side 1, on nbr at side 0
            if a == 0:
                Tc = np.kron(Mt, np.outer(V1, V1))
                Tcn = np.kron(Mt, np.outer(V1, V0))     # test c, trial nbr
                Tnc = np.kron(Mt, np.outer(V0, V1))     # test nbr, trial c
                Tn = np.kron(Mt, np.outer(V0, V0))
            else:
                Tc = np.kron(np.outer(V1, V1), Mt)
                Tcn = np.kron(np.outer(V1, V0), Mt)
                Tnc = np.kron(np.outer(V0, V1), Mt)
                Tn = np.kron(np.outer(V0, V0), Mt)
            sc = slice(c * nb, (c + 1) * nb)
            sn = slice(nbr * nb, (nbr + 1) * nb)
            if wn >= 0:     # upwind value is c's trace
                A[sc, sc] += wn * Tc
                A[sn, sc] -= wn * Tnc
            else:           # upwind value is the neighbour's trace
                A[sc, sn] += wn * Tcn
                A[sn, sn] -= wn * Tn
    return A


@pytest.mark.parametrize("k", [2, 3])
def test_lf_equals_upwind_for_constant_advection(k):
    mesh = BoxMesh(2, (3, 4), (0.0, 0.0), (1.5, 1.0), (True, True))
    d = Discretization(mesh, k, nu=1.0)
    wc = np.array([0.7, -0.4])
    w = np.zeros(d.N_u)
    W = w.reshape(d.Nc, 2, d.nbu)
    W[:, 0, :] = wc[0]
    W[:, 1, :] = wc[1]
    C = d.lf_advection(w).toarray()
    U = _upwind_matrix(d, wc)
    assert np.abs(C - U).max() <= 1e-12 * np.abs(U).max()


def test_lf_conservation_and_energy():
    d = _periodic(2, 4, 3)
    w = np.zeros(d.N_u)
    W = w.reshape(d.Nc, 2, d.nbu)
    W[:, 0, :] = 0.3
    W[:, 1, :] = -1.1
    C = d.lf_advection(w).toarray()
    s = np.abs(C).max()
    assert np.abs(C.sum(axis=1)).max() < 1e-13 * s       # C . const = 0
    assert np.abs(C.sum(axis=0)).max() < 1e-13 * s       # 1^T C = 0 (momentum conservation)
    S = 0.5 * (C + C.T)
    assert np.linalg.eigvalsh(S).min() > -1e-12 * s      # LF part dissipates
    # central part is skew and equals minus the explicit (no-upwind) form
    A0 = d.explicit_advection(w).toarray()
    assert np.abs((C - S) + A0).max() < 1e-13 * s
    assert np.abs(A0 + A0.T).max() < 1e-13 * s
    # for a variable field, C and the explicit form still conserve momentum
    wr = random_vector(d.N_u, 11)
    Cr = d.lf_advection(wr).toarray()
    assert np.abs(Cr.sum(axis=0)).max() < 1e-12 * np.abs(Cr).max()


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 4), (3, 3)])
def test_weak_gradient_is_minus_divergence_transpose(dim, k):
    d = _periodic(dim, 3 if dim == 2 else 2, k)
    Gw = d.weak_gradient().toarray()
    D = d.divergence().toarray()
    assert np.abs(Gw + D.T).max() <= 1e-13 * np.abs(D).max()
    # constant pressure test function: F_p(1) = 0 for any velocity
    assert np.abs(D.sum(axis=0)).max() <= 1e-13 * np.abs(D).max()


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 3)])
def test_projection_gives_nodal_gradient(dim, k):
    """M^{-1} P p equals grad p at the velocity nodes for p in Q_{k-1}."""
    mesh = BoxMesh(dim, (3,) * dim, (0.0,) * dim, (1.0, 2.0, 1.5)[:dim], (False,) * dim)
    d = Discretization(mesh, k, nu=1.0)
    rng = np.random.default_rng(k)
    cx = rng.standard_normal((k, k, k)) if dim == 3 else rng.standard_normal((k, k))
    def pfun(x):
        if dim == 2:
            return np.polynomial.polynomial.polyval2d(x[:, 0], x[:, 1], cx)
        return np.polynomial.polynomial.polyval3d(x[:, 0], x[:, 1], x[:, 2], cx)
    def pgrad(x):
        out = []
        for a in range(dim):
            ca = np.polynomial.polynomial.polyder(cx, axis=a)
            if dim == 2:
                out.append(np.polynomial.polynomial.polyval2d(x[:, 0], x[:, 1], ca))
            else:
                out.append(np.polynomial.polynomial.polyval3d(x[:, 0], x[:, 1], x[:, 2], ca))
        return np.stack(out, axis=1)
    p = pfun(d.node_coords("p"))
    Gp = (d.projection() @ p) / d.mass_u_vector().diagonal()
    xu = d.node_coords("u")
    ref = pgrad(xu).reshape(d.Nc, d.nbu, dim).transpose(0, 2, 1).reshape(-1)
    assert np.abs(Gp - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())


# ---------------------------------------------------------------------------
# Q1-mapped (distorted) cells: the same structural properties must survive
# the geometry map, and affine-invariant fields must be reproduced exactly.
# ---------------------------------------------------------------------------
def _sine_map(amp):
    def f(X):
        d = amp * np.sin(2 * math.pi * X[:, 0]) * np.sin(2 * math.pi * X[:, 1])
        return X + np.stack([d, d], axis=1)
    return f


def _mapped(n, k, periodic, amp=0.06, lo=(0.0, 0.0), hi=(1.0, 1.0)):
    mesh = BoxMesh(2, (n, n), lo, hi, (periodic,) * 2, vertex_map=_sine_map(amp))
    return Discretization(mesh, k, nu=1.0)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_mapped_sip_symmetric_null_space(k):
    d = _mapped(3, k, True)
    for A in (d.sip_p().toarray(), d.sip_u().toarray()):
        scale = np.abs(A).max()
        assert np.abs(A - A.T).max() <= 1e-13 * scale
        assert np.abs(A.sum(axis=1)).max() <= 1e-12 * scale
        ev = np.linalg.eigvalsh(A)
        assert ev[0] > -1e-12 * scale and ev[1] > 1e-6 * scale


@pytest.mark.parametrize("k", [2, 4])
def test_mapped_masses_measure_the_box(k):
    """The displacement vanishes on the box edges: the masses integrate 1 to
    the box area exactly."""
    d = _mapped(4, k, False, lo=(-0.5, -0.5), hi=(1.0, 1.5))
    assert abs(d.mass_u().sum() - 3.0) < 1e-13
    assert abs(d.mass_p().sum() - 3.0) < 1e-13


@pytest.mark.parametrize("k", [2, 3])
def test_mapped_projection_gives_gradient_of_linear_fields(k):
    """A physically linear pressure is bilinear in the reference coordinates
    of a Q1 cell, so it lies in the discrete space and M^{-1} P returns its
    constant gradient at every velocity node (a transposed inverse Jacobian
    would not)."""
    d = _mapped(3, k, False, amp=0.08)
    a = np.array([0.7, -1.3])
    p = d.node_coords("p") @ a + 0.25
    Gp = (d.projection() @ p) / d.mass_u_vector().diagonal()
    ref = np.tile(np.repeat(a, d.nbu), d.Nc)
    assert np.abs(Gp - ref).max() < 1e-11


@pytest.mark.parametrize("k", [2, 3])
def test_mapped_weak_gradient_is_minus_divergence_transpose(k):
    d = _mapped(3, k, True)
    Gw = d.weak_gradient().toarray()
    D = d.divergence().toarray()
    assert np.abs(Gw + D.T).max() <= 1e-13 * np.abs(D).max()
    assert np.abs(D.sum(axis=0)).max() <= 1e-13 * np.abs(D).max()


def test_mapped_lf_conservation_and_constants():
    """Constant advection of a constant field is exactly zero on a periodic
    mapped mesh (the Gauss rule integrates w . adj(J)^T grad v exactly), and
    the form conserves momentum (1^T C = 0) for any advector."""
    d = _mapped(3, 3, True)
    w = np.tile(np.repeat([0.8, -0.3], d.nbu), d.Nc)
    C = d.lf_advection(w).toarray()
    assert np.abs(C.sum(axis=1)).max() < 1e-12 * np.abs(C).max()
    assert np.abs(C.sum(axis=0)).max() < 1e-12 * np.abs(C).max()
    S = 0.5 * (C + C.T)
    assert np.linalg.eigvalsh(S)[0] > -1e-12 * np.abs(C).max()
    Cr = d.lf_advection(random_vector(d.N_u, 5)).toarray()
    assert np.abs(Cr.sum(axis=0)).max() < 1e-12 * np.abs(Cr).max()
