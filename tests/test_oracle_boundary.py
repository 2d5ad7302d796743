"""Pins of the oracle's Dirichlet-boundary branches and of its stage
ingredients that the periodic pins do not reach.

Every expected value here comes from mathematics, not from the oracle
itself:

* the symmetric interior penalty form with Nitsche boundary terms
  (eq. bilin_diff, boundary penalty 2C) is symmetric positive definite on a
  box with walls;
* a manufactured advection-diffusion-reaction solution with non-zero
  Dirichlet data, solved with the stage operator of the momentum predictor
  (mass + SIP + Lax-Friedrichs advection, eq. bilin_diff and eq. trilinear)
  and the boundary-data functional of eq. rhs1, converges at order k+1 in h
  and exponentially in k;
* discrete integration by parts: for fields that lie in the discrete space
  and are continuous across faces, the face sums of the forms cancel exactly,
  so the weak gradient and divergence with boundary faces, the explicit
  diffusion and advection functionals and the implicit operators with their
  boundary data reduce to closed forms (Gw p = -P p, D u = -M^p div u,
  L0 u = 0, A0_w u = -M (w.grad) u, (nu A + C(w)) u - F_D = M (w.grad) u);
* the advecting-velocity extrapolations reproduce fields that are linear in
  time at the stage times t^n + gamma dt / 2 and t^{n+1};
* the closed-form Kovasznay flow satisfies the steady Navier-Stokes
  equations, and the oracle's steady stage residual of that flow, with its
  exact Dirichlet data, vanishes under refinement at order k-1 or better.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synthetic
from oracle import BoxMesh, Discretization, TRBDF2, trbdf2_constants

PI = math.pi


def _walled(dim, n, k, lo=None, hi=None, nu=1.0):
    lo = lo if lo is not None else tuple(0.1 * (a + 1) for a in range(dim))
    hi = hi if hi is not None else tuple(l + 1.0 + 0.2 * a for a, l in enumerate(lo))
    mesh = BoxMesh(dim, (n,) * dim, lo, hi, (False,) * dim)
    return Discretization(mesh, k, nu=nu)


def _pack(vals, dim, nb):
    """(Nc * nb, dim) point values in [cell][node] order -> [cell][comp][node]."""
    v = np.asarray(vals).reshape(-1, nb, dim)
    return np.ascontiguousarray(v.transpose(0, 2, 1)).reshape(-1)


def _per_component(A, u, d):
    U = u.reshape(d.Nc, d.dim, d.nbu)
    out = np.empty_like(U)
    for a in range(d.dim):
        out[:, a, :] = (A @ U[:, a, :].reshape(-1)).reshape(d.Nc, d.nbu)
    return out.reshape(-1)


# ---------------------------------------------------------------------------
# SIP with Nitsche walls
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (2, 5), (3, 2), (3, 3)])
def test_sip_with_walls_is_spd(dim, k):
    """Dirichlet walls remove the constant null space of the periodic form:
    the boundary penalty 2C makes the form coercive."""
    d = _walled(dim, 3 if dim == 2 else 2, k)
    A = d.sip_u().toarray()
    scale = np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-13 * scale
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > 1e-6 * scale, ev[:3]


# ---------------------------------------------------------------------------
# manufactured solution with non-zero Dirichlet data
# ---------------------------------------------------------------------------
def _u_exact(x):
    X, Y = x[:, 0], x[:, 1]
    return np.stack([np.sin(PI * X) * np.exp(Y), np.cos(X * Y)], 1)


def _w_field(x):
    X, Y = x[:, 0], x[:, 1]
    return np.stack([np.sin(X) * np.cos(Y), -np.cos(X) * np.sin(Y)], 1)   # divergence free


def _source(x, m, nu):
    """f = m u - nu lap u + (w.grad) u for the fields above (by hand)."""
    X, Y = x[:, 0], x[:, 1]
    u1 = np.sin(PI * X) * np.exp(Y)
    u1x, u1y = PI * np.cos(PI * X) * np.exp(Y), u1
    lap1 = (1.0 - PI * PI) * u1
    u2 = np.cos(X * Y)
    u2x, u2y = -Y * np.sin(X * Y), -X * np.sin(X * Y)
    lap2 = -(X * X + Y * Y) * u2
    w = _w_field(x)
    return np.stack([m * u1 - nu * lap1 + w[:, 0] * u1x + w[:, 1] * u1y,
                     m * u2 - nu * lap2 + w[:, 0] * u2x + w[:, 1] * u2y], 1)


def _mms_error(n, k, m=1.0, nu=0.5):
    """Solve (m M + nu A + C(w)) u = M f + F_D(u_D) on a walled 2D box (the
    momentum stage system with theta = 1) and return the relative L2 error."""
    d = _walled(2, n, k, lo=(0.1, -0.3), hi=(1.1, 0.9), nu=nu)
    xu = d.node_coords("u")
    w = _pack(_w_field(xu), 2, d.nbu)
    uD = lambda c, a, s, x: _u_exact(x)
    A = (m * d.mass_u() + nu * d.sip_u() + d.lf_advection(w, uD)).tocsc()
    M = d.mass_u()
    F = _per_component(M, _pack(_source(xu, m, nu), 2, d.nbu), d) + d.dirichlet_rhs(1.0, w, uD)
    lu = spla.splu(A)
    Fr = F.reshape(d.Nc, 2, d.nbu)
    u = np.stack([lu.solve(Fr[:, a, :].reshape(-1)).reshape(d.Nc, d.nbu) for a in range(2)], 1)
    e, r = d.l2_error(u.reshape(-1), _u_exact, "u")
    return e / r


@pytest.mark.parametrize("k", [2, 3])
def test_dirichlet_mms_h_convergence(k):
    errs = [_mms_error(n, k) for n in (2, 4, 8)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > k + 1 - 0.25, (errs, rates)


def test_dirichlet_mms_k_convergence():
    """On a fixed 2 x 2 mesh each added degree cuts the error by a growing
    factor (exponential convergence of a smooth solution in k)."""
    errs = [_mms_error(2, k) for k in (2, 3, 4, 5, 6)]
    ratios = [errs[i] / errs[i + 1] for i in range(4)]
    assert min(ratios) > 6.0, (errs, ratios)
    assert errs[-1] < 1e-6, errs


def test_dirichlet_mms_3d():
    """The same boundary terms in 3D: u = (sin(pi x) e^y, cos(yz), x z^2),
    constant advection, order k + 1 = 3."""
    def uex(x):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        return np.stack([np.sin(PI * X) * np.exp(Y), np.cos(Y * Z), X * Z * Z], 1)

    wc = np.array([0.6, -0.3, 0.45])

    def src(x, m, nu):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        u1 = np.sin(PI * X) * np.exp(Y)
        g1 = np.stack([PI * np.cos(PI * X) * np.exp(Y), u1, 0 * X], 1)
        l1 = (1.0 - PI * PI) * u1
        u2 = np.cos(Y * Z)
        g2 = np.stack([0 * X, -Z * np.sin(Y * Z), -Y * np.sin(Y * Z)], 1)
        l2 = -(Y * Y + Z * Z) * u2
        u3 = X * Z * Z
        g3 = np.stack([Z * Z, 0 * X, 2 * X * Z], 1)
        l3 = 2 * X
        return np.stack([m * u - nu * l + g @ wc for (u, g, l) in ((u1, g1, l1), (u2, g2, l2), (u3, g3, l3))], 1)

    errs = []
    m, nu = 1.0, 0.5
    for n in (2, 4):
        d = _walled(3, n, 2, nu=nu)
        xu = d.node_coords("u")
        w = _pack(np.tile(wc, (xu.shape[0], 1)), 3, d.nbu)
        uD = lambda c, a, s, x: uex(x)
        A = (m * d.mass_u() + nu * d.sip_u() + d.lf_advection(w, uD)).tocsc()
        F = _per_component(d.mass_u(), _pack(src(xu, m, nu), 3, d.nbu), d) + d.dirichlet_rhs(1.0, w, uD)
        lu = spla.splu(A)
        Fr = F.reshape(d.Nc, 3, d.nbu)
        u = np.stack([lu.solve(Fr[:, a, :].reshape(-1)).reshape(d.Nc, d.nbu) for a in range(3)], 1)
        e, r = d.l2_error(u.reshape(-1), uex, "u")
        errs.append(e / r)
    assert math.log2(errs[0] / errs[1]) > 2.6, errs


# ---------------------------------------------------------------------------
# discrete integration by parts on walled boxes
# ---------------------------------------------------------------------------
def _poly_p(dim, k, x):
    """A global polynomial of degree k-1 per direction (in Q_{k-1}) and its gradient."""
    q = k - 1
    c = [0.7, -0.4, 0.3][:dim]
    val = np.ones(x.shape[0])
    grad = np.ones((x.shape[0], dim))
    for a in range(dim):
        f = x[:, a] ** q + c[a] * x[:, a] + 0.2 * a
        df = q * x[:, a] ** (q - 1) + c[a]
        val = val * f
        for b in range(dim):
            grad[:, b] *= df if a == b else f
    return val, grad


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (2, 4), (3, 2), (3, 3)])
def test_weak_gradient_of_continuous_pressure_with_walls(dim, k):
    """Gw p = sum_K int p div v - sum_E int {{p}}[[v]] equals -int grad p . v
    for a continuous p in Q_{k-1}, boundary faces included (the average on a
    boundary face is the interior trace, so the boundary integral of p v.n
    cancels the one from integrating by parts)."""
    d = _walled(dim, 3 if dim == 2 else 2, k)
    xp = d.node_coords("p")
    xu = d.node_coords("u")
    p, _ = _poly_p(dim, k, xp)
    _, gu = _poly_p(dim, k, xu)
    lhs = d.weak_gradient() @ p
    Mv = d.mass_u_vector().diagonal()
    rhs = -Mv * _pack(gu, dim, d.nbu)
    assert np.abs(lhs - rhs).max() <= 1e-11 * np.abs(rhs).max()


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_divergence_of_continuous_velocity_with_walls(dim, k):
    """D u = sum_K int u.grad q - sum_E int {{u}}.[[q]] equals -int (div u) q
    for a continuous polynomial velocity whose divergence lies in Q_{k-1}
    (component a has degree k in x_a and k-1 in the other directions)."""
    d = _walled(dim, 3 if dim == 2 else 2, k)
    xu = d.node_coords("u")
    xp = d.node_coords("p")

    def field(x):
        comps, div = [], np.zeros(x.shape[0])
        for a in range(dim):
            f, df = x[:, a] ** k + 0.3 * x[:, a], k * x[:, a] ** (k - 1) + 0.3
            g = np.ones(x.shape[0])
            for b in range(dim):
                if b != a:
                    g = g * (x[:, b] ** (k - 1) - 0.5 * x[:, b] + 0.1 * (a + b))
            comps.append(f * g)
            div = div + df * g
        return np.stack(comps, 1), div

    u, _ = field(xu)
    _, divp = field(xp)
    lhs = d.divergence() @ _pack(u, dim, d.nbu)
    rhs = -d.mass_p().diagonal() * divp
    assert np.abs(lhs - rhs).max() <= 1e-11 * np.abs(rhs).max()


def _linear_velocity(dim, x):
    """u_c(x) = b_c + sum_a G[c, a] x_a and its constant gradient G."""
    G = np.array([[0.8, -0.5, 0.3], [0.2, 0.6, -0.7], [-0.4, 0.1, 0.5]])[:dim, :dim]
    b = np.array([0.3, -0.2, 0.5])[:dim]
    return b[None, :] + x @ G.T, G


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 4), (3, 2)])
def test_explicit_functionals_on_linear_fields_with_walls(dim, k):
    """The explicit diffusion L0 (no penalty, face sum over the whole
    skeleton) annihilates a linear field, and the explicit central advection
    A0_w gives -int (w.grad u) v for a constant w (eq. rhs1)."""
    d = _walled(dim, 3 if dim == 2 else 2, k)
    xu = d.node_coords("u")
    ul, G = _linear_velocity(dim, xu)
    u = _pack(ul, dim, d.nbu)
    wc = np.array([0.6, -0.35, 0.25])[:dim]
    w = _pack(np.tile(wc, (xu.shape[0], 1)), dim, d.nbu)
    Mv = d.mass_u_vector().diagonal()
    L0u = _per_component(d.explicit_diffusion(), u, d)
    assert np.abs(L0u).max() <= 1e-11 * np.abs(Mv * u).max() * d.mesh.n_cells[0] ** 2
    A0u = _per_component(d.explicit_advection(w), u, d)
    wgu = np.tile(G @ wc, (xu.shape[0], 1))
    expect = -Mv * _pack(wgu, dim, d.nbu)
    assert np.abs(A0u - expect).max() <= 1e-11 * np.abs(expect).max()


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2)])
def test_implicit_operator_with_boundary_data_on_linear_fields(dim, k):
    """With u linear and u_D its trace, (nu A + C(w)) u equals the Dirichlet
    functional F_D (eq. rhs1 boundary terms with theta = 1) plus
    int (w.grad u) v: the SIP boundary terms (-grad u.n v - u n.grad v
    + 2C u v) meet -u_D n.grad v + 2C u_D v, and the Lax-Friedrichs boundary
    term lambda u v (lambda from the mirrored state 2 u_D - w) meets
    -u_D (w.n) v + lambda u_D v."""
    nu = 0.37
    d = _walled(dim, 3 if dim == 2 else 2, k, nu=nu)
    xu = d.node_coords("u")
    ul, G = _linear_velocity(dim, xu)
    u = _pack(ul, dim, d.nbu)
    uD = lambda c, a, s, x: _linear_velocity(dim, x)[0]
    Mv = d.mass_u_vector().diagonal()
    for wc in (np.zeros(dim), np.array([0.6, -0.35, 0.25])[:dim], np.array([-1.3, 0.9, -0.2])[:dim]):
        w = _pack(np.tile(wc, (xu.shape[0], 1)), dim, d.nbu)
        op = _per_component(nu * d.sip_u() + d.lf_advection(w, uD), u, d)
        FD = d.dirichlet_rhs(1.0, w, uD)
        expect = FD + Mv * _pack(np.tile(G @ wc, (xu.shape[0], 1)), dim, d.nbu)
        assert np.abs(op - expect).max() <= 1e-11 * np.abs(expect).max(), wc


def test_constant_state_at_rest_with_walls():
    """A constant velocity equal to its constant wall data, advected by a
    constant w: the implicit operator and the boundary-data functional cancel
    exactly, with the stage factor theta applied to both."""
    for dim, k in ((2, 3), (3, 2)):
        d = _walled(dim, 2, k, nu=0.05)
        xu = d.node_coords("u")
        uc = np.array([0.4, -1.1, 0.7])[:dim]
        u = _pack(np.tile(uc, (xu.shape[0], 1)), dim, d.nbu)
        uD = lambda c, a, s, x: np.tile(uc, (x.shape[0], 1))
        for theta in (0.5, 1.0 / math.sqrt(2.0)):
            wc = np.array([0.25, 0.8, -0.5])[:dim]
            w = _pack(np.tile(wc, (xu.shape[0], 1)), dim, d.nbu)
            op = theta * _per_component(d.nu * d.sip_u() + d.lf_advection(w, uD), u, d)
            FD = d.dirichlet_rhs(theta, w, uD)
            assert np.abs(op - FD).max() <= 1e-12 * np.abs(FD).max()


# ---------------------------------------------------------------------------
# extrapolation targets
# ---------------------------------------------------------------------------
def test_extrapolation_reaches_stage_times():
    """A field linear in time, sampled where the stepper holds it, is
    reproduced at t^n + gamma dt / 2 (stage 1, from u^n and u^{n-1+gamma})
    and at t^{n+1} (stage 2, from u^{n+gamma} and u^n)."""
    g = 2.0 - math.sqrt(2.0)
    mesh = BoxMesh(2, (1, 1), (0.0, 0.0), (1.0, 1.0), (True, True))
    ora = TRBDF2(Discretization(mesh, 1, nu=1.0), 1.0)
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(7), rng.standard_normal(7)
    for dt, tn in ((0.1, 0.0), (0.037, 1.3)):
        f = lambda t: a + b * t
        w1 = ora.extrapolate(1, f(tn), f(tn - (1.0 - g) * dt))
        assert np.abs(w1 - f(tn + 0.5 * g * dt)).max() < 1e-14 * (1 + np.abs(a).max())
        w2 = ora.extrapolate(2, f(tn + g * dt), f(tn))
        assert np.abs(w2 - f(tn + dt)).max() < 1e-14 * (1 + np.abs(a).max())
    # the two weight pairs coincide numerically (both are 1 + 1/sqrt2, -1/sqrt2)
    cst = trbdf2_constants()
    assert abs(cst["extrap1"][0] - (1 + 1 / math.sqrt(2))) < 1e-15
    assert abs(cst["extrap2"][1] + 1 / math.sqrt(2)) < 1e-15


# ---------------------------------------------------------------------------
# Kovasznay flow
# ---------------------------------------------------------------------------
def test_kovasznay_closed_form_solves_steady_navier_stokes():
    """Central differences of the closed form: div u = 0 and
    (u.grad) u + grad p - nu lap u = 0 with nu = 1/Re."""
    Re = 40.0
    rng = np.random.default_rng(5)
    x = np.stack([rng.uniform(-0.5, 1.0, 50), rng.uniform(-0.5, 1.5, 50)], 1)
    h = 1e-4

    def U(y):
        return synthetic.kovasznay(y, Re)[0]

    def P(y):
        return synthetic.kovasznay(y, Re)[1]

    ex, ey = np.array([h, 0.0]), np.array([0.0, h])
    ux = (U(x + ex) - U(x - ex)) / (2 * h)
    uy = (U(x + ey) - U(x - ey)) / (2 * h)
    lap = (U(x + ex) + U(x - ex) + U(x + ey) + U(x - ey) - 4 * U(x)) / (h * h)
    px = (P(x + ex) - P(x - ex)) / (2 * h)
    py = (P(x + ey) - P(x - ey)) / (2 * h)
    u = U(x)
    div = ux[:, 0] + uy[:, 1]
    res = u[:, :1] * ux + u[:, 1:] * uy + np.stack([px, py], 1) - lap / Re
    assert np.abs(div).max() < 1e-7
    assert np.abs(res).max() < 1e-5


def test_kovasznay_steady_residual_vanishes_under_refinement():
    """The oracle's stage-1 system evaluated at the interpolated exact
    Kovasznay flow (u_prev = w = u, the exact pressure, exact Dirichlet data
    on all four walls): the mass terms cancel and what is left is the steady
    residual theta (nu (A + L0) + C(u) - A0_u) u - Gw p - F_D.  It is the
    consistency error of the DG forms, which must vanish under refinement
    (nodal M^{-1}-weighted norm, order k - 1 or better); a sign slip in any
    boundary term leaves an O(1/h) residual at the walls."""
    Re = 40.0
    res = {}
    for k in (3, 4):
        vals = []
        for n in (4, 8):
            mesh = BoxMesh(2, (n, n), (-0.5, -0.5), (1.0, 1.5), (False, False))
            d = Discretization(mesh, k, nu=1.0 / Re)
            ora = TRBDF2(d, 0.01, uD=lambda x, t: synthetic.kovasznay(x, Re)[0], nonlinear_iters=2)
            xu, xp = d.node_coords("u"), d.node_coords("p")
            u = synthetic.nodal_velocity(synthetic.kovasznay(xu, Re)[0], 2, d.nbu)
            p = synthetic.kovasznay(xp, Re)[1]
            r = ora.apply_momentum(1, u, u, 0.0) - ora.rhs_momentum(1, u, None, u, p, 0.0, w_explicit=u)
            vals.append(math.sqrt(np.sum(r * r / ora.Mv.diagonal())))
        res[k] = vals
        rate = math.log2(vals[0] / vals[1])
        assert rate > k - 1 - 0.3, (k, vals, rate)
    assert res[4][1] < 0.01 and res[3][1] < 0.06, res
