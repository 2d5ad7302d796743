"""Pins of the oracle's learned-guess inputs and outputs against closed forms
and library routines.

* Gauss-rule cell averages and cell inner products are the exact cell means
  of pressures (and products of pressures) the space holds;
* the divergence feature of an interpolated polynomial velocity equals the
  exact cell mean of its divergence (interior cells of a periodic mesh);
* the shape features of hand-built increments take their closed-form values;
* for pressures cubic in time with a constant offset per stage, the
  network's zero output (quadratic extrapolation of the increment) has zero
  loss in every cell and reproduces the new pressure (the linear
  extrapolation does not; both are exact for quadratic pressures);
* the quadratic loss of any output equals the weighted squared error of the
  guess it injects, computed directly;
* the per-cell minimiser of the quadratic loss is the weighted least-squares
  fit of the extrapolation's error on the two increments (numpy lstsq);
* the fallback is exact for pressures linear in time with stage offsets.
"""
import numpy as np

import synthetic
from oracle import BoxMesh, Discretization, TRBDF2
from oracle import guess


def _setup(n=4, k=3):
    mesh = BoxMesh(2, (n, n), (0.0, 0.0), (1.0, 1.0), (True, True))
    disc = Discretization(mesh, k, nu=0.01)
    return disc, TRBDF2(disc, 0.01)


def _cell_bounds(disc, c):
    h = 1.0 / disc.mesh.n_cells[0]
    i, j = disc.mesh.cell_ijk(c)
    return i * h, (i + 1) * h, j * h, (j + 1) * h


def test_cell_average_and_inner_product_are_exact_means():
    disc, _ = _setup()
    xp = disc.node_coords("p")
    p = xp[:, 0] ** 2 * xp[:, 1]
    q = xp[:, 1] ** 2 + xp[:, 0]
    avg = guess.cell_average(disc, p)
    inner = guess.cell_inner(disc, p, q)
    for c in range(disc.Nc):
        x0, x1, y0, y1 = _cell_bounds(disc, c)
        hx, hy = x1 - x0, y1 - y0
        assert abs(avg[c] - (x1 ** 3 - x0 ** 3) / (3 * hx) * 0.5 * (y0 + y1)) < 1e-14
        # mean of x^2 y (y^2 + x) = mean(x^2) mean(y^3) + mean(x^3) mean(y)
        mx = lambda e: (x1 ** (e + 1) - x0 ** (e + 1)) / ((e + 1) * hx)
        my = lambda e: (y1 ** (e + 1) - y0 ** (e + 1)) / ((e + 1) * hy)
        assert abs(inner[c] - (mx(2) * my(3) + mx(3) * my(1))) < 1e-14


def test_divergence_feature_is_cell_mean_of_divergence():
    disc, ts = _setup()
    xu = disc.node_coords("u")
    u = np.stack([xu[:, 0] ** 2, xu[:, 0] * xu[:, 1]], 1)
    us = synthetic.nodal_velocity(u, 2, disc.nbu)
    p_prev = np.random.default_rng(0).standard_normal(disc.N_p)
    for s in (1, 2):
        b = ts.rhs_pressure(s, us, p_prev)
        z = np.zeros(disc.N_p)
        x, s_inc, s_div = guess.features(ts, s, b, p_prev, z + 3.0, 0.7, z + 1.0, z + 2.0)
        div = x[3] * s_div
        n = disc.mesh.n_cells[0]
        for c in range(disc.Nc):
            i, j = disc.mesh.cell_ijk(c)
            if 0 < i < n - 1 and 0 < j < n - 1:
                x0, x1, _, _ = _cell_bounds(disc, c)
                assert abs(div[c] - 1.5 * (x0 + x1)) < 1e-11, (c, div[c])
        # the increment channels are the rescaled cell averages
        bdt = ts.beta[s] * ts.dt
        assert np.allclose(x[0] * s_inc, 1.0 / bdt) and np.allclose(x[1] * s_inc, 2.0 / bdt)
        assert np.allclose(x[2] * s_inc, 3.0 / (0.7 * ts.dt))
        # d2 = 2 d1 in every cell: aligned, half the size
        assert np.allclose(x[4], 1.0) and np.allclose(x[5], np.log(0.5))


def test_shape_features_closed_forms():
    disc, _ = _setup(n=2, k=2)
    nb = disc.nbp
    rng = np.random.default_rng(4)
    d1 = rng.standard_normal(disc.N_p)
    d2 = np.empty_like(d1)
    d2[:nb] = -3.0 * d1[:nb]                    # opposite direction, three times larger
    # orthogonal in the weighted inner product: subtract the projection
    v = rng.standard_normal(nb)
    a = d1[nb:2 * nb]
    w = guess.node_weights(disc)
    d2[nb:2 * nb] = v - (np.sum(w * v * a) / np.sum(w * a * a)) * a
    d2[2 * nb:3 * nb] = 1e-9 * d1[2 * nb:3 * nb]   # growth beyond the clamp
    d2[3 * nb:] = 0.0                            # no history in this cell
    cos, lr = guess.shape_features(disc, d1, d2)
    assert abs(cos[0] + 1.0) < 1e-14 and abs(lr[0] - np.log(1.0 / 3.0)) < 1e-14
    assert abs(cos[1]) < 1e-13
    assert lr[2] == guess.LR_CLAMP and abs(cos[2] - 1.0) < 1e-14
    assert cos[3] == 0.0 and lr[3] == 0.0


def _history(disc, ts, rng, degree):
    """Pressures P(t) + o_s at stage times, P a polynomial of the given degree
    in time: returns p_prev, d1, d2, d3 and p_new of a stage-1 solve of step n."""
    q = [rng.standard_normal(disc.N_p) for _ in range(degree + 1)]
    o1, o2 = rng.standard_normal(disc.N_p), rng.standard_normal(disc.N_p)
    g, dt = ts.cst["gamma"], ts.dt
    P = lambda t: sum(qi * t ** i for i, qi in enumerate(q))
    tn = 0.4
    p_prev = P(tn) + o2
    d = [(P(tn - j * dt + g * dt) + o1) - (P(tn - j * dt) + o2) for j in (1, 2, 3)]
    p_new = P(tn + g * dt) + o1
    return p_prev, d[0], d[1], d[2], p_new


def test_extrapolation_blend_is_exact_for_cubic_in_time_pressure():
    disc, ts = _setup()
    rng = np.random.default_rng(2)
    p_prev, d1, d2, d3, p_new = _history(disc, ts, rng, degree=3)
    G = guess.gram_target(disc, p_new, p_prev, d1, d2, d3)
    y = np.zeros((2, disc.Nc))
    loss0, _ = guess.quad_loss(y, G)
    assert loss0 < 1e-24 * np.abs(G[0]).max()
    assert np.allclose(guess.inject(disc, p_prev, d1, d2, d3, y), p_new, atol=1e-12)
    assert np.allclose(guess.inject(disc, p_prev, d1, d2, d3, y), guess.extrapolate3(p_prev, d1, d2, d3))
    # the linear extrapolation misses the cubic term; for quadratic pressures
    # both are exact
    assert np.abs(guess.extrapolate2(p_prev, d1, d2) - p_new).max() > 1e-6
    p_prev, d1, d2, d3, p_new = _history(disc, ts, rng, degree=2)
    assert np.allclose(guess.extrapolate2(p_prev, d1, d2), p_new, atol=1e-12)
    assert np.allclose(guess.extrapolate3(p_prev, d1, d2, d3), p_new, atol=1e-12)


def test_loss_equals_squared_error_of_injected_guess():
    disc, ts = _setup(n=3)
    rng = np.random.default_rng(8)
    p_prev, d1, d2, d3, p_new = (rng.standard_normal(disc.N_p) for _ in range(5))
    G = guess.gram_target(disc, p_new, p_prev, d1, d2, d3)
    S = np.mean(guess.cell_inner(disc, d1, d1))
    for t in range(4):
        y = rng.standard_normal((2, disc.Nc))
        e = p_new - guess.inject(disc, p_prev, d1, d2, d3, y)
        direct = np.mean(guess.cell_inner(disc, e, e)) / S
        loss, _ = guess.quad_loss(y, G)
        assert abs(loss - direct) <= 1e-12 * max(direct, np.abs(G).max())


def test_loss_minimiser_is_the_weighted_least_squares_fit():
    disc, ts = _setup(n=3)
    rng = np.random.default_rng(6)
    p_prev, d1, d2, d3 = (rng.standard_normal(disc.N_p) for _ in range(4))
    p_new = p_prev + d1 + rng.standard_normal(disc.N_p)
    G = guess.gram_target(disc, p_new, p_prev, d1, d2, d3)
    sw = np.sqrt(guess.node_weights(disc))
    e = p_new - guess.extrapolate3(p_prev, d1, d2, d3)
    y_ls = np.empty((2, disc.Nc))
    for c in range(disc.Nc):
        sl = slice(c * disc.nbp, (c + 1) * disc.nbp)
        A = np.stack([d1[sl] * sw, d2[sl] * sw], 1)
        y_ls[:, c] = np.linalg.lstsq(A, e[sl] * sw, rcond=None)[0]
    _, grad = guess.quad_loss(y_ls, G)
    assert np.abs(grad).max() < 1e-12
    loss_ls, _ = guess.quad_loss(y_ls, G)
    for t in range(5):
        loss_y, _ = guess.quad_loss(y_ls + 0.1 * rng.standard_normal(y_ls.shape), G)
        assert loss_y > loss_ls


def test_fallback_exact_for_linear_in_time_pressure_with_stage_offsets():
    disc, ts = _setup()
    p_prev, d1, _, _, p_new = _history(disc, ts, np.random.default_rng(3), degree=1)
    assert np.allclose(guess.fallback(p_prev, d1), p_new, atol=1e-13)
