"""Pins of the oracle's learned-guess inputs and outputs against closed forms.

* Gauss-rule cell averages are exact cell means for pressures the space holds;
* the divergence feature of an interpolated polynomial velocity equals the
  exact cell mean of its divergence (interior cells of a periodic mesh);
* the training target of an injected increment returns that increment;
* the rescaled previous increment is exact for pressures linear in time.
"""
import numpy as np

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


def test_cell_average_is_exact_mean():
    disc, _ = _setup()
    xp = disc.node_coords("p")
    p = xp[:, 0] ** 2 * xp[:, 1]
    avg = guess.cell_average(disc, p)
    for c in range(disc.Nc):
        x0, x1, y0, y1 = _cell_bounds(disc, c)
        exact = (x1 ** 3 - x0 ** 3) / (3 * (x1 - x0)) * 0.5 * (y0 + y1)
        assert abs(avg[c] - exact) < 1e-14


def test_divergence_feature_is_cell_mean_of_divergence():
    disc, ts = _setup()
    xu = disc.node_coords("u")
    u = np.stack([xu[:, 0] ** 2, xu[:, 0] * xu[:, 1]], 1)
    import synthetic
    us = synthetic.nodal_velocity(u, 2, disc.nbu)
    p_prev = np.random.default_rng(0).standard_normal(disc.N_p)
    for s in (1, 2):
        b = ts.rhs_pressure(s, us, p_prev)
        z = np.zeros(disc.N_p)
        x, s_inc, s_div = guess.features(ts, s, b, p_prev, z + 1.0, 0.5, z + 2.0, 0.25)
        div = x[2] * s_div
        n = disc.mesh.n_cells[0]
        for c in range(disc.Nc):
            i, j = disc.mesh.cell_ijk(c)
            if 0 < i < n - 1 and 0 < j < n - 1:
                x0, x1, _, _ = _cell_bounds(disc, c)
                assert abs(div[c] - 1.5 * (x0 + x1)) < 1e-11, (c, div[c])
        # the increment channels are the rescaled cell averages
        assert np.allclose(x[0] * s_inc, 1.0 / (0.5 * ts.dt)) and np.allclose(x[1] * s_inc, 2.0 / (0.25 * ts.dt))


def test_target_inverts_injection():
    disc, ts = _setup()
    rng = np.random.default_rng(1)
    p_prev = rng.standard_normal(disc.N_p)
    y = rng.standard_normal(disc.Nc)
    for s in (1, 2):
        p_new = guess.inject(ts, s, p_prev, y, 3.5)
        assert np.allclose(guess.target(ts, s, p_new, p_prev, 3.5), y, atol=1e-12)


def test_fallback_exact_for_linear_in_time_pressure():
    disc, ts = _setup()
    rng = np.random.default_rng(2)
    p0, q = rng.standard_normal(disc.N_p), rng.standard_normal(disc.N_p)
    g, dt = ts.cst["gamma"], ts.dt

    def p(t):
        return p0 + t * q

    tn = 0.3
    # stage 1 of step n: the newest increment came from stage 2 of step n-1
    inc1 = p(tn) - p(tn - (1 - g) * dt)
    assert np.allclose(guess.fallback(ts, 1, p(tn), inc1, 1 - g), p(tn + g * dt), atol=1e-13)
    # stage 2: the newest increment came from stage 1 of the same step
    inc1 = p(tn + g * dt) - p(tn)
    assert np.allclose(guess.fallback(ts, 2, p(tn + g * dt), inc1, g), p(tn + dt), atol=1e-13)
