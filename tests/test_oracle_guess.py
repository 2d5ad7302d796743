"""Pins of the oracle's learned-guess inputs and outputs against closed forms.

* Gauss-rule cell averages are exact cell means for pressures the space holds;
* the divergence feature of an interpolated polynomial velocity equals the
  exact cell mean of its divergence (interior cells of a periodic mesh);
* the multilinear interpolation of cell-centre values reproduces linear data,
  and the target of an injected correction returns it;
* the same-stage increment of the previous step is exact for pressures that
  are linear in time up to a constant offset per stage.
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


def test_interpolation_and_target_reproduce_linear_cell_data():
    """Cell values linear in the cell index are reproduced exactly by the
    multilinear interpolation away from the periodic seam, and the target of
    the injected correction returns them (the cell mean of a linear function
    is its centre value); a constant is reproduced everywhere."""
    disc, ts = _setup(n=6)
    rng = np.random.default_rng(1)
    p_prev, inc2 = rng.standard_normal(disc.N_p), rng.standard_normal(disc.N_p)
    n = disc.mesh.n_cells[0]
    ij = np.array([disc.mesh.cell_ijk(c) for c in range(disc.Nc)])
    y = 0.3 + 0.7 * ij[:, 0] - 0.2 * ij[:, 1]
    inner = (ij[:, 0] > 0) & (ij[:, 0] < n - 1) & (ij[:, 1] > 0) & (ij[:, 1] < n - 1)
    for s in (1, 2):
        pg = guess.inject(ts, s, p_prev, inc2, y, 3.5)
        tgt = guess.target(ts, s, pg, p_prev, inc2, 3.5)
        assert np.allclose(tgt[inner], y[inner], atol=1e-12)
        const = guess.inject(ts, s, p_prev, inc2, np.full(disc.Nc, 2.0), 3.5)
        assert np.allclose(const - p_prev - inc2, ts.beta[s] * ts.dt * 3.5 * 2.0, atol=1e-13)


def test_fallback_exact_for_linear_in_time_pressure_with_stage_offsets():
    """p = P(t) + o_s with P linear in time and a constant offset per stage:
    the same-stage increment of the previous step predicts exactly."""
    disc, ts = _setup()
    rng = np.random.default_rng(2)
    p0, q, o1, o2 = (rng.standard_normal(disc.N_p) for _ in range(4))
    g, dt = ts.cst["gamma"], ts.dt

    def p(t, o):
        return p0 + t * q + o

    tn = 0.3
    # stage 1 of step n: p_prev = p^n (a stage-2 value), inc2 = p^{n-1+g} - p^{n-1}
    inc2 = p(tn - (1 - g) * dt, o1) - p(tn - dt, o2)
    assert np.allclose(guess.fallback(p(tn, o2), inc2), p(tn + g * dt, o1), atol=1e-13)
    # stage 2: p_prev = p^{n+g}, inc2 = p^n - p^{n-1+g}
    inc2 = p(tn, o2) - p(tn - (1 - g) * dt, o1)
    assert np.allclose(guess.fallback(p(tn + g * dt, o1), inc2), p(tn + dt, o2), atol=1e-13)
