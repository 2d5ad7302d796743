"""Inputs, outputs and fallback of the learned pressure initial guess
(oracle; TEST INFRASTRUCTURE ONLY).

Not part of the paper.  For the Helmholtz solve of stage s, with beta_s,
right-hand side b = alpha_s M^p p_prev + F_p(u**) and the two latest pressure
increments (inc1 the newest, from a solve with beta1; inc2 with beta2):

* per cell K, f0 = mean_K(inc1) / (beta1 dt), f1 = mean_K(inc2) / (beta2 dt),
  where mean_K is the Gauss-rule cell average (sum of weight * nodal value);
* div_K = -(beta_s dt / |K|) sum_{i in K} (b_i - alpha_s (M^p p_prev)_i),
  i.e. -(beta_s dt / |K|) sum_{i in K} F_p(u**)_i, which is the cell average of
  div u** in flux form (the test functions of K sum to one);
* scales s_inc = RMS over cells of f0, s_div = RMS of div (1 where zero);
* network input, cell-lexicographic: [f0 / s_inc, f1 / s_inc, div / s_div];
* training target: mean_K(p_new - p_prev) / (beta_s dt) / s_inc;
* learned guess: p_prev + beta_s dt s_inc y_K on every node of K;
* fallback: p_prev + (beta_s / beta1) inc1, the newest increment rescaled to
  the stage.
"""
import numpy as np


def cell_average(disc, p):
    """Gauss-rule cell averages of a pressure vector ([cell][node] layout)."""
    w = np.ones(1)
    for _ in range(disc.dim):
        w = np.kron(disc.wp, w)
    return p.reshape(disc.Nc, disc.nbp) @ w


def _rms_or_one(v):
    r = float(np.sqrt(np.mean(v * v)))
    return r if r > 0.0 else 1.0


def features(ts, s, b, p_prev, inc1, beta1, inc2, beta2):
    """(x [3][cells], s_inc, s_div) for stage s of the stepper ``ts``."""
    disc = ts.disc
    dt = ts.dt
    f0 = cell_average(disc, inc1) / (beta1 * dt)
    f1 = cell_average(disc, inc2) / (beta2 * dt)
    Fp = b - ts.alpha(s) * (ts.Mp @ p_prev)
    vol = np.array([disc.cell_measure(c) for c in range(disc.Nc)])
    div = -(ts.beta[s] * dt / vol) * Fp.reshape(disc.Nc, disc.nbp).sum(axis=1)
    s_inc, s_div = _rms_or_one(f0), _rms_or_one(div)
    return np.stack([f0 / s_inc, f1 / s_inc, div / s_div]), s_inc, s_div


def target(ts, s, p_new, p_prev, s_inc):
    return cell_average(ts.disc, p_new - p_prev) / (ts.beta[s] * ts.dt) / s_inc


def inject(ts, s, p_prev, y, s_inc):
    return p_prev + np.repeat(ts.beta[s] * ts.dt * s_inc * np.asarray(y), ts.disc.nbp)


def fallback(ts, s, p_prev, inc1, beta1):
    return p_prev + (ts.beta[s] / beta1) * inc1
