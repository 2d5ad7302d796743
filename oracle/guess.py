"""Inputs, outputs and fallback of the learned pressure initial guess
(oracle; TEST INFRASTRUCTURE ONLY).

Not part of the paper.  For the Helmholtz solve of stage s (beta_s, right-hand
side b = alpha_s M^p p_prev + F_p(u**)) the solver keeps the pressure
increments p_new - p_prev of its earlier solves: d1, d2 and d3 of the same
stage one, two and three steps back, d0 the newest one (of the other stage,
weight beta0).  With <a, b>_K = sum_{i in K} W_i a_i b_i (W_i the product of the
Gauss weights of node i on the unit reference cell, so <a, 1>_K is the cell
average mean_K(a)):

* network input per cell K (6 channels, cell-lexicographic):
    m1 / s_inc, m2 / s_inc, m0 / s_inc, div / s_div, cos_K, lr_K
  with m1 = mean_K(d1) / (beta_s dt), m2 = mean_K(d2) / (beta_s dt),
  m0 = mean_K(d0) / (beta0 dt), div_K = -(beta_s dt / |K|) sum_{i in K}
  (b_i - alpha_s (M^p p_prev)_i) (the cell average of div u** in flux
  form), s_inc and s_div the RMS over cells of m1 and div (1 where zero),
  cos_K = <d1, d2>_K / sqrt(<d1, d1>_K <d2, d2>_K) and
  lr_K = log(<d1, d1>_K / <d2, d2>_K) / 2 clamped to [-4, 4] (both 0 where
  a norm vanishes): the local shape and growth of the last two increments;
* network output per cell: (y0_K, y1_K), a correction along the last two
  increments of the increment extrapolated quadratically from its last
  three values, guess = p_prev + (3 + y0_K) d1 - (3 - y1_K) d2 + d3 at the
  nodes of K (y = 0: the quadratic extrapolation); the library starts the
  network's last layer at zero, i.e. from the extrapolation;
* training target: per cell the Gram data of the error
  e = p_new - (p_prev + 3 d1 - 3 d2 + d3) of the extrapolation,
    (g11, g12, g22, r1, r2, ee) = (<d1,d1>, <d1,d2>, <d2,d2>, <e,d1>, <e,d2>,
    <e,e>)_K / S,  S = the mean over cells of <d1,d1>_K (1 where zero),
  so that the squared error of the blended guess in cell K is
    l_K(y) = ee - 2 (y0 r1 + y1 r2) + y0^2 g11 + 2 y0 y1 g12 + y1^2 g22
  (times S); the loss is the mean of l_K over cells and samples.
"""
import numpy as np

LR_CLAMP = 4.0


def node_weights(disc):
    """W_i of the pressure nodes of one cell ([node] lexicographic, x fastest)."""
    w = np.ones(1)
    for _ in range(disc.dim):
        w = np.kron(disc.wp, w)
    return w


def cell_average(disc, p):
    """Gauss-rule cell averages of a pressure vector ([cell][node] layout)."""
    return p.reshape(disc.Nc, disc.nbp) @ node_weights(disc)


def cell_inner(disc, a, b):
    """<a, b>_K per cell: the Gauss-rule cell average of the product."""
    return (a.reshape(disc.Nc, disc.nbp) * b.reshape(disc.Nc, disc.nbp)) @ node_weights(disc)


def _rms_or_one(v):
    r = float(np.sqrt(np.mean(v * v)))
    return r if r > 0.0 else 1.0


def shape_features(disc, d1, d2):
    """(cos_K, lr_K) of the last two same-stage increments."""
    g11, g22, g12 = cell_inner(disc, d1, d1), cell_inner(disc, d2, d2), cell_inner(disc, d1, d2)
    ok = (g11 > 0.0) & (g22 > 0.0)
    cos = np.zeros(disc.Nc)
    lr = np.zeros(disc.Nc)
    cos[ok] = g12[ok] / np.sqrt(g11[ok] * g22[ok])
    lr[ok] = np.clip(0.5 * np.log(g11[ok] / g22[ok]), -LR_CLAMP, LR_CLAMP)
    return cos, lr


def features(ts, s, b, p_prev, d0, beta0, d1, d2):
    """(x [6][cells], s_inc, s_div) for stage s of the stepper ``ts``."""
    disc = ts.disc
    dt = ts.dt
    bs = ts.beta[s]
    m1 = cell_average(disc, d1) / (bs * dt)
    m2 = cell_average(disc, d2) / (bs * dt)
    m0 = cell_average(disc, d0) / (beta0 * dt)
    Fp = b - ts.alpha(s) * (ts.Mp @ p_prev)
    vol = np.array([disc.cell_measure(c) for c in range(disc.Nc)])
    div = -(bs * dt / vol) * Fp.reshape(disc.Nc, disc.nbp).sum(axis=1)
    s_inc, s_div = _rms_or_one(m1), _rms_or_one(div)
    cos, lr = shape_features(disc, d1, d2)
    return np.stack([m1 / s_inc, m2 / s_inc, m0 / s_inc, div / s_div, cos, lr]), s_inc, s_div


def gram_target(disc, p_new, p_prev, d1, d2, d3):
    """[6][cells]: (g11, g12, g22, r1, r2, ee) / S (module docstring)."""
    e = p_new - extrapolate3(p_prev, d1, d2, d3)
    g11 = cell_inner(disc, d1, d1)
    S = float(np.mean(g11))
    S = S if S > 0.0 else 1.0
    return np.stack([g11, cell_inner(disc, d1, d2), cell_inner(disc, d2, d2), cell_inner(disc, e, d1),
                     cell_inner(disc, e, d2), cell_inner(disc, e, e)]) / S


def inject(disc, p_prev, d1, d2, d3, y):
    """p_prev + (3 + y0_K) d1 - (3 - y1_K) d2 + d3 with y = [2][cells]."""
    a = np.repeat(np.asarray(y[0], dtype=np.float64), disc.nbp)
    c = np.repeat(np.asarray(y[1], dtype=np.float64), disc.nbp)
    return extrapolate3(p_prev, d1, d2, d3) + a * d1 + c * d2


def fallback(p_prev, d1):
    return p_prev + d1


def extrapolate2(p_prev, d1, d2):
    """The same-stage increment extrapolated linearly from its last two values."""
    return p_prev + 2.0 * d1 - d2


def extrapolate3(p_prev, d1, d2, d3):
    """The same-stage increment extrapolated quadratically from its last three
    values (the parabola through them evaluated one step on)."""
    return p_prev + 3.0 * d1 - 3.0 * d2 + d3


def quad_loss(y, G):
    """Mean over cells (and leading batch axes) of l_K(y) and its gradient.
    y: [..., 2, N], G: [..., 6, N]."""
    y0, y1 = y[..., 0, :], y[..., 1, :]
    g11, g12, g22, r1, r2, ee = (G[..., i, :] for i in range(6))
    lk = ee - 2.0 * (y0 * r1 + y1 * r2) + y0 * y0 * g11 + 2.0 * y0 * y1 * g12 + y1 * y1 * g22
    count = lk.size
    dy = np.empty_like(y, dtype=np.float64)
    dy[..., 0, :] = 2.0 * (y0 * g11 + y1 * g12 - r1) / count
    dy[..., 1, :] = 2.0 * (y0 * g12 + y1 * g22 - r2) / count
    return float(np.mean(lk)), dy
