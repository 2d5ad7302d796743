"""Inputs, outputs and fallback of the learned pressure initial guess
(oracle; TEST INFRASTRUCTURE ONLY).

Not part of the paper.  For the Helmholtz solve of stage s (beta_s, right-hand
side b = alpha_s M^p p_prev + F_p(u**)) with the two newest pressure
increments inc1 (the newest, from the other stage, weight beta1) and inc2
(the same stage one step earlier, weight beta2):

* per cell K, f0 = mean_K(inc1) / (beta1 dt), f1 = mean_K(inc2) / (beta2 dt),
  where mean_K is the Gauss-rule cell average (sum of weight * nodal value);
* div_K = -(beta_s dt / |K|) sum_{i in K} (b_i - alpha_s (M^p p_prev)_i),
  i.e. -(beta_s dt / |K|) sum_{i in K} F_p(u**)_i, which is the cell average of
  div u** in flux form (the test functions of K sum to one);
* scales s_inc = RMS over cells of f0, s_div = RMS of div (1 where zero);
* network input, cell-lexicographic: [f0 / s_inc, f1 / s_inc, div / s_div];
* fallback: p_prev + inc2 (the pressures of the two stages carry different
  offsets, so the other stage's increment predicts poorly);
* the network predicts the cell averages of the correction to the fallback,
  training target mean_K(p_new - p_prev - inc2) / (beta_s dt) / s_inc;
* learned guess: fallback + beta_s dt s_inc I(y), I the multilinear
  interpolation of the cell values from the cell centres (periodic) to the
  nodes, so the correction is continuous.
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


def target(ts, s, p_new, p_prev, inc2, s_inc):
    return cell_average(ts.disc, p_new - p_prev - inc2) / (ts.beta[s] * ts.dt) / s_inc


def interpolate_centres(disc, y):
    """Multilinear interpolation of cell values (located at the cell centres,
    periodic) to the pressure nodes, [cell][node] layout."""
    mesh = disc.mesh
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros(disc.N_p)
    z = disc.zp
    for c in range(disc.Nc):
        ijk = mesh.cell_ijk(c)
        for node in range(disc.nbp):
            loc = [(node // disc.n_p ** a) % disc.n_p for a in range(disc.dim)]
            lo, w = [], []
            for a in range(disc.dim):
                X = ijk[a] + z[loc[a]] - 0.5          # position in cell-centre units
                i0 = int(np.floor(X))
                lo.append(i0)
                w.append(X - i0)
            val = 0.0
            for corner in range(2 ** disc.dim):
                wt, idx = 1.0, []
                for a in range(disc.dim):
                    bit = (corner >> a) & 1
                    wt *= w[a] if bit else 1.0 - w[a]
                    idx.append((lo[a] + bit) % mesh.n_cells[a])
                val += wt * y[mesh.cell_index(idx)]
            out[c * disc.nbp + node] = val
    return out


def inject(ts, s, p_prev, inc2, y, s_inc):
    return fallback(p_prev, inc2) + ts.beta[s] * ts.dt * s_inc * interpolate_centres(ts.disc, y)


def fallback(p_prev, inc2):
    return p_prev + inc2
