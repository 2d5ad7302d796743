"""TR-BDF2 projection step in algebraic form (oracle; test infrastructure).

Follows Sec. 2 (eq. trbdf2, first_stage, discpress, helmholtz2a,
second_stage, discpress2, helmholtz3a) in the algebraic form at the end of
Sec. 3: per stage s, with (beta_1, theta_1) = (gamma, 1/2) and
(beta_2, theta_2) = (1 - gamma, a33),

    momentum   [ m_s M + theta_s (nu A + C(w_s)) ] u*   = m_s M u_prev + F_u^(s)
    projection u**  = u* + beta_s dt M^{-1} P p_prev
    Helmholtz  [ alpha_s M^p + K ] p_new = alpha_s M^p p_prev + F_p^(s)(u**)
    correction u_new = u** - beta_s dt M^{-1} P p_new

with m_s = 1/(beta_s dt) and alpha_s = 1/(c^2 beta_s^2 dt^2).  Every system
is solved by sparse LU (scipy ``splu``), i.e. the discrete stage solution is
reached to rounding, not to a Krylov tolerance.

Readings
--------
* Advecting velocity of stage 1: the printed extrapolation weights
  (1 + gamma/(2(1-gamma)), -gamma/(2(1-gamma))) reach the stage midpoint
  t^n + gamma dt/2 to second order only when the older level is the previous
  step's stage value u^{n-1+gamma}; that is the default (``extrap1='stage'``);
  ``extrap1='step'`` uses the literal u^{n-1}.
* Advecting velocity of stage 2: the printed weights sum to 3; the sign of
  the first is read as a typo, giving (1 + (1-gamma)/gamma) u^{n+gamma}
  - ((1-gamma)/gamma) u^n, the linear extrapolation to t^{n+1}.
* Stage-1 correction: written with the stage-2 quantity
  u~^{n+1,**}; read as u^{n+gamma} = u* - gamma dt M^{-1} P (p^{n+gamma} - p^n),
  mirroring stage 2.  Stage-2 Helmholtz "given p^n" is read as p^{n+gamma}.
* First step: the history level u^{-1+gamma} is supplied by the caller
  (the exact solution at t = -(1-gamma) dt when one is known).

Fully nonlinear stages
----------------------
Sec. 2 also allows the advecting velocity of each momentum predictor to be
the unknown itself, found by fixed-point iteration (stage 1: the implicit
advection is advected by u^{n+gamma,*} and the explicit one by u^n).  With
``nonlinear_iters`` = m > 1 a stage does up to m momentum solves: the first
advected by the extrapolated velocity, each later one by the previous
solution, stopping early once ||u*_j - u*_{j-1}||_2 <= nonlinear_tol ||u*_j||_2;
the stage-1 explicit advection then uses u^n throughout.  m = 1 is the
linearised scheme above.
"""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def trbdf2_constants(gamma=None):
    """gamma, a31, a32, a33 of eq. trbdf2 / second_stage and the two pairs of
    extrapolation weights for the advecting velocity (readings above)."""
    g = 2.0 - math.sqrt(2.0) if gamma is None else float(gamma)
    a31 = (1.0 - g) / (2.0 * (2.0 - g))
    a32 = (1.0 - g) / (2.0 * (2.0 - g))
    a33 = 1.0 / (2.0 - g)
    e1 = (1.0 + g / (2.0 * (1.0 - g)), -g / (2.0 * (1.0 - g)))
    e2 = (1.0 + (1.0 - g) / g, -(1.0 - g) / g)
    return dict(gamma=g, a31=a31, a32=a32, a33=a33, extrap1=e1, extrap2=e2)


def trbdf2_scalar_step(lam, y, dt, gamma=None):
    """One TR-BDF2 step (eq. trbdf2) of the scalar linear problem y' = lam y.

    Stage 1 (trapezoidal rule to t^n + gamma dt):
        (y_g - y) / (gamma dt) = (lam y_g + lam y) / 2
    Stage 2 (BDF2-like to t^{n+1}):
        (y_1 - y_g) / ((1-gamma) dt) = a33 lam y_1 + a32 lam y_g + a31 lam y
    """
    cst = trbdf2_constants(gamma)
    g = cst["gamma"]
    y_g = (y + 0.5 * g * dt * lam * y) / (1.0 - 0.5 * g * dt * lam)
    h2 = (1.0 - g) * dt
    rhs = y_g + h2 * lam * (cst["a32"] * y_g + cst["a31"] * y)
    return rhs / (1.0 - h2 * cst["a33"] * lam)


class TRBDF2:
    """Stage operators, right-hand sides and the full step for one mesh.

    ``uD(x, t) -> (npnt, dim)`` supplies Dirichlet data on boundary faces
    (unused on fully periodic meshes).
    """

    def __init__(self, disc, dt, gamma=None, uD=None, extrap1="stage", rows=None,
                 nonlinear_iters=1, nonlinear_tol=0.0):
        """``rows``: optional list of cells; when given, every operator is
        assembled only for the test functions of those cells (results are
        valid on those cells' entries only), which keeps large meshes cheap
        for sampled comparisons."""
        self.disc = disc
        self.rows = rows
        self.dt = float(dt)
        self.cst = trbdf2_constants(gamma)
        self.uD = uD
        self.extrap1 = extrap1
        if int(nonlinear_iters) < 1:
            raise ValueError("nonlinear_iters must be >= 1")
        self.nonlinear_iters = int(nonlinear_iters)
        self.nonlinear_tol = float(nonlinear_tol)
        g = self.cst["gamma"]
        self.beta = {1: g, 2: 1.0 - g}
        self.theta = {1: 0.5, 2: self.cst["a33"]}
        d = disc
        r = rows
        self.M = d.mass_u(r)
        self.Mv = d.mass_u_vector(r)
        self.Mp = d.mass_p(r)
        self.L = d.sip_u(r)
        self.K = d.sip_p(r)
        self.L0 = d.explicit_diffusion(r)
        self.Gw = d.weak_gradient(r)
        self.D = d.divergence(r)
        self.P = d.projection(r)
        mdiag = self.Mv.diagonal()
        if abs(sp.linalg.norm(self.Mv - sp.diags(mdiag))) > 0.0:
            raise AssertionError("velocity mass matrix is expected to be diagonal")
        # M^{-1} P: the projection of the broken pressure gradient into V_h
        inv = np.zeros_like(mdiag)
        inv[mdiag != 0.0] = 1.0 / mdiag[mdiag != 0.0]
        self.G = sp.diags(inv) @ self.P

    # -- coefficients ------------------------------------------------------
    def m(self, s):
        return 1.0 / (self.beta[s] * self.dt)

    def alpha(self, s):
        if math.isinf(self.disc.c):
            return 0.0
        return 1.0 / (self.disc.c ** 2 * self.beta[s] ** 2 * self.dt ** 2)

    # -- helpers -----------------------------------------------------------
    def per_component(self, A, u):
        d = self.disc.dim
        U = u.reshape(self.disc.Nc, d, self.disc.nbu)
        out = np.empty_like(U)
        for a in range(d):
            out[:, a, :] = (A @ U[:, a, :].reshape(-1)).reshape(self.disc.Nc, self.disc.nbu)
        return out.reshape(-1)

    def _uD_face(self, t):
        if self.uD is None:
            return None
        return lambda c, a, s, x: self.uD(x, t)

    # -- operators -----------------------------------------------------------
    def momentum_scalar(self, s, w, t_stage=None):
        """m_s M + theta_s (nu A + C(w)) for one component."""
        C = self.disc.lf_advection(w, self._uD_face(t_stage), self.rows)
        return (self.m(s) * self.M + self.theta[s] * (self.disc.nu * self.L + C)).tocsr()

    def pressure_matrix(self, s):
        return (self.alpha(s) * self.Mp + self.K).tocsr()

    def apply_momentum(self, s, w, u, t_stage=None):
        return self.per_component(self.momentum_scalar(s, w, t_stage), u)

    def apply_pressure(self, s, p):
        return self.pressure_matrix(s) @ p

    def diag_momentum(self, s, w, t_stage=None):
        """Diagonal of the scalar momentum operator (same for every component),
        in the [cell][node] layout."""
        return self.momentum_scalar(s, w, t_stage).diagonal()

    def diag_pressure(self, s):
        return self.pressure_matrix(s).diagonal()

    def grad_p(self, p):
        return self.G @ p

    def extrapolate(self, s, u_new, u_old):
        e = self.cst["extrap1"] if s == 1 else self.cst["extrap2"]
        return e[0] * u_new + e[1] * u_old

    def rhs_momentum(self, s, u_n, u_g, w, p_prev, t_stage=None, w_explicit=None):
        """m_s M u_prev + F_u^(s) (eq. rhs1 and its stage-2 analogue).

        Stage 1: u_prev = u_n, advecting field w (``w_explicit``, when given,
        replaces it in the explicit advection only).  Stage 2: u_prev = u_g
        (= u^{n+gamma}); the explicit advection uses u_g (x) u_g with a32 and
        u_n (x) u_n with a31; w enters only through the boundary terms.
        """
        d = self.disc
        nu = d.nu
        if s == 1:
            th = self.theta[1]
            A0 = d.explicit_advection(w if w_explicit is None else w_explicit, self.rows)
            F = (-th * nu * self.per_component(self.L0, u_n)
                 + th * self.per_component(A0, u_n))
            u_prev = u_n
        else:
            a31, a32 = self.cst["a31"], self.cst["a32"]
            F = (-nu * a32 * self.per_component(self.L0, u_g)
                 - nu * a31 * self.per_component(self.L0, u_n)
                 + a32 * self.per_component(d.explicit_advection(u_g, self.rows), u_g)
                 + a31 * self.per_component(d.explicit_advection(u_n, self.rows), u_n))
            u_prev = u_g
        F = F + self.Gw @ p_prev
        if self.uD is not None and any(f[0] == "B" for f in d.faces()):
            F = F + d.dirichlet_rhs(self.theta[s], w, self._uD_face(t_stage))
        return self.m(s) * (self.Mv @ u_prev) + F

    def rhs_pressure(self, s, u_ss, p_prev):
        """alpha_s M^p p_prev + F_p^(s)(u**)."""
        return (self.alpha(s) * (self.Mp @ p_prev)
                + (1.0 / (self.beta[s] * self.dt)) * (self.D @ u_ss))

    # -- solves --------------------------------------------------------------
    def solve_momentum(self, s, w, rhs, t_stage=None):
        lu = spla.splu(self.momentum_scalar(s, w, t_stage).tocsc())
        d = self.disc
        R = rhs.reshape(d.Nc, d.dim, d.nbu)
        out = np.empty_like(R)
        for a in range(d.dim):
            out[:, a, :] = lu.solve(R[:, a, :].reshape(-1)).reshape(d.Nc, d.nbu)
        return out.reshape(-1)

    def solve_pressure(self, s, rhs):
        H = self.pressure_matrix(s)
        if self.alpha(s) == 0.0:
            raise NotImplementedError("pure Poisson (c = inf) is not supported by the oracle")
        return spla.splu(H.tocsc()).solve(rhs)

    # -- one stage / one step ------------------------------------------------
    def stage(self, s, u_n, u_hist, u_g, p_prev, t):
        """One TR-BDF2 stage; returns a dict of every intermediate vector."""
        g = self.cst["gamma"]
        if s == 1:
            w = self.extrapolate(1, u_n, u_hist)
            t_stage = t + g * self.dt
            u_prev = u_n
        else:
            w = self.extrapolate(2, u_g, u_n)
            t_stage = t + self.dt
            u_prev = u_g
        solves = 1
        if self.nonlinear_iters == 1:
            rhs = self.rhs_momentum(s, u_n, u_g, w, p_prev, t_stage)
            u_star = self.solve_momentum(s, w, rhs, t_stage)
        else:
            w_ex = u_n if s == 1 else None
            rhs = self.rhs_momentum(s, u_n, u_g, w, p_prev, t_stage, w_explicit=w_ex)
            u_star = self.solve_momentum(s, w, rhs, t_stage)
            while solves < self.nonlinear_iters:
                w = u_star
                rhs = self.rhs_momentum(s, u_n, u_g, w, p_prev, t_stage, w_explicit=w_ex)
                u_star = self.solve_momentum(s, w, rhs, t_stage)
                solves += 1
                change = np.linalg.norm(u_star - w)
                if change <= self.nonlinear_tol * np.linalg.norm(u_star):
                    break
        bdt = self.beta[s] * self.dt
        u_ss = u_star + bdt * self.grad_p(p_prev)
        b = self.rhs_pressure(s, u_ss, p_prev)
        p_new = self.solve_pressure(s, b)
        u_new = u_ss - bdt * self.grad_p(p_new)
        return dict(w=w, rhs=rhs, u_star=u_star, u_ss=u_ss, b=b,
                    p=p_new, u=u_new, u_prev=u_prev, solves=solves)

    def step(self, u_n, u_hist, p_n, t):
        """Advance (u^n, u^{n-1+gamma}, p^n) at time t by dt.

        Returns (u^{n+1}, history, p^{n+1}, stages); the history level for
        the next step's stage-1 extrapolation is u^{n+gamma} (default reading)
        or u^n (literal reading).
        """
        st1 = self.stage(1, u_n, u_hist, None, p_n, t)
        st2 = self.stage(2, u_n, None, st1["u"], st1["p"], t)
        hist = st1["u"] if self.extrap1 == "stage" else u_n
        return st2["u"], hist, st2["p"], (st1, st2)
