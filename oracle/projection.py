"""The two single-stage projection schemes of Sec. 2 that the paper compares
with TR-BDF2 (oracle; test infrastructure): the Bell-Colella-Glaz method
(eq. momentum_BCG, helmholtz_BCG, Crank-Nicolson in time) and the
Guermond-Quartapelle method (eq. momentum_HI, helmholtz_HI, BDF2 in time),
on the same DG forms (Sec. 3) as the TR-BDF2 oracle.  Every system is solved
by sparse LU.

Both steps have the algebraic shape of one TR-BDF2 stage with its own
(beta, theta): momentum [ (1/(beta dt)) M + theta (nu A + C(w)) ] u* =
(1/(beta dt)) M u_base + F, projection u** = u* + beta dt M^{-1} P p^n,
Helmholtz [ alpha M^p + K ] p^{n+1} = alpha M^p p^n + (1/(beta dt)) D u**
with alpha = 1/(c^2 beta^2 dt^2), correction u^{n+1} = u** - beta dt
M^{-1} P p^{n+1}.

Bell-Colella-Glaz: beta = 1, theta = 1/2, u_base = u^n; F holds half the
explicit diffusion and advection of u^n (the unpenalised forms of eq. rhs1)
and the pressure term of p^n.  The advection is taken at the midpoint
velocity u^{n+1/2,*} = (u* + u^n)/2 in both halves (advecting field w =
u^{n+1/2,*}), so the predictor is nonlinear and is solved by fixed-point
iteration: the first solve is advected by the extrapolation
(3 u^n - u^{n-1})/2 to t^{n+1/2}, each later one by (u*_j + u^n)/2 of the
previous solution.

Guermond-Quartapelle BDF2: beta = 2/3, theta = 1, u_base = (4 u^n -
u^{n-1})/3, F the pressure term of p^n only; the advecting field is the
previous step's predictor u^{n,*} (one solve).

Readings
--------
* The BDF2 difference quotient is printed over dt; the consistent BDF2
  quotient is (3 u* - 4 u^n + u^{n-1}) / (2 dt).
* The BDF2 Helmholtz equation is printed with the coefficients of the
  Crank-Nicolson one (1/(c^2 dt^2), 1/dt); with the printed velocity update
  u^{n+1} = u** - (2/3) dt grad p^{n+1} only 1/(beta dt) with beta = 2/3
  makes u^{n+1} discretely divergence free in the incompressible limit, so
  both the Helmholtz coefficients and the divergence term use beta = 2/3.
* The BDF2 advecting field u^{n,*} is taken literally: the momentum
  predictor of the previous step (u^0 at the first step).  Its extrapolation
  2 u^n - u^{n-1} to t^{n+1}, the other natural reading, is unstable on the
  paper's Taylor-Green case at C = 1.63 with the Lax-Friedrichs form (the
  16 x 16 error grows to 0.18 against the printed 0.09), as the linearised
  TR-BDF2 stages are.
* The paper writes the advection of both schemes in non-conservative
  forms; the DG discretisation of Sec. 3 has one advection form, the
  conservative Lax-Friedrichs one, which both schemes use here with their
  advecting field.
* Dirichlet data of u* are those of t^{n+1} in both schemes.
* First step: the history level u^{-1} is supplied by the caller (the exact
  solution at t = -dt when one is known).
"""
import numpy as np

from .stepper import TRBDF2


class _SingleStage(TRBDF2):
    """A TR-BDF2 oracle whose stage 1 carries the scheme's (beta, theta)."""

    BETA = 1.0
    THETA = 1.0

    def __init__(self, disc, dt, uD=None, rows=None):
        super().__init__(disc, dt, uD=uD, rows=rows)
        self.beta = {1: self.BETA}
        self.theta = {1: self.THETA}

    def project(self, u_star, p_n):
        """Projection, Helmholtz solve and correction of the step."""
        bdt = self.beta[1] * self.dt
        u_ss = u_star + bdt * self.grad_p(p_n)
        b = self.rhs_pressure(1, u_ss, p_n)
        p_new = self.solve_pressure(1, b)
        u_new = u_ss - bdt * self.grad_p(p_new)
        return u_ss, b, p_new, u_new


class BCG(_SingleStage):
    """Bell-Colella-Glaz projection step (eq. momentum_BCG, helmholtz_BCG)."""

    BETA = 1.0
    THETA = 0.5

    def __init__(self, disc, dt, uD=None, rows=None, nonlinear_iters=10, nonlinear_tol=1e-12):
        super().__init__(disc, dt, uD=uD, rows=rows)
        if int(nonlinear_iters) < 1:
            raise ValueError("nonlinear_iters must be >= 1")
        self.nonlinear_iters = int(nonlinear_iters)
        self.nonlinear_tol = float(nonlinear_tol)

    def step(self, u_n, u_prev, p_n, t):
        """Advance (u^n, u^{n-1}, p^n) at time t by dt; returns (u^{n+1},
        u^n, p^{n+1}, intermediates)."""
        t1 = t + self.dt
        w = 1.5 * u_n - 0.5 * u_prev
        solves = 0
        while True:
            rhs = self.rhs_momentum(1, u_n, None, w, p_n, t1)
            u_star = self.solve_momentum(1, w, rhs, t1)
            solves += 1
            w_next = 0.5 * (u_star + u_n)
            change = np.linalg.norm(w_next - w)
            w_used = w
            w = w_next
            if solves >= self.nonlinear_iters or change <= self.nonlinear_tol * np.linalg.norm(w):
                break
        u_ss, b, p_new, u_new = self.project(u_star, p_n)
        return u_new, u_n, p_new, dict(w=w_used, rhs=rhs, u_star=u_star, u_ss=u_ss, b=b, p=p_new,
                                       u=u_new, solves=solves)


class BDF2GQ(_SingleStage):
    """Guermond-Quartapelle BDF2 projection step (eq. momentum_HI,
    helmholtz_HI)."""

    BETA = 2.0 / 3.0
    THETA = 1.0

    def rhs_momentum_bdf2(self, u_n, u_prev, w, p_n, t1):
        """(1/(beta dt)) M (4 u^n - u^{n-1}) / 3 + Gw p^n + boundary data."""
        d = self.disc
        F = self.Gw @ p_n
        if self.uD is not None and any(f[0] == "B" for f in d.faces()):
            F = F + d.dirichlet_rhs(1.0, w, self._uD_face(t1))
        return self.m(1) * (self.Mv @ ((4.0 * u_n - u_prev) / 3.0)) + F

    def step(self, u_n, u_prev, p_n, t, u_star_prev=None):
        """Advance (u^n, u^{n-1}, p^n) at time t by dt; ``u_star_prev`` is
        the previous step's predictor (None at the first step)."""
        t1 = t + self.dt
        w = u_n if u_star_prev is None else u_star_prev
        rhs = self.rhs_momentum_bdf2(u_n, u_prev, w, p_n, t1)
        u_star = self.solve_momentum(1, w, rhs, t1)
        u_ss, b, p_new, u_new = self.project(u_star, p_n)
        return u_new, u_n, p_new, dict(w=w, rhs=rhs, u_star=u_star, u_ss=u_ss, b=b, p=p_new,
                                       u=u_new, solves=1)
