"""Pins of the oracle's Bell-Colella-Glaz and Guermond-Quartapelle BDF2
projection steps (the comparison schemes of Sec. 2) against mathematics and
the paper's tables.

* on a shear flow that is free of advection and pressure (the projection is
  exact there), both steps reduce to their parent time integrators for the
  SIP heat equation and converge at second order in time;
* the coarsest rows of the paper's Q2-Q1 Taylor-Green tables for the two
  schemes (Sec. 4, C = 1.63): printed relative L2 velocity errors 0.48
  (Bell-Colella-Glaz) and 0.28 (BDF2), reproduced to 25 %; BCG's pressure
  (printed 0.41) as well;
* the BCG fixed point satisfies the Crank-Nicolson predictor equation with
  the advection at the midpoint velocity.
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import BCG, BDF2GQ, BoxMesh, Discretization


def _run(cls, d, dt, steps, u0, um1, p0, t0=0.0, **kw):
    ts = cls(d, dt, **kw)
    u, h, p, t = u0, um1, p0, t0
    ustar = None
    for _ in range(steps):
        if cls is BDF2GQ:
            u, h, p, st = ts.step(u, h, p, t, u_star_prev=ustar)
        else:
            u, h, p, st = ts.step(u, h, p, t)
        ustar = st["u_star"]
        t += dt
    return u, p, t


def _shear(cls, nst, T=0.4, nu=0.05):
    """u = (sin 2 pi y, 0) decaying as exp(-4 pi^2 nu t); degree 4 keeps the
    jump terms of the unpenalised explicit diffusion below the time error."""
    mesh = BoxMesh(2, (4, 4), (0.0, 0.0), (1.0, 1.0), (True, True))
    d = Discretization(mesh, 4, nu=nu)
    dt = T / nst
    xu = d.node_coords("u")

    def field(t):
        v = np.stack([np.sin(2 * math.pi * xu[:, 1]), 0 * xu[:, 0]], 1) * math.exp(-4 * math.pi ** 2 * nu * t)
        return synthetic.nodal_velocity(v, 2, d.nbu)
    u, p, _ = _run(cls, d, dt, nst, field(0.0), field(-dt), np.zeros(d.N_p))
    return u, p


@pytest.mark.parametrize("cls", [BCG, BDF2GQ], ids=["bcg", "bdf2"])
def test_shear_flow_second_order_in_time(cls):
    sols = {n: _shear(cls, n) for n in (4, 8, 16, 128)}
    for n in sols:
        assert np.ptp(sols[n][1]) < 1e-10          # no pressure gradient is generated
    e = [np.linalg.norm(sols[n][0] - sols[128][0]) for n in (4, 8, 16)]
    assert 3.3 < e[0] / e[1] < 4.8 and 3.3 < e[1] / e[2] < 4.8, e


def _paper_tg(cls, N, dt, T=3.2, Re=100.0, **kw):
    mesh = BoxMesh(2, (N, N), (0.0, 0.0), (2 * math.pi,) * 2, (True, True))
    d = Discretization(mesh, 2, nu=1.0 / Re, c=1.0e3)
    xu, xp = d.node_coords("u"), d.node_coords("p")
    U = lambda t: synthetic.nodal_velocity(synthetic.taylor_green_2d(xu, t, Re)[0], 2, d.nbu)
    u, p, t = _run(cls, d, dt, int(round(T / dt)), U(0.0), U(-dt),
                   synthetic.taylor_green_2d(xp, 0.0, Re)[1], **kw)
    eu, ru = d.l2_error(u, lambda x: synthetic.taylor_green_2d(x, t, Re)[0])
    ep, rp = d.l2_error(p, lambda x: synthetic.taylor_green_2d(x, t, Re)[1], "p", remove_mean=True)
    return eu / ru, ep / rp


def test_paper_bcg_table_coarsest():
    eu, ep = _paper_tg(BCG, 8, 0.64, nonlinear_iters=4)
    assert abs(eu / 0.48 - 1.0) < 0.25, eu
    assert abs(ep / 0.41 - 1.0) < 0.25, ep


def test_paper_bdf2_table_coarsest():
    eu, _ = _paper_tg(BDF2GQ, 8, 0.64)
    assert abs(eu / 0.28 - 1.0) < 0.25, eu


def test_bcg_fixed_point_is_the_midpoint_predictor():
    """[M/dt + (nu A + C(w))/2] u* = M u^n/dt + (-nu A0 u^n + A0_adv(w) u^n)/2
    + Gw p^n with w = (u* + u^n)/2 at the converged fixed point."""
    mesh = BoxMesh(2, (4, 4), (0.0, 0.0), (1.0, 1.0), (True, True))
    d = Discretization(mesh, 3, nu=0.01)
    dt = 0.02
    xu, xp = d.node_coords("u"), d.node_coords("p")
    u = synthetic.nodal_velocity(synthetic.taylor_green_2d_unit(xu, 0.0, 0.01)[0], 2, d.nbu)
    um1 = synthetic.nodal_velocity(synthetic.taylor_green_2d_unit(xu, -dt, 0.01)[0], 2, d.nbu)
    p = synthetic.taylor_green_2d_unit(xp, 0.0, 0.01)[1]
    ts = BCG(d, dt, nonlinear_iters=80, nonlinear_tol=1e-14)
    _, _, _, st = ts.step(u, um1, p, 0.0)
    assert st["solves"] < 80
    us = st["u_star"]
    w = 0.5 * (us + u)
    lhs = ts.per_component((1.0 / dt) * ts.M + 0.5 * (d.nu * ts.L + d.lf_advection(w)), us)
    rhs = ((1.0 / dt) * (ts.Mv @ u) - 0.5 * d.nu * ts.per_component(ts.L0, u)
           + 0.5 * ts.per_component(d.explicit_advection(w), u) + ts.Gw @ p)
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(rhs)
