"""Pins of the oracle's TR-BDF2 stepper against mathematics.

* the scalar TR-BDF2 map of eq. trbdf2 is second order and L-stable with
  gamma = 2 - sqrt(2) (the properties the paper states for it);
* the full projection step converges at second order in time in the
  Stokes regime (tiny amplitude, so the nonlinear terms vanish);
* the full step converges in space to the exact Taylor-Green vortex;
* the periodic Helmholtz step preserves the pressure mean exactly.
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import BoxMesh, Discretization, TRBDF2, trbdf2_constants, trbdf2_scalar_step


def test_scalar_trbdf2_order_and_l_stability():
    errs = []
    for z in (0.1, 0.05, 0.025):
        errs.append(abs(trbdf2_scalar_step(z, 1.0, 1.0) - math.exp(z)))
    # local error O(z^3): halving z divides it by ~8
    assert 7.0 < errs[0] / errs[1] < 9.0 and 7.0 < errs[1] / errs[2] < 9.0
    # L-stability: R(z) -> 0 as z -> -infinity, |R| <= 1 on the negative axis
    assert abs(trbdf2_scalar_step(-1e12, 1.0, 1.0)) < 1e-10
    for z in -np.logspace(-3, 6, 50):
        assert abs(trbdf2_scalar_step(z, 1.0, 1.0)) <= 1.0
    # A-stability along the imaginary axis
    for y in np.logspace(-3, 4, 40):
        assert abs(trbdf2_scalar_step(1j * y, 1.0, 1.0)) <= 1.0 + 1e-14


def test_constants_consistency():
    c = trbdf2_constants()
    assert abs(c["gamma"] - (2 - math.sqrt(2))) < 1e-16
    # stage-2 weights integrate a constant exactly
    assert abs(c["a31"] + c["a32"] + c["a33"] - 1.0) < 1e-15
    # both extrapolations reproduce constants
    for e in (c["extrap1"], c["extrap2"]):
        assert abs(e[0] + e[1] - 1.0) < 1e-15


def _tg_run(N, k, nu, dt, nst, amp=1.0):
    mesh = BoxMesh(2, (N, N), (0.0, 0.0), (1.0, 1.0), (True, True))
    d = Discretization(mesh, k, nu=nu)
    ts = TRBDF2(d, dt)
    g = ts.cst["gamma"]
    xu = d.node_coords("u")
    xp = d.node_coords("p")
    u = amp * synthetic.nodal_velocity(synthetic.taylor_green_2d_unit(xu, 0.0, nu)[0], 2, d.nbu)
    hist = amp * synthetic.nodal_velocity(synthetic.taylor_green_2d_unit(xu, -(1 - g) * dt, nu)[0], 2, d.nbu)
    p = amp * amp * synthetic.taylor_green_2d_unit(xp, 0.0, nu)[1]
    t = 0.0
    means = []
    for _ in range(nst):
        pm = float(ts.Mp.diagonal() @ p)
        u, hist, p, _st = ts.step(u, hist, p, t)
        means.append((pm, float(ts.Mp.diagonal() @ p)))
        t += dt
    return d, u, p, t, means


def _shear_run(nst, T, nu=0.05):
    """u = (sin 2 pi y, 0): discretely divergence free and free of advection,
    so the projection step is exact and the stages reduce to TR-BDF2 for
    the SIP heat equation; the exact decay is exp(-4 pi^2 nu t).

    The explicit diffusion of the stage right-hand sides carries no penalty
    (eq. rhs1), so it differs from the implicit SIP operator by terms in the
    inter-element jumps; degree 4 keeps those jumps far below the time error
    so that the order of the stage weights is visible."""
    mesh = BoxMesh(2, (4, 4), (0.0, 0.0), (1.0, 1.0), (True, True))
    d = Discretization(mesh, 4, nu=nu)
    dt = T / nst
    ts = TRBDF2(d, dt)
    g = ts.cst["gamma"]
    xu = d.node_coords("u")
    def field(t):
        v = np.stack([np.sin(2 * math.pi * xu[:, 1]), 0 * xu[:, 0]], 1) * math.exp(-4 * math.pi ** 2 * nu * t)
        return synthetic.nodal_velocity(v, 2, d.nbu)
    u, hist, p = field(0.0), field(-(1 - g) * dt), np.zeros(d.N_p)
    t = 0.0
    for _ in range(nst):
        u, hist, p, _st = ts.step(u, hist, p, t)
        t += dt
    return u, p


def test_shear_flow_second_order_in_time():
    T = 0.4
    sols = {n: _shear_run(n, T) for n in (4, 8, 16, 128)}
    for n in sols:
        assert np.ptp(sols[n][1]) < 1e-10          # no pressure gradient is generated
    e = [np.linalg.norm(sols[n][0] - sols[128][0]) for n in (4, 8, 16)]
    assert 3.5 < e[0] / e[1] < 4.6 and 3.5 < e[1] / e[2] < 4.6, e


@pytest.mark.slow
def test_taylor_green_space_convergence_and_mean():
    nu = 0.01
    errs = []
    for N in (4, 8):
        d, u, p, t, means = _tg_run(N, 3, nu, 0.002, 10)
        eu, ru = d.l2_error(u, lambda x: synthetic.taylor_green_2d_unit(x, t, nu)[0])
        errs.append(eu / ru)
        for before, after in means:
            assert abs(after - before) < 1e-12
    assert errs[1] < 5e-3 and errs[0] / errs[1] > 6.0, errs


def _paper_tg(N, k, dt, m, T=3.2, Re=100.0):
    """The 2D Taylor-Green convergence case of Sec. 4 (eq. greentaylor on
    (0, 2 pi)^2, Re = 100, c = 1e3, t = 0 .. 3.2) with fully nonlinear stages
    of at most m solves; returns the relative L2 errors of u and p (mean
    removed) at T."""
    mesh = BoxMesh(2, (N, N), (0.0, 0.0), (2 * math.pi,) * 2, (True, True))
    d = Discretization(mesh, k, nu=1.0 / Re, c=1.0e3)
    ts = TRBDF2(d, dt, nonlinear_iters=m)
    g = ts.cst["gamma"]
    xu, xp = d.node_coords("u"), d.node_coords("p")
    U = lambda t: synthetic.nodal_velocity(synthetic.taylor_green_2d(xu, t, Re)[0], 2, d.nbu)
    u, hist, p = U(0.0), U(-(1 - g) * dt), synthetic.taylor_green_2d(xp, 0.0, Re)[1]
    t = 0.0
    for _ in range(int(round(T / dt))):
        u, hist, p, st = ts.step(u, hist, p, t)
        assert st[0]["solves"] == m and st[1]["solves"] == m
        t += dt
    eu, ru = d.l2_error(u, lambda x: synthetic.taylor_green_2d(x, t, Re)[0])
    ep, rp = d.l2_error(p, lambda x: synthetic.taylor_green_2d(x, t, Re)[1], "p", remove_mean=True)
    return eu / ru, ep / rp


def test_paper_taylor_green_table_coarsest():
    """Coarsest row of the paper's Q2-Q1 Taylor-Green table at C = 1.63
    (8 x 8 cells, dt = 0.64): printed relative L2 errors 0.38 (velocity) and
    0.43 (pressure).  Reproduced to 25 % with three fixed-point solves per
    stage; the readings of the quadrature and of the projection differ from
    the paper's implementation, so the digits are not expected to agree."""
    eu, ep = _paper_tg(8, 2, 0.64, 3)
    assert abs(eu / 0.38 - 1.0) < 0.25, eu
    assert abs(ep / 0.43 - 1.0) < 0.25, ep


@pytest.mark.slow
def test_paper_taylor_green_table_second_row_velocity():
    """Second row (16 x 16, dt = 0.32): printed velocity error 0.095, i.e. a
    rate near 2 from the first row.  The velocity is reproduced to 25 % and
    the observed rate lies between 1.5 and 3."""
    e8, _ = _paper_tg(8, 2, 0.64, 3)
    e16, _ = _paper_tg(16, 2, 0.32, 3)
    assert abs(e16 / 0.095 - 1.0) < 0.25, e16
    assert 1.5 < math.log2(e8 / e16) < 3.0, (e8, e16)


def test_nonlinear_stage_solves_the_nonlinear_equation():
    """With enough fixed-point solves the stage-1 predictor satisfies the
    trapezoidal stage equation of eq. first_stage with the advecting
    velocity replaced by the unknown on the left and by u^n on the right:
    [m M + (nu A + C(u*))/2] u* = m M u^n + (-nu A0 + A0_adv(u^n)) u^n / 2 + Gw p^n."""
    mesh = BoxMesh(2, (4, 4), (0.0, 0.0), (1.0, 1.0), (True, True))
    d = Discretization(mesh, 3, nu=0.01)
    dt = 0.01
    ts = TRBDF2(d, dt, nonlinear_iters=60, nonlinear_tol=1e-14)
    g = ts.cst["gamma"]
    xu, xp = d.node_coords("u"), d.node_coords("p")
    u = synthetic.nodal_velocity(synthetic.taylor_green_2d_unit(xu, 0.0, 0.01)[0], 2, d.nbu)
    hist = synthetic.nodal_velocity(synthetic.taylor_green_2d_unit(xu, -(1 - g) * dt, 0.01)[0], 2, d.nbu)
    p = synthetic.taylor_green_2d_unit(xp, 0.0, 0.01)[1]
    st1 = ts.stage(1, u, hist, None, p, 0.0)
    assert st1["solves"] < 60
    us = st1["u_star"]
    lhs = (ts.per_component((1.0 / (g * dt)) * ts.M + 0.5 * (d.nu * ts.L + d.lf_advection(us)), us))
    rhs = ((1.0 / (g * dt)) * (ts.Mv @ u) - 0.5 * d.nu * ts.per_component(ts.L0, u)
           + 0.5 * ts.per_component(d.explicit_advection(u), u) + ts.Gw @ p)
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(rhs)
    # one solve is the linearised scheme
    lin = TRBDF2(d, dt).stage(1, u, hist, None, p, 0.0)
    one = TRBDF2(d, dt, nonlinear_iters=1).stage(1, u, hist, None, p, 0.0)
    assert np.array_equal(lin["u"], one["u"]) and one["solves"] == 1


# velocity error of the 8 x 8 Q2-Q1 config-1 run after 10 steps (t = 0.1),
# measured with this oracle; the pin below is the convergence to the exact
# solution, this value only lets the GPU test compare against it
C1_U_L2_REL_8 = 0.04263


def c1_run(N, steps=10, nu=0.01, dt=0.01):
    """Config-1 workload: the scaled Taylor-Green vortex on the periodic unit
    square, Q2-Q1, nu = 0.01, dt = 0.01; relative L2 errors of u and of the
    mean-free p against the exact solution after ``steps`` steps."""
    mesh = BoxMesh(2, (N, N), (0.0, 0.0), (1.0, 1.0), (True, True))
    d = Discretization(mesh, 2, nu=nu)
    ts = TRBDF2(d, dt)
    g = ts.cst["gamma"]
    xu, xp = d.node_coords("u"), d.node_coords("p")
    u = synthetic.nodal_velocity(synthetic.taylor_green_2d_unit(xu, 0.0, nu)[0], 2, d.nbu)
    h = synthetic.nodal_velocity(synthetic.taylor_green_2d_unit(xu, -(1 - g) * dt, nu)[0], 2, d.nbu)
    p = synthetic.taylor_green_2d_unit(xp, 0.0, nu)[1]
    t = 0.0
    for _ in range(steps):
        u, h, p, _ = ts.step(u, h, p, t)
        t += dt
    eu, ru = d.l2_error(u, lambda x: synthetic.taylor_green_2d_unit(x, t, nu)[0])
    ep, rp = d.l2_error(p, lambda x: synthetic.taylor_green_2d_unit(x, t, nu)[1], "p", remove_mean=True)
    return eu / ru, ep / rp


def test_config1_converges_to_exact_solution():
    """The config-1 run against the exact decaying vortex: halving h cuts the
    velocity error by about 2^(k+1) = 8 (measured 6.7) and the pressure error
    by about 2^k_p+1 = 4 (time step fixed, so the splitting error stays)."""
    (eu8, ep8), (eu16, ep16) = c1_run(8), c1_run(16)
    assert abs(eu8 - C1_U_L2_REL_8) < 1e-4 * C1_U_L2_REL_8 * 10
    assert eu8 / eu16 > 5.5 and ep8 / ep16 > 3.5, (eu8, eu16, ep8, ep16)
    assert eu16 < 7e-3 and ep16 < 3e-2
