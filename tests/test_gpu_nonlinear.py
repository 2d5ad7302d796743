"""GPU parity of the fully nonlinear momentum predictors (fixed-point
solves per stage) with the oracle's direct-solve stages.

* the paper's 2D Taylor-Green case at C = 1.63 (8 x 8 Q2-Q1, dt = 0.64,
  three solves per stage, five steps to t = 3.2), where the linearised
  scheme departs from the solution;
* a box with Dirichlet walls (the boundary terms follow each advector);
* the early stop on the relative change: same solve counts as the oracle.
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import BoxMesh, Discretization, TRBDF2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_paper_taylor_green_nonlinear_matches_oracle():
    from paper_2107_07776_amd import Context
    Re, N, k, dt, m = 100.0, 8, 2, 0.64, 3
    print(f"[case] nonlinear TG 2D N={N} k={k} dt={dt} m={m}", flush=True)
    ext = (2 * math.pi,) * 2
    ctx = Context(2, (N, N), (0.0, 0.0), ext, k=k, nu=1.0 / Re, dt=dt)
    ctx.set_nonlinear(m, 0.0)
    disc = Discretization(BoxMesh(2, (N, N), (0.0, 0.0), ext, (True, True)), k, nu=1.0 / Re)
    ora = TRBDF2(disc, dt, nonlinear_iters=m)
    g = ora.cst["gamma"]
    xu, xp = disc.node_coords("u"), disc.node_coords("p")
    U0 = lambda t: synthetic.nodal_velocity(synthetic.taylor_green_2d(xu, t, Re)[0], 2, disc.nbu)
    u, h, p = U0(0.0), U0(-(1 - g) * dt), synthetic.taylor_green_2d(xp, 0.0, Re)[1]
    U, H, P = _t(u), _t(h), _t(p)
    t = 0.0
    for n in range(5):
        info, st = ctx.step(U, H, P, t, n, mom_tol=1e-13, prs_tol=1e-11, mom_maxiter=5000,
                            prs_maxiter=5000, check=False)
        assert st == 0, (n, info)
        assert info[0]["solves"] == m and info[2]["solves"] == m
        u, h, p, _ = ora.step(u, h, p, t)
        t += dt
    torch.cuda.synchronize()
    Ug, Pg = U.cpu().numpy(), P.cpu().numpy()
    du = np.linalg.norm(Ug - u) / np.linalg.norm(u)
    pm = lambda v: v - v.mean()
    dp = np.linalg.norm(pm(Pg) - pm(p)) / np.linalg.norm(pm(p))
    eu, ru = disc.l2_error(Ug, lambda x: synthetic.taylor_green_2d(x, t, Re)[0])
    print(f"GPU vs oracle u {du:.2e} p {dp:.2e}; velocity L2 error vs exact {eu / ru:.3f} "
          f"(paper's table: 0.38)")
    assert du < 1e-9 and dp < 1e-7
    ctx.close()


def _uD(x, t):
    out = np.empty_like(x)
    out[:, 0] = np.sin(x[:, 0] + 2 * x[:, 1] + t)
    out[:, 1] = np.cos(x[:, 0] - x[:, 1]) * (1.0 + t)
    return out


@pytest.mark.parametrize("m,tol", [(2, 0.0), (6, 1e-4)])
def test_nonlinear_with_walls_matches_oracle(m, tol):
    """Channel (periodic in x, walls in y), Q3-Q2, time-dependent wall data:
    three steps with fixed-point stages; with tol > 0 the solve counts of
    every stage must equal the oracle's."""
    from paper_2107_07776_amd import Context
    dim, nc, ext, k, per, nu, dt = 2, (5, 4), (1.0, 1.0), 3, (1, 0), 0.02, 0.03
    print(f"[case] nonlinear walls m={m} tol={tol}", flush=True)
    ctx = Context(dim, nc, (0.0, 0.0), ext, k=k, nu=nu, dt=dt, periodic=per)
    ctx.set_nonlinear(m, tol)
    disc = Discretization(BoxMesh(dim, nc, (0.0, 0.0), ext, per), k, nu=nu)
    ora = TRBDF2(disc, dt, uD=_uD, nonlinear_iters=m, nonlinear_tol=tol)
    g = ora.cst["gamma"]
    pts = ctx.face_qpoints().cpu().numpy()
    xu = disc.node_coords("u")
    u = synthetic.nodal_velocity(_uD(xu, 0.0), 2, disc.nbu)
    h = synthetic.nodal_velocity(_uD(xu, -(1 - g) * dt), 2, disc.nbu)
    p = np.zeros(disc.N_p)
    U, H, P = _t(u), _t(h), _t(p)
    t = 0.0
    for n in range(3):
        ctx.set_dirichlet(0, _t(_uD(pts, t + g * dt)))
        ctx.set_dirichlet(1, _t(_uD(pts, t + dt)))
        info, st = ctx.step(U, H, P, t, n, mom_tol=1e-13, prs_tol=1e-11, mom_maxiter=5000,
                            prs_maxiter=5000, check=False)
        assert st == 0, (n, info)
        u, h, p, stages = ora.step(u, h, p, t)
        assert (info[0]["solves"], info[2]["solves"]) == (stages[0]["solves"], stages[1]["solves"])
        if tol == 0.0:
            assert info[0]["solves"] == m
        t += dt
    torch.cuda.synchronize()
    Ug, Pg = U.cpu().numpy(), P.cpu().numpy()
    du = np.linalg.norm(Ug - u) / np.linalg.norm(u)
    dp = np.linalg.norm(Pg - p) / np.linalg.norm(p)
    print(f"walls m={m} tol={tol}: solves {info[0]['solves']},{info[2]['solves']}; "
          f"GPU vs oracle u {du:.2e} p {dp:.2e}")
    assert du < 1e-9 and dp < 1e-7
    ctx.close()


def test_set_nonlinear_rejects_bad_arguments():
    from paper_2107_07776_amd import Context
    ctx = Context(2, (2, 2), (0.0, 0.0), (1.0, 1.0), k=2, nu=0.01, dt=0.01)
    for args in ((0, 0.0), (2, -1.0), (2, float("nan"))):
        with pytest.raises(Exception):
            ctx.set_nonlinear(*args)
    ctx.close()


@pytest.mark.parametrize("N,printed", [(8, 0.39), (16, 0.11)])
def test_paper_taylor_green_courant_3_table(N, printed):
    """The paper's Taylor-Green table at C = 3, computed with fixed-point
    iterations (Sec. 4): (0,2 pi)^2, Re = 100, Q2-Q1, dt = 3 H / (2 U)
    (1.178 on 8^2, 0.589 on 16^2), stages iterated to a relative change of
    1e-10 or 30 solves (the cap is reached on 8^2), three and five steps.  Printed relative L2 velocity errors 0.39
    and 0.11 (reproduced to 25 %: measured 0.39 and 0.086; on 32^2 and 64^2
    the converged fixed point is 4-10 times more accurate than printed)."""
    from paper_2107_07776_amd import Context
    Re, k = 100.0, 2
    dt = 3.0 * (2 * math.pi / N) / k
    nsteps = int(round(3.2 / dt))
    print(f"[case] TG C=3 N={N} dt={dt:.4f} steps={nsteps}", flush=True)
    ext = (2 * math.pi,) * 2
    ctx = Context(2, (N, N), (0.0, 0.0), ext, k=k, nu=1.0 / Re, dt=dt)
    ctx.set_nonlinear(30, 1e-10)
    disc = Discretization(BoxMesh(2, (N, N), (0.0, 0.0), ext, (True, True)), k, nu=1.0 / Re)
    g = 2.0 - math.sqrt(2.0)
    xu, xp = disc.node_coords("u"), disc.node_coords("p")
    U0 = lambda t: synthetic.nodal_velocity(synthetic.taylor_green_2d(xu, t, Re)[0], 2, disc.nbu)
    U, H, P = _t(U0(0.0)), _t(U0(-(1 - g) * dt)), _t(synthetic.taylor_green_2d(xp, 0.0, Re)[1])
    t = 0.0
    for n in range(nsteps):
        info, st = ctx.step(U, H, P, t, n, mom_tol=1e-12, prs_tol=1e-10, mom_maxiter=5000,
                            prs_maxiter=5000, check=False)
        assert st == 0, (n, info)
        t += dt
    torch.cuda.synchronize()
    eu, ru = disc.l2_error(U.cpu().numpy(), lambda x: synthetic.taylor_green_2d(x, t, Re)[0])
    print(f"TG C=3 {N}^2: velocity L2 error {eu / ru:.4f} at t = {t:.3f} (printed {printed})")
    assert abs(eu / ru / printed - 1.0) < 0.25, eu / ru
    ctx.close()
