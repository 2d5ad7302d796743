"""The single-stage comparison schemes of Sec. 2 on the GPU (tbdg_set_scheme):
Bell-Colella-Glaz (Crank-Nicolson, fixed-point midpoint advection) and the
Guermond-Quartapelle BDF2 projection, against the oracle's direct-solve
steps (periodic 2D and 3D boxes, Dirichlet walls) and against the paper's
Q2-Q1 Taylor-Green tables for the two schemes (Sec. 4, C = 1.63)."""
import math

import numpy as np
import pytest

import synthetic
from oracle import BCG, BDF2GQ, BoxMesh, Discretization

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _oracle_steps(ora, u, h, p, t, dt, steps):
    ustar = None
    for _ in range(steps):
        if isinstance(ora, BDF2GQ):
            u, h, p, st = ora.step(u, h, p, t, u_star_prev=ustar)
        else:
            u, h, p, st = ora.step(u, h, p, t)
        ustar = st["u_star"]
        t += dt
    return u, p


# (scheme, dim, cells, k): several tiles and a ragged count in 2D, a 3D box
CASES = [("bcg", 2, (6, 5), 3), ("bdf2", 2, (6, 5), 3), ("bcg", 3, (3, 2, 4), 2),
         ("bdf2", 3, (3, 2, 4), 2)]


@pytest.mark.parametrize("scheme,dim,nc,k", CASES, ids=[f"{c[0]}-d{c[1]}" for c in CASES])
def test_periodic_steps_match_oracle(scheme, dim, nc, k):
    """Six steps of a Taylor-Green field (2D: the scaled vortex on the unit
    square; 3D: the vortex of the 3D workload on [0, 2 pi]^3) with tight
    solves (line-block GMRES for the momentum; FP32 multigrid for the
    pressure in 2D, Jacobi CG on the 3D box, whose Q1 pressure on 3 x 2 x 4
    cells leaves the multigrid a single level), three fixed-point solves per
    BCG step."""
    from paper_2107_07776_amd import Context
    print(f"[case] scheme={scheme} dim={dim} cells={nc} k={k}", flush=True)
    nu, dt = (0.01, 0.02) if dim == 2 else (0.02, 0.1)
    ext = (1.0,) * dim if dim == 2 else (2 * math.pi,) * dim
    ctx = Context(dim, nc, (0.0,) * dim, ext, k=k, nu=nu, dt=dt)
    ctx.set_scheme(scheme)
    ctx.set_nonlinear(3, 0.0)
    disc = Discretization(BoxMesh(dim, nc, (0.0,) * dim, ext, (True,) * dim), k, nu=nu)
    ora = BCG(disc, dt, nonlinear_iters=3, nonlinear_tol=0.0) if scheme == "bcg" else BDF2GQ(disc, dt)
    xu, xp = disc.node_coords("u"), disc.node_coords("p")
    if dim == 2:
        f = lambda t: synthetic.nodal_velocity(synthetic.taylor_green_2d_unit(xu, t, nu)[0], 2, disc.nbu)
        u, h, p = f(0.0), f(-dt), synthetic.taylor_green_2d_unit(xp, 0.0, nu)[1]
    else:
        u = synthetic.nodal_velocity(synthetic.tgv3d_velocity(xu), 3, disc.nbu)
        h = u.copy()
        p = synthetic.tgv3d_pressure(xp)
    U, H, P = _t(u), _t(h), _t(p)
    t = 0.0
    steps = 6
    for n in range(steps):
        info, st = ctx.step(U, H, P, t, n, mom_tol=1e-13, prs_tol=1e-12, mom_maxiter=4000,
                            prs_maxiter=2000, precond="mg_fp32" if dim == 2 else "jacobi",
                            mom_precond="line", guess="previous",
                            mom_guess="previous", check=False)
        assert st == 0, (n, info)
        assert info[2]["iters"] == 0 and info[3]["iters"] == 0
        assert info[0]["solves"] == (3 if scheme == "bcg" else 1)
        t += dt
    ue, pe = _oracle_steps(ora, u, h, p, 0.0, dt, steps)
    torch.cuda.synchronize()
    du = np.linalg.norm(U.cpu().numpy() - ue) / np.linalg.norm(ue)
    dp = np.linalg.norm(P.cpu().numpy() - pe) / np.linalg.norm(pe)
    print(f"{scheme} d{dim}: GPU vs oracle u {du:.2e}, p {dp:.2e}")
    assert du < 1e-9 and dp < 1e-8
    ctx.close()


@pytest.mark.parametrize("scheme", ["bcg", "bdf2"])
def test_walled_steps_match_oracle_and_read_slot_one(scheme):
    """Kovasznay flow (Re = 40) with Dirichlet walls on 6 x 8 affine Q3-Q2
    cells: the single-stage schemes take the data of slot 1 (t^{n+1}); slot
    0 holds a wrong field that must not be read."""
    from paper_2107_07776_amd import Context
    Re, dt, k = 40.0, 0.02, 3
    lo, hi, nc = (-0.5, -0.5), (1.0, 1.5), (6, 8)
    ex = lambda x, t: synthetic.kovasznay(x, Re)[0]
    ctx = Context(2, nc, lo, hi, k=k, nu=1.0 / Re, dt=dt, periodic=(0, 0))
    ctx.set_scheme(scheme)
    ctx.set_nonlinear(2, 0.0)
    pts = ctx.face_qpoints().cpu().numpy()
    data = ex(pts, 0.0)
    ctx.set_dirichlet(0, _t(0.5 * data))
    ctx.set_dirichlet(1, _t(data))
    disc = Discretization(BoxMesh(2, nc, lo, hi, (False, False)), k, nu=1.0 / Re)
    ora = (BCG(disc, dt, uD=ex, nonlinear_iters=2, nonlinear_tol=0.0) if scheme == "bcg"
           else BDF2GQ(disc, dt, uD=ex))
    xu, xp = disc.node_coords("u"), disc.node_coords("p")
    u = synthetic.nodal_velocity(ex(xu, 0.0), 2, disc.nbu)
    h = u.copy()
    p = synthetic.kovasznay(xp, Re)[1]
    U, H, P = _t(u), _t(h), _t(p)
    t = 0.0
    for n in range(6):
        info, st = ctx.step(U, H, P, t, n, mom_tol=1e-12, prs_tol=1e-10, mom_maxiter=5000,
                            prs_maxiter=200, precond="mg_fp32", check=False)
        assert st == 0, (n, info)
        t += dt
    ue, pe = _oracle_steps(ora, u, h, p, 0.0, dt, 6)
    torch.cuda.synchronize()
    du = np.linalg.norm(U.cpu().numpy() - ue) / np.linalg.norm(ue)
    dp = np.linalg.norm(P.cpu().numpy() - pe) / np.linalg.norm(pe)
    print(f"{scheme} Kovasznay walls: GPU vs oracle u {du:.2e}, p {dp:.2e}")
    assert du < 1e-9 and dp < 1e-7
    ctx.close()


def test_scheme_errors():
    from paper_2107_07776_amd import Context
    from paper_2107_07776_amd.trbdg import TrbdgError
    ctx = Context(2, (4, 4), (0.0, 0.0), (1.0, 1.0), k=2, nu=0.01, dt=0.01)
    try:
        st = ctx.lib.tbdg_set_scheme(ctx.h, 7)
        assert st == -1   # TBDG_EINVAL
        ctx.set_scheme("bdf2")
        u = torch.zeros(ctx.N_u, dtype=torch.float64, device="cuda")
        p = torch.zeros(ctx.N_p, dtype=torch.float64, device="cuda")
        with pytest.raises(TrbdgError):
            ctx.step(u, u.clone(), p, guess="learned")
        ctx.set_scheme("trbdf2")
        info, st = ctx.step(u, u.clone(), p)
        assert st == 0 and info[2]["iters"] == 0   # zero data: nothing to solve
    finally:
        ctx.close()


def _paper_tg_gpu(scheme, N, dt, T=3.2, Re=100.0, k=2):
    """The paper's 2D Taylor-Green convergence case (Sec. 4: (0, 2 pi)^2,
    Re = 100, c = 1e3, t = 0 .. 3.2) with the given scheme; relative L2
    errors of u and of the mean-free p at T."""
    from paper_2107_07776_amd import Context
    L = 2 * math.pi
    ctx = Context(2, (N, N), (0.0, 0.0), (L, L), k=k, nu=1.0 / Re, dt=dt)
    ctx.set_scheme(scheme)
    # the Crank-Nicolson midpoint fixed point contracts slowly at C = 1.63
    # (its result after a fixed small number of solves alternates, e.g.
    # 0.10 with three and 0.21 with four on 16^2): iterate it to a tolerance
    ctx.set_nonlinear(60, 1e-8)
    disc = Discretization(BoxMesh(2, (N, N), (0.0, 0.0), (L, L), (True, True)), k, nu=1.0 / Re, c=1.0e3)
    xu, xp = ctx.node_coords(0).cpu().numpy(), ctx.node_coords(1).cpu().numpy()
    f = lambda t: synthetic.nodal_velocity(synthetic.taylor_green_2d(xu, t, Re)[0], 2, disc.nbu)
    U, H, P = _t(f(0.0)), _t(f(-dt)), _t(synthetic.taylor_green_2d(xp, 0.0, Re)[1])
    t = 0.0
    for n in range(int(round(T / dt))):
        info, st = ctx.step(U, H, P, t, n, mom_tol=1e-11, prs_tol=1e-10, mom_maxiter=5000,
                            prs_maxiter=400, precond="mg_fp32", check=False)
        assert st == 0, (n, info)
        t += dt
    torch.cuda.synchronize()
    eu, ru = disc.l2_error(U.cpu().numpy(), lambda x: synthetic.taylor_green_2d(x, t, Re)[0])
    ep, rp = disc.l2_error(P.cpu().numpy(), lambda x: synthetic.taylor_green_2d(x, t, Re)[1], "p",
                           remove_mean=True)
    ctx.close()
    return eu / ru, ep / rp


# printed relative L2 velocity errors of the paper's Q2-Q1 tables at
# C = 1.63 (dt = 0.64, 0.32, 0.16, 0.08 on 8^2 .. 64^2)
PRINTED_U = {"bcg": (0.48, 0.13, 0.0311, 0.0070), "bdf2": (0.28, 0.09, 0.023, 0.0077)}


@pytest.mark.parametrize("scheme", ["bcg", "bdf2"])
def test_paper_tables_of_the_comparison_schemes(scheme):
    """Coarsest row within 25 % of the printed value; on the finer meshes the
    observed rates lie between 1.5 and 4.5 (printed: 1.6-2.2; the BDF2 step
    converges faster than printed, 0.056 and 0.0041 on 16^2 and 32^2 against
    the printed 0.09 and 0.023, as the oracle does on 16^2)."""
    errs = []
    for i, N in enumerate((8, 16, 32)):
        eu, ep = _paper_tg_gpu(scheme, N, 0.64 / 2 ** i)
        errs.append(eu)
        print(f"{scheme} Q2-Q1 {N}^2: u {eu:.4f} (printed {PRINTED_U[scheme][i]}), p {ep:.4f}")
    assert abs(errs[0] / PRINTED_U[scheme][0] - 1.0) < 0.25, errs
    for a, b in zip(errs, errs[1:]):
        assert 1.5 < math.log2(a / b) < 4.5, errs
