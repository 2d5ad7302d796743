"""The 3D ABC (Arnold-Beltrami-Childress) convergence case of Sec. 4 on the
GPU against the paper's printed Q2-Q1 table.

(0, 2 pi)^3 with Dirichlet data from the exact solution on every wall,
Re = 1, C = 1.63 (dt = 0.32 on 8^3 cells, 0.16 on 16^3), t = 0 .. 3.2, the
linearised stages, solves to 1e-10 (momentum) and 1e-8 (pressure: the
relative floor of the all-Neumann Helmholtz system rises as the pressure
decays); the exact velocity decays as e^{-t/Re}, the pressure
(quadratic in the velocity) as e^{-2t/Re}.  Printed relative L2 velocity
errors: 0.0078 (8^3) and 0.0022 (16^3), reproduced to 25 % (as the
Taylor-Green pins; measured 0.0078 and 0.0019).  The CPU oracle gives 0.00784 on
8^3 (about four minutes, so it is not part of the CPU suite).
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import BoxMesh, Discretization

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def abc_u(x, t, nu):
    f = math.exp(-nu * t)
    return np.stack([np.sin(x[:, 2]) + np.cos(x[:, 1]), np.sin(x[:, 0]) + np.cos(x[:, 2]),
                     np.sin(x[:, 1]) + np.cos(x[:, 0])], 1) * f


def abc_p(x, t, nu):
    return -(np.sin(x[:, 0]) * np.cos(x[:, 2]) + np.sin(x[:, 1]) * np.cos(x[:, 0])
             + np.sin(x[:, 2]) * np.cos(x[:, 1])) * math.exp(-2.0 * nu * t)


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("n,dt,printed", [(8, 0.32, 0.0078), (16, 0.16, 0.0022)])
def test_abc_velocity_error_matches_paper_table(n, dt, printed):
    from paper_2107_07776_amd import Context
    nu, k, T = 1.0, 2, 3.2
    print(f"[case] ABC n={n} dt={dt}", flush=True)
    L = 2 * math.pi
    ctx = Context(3, (n,) * 3, (0.0,) * 3, (L,) * 3, k=k, nu=nu, dt=dt, periodic=(0, 0, 0))
    disc = Discretization(BoxMesh(3, (n,) * 3, (0.0,) * 3, (L,) * 3, (False,) * 3), k, nu=nu)
    g = 2.0 - math.sqrt(2.0)
    pts = ctx.face_qpoints().cpu().numpy()
    xu = ctx.node_coords(0).cpu().numpy()
    xp = ctx.node_coords(1).cpu().numpy()
    U = lambda t: synthetic.nodal_velocity(abc_u(xu, t, nu), 3, (k + 1) ** 3)
    u, h, p = _t(U(0.0)), _t(U(-(1 - g) * dt)), _t(abc_p(xp, 0.0, nu))
    t = 0.0
    for s in range(int(round(T / dt))):
        ctx.set_dirichlet(0, _t(abc_u(pts, t + g * dt, nu)))
        ctx.set_dirichlet(1, _t(abc_u(pts, t + dt, nu)))
        info, st = ctx.step(u, h, p, t, s, mom_tol=1e-10, prs_tol=1e-8, mom_maxiter=5000,
                            prs_maxiter=500, precond="mg_fp32", check=False)
        assert st == 0, (s, info)
        t += dt
    torch.cuda.synchronize()
    eu, ru = disc.l2_error(u.cpu().numpy(), lambda x: abc_u(x, t, nu))
    print(f"ABC {n}^3 Q2-Q1: velocity L2 error {eu / ru:.5f} (printed {printed})")
    assert abs(eu / ru / printed - 1.0) < 0.25, eu / ru
    ctx.close()
