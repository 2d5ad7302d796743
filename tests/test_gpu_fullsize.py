"""GPU parity at the benchmark's full size (3D periodic box, 32^3 cells,
Q3-Q2) in the benchmark's launch configuration: every operator entry point is
compared with the oracle on a sample of cells (including the corners and the
periodic wrap), which the oracle assembles row by row; the solves are checked
through their recomputed true residual."""
import math

import numpy as np
import pytest

import synthetic
from oracle import BoxMesh, Discretization, TRBDF2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 32
SAMPLE = [0, 1, N - 1, N * N - 1, N * N, 12345, N ** 3 - N * N, N ** 3 - 1]


@pytest.fixture(scope="module")
def full():
    from paper_2107_07776_amd import Context
    dt, nu = 2 * math.pi / 96, 1.0 / 1600
    print("[case] full size 32^3 Q3-Q2", flush=True)
    ctx = Context(3, (N,) * 3, (0.0,) * 3, (2 * math.pi,) * 3, k=3, nu=nu, dt=dt)
    mesh = BoxMesh(3, (N,) * 3, (0.0,) * 3, (2 * math.pi,) * 3, (True,) * 3)
    disc = Discretization(mesh, 3, nu=nu)
    ora = TRBDF2(disc, dt, rows=SAMPLE)
    yield ctx, disc, ora
    ctx.close()


def rows_u(disc):
    return np.concatenate([np.arange(c * 3 * disc.nbu, (c + 1) * 3 * disc.nbu) for c in SAMPLE])


def rows_p(disc):
    return np.concatenate([np.arange(c * disc.nbp, (c + 1) * disc.nbp) for c in SAMPLE])


def rows_s(disc):
    return np.concatenate([np.arange(c * disc.nbu, (c + 1) * disc.nbu) for c in SAMPLE])


def close(g, o, tol=1e-12):
    err = np.abs(g - o).max() / np.abs(o).max()
    assert err <= tol, f"{err:.3e}"


def t(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def h(x):
    torch.cuda.synchronize()
    return x.cpu().numpy()


@pytest.mark.parametrize("stage", [1, 2])
def test_operators_sampled(full, stage):
    ctx, disc, ora = full
    w = synthetic.random_vector(disc.N_u, 1)
    u = synthetic.random_vector(disc.N_u, 2)
    p = synthetic.random_vector(disc.N_p, 3)
    ru, rp, rs = rows_u(disc), rows_p(disc), rows_s(disc)
    close(h(ctx.apply_momentum(stage, t(w), t(u)))[ru], ora.apply_momentum(stage, w, u)[ru])
    close(h(ctx.apply_pressure(stage, t(p)))[rp], ora.apply_pressure(stage, p)[rp])
    close(h(ctx.diag_momentum(stage, t(w)))[rs], ora.diag_momentum(stage, w)[rs])
    close(h(ctx.diag_pressure(stage))[rp], ora.diag_pressure(stage)[rp])
    close(h(ctx.rhs_momentum(stage, t(u), t(w) if stage == 2 else None, t(w), t(p)))[ru],
          ora.rhs_momentum(stage, u, w if stage == 2 else None, w, p)[ru])
    close(h(ctx.rhs_pressure(stage, t(u), t(p)))[rp], ora.rhs_pressure(stage, u, p)[rp])
    close(h(ctx.grad_p(t(p)))[ru], ora.grad_p(p)[ru])


def test_full_size_solves(full):
    ctx, disc, _ = full
    b = t(synthetic.random_vector(disc.N_p, 4))
    x = torch.zeros_like(b)
    info = ctx.solve_pressure(1, b, x, tol=1e-8, maxiter=20000)
    r = b - ctx.apply_pressure(1, x)
    assert info["res_final"] <= 1e-8
    assert abs(h(r.norm() / b.norm()) - info["res_final"]) < 1e-12
    w = t(synthetic.random_vector(disc.N_u, 5)) * 0.3
    bu = t(synthetic.random_vector(disc.N_u, 6))
    xu = torch.zeros_like(bu)
    info = ctx.solve_momentum(2, w, bu, xu, tol=1e-8, maxiter=500)
    ru = bu - ctx.apply_momentum(2, w, xu)
    assert info["res_final"] <= 1e-8
    assert h(ru.norm() / bu.norm()) <= 1.01e-8


@pytest.mark.parametrize("precond", ["mg_fp32", "mg_bf16"])
def test_full_size_multigrid_solves(full, precond):
    """The benchmark's multigrid solve (5 levels down to 4^3 Q1) meets 1e-8 on
    the recomputed FP64 residual, with the V-cycle built for both stages."""
    ctx, disc, _ = full
    ctx.mg_setup()
    levels = ctx.mg_levels()
    assert [l["dofs"] for l in levels] == [884736, 262144, 32768, 4096, 512]
    for stage in (1, 2):
        b = t(synthetic.random_vector(disc.N_p, 40 + stage))
        x = torch.zeros_like(b)
        info = ctx.solve_pressure(stage, b, x, tol=1e-8, maxiter=100, precond=precond)
        r = b - ctx.apply_pressure(stage, x)
        print(f"{precond} stage {stage}: {info['iters']} iterations")
        assert info["res_final"] <= 1e-8
        assert h(r.norm() / b.norm()) <= 1.01e-8
        assert info["iters"] <= 30
