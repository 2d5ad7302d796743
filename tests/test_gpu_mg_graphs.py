"""HIP-graph replay of the multigrid V-cycles (tbdg_set_mg_graphs) against the
same kernels launched one by one.

Each check replays the captured graphs several times, with other eager
library work and host synchronisations between the replays, and compares
every replay bit for bit with the kernel-by-kernel result of the same call:
the momentum V-cycles (tbdg_mg_apply_momentum; with graphs the components'
cycles run side by side on their own streams, in 2D and 3D), the pressure
flexible CG,
the multigrid-preconditioned momentum GMRES and whole TR-BDF2 steps of the
Kovasznay flow on Q1-mapped cells.
"""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx(mapped=True):
    from paper_2107_07776_amd import Context
    Re, k = 40.0, 4
    lo, hi, nc = (-0.5, -0.5), (1.0, 1.5), (16, 16)
    print(f"[case] graphs kovasznay cells={nc} k={k} mapped={mapped}", flush=True)
    ctx = Context(2, nc, lo, hi, k=k, nu=1.0 / Re, dt=0.04, periodic=(0, 0),
                  mapping=1 if mapped else 0, map_amp=0.05 if mapped else 0.0)
    pts = ctx.face_qpoints().cpu().numpy()
    data = torch.tensor(synthetic.kovasznay(pts, Re)[0], device="cuda")
    ctx.set_dirichlet(0, data)
    ctx.set_dirichlet(1, data)
    ctx.mg_setup(degree=5)
    return ctx


def _eager_work(ctx, u, p):
    """Library and torch work between two replays, ending in a host sync."""
    y = ctx.apply_pressure(1, p)
    z = ctx.apply_momentum(2, u, u)
    torch.cuda.synchronize()
    return float(y.abs().sum().item() + z.abs().sum().item())


def test_momentum_vcycles_replay_equals_eager():
    ctx = _ctx()
    try:
        u = torch.tensor(synthetic.random_vector(ctx.N_u, 1), device="cuda")
        p = torch.tensor(synthetic.random_vector(ctx.N_p, 2), device="cuda")
        for rep in range(4):
            for stage in (1, 2):
                v = torch.tensor(synthetic.random_vector(ctx.N_u, 10 + 3 * rep + stage), device="cuda")
                ctx.set_mg_graphs(False)
                ze = ctx.mg_apply_momentum(stage, v).clone()
                _eager_work(ctx, u, p)
                ctx.set_mg_graphs(True)
                zg = ctx.mg_apply_momentum(stage, v)
                torch.cuda.synchronize()
                assert torch.equal(ze, zg), (rep, stage)
                _eager_work(ctx, u, p)
    finally:
        ctx.close()


def test_momentum_vcycles_replay_equals_eager_3d():
    """In 3D the graphs of components 1 and 2 replay on two side streams
    beside component 0's, each on its own copy of the hierarchy."""
    from paper_2107_07776_amd import Context
    print("[case] graphs 3D periodic cells=(8, 8, 8) k=2", flush=True)
    ctx = Context(3, (8, 8, 8), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), k=2, nu=0.05, dt=0.05,
                  periodic=(1, 1, 1))
    try:
        ctx.mg_setup(degree=4)
        u = torch.tensor(synthetic.random_vector(ctx.N_u, 3), device="cuda")
        p = torch.tensor(synthetic.random_vector(ctx.N_p, 4), device="cuda")
        for rep in range(3):
            for stage in (1, 2):
                v = torch.tensor(synthetic.random_vector(ctx.N_u, 40 + 3 * rep + stage), device="cuda")
                ctx.set_mg_graphs(False)
                ze = ctx.mg_apply_momentum(stage, v).clone()
                _eager_work(ctx, u, p)
                ctx.set_mg_graphs(True)
                zg = ctx.mg_apply_momentum(stage, v)
                torch.cuda.synchronize()
                assert torch.equal(ze, zg), (rep, stage)
                _eager_work(ctx, u, p)
    finally:
        ctx.close()


def test_solves_replay_equals_eager():
    ctx = _ctx()
    try:
        u = torch.tensor(synthetic.random_vector(ctx.N_u, 3), device="cuda")
        p = torch.tensor(synthetic.random_vector(ctx.N_p, 4), device="cuda")
        w = 0.5 * torch.tensor(synthetic.random_vector(ctx.N_u, 5), device="cuda")
        for rep in range(3):
            out = {}
            for graphs in (False, True):
                ctx.set_mg_graphs(graphs)
                bp = torch.tensor(synthetic.random_vector(ctx.N_p, 20 + rep), device="cuda")
                xp = torch.zeros_like(bp)
                ip = ctx.solve_pressure(1 + rep % 2, bp, xp, tol=1e-10, maxiter=500, precond="mg_fp32")
                _eager_work(ctx, u, p)
                bu = torch.tensor(synthetic.random_vector(ctx.N_u, 30 + rep), device="cuda")
                xu = torch.zeros_like(bu)
                iu = ctx.solve_momentum(2 - rep % 2, w, bu, xu, tol=1e-10, maxiter=500, restart=30,
                                        precond="mg_fp32")
                torch.cuda.synchronize()
                out[graphs] = (xp.clone(), ip["iters"], xu.clone(), iu["iters"])
                _eager_work(ctx, u, p)
            e, g = out[False], out[True]
            assert e[1] == g[1] and e[3] == g[3], (rep, e[1], g[1], e[3], g[3])
            assert torch.equal(e[0], g[0]) and torch.equal(e[2], g[2]), rep
    finally:
        ctx.close()


def test_steps_replay_equals_eager():
    """Four Kovasznay steps from rest with both multigrid preconditioners,
    kernel by kernel and with graph replays: the same fields bit for bit."""
    res = {}
    for graphs in (False, True):
        ctx = _ctx()
        try:
            ctx.set_mg_graphs(graphs)
            ctx.set_nonlinear(2, 0.0)
            U = torch.zeros(ctx.N_u, dtype=torch.float64, device="cuda")
            H = U.clone()
            P = torch.zeros(ctx.N_p, dtype=torch.float64, device="cuda")
            t = 0.0
            for n in range(4):
                info, st = ctx.step(U, H, P, t, n, mom_tol=1e-10, prs_tol=1e-10, mom_maxiter=2000,
                                    prs_maxiter=500, precond="mg_fp32", mom_precond="mg_fp32",
                                    guess="previous", mom_guess="previous", check=False)
                assert st == 0, (graphs, n, info)
                torch.cuda.synchronize()
                t += 0.04
            res[graphs] = (U.clone(), P.clone())
        finally:
            ctx.close()
    assert torch.equal(res[False][0], res[True][0]) and torch.equal(res[False][1], res[True][1])
