"""GPU parity of the momentum multigrid (tbdg_mg_apply_momentum,
TBDG_PRECOND_MG_FP32 in the momentum options) against the oracle's
velocity-component multigrid (oracle.multigrid.Multigrid, field "u").

* the hierarchy (degrees, cells, DoFs) equals the oracle's and the FP64
  Lanczos eigenvalue estimates agree to 1e-9 relative;
* one application (a V-cycle per component of v / (theta_s nu)) agrees with
  the oracle's FP64 cycles to FP32 rounding (the pressure multigrid's bound);
* GMRES preconditioned with it meets the tolerance on the oracle's CSR
  residual of the full stage operator (advection and Dirichlet data
  included) on walled, mixed and Q1-mapped meshes, in fewer iterations than
  the line preconditioner where the stage operator is diffusion-dominated;
* ten Kovasznay steps with it match the oracle's direct-solve steps.
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import BoxMesh, Discretization, TRBDF2
from oracle.multigrid import Multigrid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_VC32 = 200 * 2.0 ** -24

# (dim, cells, extent, k, periodic, coarse_cells): walls everywhere (Q3 and
# the Q4 of the Kovasznay workload), a channel with ragged cell counts, a
# single p-level, 3D boxes with walls (Q3: four nodes per direction)
CASES = [
    (2, (8, 8), (1.0, 1.0), 3, (0, 0), 16),
    (2, (12, 8), (1.5, 1.0), 4, (1, 0), 16),
    (2, (8, 8), (1.0, 1.0), 2, (0, 0), 4),
    (3, (4, 4, 4), (1.0, 1.0, 1.0), 3, (0, 1, 0), 8),
    (3, (4, 4, 4), (2 * math.pi,) * 3, 2, (1, 1, 1), 8),
]


def _ids(c):
    return f"d{c[0]}-{'x'.join(map(str, c[1]))}-k{c[3]}-p{''.join(map(str, c[4]))}"


def uD(x, t):
    d = x.shape[1]
    out = np.empty_like(x)
    out[:, 0] = np.sin(x[:, 0] + 2 * x[:, 1] + t)
    out[:, 1] = np.cos(x[:, 0] - x[:, 1]) * (1.0 + t)
    if d == 3:
        out[:, 2] = 0.5 * np.sin(x[:, 2] - t) + x[:, 0]
    return out


class UPair:
    def __init__(self, dim, nc, ext, k, per, coarse, nu=0.05, dt=0.05, t0=0.1):
        from paper_2107_07776_amd import Context
        print(f"[case] momentum multigrid dim={dim} cells={nc} k={k} periodic={per}", flush=True)
        self.gpu = Context(dim, nc, (0.0,) * dim, ext, k=k, nu=nu, dt=dt, periodic=per)
        self.gpu.mg_setup(degree=3, coarse_cells=coarse)
        mesh = BoxMesh(dim, nc, (0.0,) * dim, ext, per)
        self.disc = Discretization(mesh, k, nu=nu)
        self.ora = TRBDF2(self.disc, dt, uD=uD)
        g = self.ora.cst["gamma"]
        self.ts = {1: t0 + g * dt, 2: t0 + dt}
        if not all(per):
            pts = self.gpu.face_qpoints().cpu().numpy()
            for s in (1, 2):
                self.gpu.set_dirichlet(s - 1, torch.tensor(uD(pts, self.ts[s]), device="cuda"))
        self.tn = {s: self.ora.theta[s] * nu for s in (1, 2)}
        self.mg = {s: Multigrid(self.disc, self.ora.m(s) / self.tn[s], degree=3, coarse_cells=coarse,
                                field="u") for s in (1, 2)}

    def t(self, a):
        return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    @staticmethod
    def h(x):
        torch.cuda.synchronize()
        return x.cpu().numpy()


@pytest.fixture(scope="module", params=CASES, ids=_ids)
def up(request):
    p = UPair(*request.param)
    yield p
    p.gpu.close()


def test_hierarchy_and_eigenvalue_estimates(up):
    lv = up.gpu.mg_levels(field="u")
    ora = up.mg[1].levels
    assert len(lv) == len(ora)
    for g, o in zip(lv, ora):
        assert g["np"] == o.q + 1
        assert g["cells"][:up.disc.dim] == o.mesh.n_cells
        assert g["dofs"] == o.N
    for s in (1, 2):
        for l, lam in enumerate(up.mg[s].lam):
            assert abs(lv[l]["lam"][s - 1] - lam) <= 1e-9 * lam, (s, l, lv[l]["lam"], lam)
    # the pressure hierarchy is untouched by the momentum one
    assert up.gpu.mg_levels()[0]["np"] == up.disc.k


@pytest.mark.parametrize("stage", [1, 2])
def test_apply_matches_oracle_cycles(up, stage):
    d = up.disc
    v = synthetic.random_vector(d.N_u, 900 + stage)
    z = up.h(up.gpu.mg_apply_momentum(stage, up.t(v)))
    V = v.reshape(d.Nc, d.dim, d.nbu)
    zo = np.empty_like(V)
    for a in range(d.dim):
        zo[:, a, :] = (up.mg[stage].vcycle(V[:, a, :].reshape(-1)) / up.tn[stage]).reshape(d.Nc, d.nbu)
    zo = zo.reshape(-1)
    err = np.abs(z - zo).max() / np.abs(zo).max()
    print(f"momentum V-cycles stage {stage}: max rel diff {err:.3e}")
    assert err <= TOL_VC32


def test_preconditioned_gmres_meets_oracle_residual(up):
    d = up.disc
    tol = 1e-10
    for stage in (1, 2):
        w = 0.5 * synthetic.random_vector(d.N_u, 910 + stage)
        b = synthetic.random_vector(d.N_u, 920 + stage)
        its = {}
        for precond in ("mg_fp32", "line"):
            x = up.t(np.zeros(d.N_u))
            info = up.gpu.solve_momentum(stage, up.t(w), up.t(b), x, tol=tol, maxiter=3000,
                                         restart=30, precond=precond)
            r = b - up.ora.apply_momentum(stage, w, up.h(x), up.ts[stage])
            assert np.linalg.norm(r) <= 1.05 * tol * np.linalg.norm(b), precond
            its[precond] = info["iters"]
        print(f"stage {stage}: GMRES iterations {its}")
        assert its["mg_fp32"] <= 40, its


def test_diffusion_dominated_stage_needs_few_iterations():
    """nu dt / h^2 = 3.2 on a 32^2 walled box of Q4 (the Kovasznay
    workload's regime): the multigrid keeps GMRES at a few iterations per
    decade, the line blocks need several times more."""
    from paper_2107_07776_amd import Context
    nu, dt, n = 0.05, 0.064, 32
    ctx = Context(2, (n, n), (0.0, 0.0), (1.0, 1.0), k=4, nu=nu, dt=dt, periodic=(0, 0))
    try:
        pts = ctx.face_qpoints().cpu().numpy()
        for s in (0, 1):
            ctx.set_dirichlet(s, torch.tensor(uD(pts, 0.0), device="cuda"))
        xu = ctx.node_coords(0).cpu().numpy()
        w = torch.tensor(synthetic.nodal_velocity(uD(xu, 0.0), 2, 25), device="cuda")
        b = torch.tensor(synthetic.random_vector(ctx.N_u, 931), device="cuda")
        its = {}
        for precond in ("mg_fp32", "line"):
            x = torch.zeros_like(b)
            info = ctx.solve_momentum(2, w, b, x, tol=1e-8, maxiter=5000, restart=30, precond=precond)
            assert info["res_final"] <= 1e-8
            its[precond] = info["iters"]
        print(f"32^2 Q4 diffusion-dominated stage: GMRES iterations {its}")
        assert its["mg_fp32"] <= 30 and 3 * its["mg_fp32"] < its["line"], its
    finally:
        ctx.close()


def test_mapped_cells_gmres_meets_oracle_residual():
    """Q1-mapped Kovasznay cells (the box's levels as the preconditioner of
    the distorted operator)."""
    from paper_2107_07776_amd import Context
    lo, hi, nc, k, amp, nu, dt = (-0.5, -0.5), (1.0, 1.5), (8, 8), 4, 0.05, 0.025, 0.04
    ctx = Context(2, nc, lo, hi, k=k, nu=nu, dt=dt, periodic=(0, 0), mapping=1, map_amp=amp)
    try:
        ctx.mg_setup(degree=3, coarse_cells=16)
        vm = synthetic.sine_vertex_map(amp)
        disc = Discretization(BoxMesh(2, nc, lo, hi, (False, False), vertex_map=vm), k, nu=nu)
        ora = TRBDF2(disc, dt, uD=uD)
        g = ora.cst["gamma"]
        ts = {1: 0.1 + g * dt, 2: 0.1 + dt}
        pts = ctx.face_qpoints().cpu().numpy()
        for s in (1, 2):
            ctx.set_dirichlet(s - 1, torch.tensor(uD(pts, ts[s]), device="cuda"))
        tol = 1e-10
        for stage in (1, 2):
            w = 0.5 * synthetic.random_vector(disc.N_u, 940 + stage)
            b = synthetic.random_vector(disc.N_u, 950 + stage)
            x = torch.zeros(disc.N_u, dtype=torch.float64, device="cuda")
            info = ctx.solve_momentum(stage, torch.tensor(w, device="cuda"), torch.tensor(b, device="cuda"),
                                      x, tol=tol, maxiter=3000, precond="mg_fp32")
            torch.cuda.synchronize()
            r = b - ora.apply_momentum(stage, w, x.cpu().numpy(), ts[stage])
            assert np.linalg.norm(r) <= 1.05 * tol * np.linalg.norm(b)
            print(f"mapped stage {stage}: {info['iters']} iterations")
    finally:
        ctx.close()


def test_kovasznay_steps_with_momentum_multigrid_match_oracle():
    """Ten steps of the Kovasznay flow (Re = 40, 6 x 8 affine Q3-Q2 cells,
    exact Dirichlet data) with multigrid-preconditioned momentum and
    pressure solves against the oracle's direct-solve steps."""
    from paper_2107_07776_amd import Context
    Re, dt, k = 40.0, 0.02, 3
    lo, hi, nc = (-0.5, -0.5), (1.0, 1.5), (6, 8)
    ex = lambda x, t: synthetic.kovasznay(x, Re)[0]
    ctx = Context(2, nc, lo, hi, k=k, nu=1.0 / Re, dt=dt, periodic=(0, 0))
    try:
        pts = ctx.face_qpoints().cpu().numpy()
        data = torch.tensor(ex(pts, 0.0), device="cuda")
        ctx.set_dirichlet(0, data)
        ctx.set_dirichlet(1, data)
        disc = Discretization(BoxMesh(2, nc, lo, hi, (False, False)), k, nu=1.0 / Re)
        ora = TRBDF2(disc, dt, uD=ex)
        xu, xp = disc.node_coords("u"), disc.node_coords("p")
        u = synthetic.nodal_velocity(ex(xu, 0.0), 2, disc.nbu)
        p = synthetic.kovasznay(xp, Re)[1]
        U = torch.tensor(u, device="cuda")
        H = U.clone()
        P = torch.tensor(p, device="cuda")
        t = 0.0
        for n in range(10):
            info, st = ctx.step(U, H, P, t, n, mom_tol=1e-12, prs_tol=1e-10, mom_maxiter=2000,
                                prs_maxiter=500, precond="mg_fp32", mom_precond="mg_fp32", check=False)
            assert st == 0, (n, info)
            t += dt
        ue, he, pe = u, u.copy(), p
        t = 0.0
        for n in range(10):
            ue, he, pe, _ = ora.step(ue, he, pe, t)
            t += dt
        torch.cuda.synchronize()
        du = np.linalg.norm(U.cpu().numpy() - ue) / np.linalg.norm(ue)
        dp = np.linalg.norm(P.cpu().numpy() - pe) / np.linalg.norm(pe)
        print(f"Kovasznay with momentum multigrid: GPU vs oracle u {du:.2e}, p {dp:.2e}")
        assert du < 1e-9 and dp < 1e-7
    finally:
        ctx.close()


def test_errors():
    from paper_2107_07776_amd import Context
    from paper_2107_07776_amd.trbdg import TrbdgError
    ctx = Context(2, (4, 4), (0.0, 0.0), (1.0, 1.0), k=2, nu=0.0, dt=0.01)
    try:
        v = torch.zeros(ctx.N_u, dtype=torch.float64, device="cuda")
        with pytest.raises(TrbdgError, match="EINVAL"):
            ctx.mg_apply_momentum(1, v)
        with pytest.raises(TrbdgError, match="EUNSUPPORTED"):
            ctx.solve_momentum(1, v, v, v.clone(), precond="mg_bf16")
    finally:
        ctx.close()
