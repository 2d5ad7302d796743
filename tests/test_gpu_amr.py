"""Adaptive 2D meshes with hanging nodes on the GPU (tbdg_amr_*) against the
oracle (oracle/adaptive.py): the same flags give the same forest cell for
cell; the pressure Helmholtz operator, its diagonal, the indicator and the
field transfer agree to FP64 rounding; the marking agrees flag for flag on
the same indicator; the block- and point-Jacobi CG solves reach their
tolerance and the oracle's direct solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synthetic
from oracle.adaptive import AdaptiveDisc, QuadForest, mark, transfer

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _pair(seed, n_cells, periodic, k, max_level=3, rounds=3, lo=(0.0, 0.0), hi=(1.5, 1.0)):
    """A GPU mesh and an oracle forest driven by the same random flags."""
    from paper_2107_07776_amd import Adaptive
    print(f"[case] amr seed={seed} cells={n_cells} periodic={periodic} k={k}", flush=True)
    g = Adaptive(n_cells, lo, hi, k, max_level, periodic=periodic)
    f = QuadForest(n_cells, lo, hi, periodic, max_level)
    rng = np.random.default_rng(seed)
    for _ in range(rounds):
        flags = rng.choice([-1, 0, 1], size=f.N, p=[0.35, 0.35, 0.3]).astype(np.int8)
        g.adapt(flags)
        f = f.adapt(flags)
        assert [tuple(r) for r in g.leaves().tolist()] == f.leaves
    return g, f


CASES = [(0, (3, 2), (0, 0), 2), (1, (3, 2), (1, 0), 3), (2, (4, 3), (1, 1), 4), (3, (2, 5), (0, 1), 3)]


@pytest.mark.parametrize("seed,nc,per,k", CASES)
def test_pressure_operator_and_diagonal_match_oracle(seed, nc, per, k):
    g, f = _pair(seed, nc, per, k)
    try:
        ad = AdaptiveDisc(f, k)
        alpha = 7.5
        A = ad.helmholtz_p(alpha)
        p = synthetic.random_vector(ad.N_p, seed)
        y = g.apply_pressure(alpha, _t(p)).cpu().numpy()
        ref = A @ p
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
        d = g.diag_pressure(alpha).cpu().numpy()
        assert np.abs(d - A.diagonal()).max() <= 1e-12 * np.abs(A.diagonal()).max()
    finally:
        g.close()


def test_penalty_multiplier_and_alpha_zero():
    from paper_2107_07776_amd import Adaptive
    f = QuadForest((3, 3), (0.0, 0.0), (1.0, 1.0), (0, 0), 2)
    g = Adaptive((3, 3), (0.0, 0.0), (1.0, 1.0), 3, 2, pen_p=2.5)
    try:
        flags = np.zeros(f.N, dtype=np.int8)
        flags[4] = 1
        g.adapt(flags)
        f = f.adapt(flags)
        ad = AdaptiveDisc(f, 3, pen_p=2.5)
        p = synthetic.random_vector(ad.N_p, 9)
        y = g.apply_pressure(0.0, _t(p)).cpu().numpy()
        ref = ad.sip_p() @ p
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    finally:
        g.close()


# k <= 4: cell-block Jacobi; k = 5 (25 nodes per cell): point Jacobi
@pytest.mark.parametrize("seed,nc,per,k", CASES[:3] + [(4, (3, 2), (1, 0), 5)])
def test_cg_solve_reaches_tolerance_and_direct_solution(seed, nc, per, k):
    g, f = _pair(seed, nc, per, k)
    try:
        ad = AdaptiveDisc(f, k)
        alpha = 3.0
        A = ad.helmholtz_p(alpha)
        b = synthetic.random_vector(ad.N_p, 100 + seed)
        x = torch.zeros(ad.N_p, dtype=torch.float64, device="cuda")
        info = g.solve_pressure(alpha, _t(b), x, tol=1e-13, maxiter=20000)
        xs = x.cpu().numpy()
        assert np.linalg.norm(b - A @ xs) <= 1e-12 * np.linalg.norm(b)
        xd = spla.spsolve(A.tocsc(), b)
        assert np.abs(xs - xd).max() <= 1e-7 * np.abs(xd).max(), info
        # a converged start returns at once
        info2 = g.solve_pressure(alpha, _t(b), x, tol=1e-9)
        assert info2["iters"] == 0
    finally:
        g.close()


@pytest.mark.parametrize("k,base", [(3, (192, 160)), (5, (120, 96))])
def test_cg_solve_above_the_in_kernel_reduction_size(k, base):
    """Past 1024 blocks of partial sums the CG sums them with one-block
    kernels between its two fused kernels instead of in the consumer; the
    solve must still reach its tolerance in the true residual (the operator
    itself is pinned at large sizes by the sampled-rows test)."""
    from paper_2107_07776_amd import Adaptive
    print(f"[case] amr large CG k={k} base={base}", flush=True)
    g = Adaptive(base, (0.0, 0.0), (1.5, 1.0), k, 2, periodic=(1, 0))
    try:
        rng = np.random.default_rng(k)
        g.adapt(rng.choice([0, 1], size=g.N_c, p=[0.85, 0.15]).astype(np.int8))
        assert g.N_c * k * k > 1024 * 256       # more than 1024 operator blocks
        b = _t(rng.standard_normal(g.N_p))
        x = torch.zeros_like(b)
        info = g.solve_pressure(3.0, b, x, tol=1e-10, maxiter=50000)
        y = torch.empty_like(b)
        g.apply_pressure(3.0, x, y)
        assert (b - y).norm().item() <= 2e-10 * b.norm().item(), info
    finally:
        g.close()


@pytest.mark.parametrize("seed,nc,per,k", CASES)
def test_indicator_matches_oracle(seed, nc, per, k):
    g, f = _pair(seed, nc, per, k)
    try:
        ad = AdaptiveDisc(f, k)
        u = synthetic.random_vector(ad.N_u, 200 + seed)
        eta = g.indicator(_t(u)).cpu().numpy()
        ref = ad.indicator(u)
        assert np.abs(eta - ref).max() <= 1e-12 * np.abs(ref).max()
    finally:
        g.close()


@pytest.mark.parametrize("seed,nc,per,k", CASES[:2])
def test_marking_matches_oracle_on_the_same_indicator(seed, nc, per, k):
    g, f = _pair(seed, nc, per, k, max_level=4)
    try:
        rng = np.random.default_rng(seed)
        eta = rng.random(f.N)
        eta[::7] = eta[3]          # ties
        for rf, cf, hmin, hmax in ((0.1, 0.3, 0.0, np.inf), (0.25, 0.5, 0.1, 0.6), (0.0, 1.0, 0.0, np.inf),
                                   (1.0, 0.0, 0.0, np.inf)):
            fl = g.mark(_t(eta), rf, cf, hmin, hmax)
            ref = mark(eta, f, rf, cf, hmin, hmax)
            assert np.array_equal(fl.astype(np.int64), ref), (rf, cf, hmin, hmax)
    finally:
        g.close()


@pytest.mark.parametrize("seed,nc,per,k", CASES)
def test_adapt_transfers_fields_like_oracle(seed, nc, per, k):
    g, f = _pair(seed, nc, per, k, max_level=4, rounds=2)
    try:
        rng = np.random.default_rng(50 + seed)
        for step in range(3):
            u = synthetic.random_vector(2 * f.N * (k + 1) ** 2, 300 + step)
            p = synthetic.random_vector(f.N * k * k, 400 + step)
            flags = rng.choice([-1, 0, 1], size=f.N).astype(np.int8)
            un, pn = g.adapt(flags, [("u", _t(u)), ("p", _t(p))])
            f2 = f.adapt(flags)
            assert [tuple(r) for r in g.leaves().tolist()] == f2.leaves
            ru = transfer(f, f2, u, k + 1, 2)
            rp = transfer(f, f2, p, k, 1)
            assert np.abs(un.cpu().numpy() - ru).max() <= 1e-13 * np.abs(ru).max()
            assert np.abs(pn.cpu().numpy() - rp).max() <= 1e-13 * np.abs(rp).max()
            f = f2
        # no flags: nothing changes
        p = synthetic.random_vector(f.N * k * k, 7)
        (pn,) = g.adapt(np.zeros(f.N, dtype=np.int8), [("p", _t(p))])
        assert np.array_equal(pn.cpu().numpy(), p)
    finally:
        g.close()


def test_indicator_driven_remeshing_of_a_vortex():
    """eta of a Taylor-Green field drives three rounds of marking (10 % /
    30 %) and remeshing with transfer; the GPU and the oracle stay equal."""
    from paper_2107_07776_amd import Adaptive
    k = 3
    L = 2 * np.pi
    g = Adaptive((4, 4), (0.0, 0.0), (L, L), k, 3, periodic=(1, 1))
    f = QuadForest((4, 4), (0.0, 0.0), (L, L), (1, 1), 3)
    try:
        ad = AdaptiveDisc(f, k)
        xu = ad.node_coords("u")
        u = synthetic.nodal_velocity(synthetic.taylor_green_2d(xu, 0.0, 100.0)[0], 2, ad.nbu)
        U = _t(u)
        for _ in range(3):
            eta = g.indicator(U)
            ad = AdaptiveDisc(f, k)
            ref = ad.indicator(u)
            assert np.abs(eta.cpu().numpy() - ref).max() <= 1e-12 * ref.max()
            flags = g.mark(eta, 0.1, 0.3, 0.0, np.inf)
            (U,) = g.adapt(flags, [("u", U)])
            f2 = f.adapt(flags)
            u = transfer(f, f2, u, k + 1, 2)
            f = f2
            assert np.abs(U.cpu().numpy() - u).max() <= 1e-12 * np.abs(u).max()
        assert f.N > 16
    finally:
        g.close()


def test_errors():
    from paper_2107_07776_amd import Adaptive
    from paper_2107_07776_amd.trbdg import TrbdgError
    with pytest.raises(TrbdgError):
        Adaptive((1, 2), (0.0, 0.0), (1.0, 1.0), 2, 2, periodic=(1, 0))   # periodic needs >= 2
    with pytest.raises(TrbdgError):
        Adaptive((2, 2), (0.0, 0.0), (1.0, 1.0), 0, 2)
    g = Adaptive((2, 2), (0.0, 0.0), (1.0, 1.0), 2, 2)
    try:
        x = torch.zeros(g.N_p, dtype=torch.float64, device="cuda")
        with pytest.raises(TrbdgError):
            g.solve_pressure(0.0, x.clone(), x)      # alpha must be > 0
        assert g.lib.tbdg_amr_transfer(g.h, 1, None, None) == -1   # nothing planned
        eta = torch.full((g.N_c,), float("nan"), dtype=torch.float64, device="cuda")
        with pytest.raises(TrbdgError):
            g.mark(eta)
    finally:
        g.close()


MOM_CASES = [(4, (3, 2), (0, 0), 2), (5, (3, 2), (1, 0), 3), (6, (4, 3), (1, 1), 3), (7, (2, 5), (0, 1), 4)]


@pytest.mark.parametrize("seed,nc,per,k", MOM_CASES)
def test_momentum_operator_matches_oracle(seed, nc, per, k):
    """mc M + tnu A + th C(w) on both components, random w and u, wall data
    from a smooth field at the wall points (exported in the oracle's order)."""
    g, f = _pair(seed, nc, per, k)
    try:
        ad = AdaptiveDisc(f, k)
        xb = g.face_qpoints().cpu().numpy()
        assert np.abs(xb - ad.boundary_points()).max() < 1e-14 if len(xb) else True
        uD = np.stack([np.sin(xb[:, 0] + 2 * xb[:, 1]), np.cos(3 * xb[:, 0] - xb[:, 1])], 1) \
            if len(xb) else np.zeros((0, 2))
        w = synthetic.random_vector(ad.N_u, 500 + seed)
        u = synthetic.random_vector(ad.N_u, 600 + seed)
        for mc, tnu, th in ((3.0, 0.01, 0.5), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)):
            y = g.apply_momentum(mc, tnu, th, _t(w), _t(u), _t(uD) if len(xb) else None)
            ref = ad.apply_momentum(mc, tnu, th, w, u, uD)
            err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
            assert err <= 1e-12, (mc, tnu, th, err)
    finally:
        g.close()


def test_momentum_walls_need_data():
    from paper_2107_07776_amd import Adaptive
    from paper_2107_07776_amd.trbdg import TrbdgError
    g = Adaptive((2, 2), (0.0, 0.0), (1.0, 1.0), 2, 2, periodic=(1, 0))
    try:
        u = torch.zeros(g.N_u, dtype=torch.float64, device="cuda")
        with pytest.raises(TrbdgError):
            g.apply_momentum(1.0, 1.0, 1.0, u, u.clone())
        uD = torch.zeros((g.face_qpoints().shape[0], 2), dtype=torch.float64, device="cuda")
        with pytest.raises(TrbdgError):
            g.apply_momentum(1.0, 1.0, 1.0, u.clone(), u, uD, out=u)   # y aliases u
    finally:
        g.close()


@pytest.mark.parametrize("seed,nc,per,k", MOM_CASES[:3])
def test_momentum_gmres_reaches_tolerance_and_direct_solution(seed, nc, per, k):
    """A TR-BDF2 stage-like operator (mass 1/(gamma dt), theta nu = 0.01 / 2,
    advection 1/2) with a random advecting field: GMRES(20) to 1e-12, the
    true residual against the oracle's assembled operator and its direct
    solution per component."""
    import scipy.sparse.linalg as spla
    g, f = _pair(seed, nc, per, k)
    try:
        ad = AdaptiveDisc(f, k)
        xb = g.face_qpoints().cpu().numpy()
        uD = np.stack([np.sin(xb[:, 0]), np.cos(xb[:, 1])], 1) if len(xb) else np.zeros((0, 2))
        w = synthetic.random_vector(ad.N_u, 700 + seed)
        b = synthetic.random_vector(ad.N_u, 800 + seed)
        mc, tnu, th = 1.0 / (0.5858 * 0.02), 0.005, 0.5
        x = torch.zeros(ad.N_u, dtype=torch.float64, device="cuda")
        with pytest.raises(RuntimeError):     # the basis holds at most 60 vectors
            g.solve_momentum(mc, tnu, th, _t(w), _t(b), x, _t(uD) if len(xb) else None, tol=1e-12,
                             maxiter=4000, restart=61)
        info = g.solve_momentum(mc, tnu, th, _t(w), _t(b), x, _t(uD) if len(xb) else None, tol=1e-12,
                                maxiter=4000, restart=20)
        xs = x.cpu().numpy()
        r = b - ad.apply_momentum(mc, tnu, th, w, xs, uD)
        assert np.linalg.norm(r) <= 1.01e-12 * np.linalg.norm(b), info
        A = (mc * ad.mass_u() + tnu * ad.sip_u() + th * ad.lf_advection(w, uD)).tocsc()
        B = b.reshape(f.N, 2, ad.nbu)
        for comp in range(2):
            xd = spla.spsolve(A, B[:, comp, :].reshape(-1))
            xc = xs.reshape(f.N, 2, ad.nbu)[:, comp, :].reshape(-1)
            assert np.abs(xc - xd).max() <= 1e-9 * np.abs(xd).max()
    finally:
        g.close()


# ---------------------------------------------------------------------------
# stage functionals and the TR-BDF2 step on adapted meshes
# ---------------------------------------------------------------------------
STEP_CASES = [(8, (3, 2), (0, 0), 2), (9, (4, 3), (1, 0), 3), (10, (3, 3), (1, 1), 3)]


def _kov(x, t=0.0):
    return synthetic.kovasznay(x - 0.5, 40.0)[0]


def _kov_shifted(x, t=0.0):
    return synthetic.kovasznay(x - np.array([0.5, 0.13]), 40.0)[0]


@pytest.mark.parametrize("seed,nc,per,k", STEP_CASES)
def test_stage_functionals_match_oracle(seed, nc, per, k):
    from oracle import TRBDF2
    g, f = _pair(seed, nc, per, k, lo=(0.0, 0.0), hi=(1.5, 1.0))
    try:
        nu, dt = 0.02, 0.01
        g.set_flow(nu, dt)
        ad = AdaptiveDisc(f, k, nu=nu)
        ora = TRBDF2(ad, dt, uD=_kov)
        xb = g.face_qpoints().cpu().numpy()
        uD = _t(_kov(xb)) if len(xb) else None
        rv = lambda n, sd: synthetic.random_vector(n, sd)
        u_n, u_g, w, wex = (rv(ad.N_u, 900 + seed + 10 * q) for q in range(4))
        p = rv(ad.N_p, 950 + seed)
        for s in (1, 2):
            for we in (None, wex):
                if s == 2 and we is not None:
                    continue
                y = g.rhs_momentum(s, _t(u_n), _t(u_g), _t(w), _t(p), uD,
                                   _t(we) if we is not None else None).cpu().numpy()
                ref = ora.rhs_momentum(s, u_n, u_g, w, p, 0.0, w_explicit=we)
                assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max(), (s, we is None)
            b = g.rhs_pressure(s, _t(u_n), _t(p)).cpu().numpy()
            ref = ora.rhs_pressure(s, u_n, p)
            assert np.abs(b - ref).max() <= 1e-12 * np.abs(ref).max(), s
        y = g.add_grad_p(_t(u_g), -0.3, _t(p)).cpu().numpy()
        ref = u_g - 0.3 * ora.grad_p(p)
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    finally:
        g.close()


@pytest.mark.parametrize("seed,nc,per,k", STEP_CASES)
@pytest.mark.parametrize("nonlinear", [1, 2])
def test_trbdf2_steps_match_oracle(seed, nc, per, k, nonlinear):
    """Three steps of a Kovasznay field (walls where not periodic) on a mesh
    with hanging nodes, tight solves, against the oracle's sparse-LU steps."""
    from oracle import TRBDF2
    g, f = _pair(seed, nc, per, k, lo=(0.0, 0.0), hi=(1.5, 1.0))
    try:
        nu, dt = 0.025, 0.01
        g.set_flow(nu, dt)
        ad = AdaptiveDisc(f, k, nu=nu)
        ora = TRBDF2(ad, dt, uD=_kov, nonlinear_iters=nonlinear)
        xb = g.face_qpoints().cpu().numpy()
        uD = _t(_kov(xb)) if len(xb) else None
        xu = ad.node_coords("u")
        u = synthetic.nodal_velocity(_kov(xu), 2, ad.nbu)
        p = np.cos(xu[::ad.nbu, 0].repeat(ad.nbp))   # a cellwise-constant start
        U, H, P = _t(u), _t(u), _t(p)
        uo, ho, po = u.copy(), u.copy(), p.copy()
        t = 0.0
        for n in range(3):
            info, st = g.step(U, H, P, uD, nonlinear=nonlinear, mom_tol=1e-13, prs_tol=1e-13)
            assert st == 0, info
            uo, ho, po, _ = ora.step(uo, ho, po, t)
            t += dt
        du = np.linalg.norm(U.cpu().numpy() - uo) / np.linalg.norm(uo)
        dp = np.linalg.norm(P.cpu().numpy() - po) / np.linalg.norm(po)
        print(f"adaptive step: u {du:.2e}, p {dp:.2e}")
        assert du < 1e-9 and dp < 1e-8
    finally:
        g.close()


@pytest.mark.parametrize("check_tol", [0.0, 1e9])
def test_adaptive_schedule_matches_oracle(check_tol):
    """The schedule of Sec. 4 on a walled Kovasznay field: six steps,
    remeshing after step 4 and, while the last step changed the velocity by
    more than check_tol, after every second step (check_tol 0: steps 2, 4,
    6; 1e9: step 4 only); the oracle repeats it with its own indicator,
    marking, forest and transfer.  The field is shifted off the mesh's
    mirror line y = 1/2 (the Kovasznay flow is even in y there), so that no
    two cells tie in the indicator and both sides mark the same cells."""
    from oracle import TRBDF2
    from paper_2107_07776_amd import Adaptive
    k, nu, dt = 2, 0.025, 0.01
    lo, hi = (0.0, 0.0), (1.5, 1.0)
    g = Adaptive((3, 2), lo, hi, k, 3)
    f = QuadForest((3, 2), lo, hi, (0, 0), 3)
    try:
        g.set_flow(nu, dt)
        ad = AdaptiveDisc(f, k, nu=nu)
        xu = ad.node_coords("u")
        u = synthetic.nodal_velocity(_kov_shifted(xu), 2, ad.nbu)
        p = np.zeros(ad.N_p)
        U, H, P = _t(u), _t(u), _t(p)
        U, H, P, log = g.simulate(U, H, P, _kov_shifted, 6, remesh_every=4, check_every=2, check_tol=check_tol,
                                  refine_frac=0.2, coarsen_frac=0.2, mom_tol=1e-13, prs_tol=1e-13)
        want = [2, 4, 6] if check_tol == 0.0 else [4]
        assert [s for s, _ in log[1:]] == want
        uh = u.copy()
        t = 0.0
        for n in range(1, 7):
            ad = AdaptiveDisc(f, k, nu=nu)
            u, uh, p, _ = TRBDF2(ad, dt, uD=_kov_shifted).step(u, uh, p, t)
            t += dt
            if n in want:
                fl = mark(ad.indicator(u), f, 0.2, 0.2)
                f2 = f.adapt(fl)
                u, uh = transfer(f, f2, u, k + 1, 2), transfer(f, f2, uh, k + 1, 2)
                p = transfer(f, f2, p, k, 1)
                f = f2
        assert [tuple(r) for r in g.leaves().tolist()] == f.leaves
        assert np.linalg.norm(U.cpu().numpy() - u) <= 1e-9 * np.linalg.norm(u)
        assert np.linalg.norm(P.cpu().numpy() - p) <= 1e-8 * np.linalg.norm(p)
    finally:
        g.close()


def test_full_size_adaptive_operators_sampled():
    """The adaptive workload's mesh (512^2 base cells, Q3-Q2, two levels of
    hanging nodes, refined by the vortex field's indicator as the benchmark
    does): sampled rows of the pressure Helmholtz and momentum operators,
    coarse-fine cells included, against the oracle's row-restricted forms."""
    import bench
    from paper_2107_07776_amd import Adaptive
    k, base, maxl = 3, 512, 2
    L = 2 * np.pi
    H = L / base
    print(f"[case] amr full size base={base} k={k}", flush=True)
    g = Adaptive((base, base), (0.0, 0.0), (L, L), k, maxl, periodic=(1, 1))
    try:
        x = bench.amr_nodes(g.leaves(), H, k)
        uv = bench.amr_vortices(x)
        n = (k + 1) ** 2
        u = np.empty(g.N_u)
        u.reshape(-1, 2, n)[:, 0, :] = uv[:, 0].reshape(-1, n)
        u.reshape(-1, 2, n)[:, 1, :] = uv[:, 1].reshape(-1, n)
        U = _t(u)
        for _ in range(3):
            flags = g.mark(g.indicator(U), 0.1, 0.3, H / 4, H)
            (U,) = g.adapt(flags, [("u", U)])
        lv = g.leaves()
        assert (lv[:, 0] == 2).sum() > 0 and (lv[:, 0] == 0).sum() > 0
        f = QuadForest((base, base), (0.0, 0.0), (L, L), (1, 1), maxl, leaves=[tuple(r) for r in lv.tolist()])
        assert f.leaves == [tuple(r) for r in lv.tolist()]
        rng = np.random.default_rng(17)
        hang = [c for c in rng.choice(f.N, size=4000, replace=False).tolist()
                if any(f.neighbours(c, a, s)[0] in ("c", "f") for a in range(2) for s in (0, 1))]
        cells = sorted(set(hang[:24] + rng.choice(f.N, size=16, replace=False).tolist()))
        assert len(hang) >= 24
        ad = AdaptiveDisc(f, k)
        alpha = 3.0
        p = synthetic.random_vector(ad.N_p, 71)
        y = g.apply_pressure(alpha, _t(p)).cpu().numpy()
        ref = ad.helmholtz_p(alpha, cells) @ p
        rp = np.concatenate([np.arange(c * ad.nbp, (c + 1) * ad.nbp) for c in cells])
        assert np.abs(y[rp] - ref[rp]).max() <= 1e-12 * np.abs(ref[rp]).max()
        w = U.cpu().numpy()
        uu = synthetic.random_vector(ad.N_u, 72)
        ym = g.apply_momentum(40.0, 0.002, 0.5, U, _t(uu)).cpu().numpy()
        refm = ad.apply_momentum(40.0, 0.002, 0.5, w, uu, None, cells)
        rv = np.concatenate([np.arange(c * 2 * ad.nbu, (c + 1) * 2 * ad.nbu) for c in cells])
        assert np.abs(ym[rv] - refm[rv]).max() <= 1e-12 * np.abs(refm[rv]).max()
    finally:
        g.close()
