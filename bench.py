"""Benchmark: TR-BDF2 steps/s of the DG projection scheme on one MI355X.

Default workload (one step = both TR-BDF2 stages with all their implicit
solves): 3D periodic Taylor-Green vortex on [0, 2 pi]^3, 64^3 hexahedra,
velocity degree 3 / pressure degree 2 (50 331 648 + 7 077 888 DoFs),
nu = 1/1600, dt = 2 pi / 192 (Courant number 1), fully nonlinear momentum
predictors (two fixed-point solves per stage: at this Courant number the
linearised predictor with the extrapolated advecting velocity is unstable),
every solve to a 1e-8 relative FP64 residual.  The timed solver is the
mixed-precision one: FP32 h/p-multigrid preconditioner under FP64 flexible
CG for the pressure, started from the learned guess (3D CNN trained on the
solver's own increments, previous-increment fallback judged by the FP64
residual), line-block-preconditioned GMRES for the momentum.  Timed beside
it from the same initial state: the plain FP64 solver (Jacobi CG, Jacobi
GMRES); the two final fields are compared ("equal error").  Also reported:
the same solver with the BF16-storage smoother, the held-out evaluation of
the pressure initial guesses, the event-timed operator kernels (in a
separate run, so the timed steps carry no measurement hooks) and the CPU
oracle on a bounded sample.  Synthetic data: the closed-form initial vortex;
seeded random-phase fields for the guess network.  Inputs are resident in
HBM before timing starts.

Prints one JSON line.  `--gpus N` with N > 1 is refused: the library runs
on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TR-BDF2 steps/s & operator GDoF/s vs plain FP64 at equal L2 error"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    if name == "tgv32":
        return dict(dim=3, n=(32, 32, 32), ext=(2 * math.pi,) * 3, k=3, nu=1.0 / 1600.0,
                    dt=2 * math.pi / 96.0, tol=1e-8, nonlinear=2,
                    label="3D periodic Taylor-Green vortex, 32^3 hexes, Q3-Q2, nu=1/1600, "
                          "dt=2pi/96 (C=1), fully nonlinear stages (2 fixed-point momentum "
                          "solves per stage), solves to 1e-8 relative FP64 residual")
    if name == "tgv64":
        return dict(dim=3, n=(64, 64, 64), ext=(2 * math.pi,) * 3, k=3, nu=1.0 / 1600.0,
                    dt=2 * math.pi / 192.0, tol=1e-8, nonlinear=2,
                    label="3D periodic Taylor-Green vortex, 64^3 hexes, Q3-Q2, nu=1/1600, "
                          "dt=2pi/192 (C=1), fully nonlinear stages (2 fixed-point momentum "
                          "solves per stage), solves to 1e-8 relative FP64 residual")
    if name == "kov256":
        return dict(dim=2, n=(256, 256), lo=(-0.5, -0.5), ext=(1.5, 2.0), k=4, nu=1.0 / 40.0,
                    dt=0.04, tol=1e-8, nonlinear=2, periodic=(0, 0), mapping=1, amp=0.05, Re=40.0,
                    mom_precond="mg_fp32", restart=30, learned=False,
                    label="2D Kovasznay flow (Re=40) on [-0.5,1]x[-0.5,1.5], 256x256 quads mapped by "
                          "x+0.05 sin(2pi x) sin(2pi y) (Q1 cells), Q4-Q3, Dirichlet velocity data "
                          "from the exact solution, dt=0.04 from rest, fully nonlinear stages (2 "
                          "fixed-point momentum solves per stage), solves to 1e-8 relative FP64 residual")
    if name == "tg2d":
        return dict(dim=2, n=(8, 8), ext=(1.0, 1.0), k=2, nu=0.01, dt=0.01, tol=1e-10, nonlinear=1,
                    label="2D periodic Taylor-Green, 8x8 quads, Q2-Q1, nu=0.01, dt=0.01, tol 1e-10")
    raise SystemExit(f"unknown workload {name}")


def make_context(W):
    """Library context of the workload; Dirichlet data (time independent) set
    at the boundary points when the mesh has walls."""
    import torch

    from paper_2107_07776_amd import Context

    import synthetic
    dim = W["dim"]
    lo = W.get("lo", (0.0,) * dim)
    hi = tuple(a + e for a, e in zip(lo, W["ext"]))
    ctx = Context(dim, W["n"], lo, hi, k=W["k"], nu=W["nu"], dt=W["dt"],
                  periodic=W.get("periodic", (1,) * dim), mapping=W.get("mapping", 0),
                  map_amp=W.get("amp", 0.0))
    if "Re" in W:
        pts = ctx.face_qpoints().cpu().numpy()
        data = torch.tensor(synthetic.kovasznay(pts, W["Re"])[0], device="cuda")
        ctx.set_dirichlet(0, data)
        ctx.set_dirichlet(1, data)
    return ctx


def initial_fields(W, coords_u, coords_p):
    import numpy as np

    import synthetic
    dim = W["dim"]
    nbu = (W["k"] + 1) ** dim
    if "Re" in W:
        # impulsive start: fluid at rest, the wall data switched on at t = 0
        return np.zeros(coords_u.shape[0] * dim), np.zeros(coords_p.shape[0]), None
    if dim == 3:
        u = synthetic.tgv3d_velocity(coords_u)
        p = synthetic.tgv3d_pressure(coords_p)
        return synthetic.nodal_velocity(u, 3, nbu), p, None
    u, _ = synthetic.taylor_green_2d_unit(coords_u, 0.0, W["nu"])
    _, p = synthetic.taylor_green_2d_unit(coords_p, 0.0, W["nu"])
    g = 2.0 - math.sqrt(2.0)
    uh, _ = synthetic.taylor_green_2d_unit(coords_u, -(1 - g) * W["dt"], W["nu"])
    return synthetic.nodal_velocity(u, 2, nbu), p, synthetic.nodal_velocity(uh, 2, nbu)


def kovasznay_errors(ctx, W, U, P):
    """L2 errors of the discrete velocity and of the mean-free pressure
    against the exact Kovasznay solution, by Gauss-Legendre quadrature at the
    nodes of each field on the bilinear (Q1-mapped) cells: the nodes are the
    quadrature points, so the integrals need only the nodal values, the
    weights and det J of the bilinear map of each cell's four mapped
    vertices.  Returns (abs, relative) pairs."""
    import numpy as np

    import synthetic
    nx, ny = W["n"]
    lo, ext = np.array(W["lo"]), np.array(W["ext"])
    h = ext / np.array([nx, ny])
    vmap = synthetic.sine_vertex_map(W["amp"])

    def quad(npts, coords):
        g, w = np.polynomial.legendre.leggauss(npts)
        g, w = 0.5 * (g + 1.0), 0.5 * w
        xi, eta = np.meshgrid(g, g, indexing="xy")          # node a + npts*b: x fastest
        xi, eta = xi.reshape(-1), eta.reshape(-1)
        wq = np.outer(w, w).reshape(-1)
        i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
        i, j = i.reshape(-1), j.reshape(-1)                  # cells x fastest
        V = [vmap(np.stack([lo[0] + (i + a) * h[0], lo[1] + (j + b) * h[1]], 1))
             for (a, b) in ((0, 0), (1, 0), (0, 1), (1, 1))]
        X = sum(V[q][:, None, :] * N[None, :, None] for q, N in
                enumerate(((1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta)))
        dxi = (V[1] - V[0])[:, None, :] * (1 - eta)[None, :, None] + (V[3] - V[2])[:, None, :] * eta[None, :, None]
        deta = (V[2] - V[0])[:, None, :] * (1 - xi)[None, :, None] + (V[3] - V[1])[:, None, :] * xi[None, :, None]
        detj = dxi[..., 0] * deta[..., 1] - dxi[..., 1] * deta[..., 0]
        if np.abs(X.reshape(-1, 2) - coords).max() > 1e-11:
            raise SystemExit("quadrature nodes disagree with the library's node coordinates")
        return (wq[None, :] * detj).reshape(-1)

    xu, xp = ctx.node_coords(0).cpu().numpy(), ctx.node_coords(1).cpu().numpy()
    wu, wp = quad(W["k"] + 1, xu), quad(W["k"], xp)
    ue, pe = synthetic.kovasznay(xu, W["Re"])[0], synthetic.kovasznay(xp, W["Re"])[1]
    nb = (W["k"] + 1) ** 2
    uh = U.cpu().numpy().reshape(-1, 2, nb).transpose(0, 2, 1).reshape(-1, 2)
    ph = P.cpu().numpy()
    eu = math.sqrt(np.sum(wu[:, None] * (uh - ue) ** 2))
    nu_ = math.sqrt(np.sum(wu[:, None] * ue ** 2))
    area = wp.sum()
    ph0, pe0 = ph - np.dot(wp, ph) / area, pe - np.dot(wp, pe) / area
    ep = math.sqrt(np.sum(wp * (ph0 - pe0) ** 2))
    np_ = math.sqrt(np.sum(wp * pe0 ** 2))
    return {"u_l2": eu, "u_l2_rel": eu / nu_, "p_mean_free_l2": ep, "p_mean_free_l2_rel": ep / np_,
            "area": float(area)}


# the library's measurement hook times every third launch of an operator kernel
LAUNCH_SAMPLE_STRIDE = 3

TRAFFIC_FILES = {("momentum_apply", "tgv32"): "momentum_face_tgv32_q3_traffic.txt",
                 ("momentum_apply", "tgv64"): "momentum_face_tgv64_q3_traffic.txt",
                 ("amr_pressure", "amr2d"): "amr_pressure_amr2d_q3_traffic.txt"}

# the kernel sources each byte-counter summary depends on
TRAFFIC_SOURCES = {"momentum_apply": ("lines.hip", "lines.hpp", "internal.hpp"),
                   "amr_pressure": ("amr.hip", "amr.hpp")}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed byte-counter
    summary of this workload (rocprofv3 FETCH_SIZE and WRITE_SIZE, each
    scaled by the reading of a plain device copy of known size), or None.
    The summary names the source revision of the kernels it measured; when
    the kernel sources have changed since, the figure is not used."""
    name = TRAFFIC_FILES.get((kernel, workload))
    if not name:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    src = vals.get("kernel_source_sha256")
    if src is None or src != kernel_source_digest(TRAFFIC_SOURCES[kernel]):
        return None
    out = {"bytes_per_launch": float(vals["traffic_bytes_per_launch"]), "source": f"profiles/{name}"}
    if "traffic_bytes_per_pressure_dof" in vals:
        out["bytes_per_dof"] = float(vals["traffic_bytes_per_pressure_dof"])
    return out


def kernel_source_digest(files=("lines.hip", "lines.hpp", "internal.hpp")):
    """SHA-256 over the HIP sources of an operator kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2107_07776_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def cpu_baseline(W, seconds_budget=20.0):
    """The oracle's TR-BDF2 step on a bounded sample of the same workload: the
    same domain, degree, nu and dt on a 4^3 (3D) or at most 16^2 (2D) mesh,
    scaled to the full workload by velocity DoF count (per-DoF
    extrapolation)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synthetic
    from oracle import BoxMesh, Discretization, TRBDF2

    dim = W["dim"]
    ns = 4 if dim == 3 else min(W["n"][0], 16)
    nc = (ns,) * dim
    lo = W.get("lo", (0.0,) * dim)
    hi = tuple(a + e for a, e in zip(lo, W["ext"]))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        if "Re" in W:
            mesh = BoxMesh(dim, nc, lo, hi, (False,) * dim,
                           vertex_map=synthetic.sine_vertex_map(W["amp"]))
            uD = lambda x, t: synthetic.kovasznay(x, W["Re"])[0]
        else:
            mesh = BoxMesh(dim, nc, lo, hi, (True,) * dim)
            uD = None
        disc = Discretization(mesh, W["k"], nu=W["nu"])
        ora = TRBDF2(disc, W["dt"], nonlinear_iters=W["nonlinear"], uD=uD)
        xu, xp = disc.node_coords("u"), disc.node_coords("p")
        u, p, uh = initial_fields(W, xu, xp)
        uh = u.copy() if uh is None else uh
        setup = time.perf_counter() - t0
        steps = 0
        t1 = time.perf_counter()
        t = 0.0
        while True:
            u, uh, p, _ = ora.step(u, uh, p, t)
            t += W["dt"]
            steps += 1
            if time.perf_counter() - t1 > seconds_budget or steps >= 50:
                break
        el = time.perf_counter() - t1
    sample_sps = steps / el
    full_dofs = dim * int(np.prod(W["n"])) * (W["k"] + 1) ** dim
    scale = disc.N_u / full_dofs
    return {"value": sample_sps * scale, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpu_count": os.cpu_count(),
            "sample": f"{steps} oracle steps (assembled CSR + sparse LU, one thread) on "
                      f"{'x'.join(map(str, nc))} cells of the same workload ({disc.N_u} velocity DoFs) "
                      f"at {sample_sps:.3g} steps/s, scaled to the full workload by the velocity-DoF "
                      f"ratio {scale:.3g} (linear per-DoF extrapolation: an upper bound of the "
                      f"oracle's speed, since its sparse-LU cost grows faster than linearly in the "
                      f"DoFs); setup {setup:.1f}s excluded"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_solver(ctx, W, precond, steps, warmup, profile, mg_degree=0, guess="given", restart=30,
               mom_guess="given", mom_precond="jacobi"):
    """Fresh initial state, `warmup` untimed steps, `steps` timed steps with the
    given pressure preconditioner and initial guess.  Returns timing,
    iterations, final fields and (with `profile`) the event-timed operator
    kernels."""
    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    xu = ctx.node_coords(0).cpu().numpy()
    xp = ctx.node_coords(1).cpu().numpy()
    u0, p0, uh0 = initial_fields(W, xu, xp)
    U = torch.tensor(u0, device=dev)
    H = torch.tensor(u0 if uh0 is None else uh0, device=dev)
    P = torch.tensor(p0, device=dev)
    tol = W["tol"]
    ctx.guess_reset()
    if precond != "jacobi" and not getattr(ctx, "_mg_built", False):
        t_setup = time.perf_counter()
        ctx.mg_setup(degree=mg_degree)
        ctx._mg_built = True
        torch.cuda.synchronize()
        log(f"[bench] multigrid set-up {time.perf_counter() - t_setup:.2f}s: "
            f"{[(l['np'], l['cells'], l['dofs']) for l in ctx.mg_levels()]}")
    t = 0.0
    n = 0
    for i in range(warmup):
        info, _ = ctx.step(U, H, P, t, n, mom_tol=tol, prs_tol=tol, prs_maxiter=20000,
                           mom_maxiter=20000, precond=precond,
                           guess=guess, restart=restart, mom_guess=mom_guess,
                           mom_precond=mom_precond)
        t += W["dt"]
        n += 1
        log(f"[bench] {precond}/{guess} warmup step {i + 1}/{warmup}: iterations {[x['iters'] for x in info]}")
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True)
        for which in (0, 1):
            ctx.profile_read(which)
            ctx.profile_bytes(which)
    iters, used = [], []
    fallbacks = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U_before_last = None
    for i in range(steps):
        if i == steps - 1:
            U_before_last = U.clone()
        info, _ = ctx.step(U, H, P, t, n, mom_tol=tol, prs_tol=tol, prs_maxiter=20000,
                           mom_maxiter=20000, precond=precond,
                           guess=guess, restart=restart, mom_guess=mom_guess,
                           mom_precond=mom_precond)
        t += W["dt"]
        n += 1
        iters.append([x["iters"] for x in info])
        used += [info[1]["guess_used"], info[3]["guess_used"]]
        fallbacks += info[1].get("precond_fallbacks", 0) + info[3].get("precond_fallbacks", 0)
        log(f"[bench] {precond}/{guess} step {i + 1}/{steps}: iterations {iters[-1]}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if not np.isfinite(U.abs().max().item()):
        raise SystemExit("non-finite velocity")
    res = dict(sps=steps / elapsed, ms=1e3 * elapsed / steps, elapsed=elapsed,
               iters=[float(np.mean([it[j] for it in iters])) for j in range(4)], U=U, P=P,
               learned_rate=sum(1 for g in used if g == 2) / max(len(used), 1), fallbacks=fallbacks)
    if "Re" in W:
        res["t_final"] = t
        res["steady_rate"] = (U - U_before_last).abs().max().item() / W["dt"]
        res["state"] = dict(H=H, n=n, kw=dict(mom_tol=tol, prs_tol=tol, prs_maxiter=20000,
                                              mom_maxiter=20000, precond=precond, guess=guess,
                                              restart=restart, mom_guess=mom_guess,
                                              mom_precond=mom_precond))
    if profile:
        res["prof"] = tuple(ctx.profile_read(w) + (ctx.profile_bytes(w),) for w in (0, 1))
        ctx.profile(False)
    return res


def march_to_steady(ctx, W, run, tol=1e-4, max_steps=500):
    """Continue a run (untimed) until ||u^{n+1} - u^n||_inf / dt <= tol, the
    way the paper's steady computations stop at a tolerance, or until
    `max_steps` steps in total; the run's own steps count.  Returns the step
    count, time, rate and the L2 errors against the exact solution there."""
    st = run["state"]
    U, P, H = run["U"].clone(), run["P"].clone(), st["H"].clone()   # the run's fields stay as they are
    n, t = st["n"], run["t_final"]
    rate = run["steady_rate"]
    t0 = time.perf_counter()
    while rate > tol and n < max_steps:
        U_old = U.clone()
        ctx.step(U, H, P, t, n, **st["kw"])
        t += W["dt"]
        n += 1
        rate = (U - U_old).abs().max().item() / W["dt"]
        if not math.isfinite(rate):
            raise SystemExit("non-finite velocity while marching to the steady state")
        if n % 25 == 0:
            log(f"[bench] march to steady state: step {n}, t = {t:.2f}, rate {rate:.3e}")
    return dict(kovasznay_errors(ctx, W, U, P), steps=n, t=t, steady_rate_linf=rate,
                tolerance=tol, reached=rate <= tol, wall_s=time.perf_counter() - t0)


def random_phase_state(ctx, W, seed, peak=1.0):
    """Divergence-free random-phase field of the learned guess's training
    data (8 Fourier modes, |kappa| <= 4, amplitudes N(0,1)/|kappa|^2),
    rescaled to the largest nodal speed `peak` (that of the vortex, so the
    Courant number matches the timed workload's), zero pressure."""
    import numpy as np
    import torch

    import synthetic
    xu = ctx.node_coords(0).cpu().numpy()
    nbu = (W["k"] + 1) ** W["dim"]
    u = synthetic.random_phase_velocity(xu, seed)
    u *= peak / np.sqrt((u * u).sum(axis=1)).max()
    u = torch.tensor(synthetic.nodal_velocity(u, W["dim"], nbu), device="cuda")
    return u, u.clone(), torch.zeros(ctx.N_p, dtype=torch.float64, device="cuda")


def train_guess(ctx, W, step_kw, seeds=tuple(range(10)), steps=30, discard=5, epochs=12):
    """Generate samples with the solver (random-phase trajectories of the
    training seeds, `discard` unrecorded steps then `steps` recorded ones),
    train the guess network on the GPU by its own kernels."""
    from paper_2107_07776_amd import Net, learned_guess
    t0 = time.perf_counter()
    # the last fifth of the seeds' trajectories validate (the parameters with
    # the lowest validation loss are kept, the untrained ones included)
    n_val = max(1, len(seeds) // 5)
    fit, val = list(seeds[:-n_val]), list(seeds[-n_val:])
    gen = lambda ss: learned_guess.generate(ctx, lambda s: random_phase_state(ctx, W, s), ss, steps,
                                            discard, precond="mg_fp32", tol=W["tol"],
                                            log=lambda m: log(f"[bench] {m}"), **step_kw)
    samples, vsamples = gen(fit), gen(val)
    t1 = time.perf_counter()
    net = Net(32, seed=1)
    nx, ny, nz = (list(W["n"]) + [1, 1])[:3]
    rep = {}
    # the extrapolated increment leaves a squared error ~1e-8 of the
    # increment's: Adam's steps must stay below that scale from the start
    losses = learned_guess.train(net, samples, (nx, ny, nz), epochs=epochs, batch=8, lr=3e-5,
                                 val=vsamples, report=rep, log=lambda m: log(f"[bench] {m}"))
    t2 = time.perf_counter()
    log(f"[bench] guess network: {samples.shape[0]} + {vsamples.shape[0]} samples in {t1 - t0:.1f}s, "
        f"{epochs} epochs in {t2 - t1:.1f}s, loss {losses[0]:.3e} -> {losses[-1]:.3e}, validation "
        f"{rep['validation_losses'][0]:.3e} (untrained) -> kept epoch {rep['epoch_kept']}")
    return net, {"samples": int(samples.shape[0]), "validation_samples": int(vsamples.shape[0]),
                 "generation_s": t1 - t0, "training_s": t2 - t1,
                 "epochs": epochs, "loss_first_epoch": losses[0], "loss_last_epoch": losses[-1],
                 "validation_loss_untrained": rep["validation_losses"][0],
                 "validation_losses": rep["validation_losses"][1:], "epoch_kept": rep["epoch_kept"],
                 "train_seeds": fit, "validation_seeds": val, "train_steps_per_seed": steps,
                 "discarded_steps": discard}


def evaluate_guesses(ctx, W, step_kw, modes, seeds=(100, 101), steps=50, discard=5):
    """Held-out random-phase trajectories: mean pressure iterations, steps/s
    and (learned) the rate at which the FP64 judge took the network's guess."""
    from paper_2107_07776_amd import learned_guess
    t0 = time.perf_counter()
    res = learned_guess.evaluate(ctx, lambda s: random_phase_state(ctx, W, s), list(seeds), steps,
                                 discard, modes=modes, precond="mg_fp32", tol=W["tol"],
                                 log=lambda m: log(f"[bench] {m}"), **step_kw)
    log(f"[bench] held-out evaluation in {time.perf_counter() - t0:.1f}s: "
        + ", ".join(f"{m} {r['mean_pressure_iterations']:.2f} its" for m, r in res.items()))
    return {"seeds": list(seeds), "steps_per_seed": steps, "discarded_steps": discard, "modes": res}


AMR_LABEL = ("2D adaptive quadtree mesh with hanging nodes on (0, 2pi)^2, periodic, 512^2 base "
             "cells, Q3-Q2, at most two refinement levels (h_min = H/4, h_max = H); velocity of "
             "twelve seeded Gaussian vortices; per cycle: vorticity indicator, marking of the 10 %% "
             "largest / 30 %% smallest, remeshing with velocity and pressure transfer, then %d "
             "applications of the pressure Helmholtz operator")


def amr_vortices(x):
    """Velocity of twelve seeded Gaussian vortices (stream function sum of
    A exp(-r^2 / s^2)); x (n, 2) -> (n, 2)."""
    import numpy as np
    rng = np.random.default_rng(2107)
    u = np.zeros_like(x)
    for _ in range(12):
        c = rng.uniform(0.8, 2 * math.pi - 0.8, 2)
        A, s = rng.uniform(-1.0, 1.0), rng.uniform(0.15, 0.4)
        dx, dy = x[:, 0] - c[0], x[:, 1] - c[1]
        e = A * np.exp(-(dx * dx + dy * dy) / (s * s))
        u[:, 0] += -2.0 * dy / (s * s) * e
        u[:, 1] += 2.0 * dx / (s * s) * e
    return u


def amr_nodes(leaves, H, k):
    """Velocity node coordinates of the cells (level, i, j), x fastest."""
    import numpy as np
    z = 0.5 * (np.polynomial.legendre.leggauss(k + 1)[0] + 1.0)
    n = k + 1
    h = H / (1 << leaves[:, 0].astype(np.int64))
    ox, oy = leaves[:, 1] * h, leaves[:, 2] * h
    px = ox[:, None] + h[:, None] * np.tile(z, n)[None, :]
    py = oy[:, None] + h[:, None] * np.repeat(z, n)[None, :]
    return np.stack([px.ravel(), py.ravel()], 1)


def amr_cpu_baseline(k, seconds_budget=15.0):
    """The oracle's assembled a_p + alpha M^p (hanging-node mesh of the same
    kind: 8^2 base cells, two rounds of indicator-driven refinement) applied
    as a sparse matrix-vector product on one thread; assembly excluded."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.adaptive import AdaptiveDisc, QuadForest, mark
    with threadpool_limits(limits=1):
        L = 2 * math.pi
        f = QuadForest((8, 8), (0.0, 0.0), (L, L), (1, 1), 2)
        for _ in range(2):
            ad = AdaptiveDisc(f, k)
            xu = ad.node_coords("u")
            uv = amr_vortices(xu)
            u = np.zeros(ad.N_u)
            for c in range(f.N):
                sl = slice(c * ad.nbu, (c + 1) * ad.nbu)
                u[2 * c * ad.nbu:(2 * c + 1) * ad.nbu] = uv[sl, 0]
                u[(2 * c + 1) * ad.nbu:(2 * c + 2) * ad.nbu] = uv[sl, 1]
            f = f.adapt(mark(ad.indicator(u), f, 0.1, 0.3, L / 32, L / 8))
        ad = AdaptiveDisc(f, k)
        A = ad.helmholtz_p(1.0)
        p = np.random.default_rng(0).standard_normal(ad.N_p)
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds_budget and n < 200000:
            p = A @ p
            p /= np.abs(p).max()
            n += 1
        el = time.perf_counter() - t0
    return {"value": ad.N_p * n / el / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpu_count": os.cpu_count(),
            "sample": f"{n} products of the oracle's assembled CSR operator on an adapted mesh of "
                      f"{f.N} cells ({ad.N_p} pressure DoFs), one thread; assembly excluded"}


def run_amr(args, applies=50):
    """Adaptive-mesh workload: cycles of indicator, marking, remeshing with
    transfer and a fixed number of pressure-operator applications."""
    import numpy as np
    import torch

    from paper_2107_07776_amd import Adaptive
    k, base, maxl = 3, 512, 2
    L = 2 * math.pi
    H = L / base
    g = Adaptive((base, base), (0.0, 0.0), (L, L), k, maxl, periodic=(1, 1))

    def velocity():
        x = amr_nodes(g.leaves(), H, k)
        uv = amr_vortices(x)
        n = (k + 1) ** 2
        u = np.empty(g.N_u)
        u.reshape(-1, 2, n)[:, 0, :] = uv[:, 0].reshape(-1, n)
        u.reshape(-1, 2, n)[:, 1, :] = uv[:, 1].reshape(-1, n)
        return torch.tensor(u, device="cuda")

    U = velocity()
    P = torch.tensor(np.random.default_rng(1).standard_normal(g.N_p), device="cuda")
    alpha = 1.0
    Y = torch.empty_like(P)

    def cycle():
        nonlocal U, P, Y
        eta = g.indicator(U)
        flags = g.mark(eta, 0.1, 0.3, H / 4, H)
        U, P = g.adapt(flags, [("u", U), ("p", P)])
        Y = torch.empty_like(P)
        for i in range(applies):
            g.apply_pressure(alpha, P, Y)
            P, Y = Y, P
            if i % 10 == 9:
                P.div_(P.abs().max())   # keep the repeated products in range

    log("[bench] adaptive mesh: warm-up cycles")
    for _ in range(args.warmup):
        cycle()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cycle()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    lv = g.leaves()[:, 0]
    # the operator alone: HIP events around back-to-back launches on the
    # library's (torch's current) stream; at this size one launch outlasts
    # the host's call overhead, so the launches queue without gaps
    reps = 40
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    g.apply_pressure(alpha, P, Y)
    ev[0].record()
    for _ in range(reps):
        g.apply_pressure(alpha, P, Y)
    ev[1].record()
    torch.cuda.synchronize()
    avg_s = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
    # compulsory bytes: read p, write y (16 B per DoF) + the cell's level,
    # face kinds and neighbour ids (4 + 16 + 32 B per cell)
    bytes_launch = 16.0 * g.N_p + 52.0 * g.N_c
    gbs = bytes_launch / avg_s / 1e9
    out = {"metric": "adaptive-mesh pressure Helmholtz operator GDoF/s (hanging nodes)",
           "value": g.N_p / avg_s / 1e9, "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
           "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded Gaussian vortices; seeded random pressure)",
           "config": {"workload": AMR_LABEL % applies, "cells": int(g.N_c),
                      "cells_per_level": [int((lv == l).sum()) for l in range(maxl + 1)],
                      "pressure_dofs": int(g.N_p), "velocity_dofs": int(g.N_u), "degree": k,
                      "cycles_per_s": args.steps / el},
           "roofline": {"bound": "hbm", "kernel": "k_amr_pressure", "achieved": gbs,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                        "traffic": None, "algorithmic_bytes_per_launch": bytes_launch,
                        "avg_launch_us": avg_s * 1e6, "launches_timed": reps}}
    traffic = measured_traffic("amr_pressure", "amr2d")
    if traffic and traffic.get("bytes_per_dof"):
        # the mesh changes from cycle to cycle: the counted bytes per pressure
        # DoF of the summary's mesh, times this mesh's DoFs
        out["roofline"]["traffic"] = traffic["bytes_per_dof"] * g.N_p
        out["roofline"]["traffic_source"] = traffic["source"] + " (bytes per pressure DoF x DoFs)"
    g.close()
    if not args.no_amr_steps:
        out["adaptive_trbdf2"] = amr_steps(args)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle's operator on a bounded sample")
        out["cpu_baseline"] = amr_cpu_baseline(k)
    print(json.dumps(out), flush=True)


def amr_steps(args, base=64, k=3, maxl=2, nu=5e-3, dt=5e-4, remesh_every=5):
    """TR-BDF2 steps on an adaptive mesh with the remeshing schedule of
    Sec. 4 (every remesh_every steps: indicator, 10 % / 30 % marking,
    transfer of u, u_hist and p): Jacobi GMRES(30) and cell-block-Jacobi CG
    to 1e-8."""
    import numpy as np
    import torch

    from paper_2107_07776_amd import Adaptive
    L = 2 * math.pi
    H = L / base
    g = Adaptive((base, base), (0.0, 0.0), (L, L), k, maxl, periodic=(1, 1))
    g.set_flow(nu, dt)
    x = amr_nodes(g.leaves(), H, k)
    uv = amr_vortices(x)
    n = (k + 1) ** 2
    u = np.empty(g.N_u)
    u.reshape(-1, 2, n)[:, 0, :] = uv[:, 0].reshape(-1, n)
    u.reshape(-1, 2, n)[:, 1, :] = uv[:, 1].reshape(-1, n)
    U = torch.tensor(u, device="cuda")
    Hh = U.clone()
    P = torch.zeros(g.N_p, dtype=torch.float64, device="cuda")
    kw = dict(mom_tol=1e-8, prs_tol=1e-8, restart=30, mom_maxiter=20000, prs_maxiter=50000)
    iters, cells = [], []

    def run(nsteps, record):
        nonlocal U, Hh, P
        for i in range(1, nsteps + 1):
            info, _ = g.step(U, Hh, P, None, **kw)
            if record:
                iters.append([q["iters"] for q in info])
                cells.append(g.N_c)
            if i % remesh_every == 0:
                flags = g.mark(g.indicator(U), 0.1, 0.3, H / 4, H)
                U, Hh, P = g.adapt(flags, [("u", U), ("u", Hh), ("p", P)])

    log("[bench] adaptive TR-BDF2: warm-up")
    steps = 2 * remesh_every
    try:
        run(remesh_every * 2, False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(steps, True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    except Exception as e:   # reported, not hidden: the JSON line says what failed
        g.close()
        return {"error": str(e)}
    out = {"steps_per_s": steps / el, "ms_per_step": el / steps * 1e3, "steps": steps,
           "warmup": remesh_every * 2, "remesh_every": remesh_every,
           "mean_cells": float(np.mean(cells)), "final_cells": int(g.N_c),
           "mean_iterations_per_step": [float(v) for v in np.mean(np.asarray(iters), axis=0)],
           "config": f"(0, 2pi)^2 periodic, {base}^2 base cells, Q{k}-Q{k - 1}, <= {maxl} refinement "
                     f"levels, nu = {nu}, dt = {dt}, the twelve-vortex velocity at rest pressure; "
                     "remeshing (timed) every " + str(remesh_every) + " steps; Jacobi GMRES(30) and "
                     "cell-block-Jacobi CG to 1e-8"}
    g.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tgv64", choices=["tgv64", "tgv32", "kov256", "tg2d", "amr2d"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the separate event-timed run of the operator kernels")
    ap.add_argument("--profile-steps", type=int, default=4)
    ap.add_argument("--precond", default="mg_fp32", choices=["jacobi", "mg_fp32", "mg_bf16"],
                    help="pressure preconditioner of the timed solver")
    ap.add_argument("--mg-degree", type=int, default=5,
                    help="Chebyshev degree of the multigrid smoother (0: library default)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain FP64 (Jacobi) reference run")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16-smoother run")
    ap.add_argument("--guess", default=None, choices=["given", "previous", "learned", "extrap2", "extrap3"],
                    help="initial guess of the timed solver's pressure solves (default: learned "
                         "where the network is built, else previous)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training and evaluating the learned guess")
    ap.add_argument("--no-eval", action="store_true", help="skip the held-out guess evaluation")
    ap.add_argument("--train-seeds", type=int, default=10)
    ap.add_argument("--train-steps", type=int, default=30)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--restart", type=int, default=None,
                    help="GMRES restart length of the timed solver (default: 6; 30 on the Kovasznay mesh)")
    ap.add_argument("--mom-precond", default=None, choices=["jacobi", "line", "mg_fp32"],
                    help="momentum preconditioner of the timed solver (default: line blocks; FP32 "
                         "velocity multigrid on the Kovasznay mesh; on mapped cells both use the "
                         "undistorted box)")
    ap.add_argument("--mom-guess", default="previous", choices=["given", "previous"],
                    help="momentum initial guess of the timed solver")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the run, copy a MIB-sized device buffer 5 times (a plain copy "
                         "kernel of known size, the reference for hardware byte counters)")
    ap.add_argument("--no-steady", action="store_true",
                    help="Kovasznay workload: skip the untimed march to the steady state")
    ap.add_argument("--no-amr-steps", action="store_true",
                    help="adaptive workload: skip the TR-BDF2 steps on the small adaptive mesh")
    ap.add_argument("--nonlinear", type=int, default=0,
                    help="momentum solves per stage (fixed point; 0 = the workload's setting)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on exactly one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_calibration} MiB five times")
        del src, dst
    if args.workload == "amr2d":
        run_amr(args)
        return
    W = workload(args.workload)
    log(f"[bench] setting up {W['label']}")
    if args.nonlinear > 0:
        W["nonlinear"] = args.nonlinear
    ctx = make_context(W)
    if args.restart is None:
        args.restart = W.get("restart", 6)
    if args.mom_precond is None:
        args.mom_precond = W.get("mom_precond", "line")
    ctx.set_nonlinear(W["nonlinear"], 0.0)
    learned_ok = W.get("learned", True) and args.precond != "jacobi"
    if args.guess is None:
        args.guess = "learned" if learned_ok and not args.no_learned else "previous"
    if args.guess == "learned" and not learned_ok:
        raise SystemExit("the learned guess is built for 3D affine boxes with the multigrid solver")
    step_kw = dict(restart=args.restart, mom_guess=args.mom_guess, mom_precond=args.mom_precond,
                   mom_maxiter=20000)
    plain = None
    if not args.no_compare and args.precond != "jacobi":
        plain = run_solver(ctx, W, "jacobi", args.steps, args.warmup, False)
    net = None
    learned_info = None
    if learned_ok and (args.guess == "learned" or not args.no_learned):
        net, learned_info = train_guess(ctx, W, step_kw, seeds=tuple(range(args.train_seeds)),
                                        steps=args.train_steps, epochs=args.epochs)
        ctx.set_guess_net(net)
    # the timed run carries no measurement hooks
    main_run = run_solver(ctx, W, args.precond, args.steps, args.warmup, False, args.mg_degree,
                          args.guess, args.restart, args.mom_guess, args.mom_precond)
    prof_run = None
    if not args.no_profile:
        prof_run = run_solver(ctx, W, args.precond, args.profile_steps, 1, True, args.mg_degree,
                              args.guess, args.restart, args.mom_guess, args.mom_precond)
    solver = {"jacobi": "Jacobi-preconditioned FP64 CG",
              "mg_fp32": "FP32 h/p-multigrid V-cycle (Chebyshev smoother) under FP64 flexible CG",
              "mg_bf16": "h/p-multigrid V-cycle with BF16 storage on the finest level under FP64 "
                         "flexible CG"}[args.precond]
    guess_desc = {
        "given": "previous pressure",
        "previous": "previous pressure + the same stage's increment of the previous step",
        "learned": "learned (3D CNN, bf16 MFMA) correction of the quadratically extrapolated "
                   "increment, previous pressure + the same stage's last increment as fallback, "
                   "the smaller FP64 residual decides",
        "extrap2": "previous pressure + the same stage's increment extrapolated linearly from its "
                   "last two values",
        "extrap3": "previous pressure + the same stage's increment extrapolated quadratically from "
                   "its last three values"}
    out = {"metric": METRIC, "value": main_run["sps"], "unit": "steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_run["ms"],
           "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (closed-form Taylor-Green initial field; seeded random-phase fields train "
                   "and evaluate the guess network)",
           "config": {"workload": W["label"], "pressure_solver": solver,
                      "pressure_initial_guess": guess_desc[args.guess],
                      "momentum_solver": {"line": "line-block", "jacobi": "Jacobi",
                                          "mg_fp32": "FP32 velocity-multigrid (one V-cycle per component)"}[args.mom_precond]
                                         + f"-preconditioned FP64 GMRES({args.restart})",
                      "momentum_initial_guess": {"given": "previous stage value",
                                                 "previous": "linear extrapolation to the stage time"}[args.mom_guess],
                      "momentum_solves_per_stage": W["nonlinear"],
                      "mg_chebyshev_degree": args.mg_degree if args.precond != "jacobi" else None,
                      "tolerance": W["tol"], "cells": list(W["n"]), "degree": W["k"],
                      "velocity_dofs": ctx.N_u, "pressure_dofs": ctx.N_p,
                      "mean_iterations_per_step": main_run["iters"]}}
    if args.guess == "learned":
        out["config"]["learned_guess_used_rate"] = main_run["learned_rate"]
    if args.precond != "jacobi":
        out["preconditioner_dtype"] = "f32" if args.precond == "mg_fp32" else "bf16 storage, f32 arithmetic"
    if args.precond == "mg_fp32" and not args.no_bf16:
        bf = run_solver(ctx, W, "mg_bf16", args.steps, args.warmup, False, args.mg_degree, args.guess,
                        args.restart, args.mom_guess, args.mom_precond)
        out["bf16_smoother"] = {"steps_per_s": bf["sps"], "ms_per_step": bf["ms"],
                                "mean_iterations_per_step": bf["iters"],
                                "precond_fallbacks": bf["fallbacks"],
                                "u_rel_l2_diff_vs_fp32": (bf["U"] - main_run["U"]).norm().item()
                                                         / main_run["U"].norm().item()}
    if learned_info is not None and not args.no_eval:
        modes = ("given", "previous", "extrap2", "extrap3", "learned")
        learned_info["held_out"] = evaluate_guesses(ctx, W, step_kw, modes)
    if not W.get("learned", True):
        out["learned_guess"] = {"built": False,
                                "reason": "the guess network is a 3D convolution on affine boxes; this "
                                          "2D mapped workload runs with the multigrid preconditioner only"}
    if "Re" in W:
        out["data"] = "synthetic (exact Kovasznay solution as wall data, fluid at rest at t=0)"
        out["l2_error_vs_exact"] = dict(kovasznay_errors(ctx, W, main_run["U"], main_run["P"]),
                                        t_final=main_run["t_final"],
                                        steady_rate_linf=main_run["steady_rate"])
        if plain is not None:
            out["plain_fp64_l2_error_vs_exact"] = dict(kovasznay_errors(ctx, W, plain["U"], plain["P"]),
                                                       steady_rate_linf=plain["steady_rate"])
        if not args.no_steady:
            out["steady_state"] = march_to_steady(ctx, W, main_run)
    if learned_info is not None:
        out["learned_guess"] = learned_info
    if plain is not None:
        du = (main_run["U"] - plain["U"]).norm().item() / plain["U"].norm().item()
        dp = (main_run["P"] - plain["P"]).norm().item() / plain["P"].norm().item()
        p0 = plain["P"] - plain["P"].mean()
        dp0 = (main_run["P"] - main_run["P"].mean() - p0).norm().item() / p0.norm().item()
        out["plain_fp64"] = {"steps_per_s": plain["sps"], "ms_per_step": plain["ms"],
                             "mean_iterations_per_step": plain["iters"],
                             "pressure_solver": "Jacobi-preconditioned FP64 CG from the previous pressure",
                             "momentum_solver": "Jacobi-preconditioned FP64 GMRES(30) from the previous "
                                                "stage value"}
        out["speedup_vs_plain_fp64"] = main_run["sps"] / plain["sps"]
        out["equal_error"] = {"u_rel_l2_diff_vs_plain": du, "p_rel_l2_diff_vs_plain": dp,
                              "p_mean_free_rel_l2_diff_vs_plain": dp0,
                              "after_steps": args.steps + args.warmup}
    if prof_run is not None:
        (ms_p, n_p, b_p), (ms_u, n_u, b_u) = prof_run["prof"]
        kern = {
            "pressure_apply": dict(ms=ms_p, n=n_p, bytes=b_p / max(n_p, 1), dofs=ctx.N_p, unit_bytes=16),
            "momentum_apply": dict(ms=ms_u, n=n_u, bytes=b_u / max(n_u, 1), dofs=ctx.N_u, unit_bytes=24),
        }
        for name, kd in kern.items():
            avg_s = kd["ms"] * 1e-3 / max(kd["n"], 1)
            kd["avg_us"] = avg_s * 1e6
            kd["gdofs"] = kd["dofs"] / avg_s / 1e9 if avg_s > 0 else 0.0
            kd["gbs"] = kd["bytes"] / avg_s / 1e9 if avg_s > 0 else 0.0
            # the operator's own compulsory bytes (read the operand(s), write
            # the result) without the fused Krylov work of the launch
            kd["apply_gbs"] = kd["unit_bytes"] * kd["dofs"] / avg_s / 1e9 if avg_s > 0 else 0.0
        dom = max(kern, key=lambda k: kern[k]["ms"])
        kd = kern[dom]
        traffic = measured_traffic(dom, args.workload)
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": kd["gbs"], "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": kd["gbs"] / HBM_PEAK_GBS,
                           "traffic": traffic["bytes_per_launch"] if traffic else None,
                           "traffic_source": traffic["source"] if traffic else None,
                           "algorithmic_bytes_per_launch": kd["bytes"], "avg_launch_us": kd["avg_us"],
                           "apply_only_achieved": kd["apply_gbs"],
                           "apply_only_frac": kd["apply_gbs"] / HBM_PEAK_GBS,
                           "launches_timed": kd["n"], "launch_sample_stride": LAUNCH_SAMPLE_STRIDE,
                           "sampled_run_steps": args.profile_steps,
                           # the timed launches are every third one: their time
                           # scaled by the stride estimates the kernel's total
                           "share_of_step_time": LAUNCH_SAMPLE_STRIDE * kd["ms"] * 1e-3 / prof_run["elapsed"]}
        out["operator_gdofs"] = {k: round(v["gdofs"], 3) for k, v in kern.items()}
        out["operator_avg_us"] = {k: round(v["avg_us"], 3) for k, v in kern.items()}
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(W)
    ctx.set_guess_net(None)
    if net is not None:
        net.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
