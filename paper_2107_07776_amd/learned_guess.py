"""Training and evaluation of the learned pressure initial guess.

Samples come from the solver itself: ``tbdg_step`` runs from seeded initial
states with sample recording on (network input and the converged increment
of every Helmholtz solve).  The network is trained on the GPU by its own
kernels (forward, backward, Adam through the C ABI); the evaluation runs
held-out trajectories with the three initial-guess modes and reports the
pressure-solve iterations.  Orchestration only: every computation happens in
the library.
"""
import time

import torch


def generate(ctx, initial_state, seeds, steps, discard, precond="mg_fp32", tol=1e-8, maxiter=20000,
             log=None, **step_kw):
    """Samples [S][12][N_c] (float32, device: network input [6][N_c], Gram
    target [6][N_c]) from ``steps`` recorded steps per
    seed after ``discard`` unrecorded ones.  ``initial_state(seed)`` returns
    device tensors (u, u_hist, p); ``step_kw`` go to ``ctx.step`` (momentum
    solver settings).  A trajectory whose step fails (a solve that does not
    converge) ends there; its samples so far are kept."""
    cap = 2 * steps * len(seeds)
    buf = torch.zeros((cap, 12, ctx.N_c), dtype=torch.float32, device=ctx.device)
    total = 0
    for seed in seeds:
        u, uh, p = initial_state(seed)
        ctx.guess_record(None)
        ctx.guess_reset()
        t = 0.0
        for n in range(discard + steps + 3):
            if n == discard:
                # recording clears the history; the network's input needs the
                # same stage's last three increments: three steps refill it
                ctx.guess_record(buf[total:])
            info, st = ctx.step(u, uh, p, t, n, mom_tol=tol, prs_tol=tol, prs_maxiter=maxiter,
                                precond=precond, guess="previous", check=False, **step_kw)
            if st != 0:
                if log:
                    log(f"seed {seed}: step {n} failed with status {st} (iterations "
                        f"{[i['iters'] for i in info]}); trajectory ends")
                break
            t += ctx.dt
        total += ctx.guess_recorded()
        ctx.guess_record(None)
    return buf[:total]


def mean_loss(net, samples, grid, batch=8):
    """Mean per-cell quadratic loss of the network's output over samples."""
    nx, ny, nz = grid
    S = samples.shape[0]
    x_all = samples[:, :6].reshape(S, 6, nz, ny, nx)
    y_all = samples[:, 6:].reshape(S, 6, nz, ny, nx)
    tot = 0.0
    for i in range(0, S, batch):
        x = x_all[i:i + batch].contiguous()
        y = y_all[i:i + batch].contiguous()
        loss, _ = net.quad_loss(net.forward(x), y)
        tot += loss * x.shape[0]
    return tot / max(S, 1)


def train(net, samples, grid, epochs, batch=8, lr=1e-3, seed=0, log=None, val=None, report=None):
    """Adam on the per-cell quadratic loss of the recorded Gram targets (the
    squared nodal error of the injected guess); returns the mean loss of
    every epoch.  ``grid`` = (nx, ny, nz) of the cell grid.  With validation
    samples ``val`` (other trajectories), the parameters with the lowest
    validation loss are kept, the untrained ones (zero output: the
    extrapolated increment itself) included; ``report`` (a dict) receives the
    validation losses and the epoch kept."""
    nx, ny, nz = grid
    S = samples.shape[0]
    x_all = samples[:, :6].reshape(S, 6, nz, ny, nx)
    y_all = samples[:, 6:].reshape(S, 6, nz, ny, nx)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    losses, vlosses = [], []
    best = None
    if val is not None:
        vlosses.append(mean_loss(net, val, grid, batch))
        best = (vlosses[0], net.params().clone(), 0)
    for ep in range(epochs):
        perm = torch.randperm(S, generator=gen)
        tot, cnt = 0.0, 0
        for i in range(0, S, batch):
            idx = perm[i:i + batch].to(samples.device)
            x = x_all.index_select(0, idx).contiguous()
            y = y_all.index_select(0, idx).contiguous()
            yhat = net.forward(x)
            loss, dy = net.quad_loss(yhat, y)
            net.zero_grad()
            net.backward(dy)
            net.adam_step(lr)
            tot += loss * len(idx)
            cnt += len(idx)
        losses.append(tot / cnt)
        msg = f"epoch {ep + 1}/{epochs}: loss {losses[-1]:.4e}"
        if val is not None:
            vlosses.append(mean_loss(net, val, grid, batch))
            msg += f", validation {vlosses[-1]:.4e}"
            if vlosses[-1] < best[0]:
                best = (vlosses[-1], net.params().clone(), ep + 1)
        if log:
            log(msg)
    if best is not None:
        net.set_params(best[1])
    if report is not None:
        report.update(validation_losses=vlosses, epoch_kept=best[2] if best else epochs)
    return losses


def evaluate(ctx, initial_state, seeds, steps, discard, modes=("given", "previous", "learned"),
             precond="mg_fp32", tol=1e-8, maxiter=20000, log=None, **step_kw):
    """Mean pressure-solve iterations, fallback rate and steps/s per guess
    mode over held-out trajectories (identical trajectories for every mode
    up to the solver tolerance); ``step_kw`` go to ``ctx.step``.  A step
    that fails (a solve that does not converge) ends that trajectory for
    every mode: the statistics cover the steps all modes completed."""
    per = {m: {} for m in modes}      # mode -> seed -> list of (iters, used, secs) per step
    limit = {seed: discard + steps for seed in seeds}
    for mode in modes:
        for seed in seeds:
            u, uh, p = initial_state(seed)
            ctx.guess_reset()
            t = 0.0
            rec = []
            for n in range(limit[seed]):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info, st = ctx.step(u, uh, p, t, n, mom_tol=tol, prs_tol=tol, prs_maxiter=maxiter,
                                    precond=precond, guess=mode, check=False, **step_kw)
                torch.cuda.synchronize()
                t += ctx.dt
                if st != 0:
                    if log:
                        log(f"{mode}, seed {seed}: step {n} failed with status {st} "
                            f"(iterations {[i['iters'] for i in info]}); trajectory ends")
                    limit[seed] = n
                    break
                rec.append(([info[j]["iters"] for j in (1, 3)], [info[j]["guess_used"] for j in (1, 3)],
                            time.perf_counter() - t0))
            per[mode][seed] = rec
    out = {}
    for mode in modes:
        iters, used, secs, nsteps = [], [], 0.0, 0
        for seed in seeds:
            for its, us, dt_s in per[mode][seed][discard:limit[seed]]:
                iters += its
                used += us
                secs += dt_s
                nsteps += 1
        res = {"mean_pressure_iterations": sum(iters) / max(len(iters), 1),
               "steps_per_s": nsteps / secs if secs > 0 else 0.0, "solves": len(iters), "steps": nsteps}
        if mode == "learned":
            res["learned_used_rate"] = sum(1 for g in used if g == 2) / max(len(used), 1)
            res["fallback_rate"] = 1.0 - res["learned_used_rate"]
        out[mode] = res
    return out
