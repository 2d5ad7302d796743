"""GPU parity and gain of the learned pressure initial guess.

* the network input computed by the library equals the oracle's (FP32
  output of FP64 cell sums: 1e-6 relative) and so do its scales (1e-12);
* the injection of a cell-wise increment equals the oracle's (1e-12);
* recorded samples are consistent: the target of one solve plus the
  same-stage channel, rescaled, is the newest-increment channel of the next;
* a network trained on the solver's own samples (seeds 0-2) reaches a
  training loss below half its initial value, and on a held-out trajectory
  (seed 100) the learned mode needs fewer pressure-solve iterations than
  starting from the previous pressure and no more than the same-stage
  previous increment (the residual judge keeps the better candidate).
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import BoxMesh, Discretization, TRBDF2
from oracle import guess as oguess

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [(2, (8, 8), (1.0, 1.0), 3), (3, (6, 4, 4), (2 * math.pi,) * 3, 3), (3, (4, 4, 4), (1.0,) * 3, 2)]


def _ids(c):
    return f"d{c[0]}-{'x'.join(map(str, c[1]))}-k{c[3]}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_features_and_injection_match_oracle(case):
    from paper_2107_07776_amd import Context
    dim, nc, ext, k = case
    print(f"[case] guess features {case}", flush=True)
    dt = 0.02
    ctx = Context(dim, nc, (0.0,) * dim, ext, k=k, nu=0.01, dt=dt)
    mesh = BoxMesh(dim, nc, (0.0,) * dim, ext, (True,) * dim)
    disc = Discretization(mesh, k, nu=0.01)
    ts = TRBDF2(disc, dt)
    N = disc.N_p
    b, p, i1, i2 = (synthetic.random_vector(N, 500 + j) for j in range(4))
    t = lambda a: torch.tensor(a, device="cuda")
    g = ts.cst["gamma"]
    for s, (b1, b2) in ((1, (1 - g, g)), (2, (g, 1 - g))):
        x, (si, sd) = ctx.guess_features(s, t(b), t(p), t(i1), b1, t(i2), b2)
        xo, sio, sdo = oguess.features(ts, s, b, p, i1, b1, i2, b2)
        x = x.cpu().numpy()
        assert abs(si - sio) <= 1e-12 * sio and abs(sd - sdo) <= 1e-12 * sdo
        assert np.abs(x - xo).max() <= 1e-6 * np.abs(xo).max()
        y = np.random.default_rng(s).standard_normal(disc.Nc).astype(np.float32)
        out = ctx.guess_inject(s, t(p), t(i2), torch.tensor(y, device="cuda"), 2.5).cpu().numpy()
        ref = oguess.inject(ts, s, p, i2, y.astype(np.float64), 2.5)
        assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
    ctx.close()


def _initial_state(ctx, seed):
    xu = ctx.node_coords(0).cpu().numpy()
    nbu = (ctx.k + 1) ** ctx.dim
    u = synthetic.nodal_velocity(synthetic.random_phase_velocity(xu, seed), ctx.dim, nbu)
    U = torch.tensor(u, device="cuda")
    return U, U.clone(), torch.zeros(ctx.N_p, dtype=torch.float64, device="cuda")


def _box(n, k=3):
    from paper_2107_07776_amd import Context
    L = 2 * math.pi
    return Context(3, (n,) * 3, (0.0,) * 3, (L,) * 3, k=k, nu=1.0 / 1600, dt=L / (10 * n))


def test_recorded_samples_are_consistent():
    from paper_2107_07776_amd import learned_guess
    print("[case] sample recording 8^3 Q3-Q2", flush=True)
    ctx = _box(8)
    S = learned_guess.generate(ctx, lambda s: _initial_state(ctx, s), seeds=[7], steps=4, discard=2)
    assert S.shape == (8, 4, ctx.N_c)
    S = S.cpu().numpy().astype(np.float64)
    assert np.isfinite(S).all()
    for j in range(S.shape[0] - 1):
        # mean(p_new - p_prev) / (beta dt), in units of solve j's scale, is
        # target + f1 (the same-stage channel has the same weight beta)
        inc = S[j, 3] + S[j, 1]
        f0 = S[j + 1, 0]
        c = (inc @ f0) / (f0 @ f0)          # the ratio of the two solves' scales
        assert np.linalg.norm(inc - c * f0) <= 1e-5 * np.linalg.norm(inc), j
    ctx.close()


def test_trained_network_gains_on_held_out_trajectory():
    from paper_2107_07776_amd import Net, learned_guess
    n = 16
    print(f"[case] learned guess {n}^3 Q3-Q2: generate, train, evaluate", flush=True)
    ctx = _box(n)
    init = lambda s: _initial_state(ctx, s)
    samples = learned_guess.generate(ctx, init, seeds=[0, 1, 2], steps=12, discard=3)
    net = Net(32, seed=1)
    losses = learned_guess.train(net, samples, (n, n, n), epochs=25, batch=8, lr=1e-3,
                                 log=lambda m: print(m, flush=True))
    assert losses[-1] < 0.5 * losses[0]
    ctx.set_guess_net(net)
    res = learned_guess.evaluate(ctx, init, seeds=[100], steps=10, discard=3)
    print("held-out evaluation:", res)
    print("last residuals (learned, fallback):", ctx.guess_last())
    g, p, l = (res[m]["mean_pressure_iterations"] for m in ("given", "previous", "learned"))
    assert l < g
    assert l <= p + 0.25
    ctx.set_guess_net(None)
    net.close()
    ctx.close()
