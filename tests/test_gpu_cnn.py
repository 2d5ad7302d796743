"""GPU parity of the learned-guess network against the FP64 oracle network.

The oracle runs on the same bf16-rounded parameters and inputs (the GPU
stores both in bf16); with the hidden activations rounded to bf16 at the same
points the forward pass agrees to a bf16 rounding flip (TOL_FWD_ROUNDED),
and without that rounding to the accumulated bf16 error of three layers
(TOL_FWD).  Parameter gradients carry the extra bf16 rounding of the
back-propagated signals (TOL_GRAD, relative to each layer's largest entry).
"""
import time

import numpy as np
import pytest

from oracle import cnn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8                      # unit roundoff of bfloat16
TOL_FWD_ROUNDED = 4 * U_BF16             # one rounding flip of an activation, propagated
TOL_FWD = 12 * U_BF16                    # three layers of activation rounding
TOL_GRAD = 16 * U_BF16

# (B, nz, ny, nx): x rows of 16 and of a ragged length, a total voxel count
# that is not a multiple of the 16-voxel strips, several samples
SHAPES = [(1, 4, 4, 16), (2, 3, 5, 7), (1, 8, 8, 8)]
# the weight-gradient kernel gives each block rows / 256 (at least one) x-rows
# of B * ny * nz: these shapes run 4 rows per block (B = 2, 32 x 32 x 16) and
# 2 rows per block with a ragged last block (585 rows)
BACKWARD_SHAPES = SHAPES[:2] + [(2, 16, 32, 32), (3, 15, 13, 11)]


def _theta(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    th = np.zeros(cnn.n_params())
    for W, b in cnn.unpack(th):
        W[...] = rng.uniform(-1, 1, W.shape) * scale * np.sqrt(6.0 / (27 * W.shape[1]))
        b[...] = rng.uniform(-0.1, 0.1, b.shape)
    return th.astype(np.float32)


def _net(theta):
    from paper_2107_07776_amd import Net
    net = Net(32, seed=1)
    net.set_params(torch.tensor(theta, device="cuda"))
    return net


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_forward_matches_oracle(shape):
    B, nz, ny, nx = shape
    print(f"[case] forward B={B} grid={nx}x{ny}x{nz}", flush=True)
    theta = _theta(10)
    x = np.random.default_rng(11).standard_normal((B, cnn.N_IN, nz, ny, nx)).astype(np.float32)
    net = _net(theta)
    y = net.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    p = cnn.unpack(cnn.bf16_round(theta))
    xo = cnn.bf16_round(x)
    yr, _ = cnn.forward(p, xo, act_round=cnn.bf16_round)
    y64, _ = cnn.forward(p, xo)
    e1, e2 = _rel(y, yr), _rel(y, y64)
    print(f"forward: vs rounded-activation oracle {e1:.2e}, vs FP64 oracle {e2:.2e}")
    assert e1 <= TOL_FWD_ROUNDED and e2 <= TOL_FWD
    net.close()


@pytest.mark.parametrize("shape", BACKWARD_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_backward_matches_oracle(shape):
    B, nz, ny, nx = shape
    print(f"[case] backward B={B} grid={nx}x{ny}x{nz}", flush=True)
    theta = _theta(20)
    rng = np.random.default_rng(21)
    x = rng.standard_normal((B, cnn.N_IN, nz, ny, nx)).astype(np.float32)
    target = rng.standard_normal((B, cnn.N_OUT, nz, ny, nx)).astype(np.float32)
    net = _net(theta)
    yt = net.forward(torch.tensor(x, device="cuda"))
    loss, dy = net.mse(yt, torch.tensor(target, device="cuda"))
    net.zero_grad()
    net.backward(dy)
    g = net.grads().cpu().numpy()
    p = cnn.unpack(cnn.bf16_round(theta))
    yo, acts = cnn.forward(p, cnn.bf16_round(x), act_round=cnn.bf16_round)
    lo, dyo = cnn.mse(yo, target)
    assert abs(loss - lo) <= 1e-2 * lo
    go = cnn.backward(p, acts, dyo)
    for l, ((gw, gb), (Wg, bg)) in enumerate(zip(go, cnn.unpack(g.astype(np.float64)))):
        ew, eb = _rel(Wg, gw), _rel(bg, gb)
        print(f"layer {l}: weight-gradient rel err {ew:.2e}, bias {eb:.2e}")
        assert ew <= TOL_GRAD and eb <= TOL_GRAD
    net.close()


def test_adam_step_and_training_reduce_loss():
    B, nz, ny, nx = 2, 8, 8, 8
    theta = _theta(30)
    rng = np.random.default_rng(31)
    x = rng.standard_normal((B, cnn.N_IN, nz, ny, nx)).astype(np.float32)
    # a target the network can represent: a smooth function of the inputs
    target = np.stack([0.5 * x[:, 0] - 0.25 * np.roll(x[:, 1], 1, axis=-1),
                       0.3 * x[:, 4] + 0.2 * x[:, 2]], 1).astype(np.float32)
    net = _net(theta)
    xt, tt = torch.tensor(x, device="cuda"), torch.tensor(target, device="cuda")
    lr = 1e-3
    # first Adam step: every parameter moves by about lr * sign(g) (oracle gradients)
    y = net.forward(xt)
    _, dy = net.mse(y, tt)
    net.zero_grad()
    net.backward(dy)
    net.adam_step(lr)
    step = (net.params().cpu().numpy() - theta) / lr
    p = cnn.unpack(cnn.bf16_round(theta))
    yo, acts = cnn.forward(p, cnn.bf16_round(x), act_round=cnn.bf16_round)
    _, dyo = cnn.mse(yo, target)
    go = cnn.pack(cnn.backward(p, acts, dyo))
    expect = (cnn.adam_step(theta.astype(np.float64), go, np.zeros_like(go), np.zeros_like(go), 1, lr)
              - theta) / lr
    big = np.abs(go) > 1e-3 * np.abs(go).max()
    assert np.mean(np.abs(step - expect)[big] > 0.05) < 0.01
    losses = []
    for _ in range(60):
        y = net.forward(xt)
        loss, dy = net.mse(y, tt)
        losses.append(loss)
        net.zero_grad()
        net.backward(dy)
        net.adam_step(lr)
    print("training losses:", [round(v, 4) for v in losses[::10]], round(losses[-1], 4))
    assert losses[-1] < 0.3 * losses[0]
    net.close()


def test_throughput_report():
    """Forward and forward+backward times at 32^3 and 48^3 (report only)."""
    for n in (32, 48):
        net = _net(_theta(40))
        x = torch.randn((1, cnn.N_IN, n, n, n), device="cuda", dtype=torch.float32)
        y = net.forward(x)
        _, dy = net.mse(y, torch.zeros_like(y))
        net.backward(dy)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            net.forward(x)
        torch.cuda.synchronize()
        tf = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            net.forward(x)
            net.backward(dy)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / reps
        flops = 2 * n ** 3 * 27 * (cnn.N_IN * 32 + 2 * 32 * 32 + 32 * cnn.N_OUT)
        print(f"{n}^3: forward {tf * 1e3:.3f} ms ({flops / tf / 1e12:.1f} TFLOP/s), "
              f"forward+backward {tb * 1e3:.3f} ms")
        net.close()


def test_quad_loss_matches_oracle():
    """The guess's training loss and its gradient against oracle.guess.quad_loss
    (FP32 data, FP64 accumulation of the loss: 1e-6 relative)."""
    from oracle import guess as oguess
    from paper_2107_07776_amd import Net
    rng = np.random.default_rng(50)
    B, n = 3, 1000
    A = rng.standard_normal((3, B, n, 5))                  # d1, d2, e at 5 nodes per cell
    G = np.stack([(A[0] ** 2).sum(-1), (A[0] * A[1]).sum(-1), (A[1] ** 2).sum(-1),
                  (A[2] * A[0]).sum(-1), (A[2] * A[1]).sum(-1), (A[2] ** 2).sum(-1)], 1).astype(np.float32)
    y = rng.standard_normal((B, 2, n)).astype(np.float32)
    net = Net(32, seed=1)
    loss, dy = net.quad_loss(torch.tensor(y, device="cuda"), torch.tensor(G, device="cuda"))
    lo, dyo = oguess.quad_loss(y.astype(np.float64), G.astype(np.float64))
    assert abs(loss - lo) <= 1e-6 * abs(lo)
    assert _rel(dy.cpu().numpy(), dyo) <= 1e-6
    net.close()
