"""Small 3D convolutional network of the learned pressure initial guess
(oracle; TEST INFRASTRUCTURE ONLY).

The network is not part of the paper; it predicts, per cell, how to blend
the solver's last two pressure increments into the next one, from cell
statistics of its own history.  This module is its plain FP64 definition,
written with numpy:

* layers N_IN -> C -> C -> C -> N_OUT (6 -> 32 -> 32 -> 32 -> 2 in the
  library), 3x3x3 kernels, circular (periodic) padding, ReLU after every
  layer but the last;
* convolution as cross-correlation, the layout of the weights being
  [out][in][dz][dy][dx] and of the activations [batch][channel][z][y][x]:
      y[o, z, y, x] = b[o] + sum_{i, dz, dy, dx} W[o, i, dz+1, dy+1, dx+1]
                              * X[i, (z+dz) mod nz, (y+dy) mod ny, (x+dx) mod nx];
* mean-squared-error loss L = mean((yhat - y)^2) (the guess's own loss,
  a quadratic form per cell, is ``oracle.guess.quad_loss``);
* Adam (Kingma and Ba 2015) with bias correction;
* round-to-nearest-even to bfloat16 (the upper 16 bits of an IEEE binary32).
"""
import numpy as np

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]

N_IN, N_OUT = 6, 2


def layer_shapes(channels=32, n_in=N_IN, n_out=N_OUT):
    """(out, in) of the four layers."""
    return [(channels, n_in), (channels, channels), (channels, channels), (n_out, channels)]


def n_params(channels=32, n_in=N_IN, n_out=N_OUT):
    return sum(o * i * 27 + o for o, i in layer_shapes(channels, n_in, n_out))


def unpack(theta, channels=32, n_in=N_IN, n_out=N_OUT):
    """Split the flat parameter vector into [(W, b)] per layer, W in
    [out][in][3][3][3] order followed by b[out], layer after layer."""
    out, k = [], 0
    for o, i in layer_shapes(channels, n_in, n_out):
        W = theta[k:k + o * i * 27].reshape(o, i, 3, 3, 3)
        k += o * i * 27
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    return out


def pack(params):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in params])


def shift(X, off):
    """X shifted so that entry (z, y, x) holds X[(z+dz), (y+dy), (x+dx)] (periodic)."""
    dz, dy, dx = off
    return np.roll(X, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


def conv3d(X, W, b):
    """Circular 3x3x3 cross-correlation, X: [B][in][nz][ny][nx]."""
    Y = np.broadcast_to(b[None, :, None, None, None], (X.shape[0], W.shape[0]) + X.shape[2:]).copy()
    for off in OFFSETS:
        Wk = W[:, :, off[0] + 1, off[1] + 1, off[2] + 1]
        Y += np.einsum("oi,bizyx->bozyx", Wk, shift(X, off))
    return Y


def conv3d_grad(X, W, dY):
    """Gradients of sum(dY * conv3d(X, W, b)) with respect to X, W and b."""
    dX = np.zeros_like(X)
    dW = np.zeros_like(W)
    for off in OFFSETS:
        Wk = W[:, :, off[0] + 1, off[1] + 1, off[2] + 1]
        Xs = shift(X, off)
        dW[:, :, off[0] + 1, off[1] + 1, off[2] + 1] = np.einsum("bozyx,bizyx->oi", dY, Xs)
        # d/dX of X shifted by +off is the adjoint shift by -off
        dX += shift(np.einsum("oi,bozyx->bizyx", Wk, dY), (-off[0], -off[1], -off[2]))
    db = dY.sum(axis=(0, 2, 3, 4))
    return dX, dW, db


def forward(params, X, act_round=None):
    """Returns the output [B][n_out][nz][ny][nx] and the inputs of every layer.
    ``act_round`` (e.g. bf16_round) is applied to every hidden activation,
    modelling storage of the activations in a narrower format."""
    acts = [X]
    A = X
    for li, (W, b) in enumerate(params):
        Z = conv3d(A, W, b)
        A = np.maximum(Z, 0.0) if li < len(params) - 1 else Z
        if li < len(params) - 1:
            if act_round is not None:
                A = act_round(A)
            acts.append(A)
    return A, acts


def backward(params, acts, dY):
    """Parameter gradients of sum(dY * forward(params, X)); ReLU'(z) is taken
    as (relu(z) > 0), i.e. 0 at z = 0."""
    grads = [None] * len(params)
    G = dY
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        dX, dW, db = conv3d_grad(acts[li], W, G)
        grads[li] = (dW, db)
        if li > 0:
            G = dX * (acts[li] > 0.0)
    return grads


def mse(yhat, y):
    """L = mean((yhat - y)^2) and dL/dyhat."""
    d = yhat - y
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the flat parameters at step t >= 1 (in place on m, v);
    returns the new parameters."""
    m *= beta1
    m += (1.0 - beta1) * grad
    v *= beta2
    v += (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps)


def bf16_round(x):
    """Round float32 values to the nearest bfloat16, ties to even, returned as
    float64 (NaN stays NaN)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)
