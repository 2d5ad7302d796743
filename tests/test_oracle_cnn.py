"""Pins of the oracle's convolutional network against brute force, finite
differences and closed forms.

* the vectorised circular convolution equals an explicit seven-fold loop;
* the network commutes with periodic translations;
* the hand-written backward pass equals central finite differences of the
  loss for every parameter of a small network;
* Adam's first step moves every parameter by lr * g / (|g| + eps);
* bfloat16 rounding reproduces exactly representable values and rounds ties
  to even.
"""
import numpy as np

from oracle import cnn


def _params(rng, channels, n_in=3, n_out=1, scale=0.3):
    theta = rng.standard_normal(cnn.n_params(channels, n_in, n_out)) * scale
    return theta, cnn.unpack(theta, channels, n_in, n_out)


def test_conv_equals_brute_force_loops():
    rng = np.random.default_rng(0)
    B, ci, co, nz, ny, nx = 2, 2, 3, 3, 4, 5
    X = rng.standard_normal((B, ci, nz, ny, nx))
    W = rng.standard_normal((co, ci, 3, 3, 3))
    b = rng.standard_normal(co)
    Y = cnn.conv3d(X, W, b)
    ref = np.zeros_like(Y)
    for n in range(B):
        for o in range(co):
            for z in range(nz):
                for y in range(ny):
                    for x in range(nx):
                        s = b[o]
                        for i in range(ci):
                            for kz in range(3):
                                for ky in range(3):
                                    for kx in range(3):
                                        s += W[o, i, kz, ky, kx] * X[n, i, (z + kz - 1) % nz,
                                                                     (y + ky - 1) % ny, (x + kx - 1) % nx]
                        ref[n, o, z, y, x] = s
    assert np.allclose(Y, ref, rtol=0, atol=1e-12)


def test_translation_equivariance():
    rng = np.random.default_rng(1)
    _, params = _params(rng, 4)
    X = rng.standard_normal((1, 3, 4, 5, 6))
    Y, _ = cnn.forward(params, X)
    Xs = np.roll(X, shift=(1, 2, 3), axis=(2, 3, 4))
    Ys, _ = cnn.forward(params, Xs)
    assert np.allclose(Ys, np.roll(Y, shift=(1, 2, 3), axis=(2, 3, 4)), atol=1e-12)


def test_backward_equals_finite_differences():
    rng = np.random.default_rng(2)
    ch = 3
    theta, params = _params(rng, ch)
    X = rng.standard_normal((2, 3, 3, 3, 4))
    target = rng.standard_normal((2, 1, 3, 3, 4))

    def loss(th):
        out, _ = cnn.forward(cnn.unpack(th, ch, 3, 1), X)
        return cnn.mse(out, target)[0]

    out, acts = cnn.forward(params, X)
    _, dY = cnn.mse(out, target)
    g = cnn.pack(cnn.backward(params, acts, dY))
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        fd[k] = (loss(theta + e) - loss(theta - e)) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max(), np.abs(g - fd).max()


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m, v = np.zeros(50), np.zeros(50)
    lr, eps = 1e-3, 1e-8
    new = cnn.adam_step(theta, g, m, v, 1, lr, eps=eps)
    assert np.allclose(new, theta - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # second step with the same gradient: bias-corrected moments are still g and g^2
    new2 = cnn.adam_step(new, g, m, v, 2, lr, eps=eps)
    assert np.allclose(new2, new - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)


def test_bf16_rounding():
    one = 1.0
    vals = np.array([one, one + 2.0 ** -8, one + 3 * 2.0 ** -9, one + 2.0 ** -7 + 2.0 ** -8,
                     -2.5, 3.0e38], dtype=np.float32)
    r = cnn.bf16_round(vals)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to the even mantissa (1)
    # 1 + 3*2^-9 lies above the midpoint: up to 1 + 2^-7
    # 1 + 2^-7 + 2^-8 is halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even): up
    assert r.tolist()[:5] == [1.0, 1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -6, -2.5]
    assert abs(r[5] - 3.0e38) <= 3.0e38 * 2.0 ** -8
    assert np.isnan(cnn.bf16_round(np.array([np.nan], dtype=np.float32))[0])


def test_backward_with_the_guess_loss_equals_finite_differences():
    """The library's shapes (6 inputs, 2 outputs) under the guess's
    quadratic loss (oracle.guess.quad_loss, Gram data of a random
    positive semi-definite form per cell)."""
    from oracle import guess
    rng = np.random.default_rng(5)
    ch = 2
    theta, params = _params(rng, ch, cnn.N_IN, cnn.N_OUT)
    X = rng.standard_normal((2, cnn.N_IN, 2, 3, 3))
    A = rng.standard_normal((2, 3, 2, 18))          # per cell: d1, d2, e at 3 "nodes"
    G = np.stack([(A[:, :, 0] ** 2).sum(1), (A[:, :, 0] * A[:, :, 1]).sum(1), (A[:, :, 1] ** 2).sum(1),
                  (A[:, :, 0] * A[:, :, 1]).sum(1) * 0.3, (A[:, :, 1] ** 2).sum(1) * -0.2,
                  (A[:, :, 0] ** 2).sum(1) + 1.0], 1)

    def loss(th):
        out, _ = cnn.forward(cnn.unpack(th, ch), X)
        return guess.quad_loss(out.reshape(2, 2, -1), G)[0]

    out, acts = cnn.forward(params, X)
    _, dy = guess.quad_loss(out.reshape(2, 2, -1), G)
    g = cnn.pack(cnn.backward(params, acts, dy.reshape(out.shape)))
    h = 1e-6
    fd = np.array([(loss(theta + h * e) - loss(theta - h * e)) / (2 * h) for e in np.eye(theta.size)])
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max(), np.abs(g - fd).max()


def test_parameter_count():
    assert cnn.n_params(32, 3, 1) == 58849
    assert cnn.n_params() == 32 * 6 * 27 + 32 + 2 * (32 * 32 * 27 + 32) + 2 * 32 * 27 + 2
