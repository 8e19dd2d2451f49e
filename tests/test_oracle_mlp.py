"""Pins of the learned-guess network oracle (oracle/mlp.py): gradients against
central finite differences, the loss where it is known in closed form, and
Adam against its published update written out step by step."""

import numpy as np

from oracle import mlp

RNG = np.random.default_rng(2000)


def _problem(rows=7, din=5, hidden=6, dout=4):
    theta = mlp.init(din, hidden, dout, RNG)
    # a larger last layer so every parameter has a visible effect
    W1, b1, W2, b2, W3, b3 = mlp.unflatten(theta, din, hidden, dout)
    W3 = RNG.standard_normal(W3.shape)
    b1 = RNG.standard_normal(b1.shape) * 0.1
    b2 = RNG.standard_normal(b2.shape) * 0.1
    b3 = RNG.standard_normal(b3.shape) * 0.1
    theta = mlp.flatten([W1, b1, W2, b2, W3, b3])
    x = RNG.standard_normal((rows, din))
    t = RNG.standard_normal((rows, dout))
    mask = (RNG.random((rows, dout)) < 0.7).astype(float)
    mask[0, 0] = 1.0
    return theta, x, t, mask, din, hidden, dout


def test_gradient_against_central_differences():
    theta, x, t, mask, din, hidden, dout = _problem()
    _, g = mlp.gradient(theta, x, t, mask, din, hidden, dout)
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        tp = theta.copy()
        tp[k] += h
        tm = theta.copy()
        tm[k] -= h
        fd[k] = (mlp.loss(tp, x, t, mask, din, hidden, dout) -
                 mlp.loss(tm, x, t, mask, din, hidden, dout)) / (2 * h)
    # ReLU kinks are measure-zero for random inputs; central differences are O(h^2)
    assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())


def test_loss_closed_form():
    """With zero weights the network outputs b3 plus the skipped inputs (the
    last dout columns of x) for every row."""
    din, hidden, dout = 3, 4, 2
    b3 = np.array([0.5, -1.5])
    theta = mlp.flatten([np.zeros((din, hidden)), np.zeros(hidden), np.zeros((hidden, hidden)),
                         np.zeros(hidden), np.zeros((hidden, dout)), b3])
    x = RNG.standard_normal((5, din))
    t = RNG.standard_normal((5, dout))
    mask = np.ones((5, dout))
    mask[2, 1] = 0.0
    y = b3 + x[:, 1:3]
    ref = np.sum(mask * (y - t) ** 2) / mask.sum()
    assert abs(mlp.loss(theta, x, t, mask, din, hidden, dout) - ref) < 1e-14
    # and the gradient is 2 (y - t) averaged over the masked entries for b3 only
    _, g = mlp.gradient(theta, x, t, mask, din, hidden, dout)
    gb3 = g[-dout:]
    assert np.allclose(gb3, (2 * mask * (y - t)).sum(axis=0) / mask.sum(), atol=1e-14)
    assert np.abs(g[:-dout]).max() == 0.0


def test_adam_against_published_update():
    """Two Adam steps on a 2-vector, each written out from Algorithm 1."""
    th = np.array([1.0, -2.0])
    g1 = np.array([0.3, -0.1])
    g2 = np.array([-0.2, 0.4])
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    t1, m1, v1 = mlp.adam_step(th, g1, np.zeros(2), np.zeros(2), 1, lr, b1, b2, eps)
    # step 1: m = 0.1 g, v = 0.001 g^2, mhat = g, vhat = g^2 -> th - lr g/(|g|+eps)
    assert np.allclose(t1, th - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    t2, _, _ = mlp.adam_step(t1, g2, m1, v1, 2, lr, b1, b2, eps)
    m = b1 * (1 - b1) * g1 + (1 - b1) * g2
    v = b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2
    ref = t1 - lr * (m / (1 - b1 ** 2)) / (np.sqrt(v / (1 - b2 ** 2)) + eps)
    assert np.allclose(t2, ref, rtol=0, atol=1e-15)


def test_training_reduces_loss():
    theta, x, t, mask, din, hidden, dout = _problem(rows=32)
    _, losses = mlp.train(theta, x, t, mask, din, hidden, dout, steps=200, lr=1e-2)
    assert losses[-1] < 0.5 * losses[0]
