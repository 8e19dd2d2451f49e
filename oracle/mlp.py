"""Oracle of the learned-guess network: a two-hidden-layer perceptron with ReLU
activations, a masked mean-squared-error loss and the Adam optimiser, in
NumPy FP64.

Test infrastructure only (tests, the smoke check and the CPU baseline use it;
the product path never does).  Written from the definitions:
  h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3 + x_skip,
  loss = sum(mask * (y - t)^2) / sum(mask),
where x_skip is the last dout input columns (a residual connection: the
in-run inputs end with the previous step's residual block, so an untrained
network extrapolates it and training learns the correction);
back-propagation by the chain rule, and Adam as published by Kingma and Ba
(2015, Algorithm 1: first and second moment estimates with bias correction).

Parameters travel as one flat FP32/FP64 vector in the order
W1 (din x h), b1 (h), W2 (h x h), b2 (h), W3 (h x dout), b3 (dout), each
matrix row-major; this is the layout of bscf_guess_set_params.

Pins (tests/test_oracle_mlp.py): gradients against central finite
differences, the loss at a point where it is known in closed form, and Adam
steps against the published update written out by hand.
"""

import numpy as np


def shapes(din, hidden, dout):
    return [(din, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, dout), (dout,)]


def n_params(din, hidden, dout):
    return sum(int(np.prod(s)) for s in shapes(din, hidden, dout))


def unflatten(theta, din, hidden, dout):
    out, k = [], 0
    for s in shapes(din, hidden, dout):
        m = int(np.prod(s))
        out.append(np.asarray(theta[k:k + m], dtype=np.float64).reshape(s))
        k += m
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def init(din, hidden, dout, rng):
    """He-style initial weights (scale sqrt(2/fan_in)), zero biases, a small
    last layer so the first predictions are near zero."""
    W1 = rng.standard_normal((din, hidden)) * np.sqrt(2.0 / din)
    W2 = rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden)
    W3 = rng.standard_normal((hidden, dout)) * np.sqrt(2.0 / hidden) * 0.01
    return flatten([W1, np.zeros(hidden), W2, np.zeros(hidden), W3, np.zeros(dout)])


def forward(theta, x, din, hidden, dout):
    """Outputs y and the activations (h1, h2) of the rows x (rows x din)."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, din, hidden, dout)
    h1 = np.maximum(x @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ W3 + b3 + x[:, din - dout:], h1, h2


def loss(theta, x, t, mask, din, hidden, dout):
    y, _, _ = forward(theta, x, din, hidden, dout)
    return float(np.sum(mask * (y - t) ** 2) / np.sum(mask))


def gradient(theta, x, t, mask, din, hidden, dout):
    """Loss and its gradient with respect to the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, din, hidden, dout)
    y, h1, h2 = forward(theta, x, din, hidden, dout)
    cnt = np.sum(mask)
    dy = 2.0 * mask * (y - t) / cnt
    gW3 = h2.T @ dy
    gb3 = dy.sum(axis=0)
    dh2 = (dy @ W3.T) * (h2 > 0)
    gW2 = h1.T @ dh2
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (h1 > 0)
    gW1 = x.T @ dh1
    gb1 = dh1.sum(axis=0)
    return float(np.sum(mask * (y - t) ** 2) / cnt), flatten([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(theta, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new theta, m, v."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(theta, x, t, mask, din, hidden, dout, steps, lr=1e-3):
    """Full-batch Adam from zero moments; returns the final parameters and the
    loss before each step."""
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    for k in range(1, steps + 1):
        L, g = gradient(theta, x, t, mask, din, hidden, dout)
        losses.append(L)
        theta, m, v = adam_step(theta, g, m, v, k, lr)
    return theta, losses
