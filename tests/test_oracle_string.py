"""Pins of the string-method oracle (oracle/string_method.py).

* Reparametrisation: points on a straight line end equally spaced (closed
  form); a dense unevenly sampled circle arc ends uniformly sampled in angle;
  end images, strings of two images and of zero length are left alone; an
  equal-arc string is a fixed point.
* Evolution: a steepest-descent step of every image, ends held if asked.
* On the two-dimensional Mueller-Brown surface (Mueller and Brown 1979) the
  iterated string from one minimum's basin to another's becomes a minimum
  energy path: its ends settle in the minima that scipy's minimiser finds
  independently, the force perpendicular to the path vanishes at every
  interior image, and its highest image lies next to the saddle point that
  scipy's root finder locates on grad V = 0 from there, below it in energy by
  no more than the discretisation allows.
"""

import math

import numpy as np
import pytest
import scipy.optimize

from oracle import string_method as sm

# Mueller-Brown: V = sum_k A_k exp(a_k (x - x0_k)^2 + b_k (x - x0_k)(y - y0_k) + c_k (y - y0_k)^2)
MB_A = np.array([-200.0, -100.0, -170.0, 15.0])
MB_a = np.array([-1.0, -1.0, -6.5, 0.7])
MB_b = np.array([0.0, 0.0, 11.0, 0.6])
MB_c = np.array([-10.0, -10.0, -6.5, 0.7])
MB_x0 = np.array([1.0, 0.0, -0.5, -1.0])
MB_y0 = np.array([0.0, 0.5, 1.5, 1.0])


def mb_v(p):
    x, y = p[..., 0:1], p[..., 1:2]
    dx, dy = x - MB_x0, y - MB_y0
    return np.sum(MB_A * np.exp(MB_a * dx * dx + MB_b * dx * dy + MB_c * dy * dy), axis=-1)


def mb_grad(p):
    x, y = p[..., 0:1], p[..., 1:2]
    dx, dy = x - MB_x0, y - MB_y0
    e = MB_A * np.exp(MB_a * dx * dx + MB_b * dx * dy + MB_c * dy * dy)
    gx = np.sum(e * (2 * MB_a * dx + MB_b * dy), axis=-1)
    gy = np.sum(e * (MB_b * dx + 2 * MB_c * dy), axis=-1)
    return np.stack([gx, gy], axis=-1)


def test_straight_line_becomes_equally_spaced():
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(6), rng.standard_normal(6)
    t = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, 9)]))
    x = a[None] + t[:, None] * (b - a)[None]
    y = sm.reparametrize(x)
    want = a[None] + np.linspace(0, 1, 11)[:, None] * (b - a)[None]
    assert np.abs(y - want).max() < 1e-13
    assert np.abs(sm.reparametrize(y) - y).max() < 1e-13       # a fixed point
    assert np.allclose(sm.arc_positions(y), np.linspace(0, 1, 11), atol=1e-14)


def test_dense_arc_ends_uniform_in_angle():
    n = 2001
    th = np.sort(np.concatenate([[0.0, math.pi / 2], np.random.default_rng(2).uniform(0, math.pi / 2, n - 2)]))
    x = np.stack([np.cos(th), np.sin(th)], axis=1)
    y = sm.reparametrize(x)
    ang = np.arctan2(y[:, 1], y[:, 0])
    assert np.abs(ang - np.linspace(0, math.pi / 2, n)).max() < 1e-5
    assert np.array_equal(y[0], x[0]) and np.array_equal(y[-1], x[-1])


def test_degenerate_strings():
    x = np.ones((5, 3, 3))
    assert np.array_equal(sm.reparametrize(x), x)                 # zero length
    two = np.random.default_rng(3).standard_normal((2, 4, 3))
    assert np.array_equal(sm.reparametrize(two), two)
    # coincident images inside the string are spread out again
    x = np.array([[0.0], [0.0], [0.0], [1.0], [3.0]])
    assert np.allclose(sm.reparametrize(x)[:, 0], [0.0, 0.75, 1.5, 2.25, 3.0])


def test_evolution_step():
    rng = np.random.default_rng(4)
    x, F = rng.standard_normal((6, 2, 3)), rng.standard_normal((6, 2, 3))
    y = sm.evolve(x, F, 0.1)
    assert np.allclose(y, x + 0.1 * F)
    y = sm.evolve(x, F, 0.1, fix_ends=True)
    assert np.array_equal(y[0], x[0]) and np.array_equal(y[-1], x[-1])
    assert np.allclose(y[1:-1], x[1:-1] + 0.1 * F[1:-1])


def _mb_string(n, h=1e-4, iters=20000):
    a, b = np.array([-0.5, 1.5]), np.array([0.6, 0.1])     # inside the basins of two minima
    x = a[None] + np.linspace(0, 1, n)[:, None] * (b - a)[None]
    for _ in range(iters):
        x = sm.step(x, -mb_grad(x), h)
    return x, a, b


def _fperp_max(x):
    """Largest force component perpendicular to the path (central-difference
    tangents) over the interior images."""
    F = -mb_grad(x)
    out = 0.0
    for i in range(1, len(x) - 1):
        tau = x[i + 1] - x[i - 1]
        tau /= np.linalg.norm(tau)
        out = max(out, np.linalg.norm(F[i] - np.dot(F[i], tau) * tau))
    return out


def test_mueller_brown_minimum_energy_path():
    x21, a, b = _mb_string(21)
    x, _, _ = _mb_string(41)
    # ends in the minima found independently
    for end, start in ((x[0], a), (x[-1], b)):
        m = scipy.optimize.minimize(lambda p: mb_v(p[None])[0], start, jac=lambda p: mb_grad(p[None])[0],
                                    method="BFGS", options={"gtol": 1e-10}).x
        assert np.abs(end - m).max() < 1e-4, (end, m)
    # the force perpendicular to the discretised path vanishes at first
    # order in the image spacing (the tangents and the polygon both carry an
    # error of order spacing x curvature): twice the images, half of it
    r = _fperp_max(x) / _fperp_max(x21)
    assert 0.35 < r < 0.75, r
    # the highest image sits next to the saddle point
    E = mb_v(x)
    k = int(np.argmax(E[1:-1])) + 1
    sp = scipy.optimize.root(lambda p: mb_grad(p[None])[0], x[k], tol=1e-12).x
    H = np.array([[mb_grad(sp[None] + e[None])[0] - mb_grad(sp[None] - e[None])[0]]
                  for e in (np.array([1e-6, 0]), np.array([0, 1e-6]))])[:, 0] / 2e-6
    assert np.sum(np.linalg.eigvalsh(0.5 * (H + H.T)) < 0) == 1       # a first-order saddle
    Es = mb_v(sp[None])[0]
    seg = np.linalg.norm(x[1] - x[0])
    assert np.linalg.norm(x[k] - sp) < seg
    assert Es - 2.0 < E[k] <= Es + 1e-9
