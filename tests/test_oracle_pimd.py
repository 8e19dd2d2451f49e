"""Pins of the ring-polymer integrator oracle (oracle/pimd.py).

* Philox4x32-10 against the published known-answer vectors (golden file).
* Box-Muller deviates: moments of a large sample.
* Normal modes: C orthogonal, and C^T L C diagonal with the closed-form
  eigenvalues 4 sin^2(k pi / P) of the cyclic bead Laplacian L.
* The free ring-polymer step A against the matrix exponential of the linear
  equations of motion in bead coordinates (scipy.linalg.expm), which uses no
  normal modes.
* NVE: time reversibility, and the conserved H of a ring polymer in a
  harmonic well fluctuating at O(dt^2) without drift.
* PILE-L: in a harmonic well the thermostatted run samples the exact
  quantum-classical (ring-polymer) averages: <p^2/2m> = k_B T/2 per bead
  degree of freedom and the centroid variance of the discretised path
  integral, which has a closed form for a harmonic oscillator.
"""

import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import pimd

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KB = 3.166811563e-6


def test_philox_known_answers():
    g = json.load(open(os.path.join(GOLD, "philox4x32_10_kat.json")))
    for v in g["vectors"]:
        ctr = [int(h, 16) for h in v["ctr"]]
        key = [int(h, 16) for h in v["key"]]
        assert pimd.philox4x32_10(ctr, key) == [int(h, 16) for h in v["out"]]


def test_gaussian_deviates_moments():
    z = np.concatenate([pimd.gaussians(7, h, 5001) for h in range(20)])
    n = z.size
    assert abs(z.mean()) < 4 / math.sqrt(n)
    assert abs(z.var() - 1) < 4 * math.sqrt(2 / n)
    assert abs(np.mean(z ** 4) - 3) < 4 * math.sqrt(96 / n)
    # odd number of deviates: the last pair is cut, the rest unchanged
    assert np.array_equal(pimd.gaussians(3, 5, 7), pimd.gaussians(3, 5, 8)[:7])
    # different half-steps and seeds give different deviates
    assert not np.allclose(pimd.gaussians(3, 5, 8), pimd.gaussians(3, 6, 8))
    assert not np.allclose(pimd.gaussians(3, 5, 8), pimd.gaussians(4, 5, 8))


@pytest.mark.parametrize("P", [1, 2, 3, 4, 7, 16, 32])
def test_normal_modes_diagonalise_the_ring(P):
    C = pimd.normal_mode_matrix(P)
    assert np.abs(C.T @ C - np.eye(P)).max() < 1e-13
    L = 2 * np.eye(P) - np.roll(np.eye(P), 1, axis=0) - np.roll(np.eye(P), -1, axis=0)
    if P == 1:
        L = np.zeros((1, 1))
    if P == 2:
        L = np.array([[2.0, -2.0], [-2.0, 2.0]])   # both neighbours are the other bead
    D = C.T @ L @ C
    lam = np.array([4 * math.sin(k * math.pi / P) ** 2 for k in range(P)])
    assert np.abs(D - np.diag(lam)).max() < 1e-12
    w = pimd.mode_frequencies(P, 1.0)
    assert np.allclose(w ** 2, lam)


def _rand_state(P, N, seed):
    rng = np.random.default_rng(seed)
    m = rng.uniform(1000.0, 30000.0, N)
    x = rng.standard_normal((P, N, 3))
    p = rng.standard_normal((P, N, 3)) * np.sqrt(m)[None, :, None] * 0.01
    return m, x, p


@pytest.mark.parametrize("P", [1, 4, 6])
def test_free_ring_step_against_matrix_exponential(P):
    N, T, dt = 2, 300.0, 20.0
    m, x, p = _rand_state(P, N, 3)
    sim = pimd.PileL(m, x, p, T, dt, KB, thermostat=False)
    sim.A()
    # bead-space linear system: dq/dt = p/m, dp/dt = -m wp^2 L q
    wp = pimd.omega_p(P, T, KB)
    L = 2 * np.eye(P) - np.roll(np.eye(P), 1, axis=0) - np.roll(np.eye(P), -1, axis=0)
    if P == 1:
        L = np.zeros((1, 1))
    for a in range(N):
        M = np.zeros((2 * P, 2 * P))
        M[:P, P:] = np.eye(P) / m[a]
        M[P:, :P] = -m[a] * wp ** 2 * L
        U = scipy.linalg.expm(M * dt)
        for d in range(3):
            y = U @ np.concatenate([x[:, a, d], p[:, a, d]])
            assert np.abs(sim.x[:, a, d] - y[:P]).max() < 1e-10
            assert np.abs(sim.p[:, a, d] - y[P:]).max() < 1e-10 * np.abs(p).max() + 1e-14


def _harmonic(k):
    return lambda x: (-k[None, :, None] * x, 0.5 * np.sum(k[None, :, None] * x * x, axis=(1, 2)))


def _run(sim, force, n):
    F, V = force(sim.x)
    Hs = []
    for _ in range(n):
        sim.begin(F)
        F, V = force(sim.x)
        sim.end(F)
        Hs.append(sim.hamiltonian(V))
    return np.array(Hs)


def test_nve_reversible_and_conserving():
    P, N, T, dt = 8, 3, 300.0, 10.0
    m, x, p = _rand_state(P, N, 5)
    k = m * (0.01 ** 2)            # harmonic wells of frequency 0.01 Eh/hbar
    force = _harmonic(k)
    sim = pimd.PileL(m, x, p, T, dt, KB, thermostat=False)
    H = _run(sim, force, 400)
    assert (H.max() - H.min()) < 2e-3 * abs(H.mean())
    # no drift: the first and last quarters fluctuate about the same mean
    assert abs(H[:100].mean() - H[-100:].mean()) < 2e-4 * abs(H.mean())
    # halving dt cuts the fluctuation by about four (second-order splitting)
    sim2 = pimd.PileL(m, x, p, T, dt / 2, KB, thermostat=False)
    H2 = _run(sim2, force, 800)
    r = (H.max() - H.min()) / (H2.max() - H2.min())
    assert 3.0 < r < 5.0, r
    # reversibility: flip the momenta and integrate back
    sim.p = -sim.p
    _run(sim, force, 400)
    assert np.abs(sim.x - x).max() < 1e-9
    assert np.abs(sim.p + p).max() < 1e-9 * np.abs(p).max()


def test_pile_samples_the_harmonic_ring_polymer():
    """One particle of mass m in a 3-D well of frequency w0 at temperature T
    as a P-bead ring polymer (all in the module's convention).  Exact:
    <p^2/2m> = k_B T / 2 per bead degree of freedom, and the centroid
    variance per direction <qc^2> = k_B T / (m w0^2) (the centroid of the
    discretised path is a classical coordinate in the full potential)."""
    P, T, dt = 4, 300.0, 20.0
    m = np.array([1836.0])
    w0 = 0.005
    k = m * w0 ** 2
    force = _harmonic(k)
    x = np.zeros((P, 1, 3))
    p = np.zeros((P, 1, 3))
    sim = pimd.PileL(m, x, p, T, dt, KB, thermostat=True, tau0=1.0 / (2 * w0), seed=11)
    F, _ = force(sim.x)
    ke, qc2 = [], []
    for s in range(40000):
        sim.begin(F)
        F, _ = force(sim.x)
        sim.end(F)
        if s >= 2000:
            ke.append(sim.kinetic())
            qc2.append(np.mean(sim.x[:, 0, :].mean(axis=0) ** 2))
    kt = KB * T
    ke, qc2 = np.array(ke), np.array(qc2)
    assert abs(ke.mean() / (1.5 * P * kt) - 1) < 0.03, ke.mean() / (1.5 * P * kt)
    assert abs(qc2.mean() / (kt / (m[0] * w0 ** 2)) - 1) < 0.08, qc2.mean() * m[0] * w0 ** 2 / kt
