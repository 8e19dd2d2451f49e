"""Pins of the oracle's J/K, SCF and gradient against invariants and brute force.

* J and K against an einsum over the full ERI tensor (plain definition).
* SCF: Tr(PS) = N_e, PSP = 2P, vanishing commutator, invariance of E under a
  rigid rotation plus translation, independence of the converged E from the
  starting guess.
* Gradient: central finite differences of converged energies; zero net force
  and zero torque; rotation covariance.
"""

import numpy as np
import pytest

import inputs
import oracle
from inputs.geometry import random_rotation


def _rand_density(n, rng):
    A = rng.standard_normal((n, n))
    return 0.1 * (A + A.T)


@pytest.mark.parametrize("case", ["h2o_sto3g", "w2"])
def test_jk_against_full_tensor(case, sto3g, b631gs):
    w = inputs.workload(case)
    Z, x = w["instances"][0]
    b = oracle.build_basis(sto3g if w["basis"] == "sto-3g" else b631gs, Z, x)
    g = oracle.eri_tensor(b)
    P = _rand_density(b["nbf"], np.random.default_rng(3))
    Jr = np.einsum("ijkl,kl->ij", g, P)
    Kr = np.einsum("ikjl,kl->ij", g, P)
    J, K, nq = oracle.jk(b, P, tau=0.0)
    assert np.abs(J - Jr).max() < 1e-12 and np.abs(K - Kr).max() < 1e-12
    assert np.abs(J - J.T).max() < 1e-13 and np.abs(K - K.T).max() < 1e-13
    ns = b["nsh"]
    npair = ns * (ns + 1) // 2
    assert nq == npair * (npair + 1) // 2
    # screened build differs by less than the dropped bound
    Js, Ks, nqs = oracle.jk(b, P, tau=1e-12)
    assert nqs <= nq
    assert np.abs(Js - Jr).max() < 1e-9 and np.abs(Ks - Kr).max() < 1e-9


@pytest.fixture(scope="module")
def h2o_scf(sto3g):
    w = inputs.workload("h2o_sto3g")
    Z, x = w["instances"][0]
    b = oracle.build_basis(sto3g, Z, x)
    return b, oracle.scf(b, w["e_tol"], w["comm_tol"])


def test_scf_density_properties(h2o_scf):
    b, r = h2o_scf
    assert r["converged"]
    P, S, F = r["P"], r["S"], r["F"]
    assert np.trace(P @ S) == pytest.approx(10.0, abs=1e-10)
    assert np.abs(P @ S @ P - 2 * P).max() < 1e-9
    assert np.abs(F @ P @ S - S @ P @ F).max() < 1e-7
    # energy expression against J/K at the same P
    J, K, _ = oracle.jk(b, P, 0.0)
    H = r["H"]
    e = 0.5 * np.sum(P * (2 * H + J - 0.5 * K)) + oracle.nuclear_repulsion(b["Z"], b["xyz"])
    assert e == pytest.approx(r["E"], abs=1e-11)


def test_scf_rigid_motion_invariance(h2o_scf, sto3g):
    b, r = h2o_scf
    R = random_rotation(np.random.default_rng(11))
    x2 = b["xyz"] @ R.T + np.array([0.7, -1.3, 2.1])
    b2 = oracle.build_basis(sto3g, b["Z"], x2)
    r2 = oracle.scf(b2, 1e-10, 1e-8)
    assert r2["E"] == pytest.approx(r["E"], abs=1e-10)


def test_scf_guess_independence(h2o_scf):
    b, r = h2o_scf
    rng = np.random.default_rng(5)
    P0 = r["P"] + 0.05 * _rand_density(b["nbf"], rng)
    r2 = oracle.scf(b, 1e-10, 1e-8, guess=P0)
    assert r2["E"] == pytest.approx(r["E"], abs=1e-9)


def test_gradient_finite_difference(b631gs):
    Z, x = inputs.workload("h2o_sto3g")["instances"][0]
    b = oracle.build_basis(b631gs, Z, x)
    r = oracle.scf(b, 1e-12, 1e-10)
    g = oracle.gradient(b, r["P"], r["F"])
    h = 1e-4
    for a, d in [(0, 0), (0, 2), (1, 1), (2, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[a, d] += h
        xm[a, d] -= h
        ep = oracle.scf(oracle.build_basis(b631gs, Z, xp), 1e-12, 1e-10, guess=r["P"])["E"]
        em = oracle.scf(oracle.build_basis(b631gs, Z, xm), 1e-12, 1e-10, guess=r["P"])["E"]
        assert g[a, d] == pytest.approx((ep - em) / (2 * h), abs=1e-7)


def test_gradient_net_force_torque_and_rotation(sto3g):
    Z, x = inputs.water_cluster(2, 21)
    b = oracle.build_basis(sto3g, Z, x)
    r = oracle.scf(b, 1e-11, 1e-9)
    g = oracle.gradient(b, r["P"], r["F"])
    assert np.abs(g.sum(axis=0)).max() < 1e-10
    assert np.abs(np.cross(x, g).sum(axis=0)).max() < 1e-8
    R = random_rotation(np.random.default_rng(2))
    b2 = oracle.build_basis(sto3g, Z, x @ R.T + 1.0)
    r2 = oracle.scf(b2, 1e-11, 1e-9)
    g2 = oracle.gradient(b2, r2["P"], r2["F"])
    assert np.abs(g2 - g @ R.T).max() < 1e-8


@pytest.mark.parametrize("tau", [0.0, 1e-12, 1e-6])
def test_jk_pairs_against_full_tensor_and_canonical_build(b631gs, tau):
    """The sampled-block J/K (direct sums over every ket pair) equal the
    einsum over the full ERI tensor at tau = 0 and the canonical-quartet build
    at the same Schwarz cutoff, for every shell pair of (H2O)2, diagonal and
    off-diagonal, in both orders."""
    z, x = inputs.workload("w2")["instances"][0]
    b = oracle.build_basis(b631gs, z, x)
    P = _rand_density(b["nbf"], np.random.default_rng(17))
    Q = oracle.schwarz(b)
    ns = b["nsh"]
    pairs = [(a, c) for a in range(ns) for c in range(ns)]
    Jp, Kp = oracle.jk_pairs(b, P, pairs, tau, Q)
    assert not np.isnan(Jp).any() and not np.isnan(Kp).any()
    J, K, _ = oracle.jk(b, P, tau, Q)
    assert np.abs(Jp - J).max() < 1e-12 and np.abs(Kp - K).max() < 1e-12
    if tau == 0.0:
        g = oracle.eri_tensor(b)
        assert np.abs(Jp - np.einsum("ijkl,kl->ij", g, P)).max() < 1e-12
        assert np.abs(Kp - np.einsum("ikjl,kl->ij", g, P)).max() < 1e-12
    # a subset fills only its own blocks
    Js, Ks = oracle.jk_pairs(b, P, [(3, 0), (5, 5)], tau, Q)
    bf, l = b["bf"], b["l"]
    nc = lambda s: (int(l[s]) + 1) * (int(l[s]) + 2) // 2
    for a, c in [(3, 0), (5, 5)]:
        blk = np.s_[bf[a]:bf[a] + nc(a), bf[c]:bf[c] + nc(c)]
        # (threads add their partial sums in any order: equal to rounding)
        assert np.abs(Js[blk] - Jp[blk]).max() < 1e-14 and np.abs(Ks[blk] - Kp[blk]).max() < 1e-14
    assert np.isnan(Js).sum() == b["nbf"] ** 2 - nc(3) * nc(0) - nc(5) ** 2


def test_gradient_of_selected_atoms_equals_full_gradient_rows(b631gs):
    """The atom-restricted gradient (quartets touching the selected atoms,
    their one-electron and operator terms) reproduces those rows of the full
    gradient at an arbitrary density and Fock matrix, and leaves the rest NaN."""
    z, x = inputs.water_cluster(2, 5)
    b = oracle.build_basis(b631gs, z, x)
    rng = np.random.default_rng(23)
    P = _rand_density(b["nbf"], rng)
    F = _rand_density(b["nbf"], rng)
    g = oracle.gradient(b, P, F)
    for atoms in ([1], [0, 4], [5, 2, 3]):
        ga = oracle.gradient(b, P, F, atoms=atoms)
        assert np.abs(ga[atoms] - g[atoms]).max() < 1e-11, atoms
        others = [k for k in range(len(z)) if k not in atoms]
        assert np.isnan(ga[others]).all()


def test_jk_sample_with_stride_one_is_the_full_build(b631gs):
    """The timing sample at stride 1 is the canonical build itself; at
    stride s it evaluates ceil(n / s) quartets."""
    z, x = inputs.workload("w2")["instances"][0]
    b = oracle.build_basis(b631gs, z, x)
    P = _rand_density(b["nbf"], np.random.default_rng(29))
    J, K, nq = oracle.jk(b, P)
    Js, Ks, ns = oracle.jk_sample(b, P, 1, 2)
    assert ns == nq and np.abs(Js - J).max() < 1e-13 and np.abs(Ks - K).max() < 1e-13
    _, _, n7 = oracle.jk_sample(b, P, 7, 1)
    assert n7 == (nq + 6) // 7
