"""Deterministic J and K (bscf_set_deterministic / bscf_scf_opts.deterministic):
the class kernels accumulate into exact 128-bit fixed point instead of FP64
atomics, so repeated builds at the same densities give bitwise equal J and K
whatever order the workgroups finish in, equal to the atomic build to
rounding and to the oracle's J and K.  An SCF in deterministic mode reaches
the energies of the default mode."""

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def beadscf():
    from paper_1601_02713_amd import beadscf as b
    return b


def _rand_sym(n, seed):
    A = np.random.default_rng([77, seed]).standard_normal((n, n))
    return 0.02 * (A + A.T)


@pytest.mark.parametrize("variant", ["auto", "coop"])
def test_bitwise_repeatable_and_equal_to_atomic_build(beadscf, b631gs, variant, monkeypatch):
    if variant != "auto":
        monkeypatch.setenv("BSCF_VARIANT", variant)
    w = inputs.workload("w8_beads", n_beads=4)
    inst = w["instances"] + inputs.workload("w3")["instances"]
    e = beadscf.Engine(0)
    try:
        e.load_basis(b631gs)
        e.set_instances([z for z, _ in inst])
        e.set_geometries([x for _, x in inst])
        Ps = [_rand_sym(n, k) for k, n in enumerate(e.nbf)]
        J0, K0 = e.build_jk(Ps)                 # FP64 atomics
        e.set_deterministic(True)
        J1, K1 = e.build_jk(Ps)
        J2, K2 = e.build_jk(Ps)
        e.set_deterministic(False)
        for k in range(len(inst)):
            assert np.array_equal(J1[k], J2[k]) and np.array_equal(K1[k], K2[k]), k
            assert np.abs(J1[k] - J0[k]).max() <= 1e-12 * np.abs(J0[k]).max(), k
            assert np.abs(K1[k] - K0[k]).max() <= 1e-12 * np.abs(K0[k]).max(), k
        b = oracle.build_basis(b631gs, *inst[-1])
        J, K, _ = oracle.jk(b, Ps[-1])
        assert np.abs(J1[-1] - J).max() <= 1e-12 * np.abs(J).max()
        assert np.abs(K1[-1] - K).max() <= 1e-12 * np.abs(K).max()
    finally:
        e.close()


def test_deterministic_scf_matches_default(beadscf, b631gs):
    z, x = inputs.water_cluster(3, 13)
    bx = inputs.beads(z, x, 4, 13)
    e = beadscf.Engine(0)
    try:
        e.load_basis(b631gs)
        e.set_instances([z] * 4)
        e.set_geometries(list(bx))
        E0, it0, st0 = e.run_scf(e_tol=1e-10, comm_tol=1e-8)
        F0 = e.forces()
        E1, it1, st1 = e.run_scf(e_tol=1e-10, comm_tol=1e-8, deterministic=1)
        F1 = e.forces()
        assert (st0 == 0).all() and (st1 == 0).all()
        assert np.abs(E1 - E0).max() < 1e-10
        for a, c in zip(F0, F1):
            assert np.abs(a - c).max() < 1e-8
        with pytest.raises(beadscf.BscfError):
            e.run_scf(deterministic=2)
    finally:
        e.close()
