"""GPU parity at the full problem sizes, in the launch configurations the
benchmark uses.

At these sizes the library takes paths the small parity cases never reach:
lane-kernel LDS rows sized by the batch's largest basis (a 608-function
instance pushes the d-shell bra units past 64 KB, to one or two workgroups
per CU, and changes which classes run cooperatively), many instances per
launch, and ragged batches.  The oracle cannot build a 608-function Fock
matrix or gradient in test time, so it checks what it can compute one by
one at every size:

  * J and K blocks of sampled shell pairs (direct sums over every ket pair,
    the definition J_mn = sum (mn|ls) P_ls, K_mn = sum (ml|ns) P_ls);
  * the gradient rows of sampled atoms;
  * whole Fock matrices, energies and gradients of the smaller instances.

Every oracle input is seeded here (random symmetric densities) or computed
by the oracle itself (its core-guess density and its own SCF); nothing the
GPU computes is handed to the oracle.  Properties that hold at any size
(Tr(PS) = N, zero net force) cover the rest of the largest instances.
"""

import numpy as np
import pytest

import inputs
import oracle
from oracle import rhf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def beadscf():
    from paper_1601_02713_amd import beadscf as b
    return b


def _rand_sym(n, seed, scale=0.05):
    rng = np.random.default_rng([4242, seed])
    A = rng.standard_normal((n, n))
    return scale * (A + A.T)


def _core_density(b, nocc):
    """The oracle's core-Hamiltonian guess density (and S, H)."""
    S, T, V = oracle.one_electron(b)
    X = rhf.orthogonaliser(S)
    P, _, _ = rhf._density(X.T @ (T + V) @ X, X, nocc)
    return P, S, T + V


def _sampled_pairs(b, rng, n_random=6):
    """Shell pairs that cover the d-shell classes: each d shell with itself,
    d with a d and a p shell of the next water, plus random pairs."""
    l = b["l"]
    d = [s for s in range(b["nsh"]) if l[s] == 2]
    p = [s for s in range(b["nsh"]) if l[s] == 1]
    pairs = [(d[0], d[0]), (d[1], d[0]), (d[-1], p[-2]), (0, 0), (b["nsh"] - 1, 0)]
    for _ in range(n_random):
        a, c = rng.integers(0, b["nsh"], size=2)
        pairs.append((int(a), int(c)))
    return pairs


def _block_mask(b, pairs):
    m = np.zeros((b["nbf"],) * 2, bool)
    for a, c in pairs:
        na = (b["l"][a] + 1) * (b["l"][a] + 2) // 2
        nc = (b["l"][c] + 1) * (b["l"][c] + 2) // 2
        m[b["bf"][a]:b["bf"][a] + na, b["bf"][c]:b["bf"][c] + nc] = True
    return m


def _big_ragged_batch():
    """One (H2O)32 bead (608 functions) beside (H2O)2 and (H2O)3."""
    big = inputs.workload("w32_beads", n_beads=1)["instances"][0]
    return [big] + inputs.workload("w2")["instances"] + inputs.workload("w3")["instances"]


@pytest.mark.parametrize("variant", ["auto", "lane", "coop"])
def test_608_function_instance_in_a_ragged_batch(beadscf, b631gs, variant, monkeypatch):
    """J/K and forces at seeded densities for a batch whose largest instance
    has 608 functions, with each kernel form the autotuner may choose.  The
    small instances match the oracle element by element; the 608-function one
    on sampled J/K blocks and on the gradient of one hydrogen atom."""
    if variant != "auto":
        monkeypatch.setenv("BSCF_VARIANT", variant)
    inst = _big_ragged_batch()
    e = beadscf.Engine(0)
    try:
        e.load_basis(b631gs)
        e.set_instances([z for z, _ in inst])
        e.set_geometries([x for _, x in inst])
        assert e.nbf == [608, 38, 57]
        Ps = [_rand_sym(n, 10 + k) for k, n in enumerate(e.nbf)]
        Fs = [_rand_sym(n, 20 + k) for k, n in enumerate(e.nbf)]
        Jg, Kg = e.build_jk(Ps, schwarz_tol=1e-12)
        G = e.forces_at(Ps, Fs, schwarz_tol=1e-12)
        for k, (z, x) in enumerate(inst):
            b = oracle.build_basis(b631gs, z, x)
            Q = oracle.schwarz(b)
            if k == 0:
                pairs = _sampled_pairs(b, np.random.default_rng(7))
                J, K = oracle.jk_pairs(b, Ps[k], pairs, 1e-12, Q)
                m = _block_mask(b, pairs)
                sJ, sK = np.abs(J[m]).max(), np.abs(K[m]).max()
                assert np.abs(Jg[k][m] - J[m]).max() <= 1e-12 * sJ, np.abs(Jg[k][m] - J[m]).max()
                assert np.abs(Kg[k][m] - K[m]).max() <= 1e-12 * sK, np.abs(Kg[k][m] - K[m]).max()
                atoms = [1]
            else:
                J, K, _ = oracle.jk(b, Ps[k], 1e-12, Q)
                assert np.abs(Jg[k] - J).max() <= 1e-12 * np.abs(J).max()
                assert np.abs(Kg[k] - K).max() <= 1e-12 * np.abs(K).max()
                atoms = list(range(len(z)))
            g = oracle.gradient(b, Ps[k], Fs[k], 1e-12, Q, atoms=atoms)
            err = np.abs(G[k][atoms] + g[atoms]).max()
            # the device also skips quartets whose density-weighted bound is
            # below the cutoff (the oracle applies the Schwarz test alone); at
            # these random densities that moves the 608-function gradient by
            # about 6e-11 Eh/bohr
            assert err <= 1e-11 * np.abs(g[atoms]).max() + 2e-10, (k, err)
        if variant == "auto":
            _scf_part(e, inst, b631gs)
    finally:
        e.close()


def _scf_part(e, inst, b631gs):
    """The same batch through the SCF in the benchmark's options: every
    instance converges; the small ones reach the oracle's converged energy and
    forces, the 608-function one holds Tr(PS) = N and zero net force."""
    E, it, st = e.run_scf(e_tol=1e-10, comm_tol=1e-8, max_iter=80)
    assert (st == 0).all(), (st, it)
    F = e.forces()
    for k, (z, x) in enumerate(inst):
        S, _ = e.one_electron(k)
        P = e.density(k)
        assert abs(np.sum(P * S) - z.sum()) < 1e-8
        assert np.abs(F[k].sum(axis=0)).max() < 1e-8
        if k == 0:
            continue
        b = oracle.build_basis(b631gs, z, x)
        r = oracle.scf(b, 1e-10, 1e-8)
        assert r["converged"]
        g = oracle.gradient(b, r["P"], r["F"])
        assert abs(E[k] - r["E"]) < 1e-8, (k, E[k], r["E"])
        assert np.abs(F[k] + g).max() < 1e-7, k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_w16_beads_fock_and_forces_at_oracle_densities(beadscf, b631gs, precision):
    """All 32 beads of (H2O)16 (304 functions) in one batch.  Two sampled
    beads get the oracle's core-guess density; the others seeded random
    ones.  The Fock matrix and energy of the sampled beads match the oracle's
    (FP64: 1e-9 / 1e-8 Eh; mixed precision with its default FP32 split:
    1e-6 Eh), and their forces at the oracle's density and Fock matrix match
    the oracle's gradient rows of a sampled O and H atom (3e-9 Eh/bohr, the
    size of the density-weighted quartet skipping)."""
    w = inputs.workload("w16_beads")
    inst = w["instances"]
    assert len(inst) == 32
    prec = beadscf.BSCF_FP64 if precision == "fp64" else beadscf.BSCF_MIXED
    e = beadscf.Engine(0)
    try:
        e.load_basis(b631gs)
        e.set_instances([z for z, _ in inst])
        e.set_geometries([x for _, x in inst])
        assert e.nbf == [304] * 32
        sampled = (3, 26)
        ref = {}
        Ps = [_rand_sym(304, 40 + k, 0.01) for k in range(32)]
        Fs = [_rand_sym(304, 80 + k, 0.01) for k in range(32)]
        for k in sampled:
            z, x = inst[k]
            b = oracle.build_basis(b631gs, z, x)
            Q = oracle.schwarz(b)
            P, S, H = _core_density(b, int(z.sum()) // 2)
            Fo, Eo = oracle.fock_energy(b, H, P, 1e-12, Q)
            Ps[k], Fs[k] = P, Fo
            ref[k] = (b, Q, Fo, Eo)
        Fg, Eg = e.build_fock(Ps, schwarz_tol=1e-12, precision=prec)
        G = e.forces_at(Ps, Fs, schwarz_tol=1e-12)
        for k in sampled:
            b, Q, Fo, Eo = ref[k]
            dF, dE = np.abs(Fg[k] - Fo).max(), abs(Eg[k] - Eo)
            print(f"bead {k} {precision}: max|dF| {dF:.2e}, |dE| {dE:.2e} Eh")
            if precision == "fp64":
                assert dF < 1e-9 and dE < 1e-8, (k, dF, dE)
            else:
                assert dF < 1e-6 and dE < 1e-6, (k, dF, dE)
            atoms = [0, 4] if k == sampled[0] else [3, 47]
            g = oracle.gradient(b, Ps[k], Fs[k], 1e-12, Q, atoms=atoms)
            # the device's density-weighted skipping of quartets below the
            # cutoff (the oracle applies the Schwarz test alone) moves these
            # rows by about 1e-9 Eh/bohr
            assert np.abs(G[k][atoms] + g[atoms]).max() < 3e-9, k
    finally:
        e.close()


@pytest.mark.timeout(600)
def test_w16_beads_converged_fp64_and_mixed_against_oracle_scf(beadscf, b631gs):
    """The 32-bead (H2O)16 batch through the SCF in FP64 and in mixed
    precision (the benchmark's options: incremental builds, graph replay,
    SP2).  Every bead converges in both; per bead the mixed energy and forces
    are within 1e-6 Eh and 1e-5 Eh/bohr of FP64.  One sampled bead's
    converged FP64 and mixed energies are compared with the oracle's own SCF,
    and its forces on a sampled H atom with the oracle gradient."""
    w = inputs.workload("w16_beads")
    inst = w["instances"]
    e = beadscf.Engine(0)
    try:
        e.load_basis(b631gs)
        e.set_instances([z for z, _ in inst])
        e.set_geometries([x for _, x in inst])
        out = {}
        for prec in (beadscf.BSCF_FP64, beadscf.BSCF_MIXED):
            E, it, st = e.run_scf(e_tol=1e-10, comm_tol=1e-8, max_iter=80, precision=prec)
            assert (st == 0).all(), (prec, st)
            out[prec] = (E, e.forces())
        E64, F64 = out[beadscf.BSCF_FP64]
        Emx, Fmx = out[beadscf.BSCF_MIXED]
        dE = np.abs(Emx - E64)
        dF = np.array([np.abs(a - c).max() for a, c in zip(Fmx, F64)])
        print("mixed vs FP64 per bead: max |dE| %.2e Eh, max |dF| %.2e Eh/bohr" % (dE.max(), dF.max()))
        assert dE.max() < 1e-6 and dF.max() < 1e-5
        k = 9
        z, x = inst[k]
        b = oracle.build_basis(b631gs, z, x)
        r = oracle.scf(b, 1e-10, 1e-8)
        assert r["converged"]
        g = oracle.gradient(b, r["P"], r["F"], atoms=[2])
        print(f"bead {k}: FP64 |dE| {abs(E64[k] - r['E']):.2e}, mixed |dE| {abs(Emx[k] - r['E']):.2e} Eh; "
              f"FP64 |dF| {np.abs(F64[k][2] + g[2]).max():.2e}, "
              f"mixed |dF| {np.abs(Fmx[k][2] + g[2]).max():.2e} Eh/bohr")
        assert abs(E64[k] - r["E"]) < 1e-8
        assert abs(Emx[k] - r["E"]) < 1e-6
        assert np.abs(F64[k][2] + g[2]).max() < 1e-6
        assert np.abs(Fmx[k][2] + g[2]).max() < 1e-5
    finally:
        e.close()


@pytest.mark.timeout(600)
def test_uneven_batch_sampled_instances(beadscf, b631gs):
    """The full uneven batch (48 clusters of 2-24 waters, 4 beads each, 192
    instances of 38-456 functions) in one context.  J/K at seeded densities:
    the smallest instance and a mid-sized one element by element, the largest
    on sampled blocks.  Then the SCF of all 192 instances: every instance
    converges with Tr(PS) = N and zero net force, and the smallest and the
    mid-sized instance reach the oracle's converged energy and forces."""
    w = inputs.workload("uneven")
    inst = w["instances"]
    assert len(inst) == 192
    nw = [len(z) // 3 for z, _ in inst]
    small = int(np.argmin(nw))
    big = int(np.argmax(nw))
    mid = int(np.argmin([abs(v - 8) for v in nw]))
    e = beadscf.Engine(0)
    try:
        e.load_basis(b631gs)
        e.set_instances([z for z, _ in inst])
        e.set_geometries([x for _, x in inst])
        assert e.nbf[small] == 38 and e.nbf[big] == 456
        Ps = [_rand_sym(n, 200 + k, 0.02) for k, n in enumerate(e.nbf)]
        Jg, Kg = e.build_jk(Ps, schwarz_tol=1e-12)
        for k in (small, mid, big):
            z, x = inst[k]
            b = oracle.build_basis(b631gs, z, x)
            Q = oracle.schwarz(b)
            if k == big:
                pairs = _sampled_pairs(b, np.random.default_rng(9))
                J, K = oracle.jk_pairs(b, Ps[k], pairs, 1e-12, Q)
                m = _block_mask(b, pairs)
                assert np.abs(Jg[k][m] - J[m]).max() <= 1e-12 * np.abs(J[m]).max()
                assert np.abs(Kg[k][m] - K[m]).max() <= 1e-12 * np.abs(K[m]).max()
            else:
                J, K, _ = oracle.jk(b, Ps[k], 1e-12, Q)
                assert np.abs(Jg[k] - J).max() <= 1e-12 * np.abs(J).max(), k
                assert np.abs(Kg[k] - K).max() <= 1e-12 * np.abs(K).max(), k
        E, it, st = e.run_scf(e_tol=w["e_tol"], comm_tol=w["comm_tol"], max_iter=80)
        assert (st == 0).all(), st
        F = e.forces()
        for k, (z, x) in enumerate(inst):
            S, _ = e.one_electron(k)
            assert abs(np.sum(e.density(k) * S) - z.sum()) < 1e-7, k
            assert np.abs(F[k].sum(axis=0)).max() < 1e-7, k
        for k in (small, mid):
            z, x = inst[k]
            b = oracle.build_basis(b631gs, z, x)
            r = oracle.scf(b, 1e-10, 1e-8)
            g = oracle.gradient(b, r["P"], r["F"])
            print(f"instance {k} ({nw[k]} waters): |dE| {abs(E[k] - r['E']):.2e} Eh, "
                  f"max |dF| {np.abs(F[k] + g).max():.2e} Eh/bohr, {it[k]} iterations")
            assert abs(E[k] - r["E"]) < 1e-8, k
            assert np.abs(F[k] + g).max() < 1e-5, k
    finally:
        e.close()
