"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Layered: Boys function (against mpmath) -> full ERI tensors -> one-electron
matrices and Schwarz bounds -> J/K at fixed densities (screened and
unscreened, batched instances of different sizes) -> converged SCF energies.
Tolerances follow from FP64 rounding of the quantities compared.
"""

import mpmath
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def beadscf():
    from paper_1601_02713_amd import beadscf as b
    return b


@pytest.fixture(scope="module")
def eng(beadscf):
    e = beadscf.Engine(0)
    yield e
    e.close()


def _setup(eng, basis_name, instances):
    eng.load_basis(inputs.load_basis(basis_name))
    eng.set_instances([z for z, _ in instances])
    eng.set_geometries([x for _, x in instances])


def _rand_density(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return 0.05 * (A + A.T)


def test_device_boys_against_mpmath(eng):
    mpmath.mp.dps = 40
    T = np.concatenate([[0.0, 1e-10, 0.04999, 0.05001, 39.95, 39.9999, 40.0, 40.0001, 55.0, 300.0],
                        np.random.default_rng(1).uniform(0, 45, 200)])
    F64 = eng.boys(12, T, 0)
    F32 = eng.boys(12, T, 1)
    for i, t in enumerate(T):
        for m in range(13):
            tt = mpmath.mpf(float(t))
            ref = float(mpmath.mpf(1) / (2 * m + 1) if tt == 0 else
                        mpmath.gammainc(m + mpmath.mpf(1) / 2, 0, tt) / (2 * tt ** (m + mpmath.mpf(1) / 2)))
            assert abs(F64[i, m] - ref) <= 2e-14 * ref, (t, m, F64[i, m], ref)
            assert abs(F32[i, m] - ref) <= 2e-6 * ref, (t, m, F32[i, m], ref)
    # F_0 alone (the body the classes with total angular momentum 0 use),
    # around the grid points and the large-T branch
    T0 = np.concatenate([T, [1e-6, 0.005, 0.009999, 0.01, 0.010001, 0.02, 1.0, 12.5]])
    F0 = eng.boys(0, T0, 0)
    for i, t in enumerate(T0):
        tt = mpmath.mpf(float(t))
        ref = float(1 if tt == 0 else
                    mpmath.gammainc(mpmath.mpf(1) / 2, 0, tt) / (2 * tt ** (mpmath.mpf(1) / 2)))
        assert abs(F0[i, 0] - ref) <= 2e-14 * ref, (t, F0[i, 0], ref)


@pytest.mark.parametrize("case,basis", [("h2o_sto3g", "sto-3g"), ("h2o_sto3g", "6-31g*")])
def test_eri_tensor(eng, case, basis):
    inst = inputs.workload(case)["instances"]
    _setup(eng, basis, inst)
    b = oracle.build_basis(inputs.load_basis(basis), *inst[0])
    ref = oracle.eri_tensor(b)
    got = eng.eri_tensor(0)
    assert np.abs(got - ref).max() < 1e-13


def test_one_electron_and_schwarz(eng, b631gs):
    inst = inputs.workload("w2")["instances"]
    _setup(eng, "6-31g*", inst)
    b = oracle.build_basis(b631gs, *inst[0])
    S, T, V = oracle.one_electron(b)
    Sg, Hg = eng.one_electron(0)
    assert np.abs(Sg - S).max() < 1e-13
    assert np.abs(Hg - (T + V)).max() < 1e-12
    Q = oracle.schwarz(b)
    Qg = eng.schwarz(0)
    assert np.allclose(Qg, Q, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("tau", [0.0, 1e-12])
def test_jk_fixed_density(eng, b631gs, tau):
    inst = inputs.workload("w2")["instances"]
    _setup(eng, "6-31g*", inst)
    b = oracle.build_basis(b631gs, *inst[0])
    P = _rand_density(b["nbf"], 4)
    J, K, _ = oracle.jk(b, P, tau=tau)
    Jg, Kg = eng.build_jk([P], schwarz_tol=tau)
    assert np.abs(Jg[0] - J).max() < 1e-11
    assert np.abs(Kg[0] - K).max() < 1e-11


def test_jk_batched_uneven(eng, b631gs):
    """Instances of 1, 3 and 2 waters in one batch, each against the oracle."""
    inst = []
    for nw in (1, 3, 2):
        inst += inputs.workload(f"w{nw}")["instances"]
    _setup(eng, "6-31g*", inst)
    Ps = []
    for i, (z, x) in enumerate(inst):
        n = oracle.build_basis(b631gs, z, x)["nbf"]
        Ps.append(_rand_density(n, 10 + i))
    Jg, Kg = eng.build_jk(Ps)
    Fg, Eg = eng.build_fock(Ps)
    for i, (z, x) in enumerate(inst):
        b = oracle.build_basis(b631gs, z, x)
        J, K, _ = oracle.jk(b, Ps[i])
        assert np.abs(Jg[i] - J).max() < 1e-11
        assert np.abs(Kg[i] - K).max() < 1e-11
        S, T, V = oracle.one_electron(b)
        F, E = oracle.fock_energy(b, T + V, Ps[i])
        assert np.abs(Fg[i] - F).max() < 1e-11
        assert abs(Eg[i] - E) < 1e-10


def test_scf_h2o_sto3g(eng, sto3g):
    w = inputs.workload("h2o_sto3g")
    _setup(eng, "sto-3g", w["instances"])
    b = oracle.build_basis(sto3g, *w["instances"][0])
    r = oracle.scf(b, 1e-11, 1e-9)
    E, it, st = eng.run_scf(e_tol=1e-11, comm_tol=1e-9)
    assert st[0] == 0
    assert abs(E[0] - r["E"]) < 1e-10
    assert np.abs(eng.density(0) - r["P"]).max() < 1e-7


def test_scf_batched_beads(eng, b631gs):
    """Four (H2O)2 beads in one batch: each equals its own oracle SCF."""
    z, x = inputs.water_cluster(2, 7)
    bx = inputs.beads(z, x, 4, 7)
    inst = [(z, bx[k]) for k in range(4)]
    _setup(eng, "6-31g*", inst)
    E, it, st = eng.run_scf(e_tol=1e-10, comm_tol=1e-8)
    assert (st == 0).all()
    for k in range(4):
        b = oracle.build_basis(b631gs, *inst[k])
        r = oracle.scf(b, 1e-10, 1e-8)
        assert abs(E[k] - r["E"]) < 1e-8


@pytest.mark.parametrize("basis", ["sto-3g", "6-31g*"])
def test_forces_single_water(eng, basis):
    w = inputs.workload("h2o_sto3g")
    _setup(eng, basis, w["instances"])
    b = oracle.build_basis(inputs.load_basis(basis), *w["instances"][0])
    r = oracle.scf(b, 1e-11, 1e-9)
    g = oracle.gradient(b, r["P"], r["F"])
    E, it, st = eng.run_scf(e_tol=1e-11, comm_tol=1e-9)
    F = eng.forces()[0]
    assert abs(E[0] - r["E"]) < 1e-9
    assert np.abs(F + g).max() < 1e-8
    assert np.abs(F.sum(axis=0)).max() < 1e-9


def test_forces_batched_beads(eng, b631gs):
    z, x = inputs.water_cluster(2, 9)
    bx = inputs.beads(z, x, 2, 9)
    inst = [(z, bx[k]) for k in range(2)]
    _setup(eng, "6-31g*", inst)
    E, it, st = eng.run_scf(e_tol=1e-11, comm_tol=1e-9)
    F = eng.forces()
    for k in range(2):
        b = oracle.build_basis(b631gs, *inst[k])
        r = oracle.scf(b, 1e-11, 1e-9)
        g = oracle.gradient(b, r["P"], r["F"])
        assert abs(E[k] - r["E"]) < 1e-9
        assert np.abs(F[k] + g).max() < 1e-8


def test_scf_staggered_convergence(eng, b631gs):
    """Instances that converge at different iterations keep the energy and
    Fock matrix of their own last build while the others iterate on."""
    inst = inputs.workload("w1")["instances"] + inputs.workload("w3")["instances"]
    z, x = inputs.water_cluster(2, 9)
    inst += [(z, b) for b in inputs.beads(z, x, 2, 9)]
    _setup(eng, "6-31g*", inst)
    E, it, st = eng.run_scf(e_tol=1e-11, comm_tol=1e-9)
    assert len(set(it.tolist())) > 1, it
    for k, (zz, xx) in enumerate(inst):
        b = oracle.build_basis(b631gs, zz, xx)
        r = oracle.scf(b, 1e-11, 1e-9)
        assert st[k] == 0
        assert abs(E[k] - r["E"]) < 1e-9, (k, it, E[k], r["E"])


@pytest.mark.parametrize("variant", ["lane", "coop"])
def test_jk_and_forces_each_kernel_variant(beadscf, b631gs, variant, monkeypatch):
    """Both kernel forms of every class (one quartet per lane, one per
    wavefront) against the oracle: J/K at a fixed density for a 3-water
    cluster, and forces of a 2-water cluster."""
    monkeypatch.setenv("BSCF_VARIANT", variant)
    e = beadscf.Engine(0)
    try:
        inst = inputs.workload("w3")["instances"]
        _setup(e, "6-31g*", inst)
        b = oracle.build_basis(b631gs, *inst[0])
        P = _rand_density(b["nbf"], 21)
        J, K, _ = oracle.jk(b, P)
        Jg, Kg = e.build_jk([P])
        assert np.abs(Jg[0] - J).max() < 1e-11
        assert np.abs(Kg[0] - K).max() < 1e-11
        st = e.stats()["classes"]
        for tag, v in st.items():
            if v["items"]:
                lane_exists = sum(map(int, tag)) <= 5
                assert v["variant"][0] == (1 if variant == "coop" or not lane_exists else 0), tag
        z, x = inputs.water_cluster(2, 13)
        _setup(e, "6-31g*", [(z, x)])
        E, it, status = e.run_scf(e_tol=1e-11, comm_tol=1e-9)
        F = e.forces()[0]
        bb = oracle.build_basis(b631gs, z, x)
        r = oracle.scf(bb, 1e-11, 1e-9)
        g = oracle.gradient(bb, r["P"], r["F"])
        assert abs(E[0] - r["E"]) < 1e-9
        assert np.abs(F + g).max() < 1e-8
    finally:
        e.close()


def test_density_methods_agree(eng, b631gs):
    """SP2 purification and the eigenvector route give the same SCF: four
    (H2O)2 beads, energies, densities and forces of the two runs agree to
    rounding, and each energy matches the oracle (whose density comes from
    eigenvectors)."""
    z, x = inputs.water_cluster(2, 11)
    bx = inputs.beads(z, x, 4, 11)
    inst = [(z, bx[k]) for k in range(4)]
    _setup(eng, "6-31g*", inst)
    from paper_1601_02713_amd import beadscf as b
    out = {}
    for method in (b.DENSITY_EIG, b.DENSITY_SP2):
        eng.reset_stats()
        E, it, st = eng.run_scf(e_tol=1e-11, comm_tol=1e-9, density=method)
        assert (st == 0).all()
        out[method] = (E, [eng.density(k) for k in range(4)], eng.forces(), eng.stats())
    Ee, Pe, Fe, se = out[b.DENSITY_EIG]
    Es, Ps, Fs, ss = out[b.DENSITY_SP2]
    assert se["sp2_calls"] == 0
    assert ss["sp2_calls"] > 0 and ss["sp2_fallbacks"] == 0
    assert np.abs(Ee - Es).max() < 1e-10
    for k in range(4):
        assert np.abs(Pe[k] - Ps[k]).max() < 1e-8
        assert np.abs(Fe[k] - Fs[k]).max() < 1e-9
        r = oracle.scf(oracle.build_basis(b631gs, *inst[k]), 1e-11, 1e-9)
        assert abs(Es[k] - r["E"]) < 1e-9


def test_density_without_gap(eng):
    """Oxygen atom, core guess: two of three degenerate 2p levels are
    occupied, so the guess density has no gap at the Fermi level.  SP2 either
    hands such a replica to the eigenvector route or settles on two orbitals of
    the degenerate set; either way the energy of the density is that of the
    eigenvector route (every choice is equivalent by symmetry)."""
    from paper_1601_02713_amd import beadscf as b
    _setup(eng, "6-31g*", [(np.array([8]), np.zeros((1, 3)))])
    E = {}
    for method in (b.DENSITY_EIG, b.DENSITY_SP2):
        eng.reset_stats()
        E[method], _, _ = eng.run_scf(max_iter=1, density=method)
        print(method, eng.stats()["sp2_fallbacks"])
    assert np.isfinite(E[b.DENSITY_SP2]).all()
    assert abs(E[b.DENSITY_SP2][0] - E[b.DENSITY_EIG][0]) < 1e-9


def test_incremental_builds_agree(eng, b631gs):
    """Incremental Fock builds (J and K from the density change, quartets
    screened by their Schwarz bound times max |dP|, a full build every 12
    iterations) converge to what full builds give: four (H2O)3 beads, energies
    within 1e-9 Eh, densities 1e-6, forces 1e-7 Eh/bohr, the first bead within
    1e-8 Eh of the oracle, and fewer quartets evaluated."""
    z, x = inputs.water_cluster(3, 13)
    bx = inputs.beads(z, x, 4, 13)
    inst = [(z, bx[k]) for k in range(4)]
    _setup(eng, "6-31g*", inst)
    out = {}
    for inc in (0, 1):
        eng.reset_stats()
        E, it, st = eng.run_scf(e_tol=1e-10, comm_tol=1e-8, incremental=inc)
        assert (st == 0).all()
        F = eng.forces()
        s = eng.stats()
        done = sum(v["done_quartets"] for v in s["classes"].values())
        out[inc] = (E, [eng.density(k) for k in range(4)], F, s["incremental_builds"], done, it)
    E0, P0, F0, n0, d0, it0 = out[0]
    E1, P1, F1, n1, d1, it1 = out[1]
    print("iterations", it0.tolist(), it1.tolist(), "quartets", d0, d1)
    assert n0 == 0 and n1 > 0
    assert d1 < d0
    assert np.abs(E0 - E1).max() < 1e-9
    for k in range(4):
        assert np.abs(P0[k] - P1[k]).max() < 1e-6
        assert np.abs(F0[k] - F1[k]).max() < 1e-7
    r = oracle.scf(oracle.build_basis(b631gs, *inst[0]), 1e-10, 1e-8)
    assert abs(E1[0] - r["E"]) < 1e-8


def test_graph_replay_matches_eager(eng):
    """The steps of each SCF iteration after the Fock build replayed from a
    captured HIP graph give what the same launches one by one give: four
    (H2O)3 beads, a core-guess SCF and then, at displaced geometries, a
    previous-step-guess SCF (so one graph is replayed across iterations and
    calls, with eager Fock builds and host synchronisations between the
    replays).  Energies within 1e-10 Eh, densities and forces within 1e-8,
    equal iteration counts, and every iteration one graph launch."""
    z, x = inputs.water_cluster(3, 17)
    bx = inputs.beads(z, x, 4, 17)
    by = inputs.beads(z, x, 4, 18)
    out = {}
    for graph in (0, 1):
        _setup(eng, "6-31g*", [(z, bx[k]) for k in range(4)])
        eng.reset_stats()
        res = []
        for geoms, guess in ((None, 0), (by, 1)):
            if geoms is not None:
                eng.set_geometries([geoms[k] for k in range(4)])
            E, it, st = eng.run_scf(e_tol=1e-10, comm_tol=1e-8, graph=graph, guess=guess)
            assert (st == 0).all()
            res.append((E, it, [eng.density(k) for k in range(4)], eng.forces()))
        s = eng.stats()
        assert s["graph_memset_nodes"] == 0   # fills are kernels, also inside the libraries
        out[graph] = (res, s["graph_launches"], s["graph_captures"], s["scf_iterations"])
    (r0, l0, c0, n0), (r1, l1, c1, n1) = out[0], out[1]
    print("graph launches", l1, "captures", c1, "iterations", n1)
    assert l0 == 0 and c0 == 0
    assert l1 == n1 and 1 <= c1 < l1
    for (E0, it0, P0, F0), (E1, it1, P1, F1) in zip(r0, r1):
        assert (it0 == it1).all()
        assert np.abs(E0 - E1).max() < 1e-10
        for k in range(4):
            assert np.abs(P0[k] - P1[k]).max() < 1e-8
            assert np.abs(F0[k] - F1[k]).max() < 1e-8


@pytest.mark.parametrize("mode", ["fp64_deterministic", "mixed"])
def test_fock_build_graph_matches_eager(eng, beadscf, mode, monkeypatch):
    """Fock builds whose J and K launches replay captured graphs (graph 2)
    against the same launches one by one (graph 1): four (H2O)3 beads, a
    core-guess SCF and then a previous-step-guess SCF at displaced
    geometries, so full and incremental builds are each captured once per
    geometry and replayed across iterations, with eager work and host
    synchronisations between the replays.  Both runs agree to rounding (the
    energy sums and SP2 traces use atomics in both, so not bitwise even
    with deterministic J and K): energies within 1e-11 Eh, densities within
    1e-9, in FP64 with deterministic J and K (kernel forms fixed) and in
    mixed precision (tuned forms)."""
    det = mode == "fp64_deterministic"
    if det:
        monkeypatch.setenv("BSCF_VARIANT", "coop")
    prec = 0 if det else 1
    z, x = inputs.water_cluster(3, 19)
    bx = inputs.beads(z, x, 4, 19)
    by = inputs.beads(z, x, 4, 20)
    out = {}
    for graph in (1, 2):
        _setup(eng, "6-31g*", [(z, bx[k]) for k in range(4)])
        eng.reset_stats()
        res = []
        for geoms, guess in ((None, 0), (by, 1)):
            if geoms is not None:
                eng.set_geometries([geoms[k] for k in range(4)])
            E, it, st = eng.run_scf(e_tol=1e-10, comm_tol=1e-8, graph=graph, guess=guess,
                                    precision=prec, deterministic=int(det))
            assert (st == 0).all()
            res.append((E, it, [eng.density(k) for k in range(4)]))
        s = eng.stats()
        assert s["graph_memset_nodes"] == 0
        out[graph] = (res, s["fock_graph_launches"], s["fock_graph_captures"], s["fock_builds"])
    (r1, l1, c1, _), (r2, l2, c2, n2) = out[1], out[2]
    print("fock graph launches", l2, "captures", c2, "builds", n2)
    assert l1 == 0 and c1 == 0
    assert l2 == n2 and 2 <= c2 < l2
    for (E1, it1, P1), (E2, it2, P2) in zip(r1, r2):
        print("max dE", np.abs(E1 - E2).max(),
              "max dP", max(np.abs(P1[k] - P2[k]).max() for k in range(4)))
        assert (it1 == it2).all()
        assert np.abs(E1 - E2).max() < 1e-11
        for k in range(4):
            assert np.abs(P1[k] - P2[k]).max() < 1e-9
    with pytest.raises(beadscf.BscfError):
        eng.run_scf(graph=3)


def test_full_size_bead_batch(eng, b631gs):
    """The benchmark's batch at full size, in its launch configuration: 16
    beads of (H2O)8 in 6-31G* (152 functions), FP64, core guess, SCF to
    1e-8 Eh with incremental builds and graph replay.  Every bead converges
    with Tr(PS) = 80 electrons and zero net force.  Two sampled beads get the
    oracle's core-guess density in one batched Fock build (the other beads
    seeded random densities): Fock matrices and energies within 1e-9 and
    1e-8 Eh of the oracle's.  Then the batch's SCF is tightened (1e-10 Eh,
    commutator 1e-8) and one bead's energy and forces are compared with the
    oracle's own SCF and gradient (1e-8 Eh, 1e-7 Eh/bohr)."""
    from oracle import rhf
    w = inputs.workload("w8_beads")
    inst = w["instances"]
    assert len(inst) == 16
    _setup(eng, w["basis"], inst)
    E, it, st = eng.run_scf(e_tol=w["e_tol"], comm_tol=w["comm_tol"], max_iter=60)
    assert (st == 0).all(), st
    F = eng.forces()
    for k in range(16):
        S, _ = eng.one_electron(k)
        assert abs(np.sum(eng.density(k) * S) - 80.0) < 1e-8
        assert np.abs(F[k].sum(axis=0)).max() < 1e-8
    Ps = [_rand_density(152, 300 + k) for k in range(16)]
    ref = {}
    for k in (0, 11):
        b = oracle.build_basis(b631gs, *inst[k])
        S, T, V = oracle.one_electron(b)
        X = rhf.orthogonaliser(S)
        Ps[k], _, _ = rhf._density(X.T @ (T + V) @ X, X, 40)
        ref[k] = oracle.fock_energy(b, T + V, Ps[k])
    Fg, Eg = eng.build_fock(Ps)
    for k, (Fo, Eo) in ref.items():
        assert np.abs(Fg[k] - Fo).max() < 1e-9
        assert abs(Eg[k] - Eo) < 1e-8
    E, it, st = eng.run_scf(e_tol=1e-10, comm_tol=1e-8, max_iter=60, guess=1)
    assert (st == 0).all(), st
    F = eng.forces()
    k = 11
    b = oracle.build_basis(b631gs, *inst[k])
    r = oracle.scf(b, 1e-10, 1e-8)
    assert r["converged"]
    g = oracle.gradient(b, r["P"], r["F"])
    assert abs(E[k] - r["E"]) < 1e-8
    assert np.abs(F[k] + g).max() < 1e-7


@pytest.mark.parametrize("threads", ["64", "128", "256"])
def test_lane_units_of_each_width(beadscf, b631gs, threads, monkeypatch):
    """Lane units of one, two and four wavefronts sharing their LDS rows give
    the oracle's J and K, in FP64 and in mixed precision (all lane forms
    forced), on a ragged batch of 3- and 2-water clusters, and the oracle's
    forces through the gradient's lane units of the same width."""
    monkeypatch.setenv("BSCF_VARIANT", "lane")
    monkeypatch.setenv("BSCF_UNIT_THREADS", threads)
    e = beadscf.Engine(0)
    try:
        inst = inputs.workload("w3")["instances"] + inputs.workload("w2")["instances"]
        _setup(e, "6-31g*", inst)
        Ps = [_rand_density(n, 40 + k) for k, n in enumerate(e.nbf)]
        Jg, Kg = e.build_jk(Ps)
        Jm, Km = e.build_jk(Ps, precision=beadscf.BSCF_MIXED)
        for k, (z, x) in enumerate(inst):
            b = oracle.build_basis(b631gs, z, x)
            J, K, _ = oracle.jk(b, Ps[k])
            assert np.abs(Jg[k] - J).max() < 1e-11 and np.abs(Kg[k] - K).max() < 1e-11, k
            assert np.abs(Jm[k] - J).max() < 1e-7 and np.abs(Km[k] - K).max() < 1e-7, k
        # the gradient's lane units of the same width
        z, x = inputs.water_cluster(2, 13)
        _setup(e, "6-31g*", [(z, x)])
        E, _, st = e.run_scf(e_tol=1e-11, comm_tol=1e-9)
        F = e.forces()[0]
        b = oracle.build_basis(b631gs, z, x)
        r = oracle.scf(b, 1e-11, 1e-9)
        g = oracle.gradient(b, r["P"], r["F"])
        assert st[0] == 0 and abs(E[0] - r["E"]) < 1e-9
        assert np.abs(F + g).max() < 1e-8
    finally:
        e.close()
