"""GPU edge cases through the C ABI: the smallest and degenerate instances
(one atom, two basis functions, ions) in one ragged batch against the FP64
oracle, and rejected calls that must leave the context as it was.

Energies and forces follow the closed-shell RHF energy and its analytic
gradient (Szabo and Ostlund, ch. 3; Pople et al. for the gradient), the same
definitions the oracle writes out.  Properties that hold at any size are
checked too: a lone atom feels no force, and the forces of every instance sum
to zero (translational invariance).
"""

import copy

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

# Closed-shell instances (Z, xyz in bohr, total charge) of very different
# sizes: 2, 4, 6, 17, 15 and 19 Cartesian 6-31G* functions.
_SMALL = [
    ([1], [[0.3, -0.2, 0.1]], -1),                                        # H-
    ([1, 1], [[0.0, 0.0, 0.0], [0.1, -0.05, 1.4]], 0),                    # H2
    ([1, 1, 1], [[0.0, 0.0, 0.0], [1.65, 0.0, 0.0], [0.80, 1.45, 0.05]], 1),  # H3+
    ([8, 1], [[0.0, 0.0, 0.0], [0.05, 0.0, 1.83]], -1),                   # OH-
    ([8], [[1.0, 2.0, -0.5]], -2),                                        # O2-
    ([8, 1, 1], [[0.0, 0.0, 0.0], [1.43, 0.0, 1.11], [-1.50, 0.10, 1.05]], 0),  # H2O
]


@pytest.fixture(scope="module")
def beadscf():
    from paper_1601_02713_amd import beadscf as b
    return b


@pytest.fixture(scope="module")
def eng(beadscf):
    e = beadscf.Engine(0)
    yield e
    e.close()


def _setup(eng, basis, inst, charges=None):
    eng.load_basis(basis)
    eng.set_instances([np.asarray(z) for z, _ in inst], charges)
    eng.set_geometries([np.asarray(x, float) for _, x in inst])


def test_small_ions_and_lone_atoms_in_one_batch(eng, b631gs):
    inst = [(z, x) for z, x, _ in _SMALL]
    charges = [q for _, _, q in _SMALL]
    _setup(eng, b631gs, inst, charges)
    assert eng.nbf == [2, 4, 6, 17, 15, 19]
    E, it, st = eng.run_scf(e_tol=1e-11, comm_tol=1e-9)
    assert (st == 0).all(), st
    F = eng.forces()
    for k, (z, x, q) in enumerate(_SMALL):
        b = oracle.build_basis(b631gs, np.asarray(z), np.asarray(x, float))
        r = oracle.scf(b, 1e-11, 1e-9, charge=q)
        assert r["converged"]
        g = oracle.gradient(b, r["P"], r["F"])
        assert abs(E[k] - r["E"]) < 1e-9, (k, E[k], r["E"])
        assert np.abs(eng.density(k) - r["P"]).max() < 1e-6, k
        assert np.abs(F[k] + g).max() < 1e-8, (k, F[k], -g)
        assert np.abs(F[k].sum(axis=0)).max() < 1e-9, k
        if len(z) == 1:
            assert np.abs(F[k]).max() < 1e-10, (k, F[k])


def test_rejected_calls_leave_the_context_usable(eng, beadscf, b631gs):
    inst = [(z, x) for z, x, _ in _SMALL[-1:]]
    _setup(eng, b631gs, inst)
    E0, _, st = eng.run_scf(e_tol=1e-11, comm_tol=1e-9)
    assert st[0] == 0
    F0 = eng.forces()[0]

    def rejected(code, fn, *args, **kw):
        with pytest.raises(beadscf.BscfError) as ei:
            fn(*args, **kw)
        assert ei.value.code == code, str(ei.value)

    # instance sets the library must refuse before it changes anything:
    # an element outside the basis, an odd electron count, no electrons, an
    # instance without atoms (the last after a valid first instance)
    rejected(-2, eng.set_instances, [np.array([6, 1, 1, 1, 1])])
    rejected(-2, eng.set_instances, [np.array([8, 1])])
    rejected(-2, eng.set_instances, [np.array([1])], [1])
    rejected(-1, eng.set_instances, [np.array([8, 1, 1]), np.array([], np.int32)])
    # a non-finite coordinate and out-of-range SCF options
    bad = np.asarray(inst[0][1], float).copy()
    bad[1, 2] = np.nan
    rejected(-1, eng.set_geometries, [bad])
    rejected(-1, eng.run_scf, diis_size=9)
    rejected(-1, eng.run_scf, max_iter=0)
    # a basis with an f shell is refused and the loaded basis stays
    fb = copy.deepcopy(b631gs)
    fb["elements"]["O"]["shells"].append({"l": 3, "exponents": [0.8], "coefficients": [1.0]})
    rejected(-2, eng.load_basis, fb)

    # the instance set, geometry and converged state are those of before
    assert eng.nbf == [19]
    F1 = eng.forces()[0]
    assert np.abs(F1 - F0).max() < 1e-12
    E1, _, st = eng.run_scf(e_tol=1e-11, comm_tol=1e-9)
    assert st[0] == 0 and abs(E1[0] - E0[0]) < 1e-10

    # a Fock build at a caller's density replaces the SCF's: no forces until
    # the next SCF, which gives them back
    P = eng.density(0)
    eng.build_fock([0.5 * P])
    rejected(-4, eng.forces)
    eng.run_scf(e_tol=1e-11, comm_tol=1e-9)
    assert np.abs(eng.forces()[0] - F0).max() < 1e-9

    # a new instance set discards the geometry and the converged state, and
    # its density is zero until one is computed or given
    eng.set_instances([np.array([8, 1, 1])])
    assert not eng.density(0).any()
    rejected(-4, eng.forces)
    rejected(-1, eng.run_scf)
    eng.set_geometries([np.asarray(inst[0][1], float)])
    E2, _, st = eng.run_scf(e_tol=1e-11, comm_tol=1e-9)
    assert st[0] == 0 and abs(E2[0] - E0[0]) < 1e-10


@pytest.mark.parametrize("z,x,q", [
    ([1, 1], [[0.0, 0.0, 0.0], [0.1, -0.05, 1.4]], 0),    # H2: 4 matrix elements, 6 force components
    ([1], [[0.3, -0.2, 0.1]], -1),                         # H-: 1 matrix element, 3 force components
])
def test_batches_with_fewer_matrix_elements_than_force_components(eng, sto3g, z, x, q):
    # In STO-3G these batches hold fewer density-matrix elements than force
    # components; the first forces call of a batch also times every gradient
    # kernel alone, into a buffer of the batch's force components.
    _setup(eng, sto3g, [(z, x)], [q])
    E, _, st = eng.run_scf(e_tol=1e-11, comm_tol=1e-9)
    assert st[0] == 0
    F = eng.forces()[0]
    b = oracle.build_basis(sto3g, np.asarray(z), np.asarray(x, float))
    r = oracle.scf(b, 1e-11, 1e-9, charge=q)
    g = oracle.gradient(b, r["P"], r["F"])
    assert abs(E[0] - r["E"]) < 1e-9
    assert np.abs(F + g).max() < 1e-8, (F, -g)
    assert np.abs(F.sum(axis=0)).max() < 1e-10


def test_lane_kernels_over_the_scratch_bound_never_run(beadscf, eng, b631gs, monkeypatch):
    """Every class whose lane kernel needs more private memory per lane than
    the context's bound (4096 bytes, or less through BSCF_LANE_SCRATCH_MAX)
    runs cooperatively, for the Fock build in both precisions and for the
    gradient.  No lane kernel of the library is over 4096 bytes, so a bound
    of 1024 bytes routes some classes (among them the (pp|pp) and (dp|ds)
    gradients) to the cooperative form; the forces stay those of the
    default routing."""
    inst = inputs.workload("w3")["instances"]

    def run(e):
        _setup(e, b631gs, inst)
        e.run_scf(e_tol=1e-9, comm_tol=1e-7)
        F = e.forces()
        e.run_scf(e_tol=1e-9, comm_tol=1e-7, precision=1)
        return F, e.stats()["classes"]

    F0, st0 = run(eng)
    monkeypatch.setenv("BSCF_LANE_SCRATCH_MAX", "1024")
    e1 = beadscf.Engine(0)
    try:
        F1, st1 = run(e1)
    finally:
        e1.close()
    for bound, st in ((4096, st0), (1024, st1)):
        over = 0
        for tag, v in st.items():
            if not v["items"]:
                continue
            for k in range(3):
                if v["private_bytes"][k] > bound:
                    over += 1
                    assert v["variant"][k] == 1, (bound, tag, k, v["private_bytes"], v["variant"])
        if bound == 1024:
            assert over >= 1
    for a, b in zip(F0, F1):
        assert np.abs(a - b).max() < 1e-10
