"""Second-order orbital extrapolation (BSCF_GUESS_EXTRAPOLATED) along a
smooth sequence of geometries, as in MD: the SCF converges to the energies of
a core-guess SCF at the same geometries (the guess changes the start, not the
answer), and it starts closer than the previous-step guess (no more
iterations summed over the beads)."""

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


def _path(nb=4, steps=5):
    z, x = inputs.water_cluster(2, 7)
    bx = inputs.beads(z, x, nb, 7)
    v = np.random.default_rng(9).standard_normal(bx.shape) * 0.004   # bohr per step
    return z, [bx + k * v + 0.5 * k * k * 0.02 * v for k in range(steps)]


def _run(beadscf, basis, z, geoms, guess):
    e = beadscf.Engine(0)
    try:
        e.load_basis(basis)
        e.set_instances([z] * len(geoms[0]))
        Es, its = [], []
        for k, g in enumerate(geoms):
            e.set_geometries(list(g))
            gk = beadscf.GUESS_CORE if k == 0 else guess
            E, it, st = e.run_scf(beadscf.default_opts(e_tol=1e-10, comm_tol=1e-8, guess=gk))
            assert np.all(st == 0), (k, st)
            Es.append(E)
            its.append(it)
        return np.array(Es), np.array(its)
    finally:
        e.close()


def test_extrapolated_guess_converges_to_the_same_energies(b631gs):
    from paper_1601_02713_amd import beadscf
    z, geoms = _path()
    Ex, itx = _run(beadscf, b631gs, z, geoms, beadscf.GUESS_EXTRAPOLATED)
    Ep, itp = _run(beadscf, b631gs, z, geoms, beadscf.GUESS_PREVIOUS)
    for k, g in enumerate(geoms):
        Ec, _ = _run(beadscf, b631gs, z, [g], beadscf.GUESS_CORE)
        assert np.abs(Ex[k] - Ec[0]).max() < 1e-8, k
        assert np.abs(Ep[k] - Ec[0]).max() < 1e-8, k
    # steps 2.. extrapolate (step 1 has one stored SCF: the previous-step guess)
    assert itx[1].sum() == itp[1].sum()
    assert itx[2:].sum() <= itp[2:].sum(), (itx, itp)
