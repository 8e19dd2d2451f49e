"""The device string method (bscf_string_*) against the NumPy oracle of
oracle/string_method.py (the simplified string method in code of its own).

* With caller forces that depend on the positions, 40 device iterations and
  40 oracle iterations from the same path agree to rounding.
* With this library's SCF forces (proton transfer in H5O2+, STO-3G, 7
  images), three iterations agree with the oracle string driven by the
  oracle's own SCF and gradient per image.
* Proton transfer in H5O2+ in 6-31G* (ends held) is symmetric under the
  mirror that exchanges reactant and product, so the energy profile of the
  evolving string stays symmetric while the interior relaxes; the images stay
  equally spaced in arc length.  Images need different SCF iteration counts,
  which the batch absorbs.  The same at B3LYP (its forces and grid).
* Refusals: one image, images of different systems, an update before init.
"""

import numpy as np
import pytest

import inputs
import oracle
from oracle import string_method as osm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def beadscf():
    from paper_1601_02713_amd import beadscf as b
    return b


def _engine(beadscf, basis, z, x):
    """Images of H5O2+ (charge +1) as the batch."""
    e = beadscf.Engine(0)
    e.load_basis(basis)
    e.set_instances([z] * len(x), [1] * len(x))
    e.set_geometries(list(x))
    return e


def test_caller_force_iterations_match_oracle(beadscf, sto3g):
    z, x0 = inputs.zundel_path(9)
    ref = x0[4].copy()
    # a weak pull towards the middle image plus a position-dependent term,
    # so the path bends but keeps its length
    force = lambda x: -0.02 * (x - ref[None]) + 0.05 * np.sin(3.0 * x)
    e = _engine(beadscf, sto3g, z, x0)
    try:
        e.string_init(step=0.7)
        x = x0.copy()
        for _ in range(40):
            xg, _ = e.string_state()
            e.string_evolve(force(xg))
            x = osm.step(x, force(x), 0.7)
        xg, s = e.string_state()
        assert np.abs(xg - x).max() < 1e-11
        assert np.abs(s - osm.arc_positions(x)).max() < 1e-12
        assert np.abs(xg[0] - x0[0]).max() > 1e-3        # free ends moved
        e.string_init(step=0.7, fix_ends=1)
        xs, _ = e.string_state()
        e.string_evolve(force(xs))
        xg, _ = e.string_state()
        assert np.array_equal(xg[0], xs[0]) and np.array_equal(xg[-1], xs[-1])
        assert np.abs(xg - osm.step(xs, force(xs), 0.7, fix_ends=True)).max() < 1e-12
    finally:
        e.close()


def test_scf_driven_iterations_match_oracle(beadscf, sto3g):
    n, h = 7, 0.5
    z, x0 = inputs.zundel_path(n)
    e = _engine(beadscf, sto3g, z, x0)
    try:
        e.string_init(step=h)
        so = beadscf.default_opts(e_tol=1e-12, comm_tol=1e-10, guess=beadscf.GUESS_PREVIOUS)
        out = [e.string_step(so) for _ in range(3)]
        xg, _ = e.string_state()
    finally:
        e.close()
    x = x0.copy()
    for k in range(3):
        F, En = [], []
        for i in range(n):
            b = oracle.build_basis(sto3g, z, x[i])
            r = oracle.scf(b, 1e-12, 1e-10, charge=1)
            assert r["converged"]
            F.append(-oracle.gradient(b, r["P"], r["F"]))
            En.append(r["E"])
        Eg, _, st, Fg = out[k]
        assert (st == 0).all()
        assert np.abs(Eg - np.array(En)).max() < 1e-9, k
        assert np.abs(Fg - np.array(F)).max() < 1e-7, k
        x = osm.step(x, np.array(F), h)
    assert np.abs(xg - x).max() < 1e-8


@pytest.mark.parametrize("xc", ["hf", "b3lyp"])
def test_symmetric_proton_transfer_path(beadscf, b631gs, xc):
    n = 9
    z, x0 = inputs.zundel_path(n)
    e = _engine(beadscf, b631gs, z, x0)
    try:
        if xc == "b3lyp":   # the grid is symmetric under the mirror x -> R - x too
            e.set_xc(beadscf.XC_B3LYP)
        e.string_init(step=0.5, fix_ends=1)
        so = beadscf.default_opts(e_tol=1e-10, comm_tol=1e-8, guess=beadscf.GUESS_PREVIOUS)
        E0 = None
        iters = []
        for k in range(12):
            E, it, st, F = e.string_step(so)
            assert (st == 0).all()
            iters.append(it.copy())
            if E0 is None:
                E0 = E
        x, s = e.string_state()
    finally:
        e.close()
    print("energies (Eh):", np.round(E, 6).tolist(), "iterations:", iters[-1].tolist())
    assert np.abs(E - E[::-1]).max() < 1e-7          # mirror symmetry of the profile
    assert np.abs(E0 - E0[::-1]).max() < 1e-9
    assert E[1:-1].sum() < E0[1:-1].sum() - 1e-3      # the interior relaxed
    assert abs(E[0] - E0[0]) < 1e-9                   # ends held
    assert np.abs(s - np.linspace(0, 1, n)).max() < 0.05
    assert len({int(v) for v in np.concatenate(iters)}) > 1   # uneven SCF counts in one batch


def test_refusals(beadscf, sto3g):
    z, x = inputs.zundel_path(3)
    e = _engine(beadscf, sto3g, z, x[:1])
    try:
        with pytest.raises(beadscf.BscfError) as ei:
            e.string_init()
        assert ei.value.code == -1
        zw, xw = inputs.workload("h2o_sto3g")["instances"][0]
        e.set_instances([z, zw], [1, 0])
        e.set_geometries([x[0], xw])
        with pytest.raises(beadscf.BscfError) as ei:
            e.string_init()
        assert ei.value.code == -1
        with pytest.raises(beadscf.BscfError) as ei:
            e.string_state()
        assert ei.value.code == -4
        with pytest.raises(beadscf.BscfError) as ei:
            e.string_init(step=-1.0)
        assert ei.value.code == -1
    finally:
        e.close()
