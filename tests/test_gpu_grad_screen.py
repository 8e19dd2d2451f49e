"""Density-weighted screening of the two-electron gradient.

A gradient quartet is skipped when Q_ab Q_cd (Pm_ab Pm_cd + (Pm_ac Pm_bd +
Pm_ad Pm_bc) / 4) falls below the integral cutoff, Pm being the largest |P|
of each shell-pair block: the cutoff applied to the density-weighted
contribution, as for the incremental Fock builds.  Against the gradient with
no screening at all (cutoff 0: every shell quartet, Schwarz included) the
forces of converged (H2O)8 beads move by less than 1e-9 Eh/bohr, in both
kernel forms.  (The oracle's estimate for (H2O)4, summing the skipped
quartets' contributions: 3.9e-10 Eh/bohr.)
"""

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", ["auto", "coop"])
def test_screened_forces_match_unscreened(b631gs, variant, monkeypatch):
    if variant != "auto":
        monkeypatch.setenv("BSCF_VARIANT", variant)
    from paper_1601_02713_amd import beadscf
    w = inputs.workload("w8_beads", n_beads=2)
    e = beadscf.Engine(0)
    try:
        e.load_basis(b631gs)
        e.set_instances([z for z, _ in w["instances"]])
        e.set_geometries([x for _, x in w["instances"]])
        E, it, st = e.run_scf(e_tol=1e-10, comm_tol=1e-8)
        assert np.all(st == 0)
        F0 = e.forces()
        Ps = [e.density(i) for i in range(e.n_inst)]
        Fs, _ = e.build_fock(Ps)
        Fa = e.forces_at(Ps, Fs, schwarz_tol=1e-12)
        Fb = e.forces_at(Ps, Fs, schwarz_tol=0.0)
    finally:
        e.close()
    for k in range(len(Ps)):
        assert np.abs(Fa[k] - Fb[k]).max() < 1e-9, k
        # the SCF's own forces (same density, its last Fock matrix) agree too
        assert np.abs(F0[k] - Fa[k]).max() < 1e-6, k
        # net force vanishes
        assert np.abs(Fa[k].sum(axis=0)).max() < 1e-8
